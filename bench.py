#!/usr/bin/env python3
"""Benchmark: Fresnel planes/s at 4096^2 c64, forward + adjoint, batched vs plain, as a fraction
of the HBM roofline; the FP64 oracle timed on the host beside it.

Step (one pass of the timed workload): 42 Fresnel planes at 4096^2 complex64, 21 forward and
21 adjoint angular-spectrum steps (Sec. 1.1; wavelengths uniform over 500-600 nm as in the
broadband model of Sec. 1.2, z = 1 m, pitch 25 um), each with a dense optic (Eq. 3: amplitude and
OPD maps of the whole plane, read by the row sweep), on 42 fields resident in HBM.
  batched form (`value`): one fresnel_step_batched_graph call per step (the call's launches
      recorded once as a graph and replayed);
  plain form: 42 fresnel_step calls per step, stream-ordered, no graph.
Beside it: per-iteration spread (median / IQR over 50 steps) and the paper's own timing style
(mean +- sigma over 7 runs); the same 42 planes on 512^2 grids, batched against plain (where
the launches, not the sweeps, set the plain form's time); the same 42 planes on the uneven
per-wavelength grids 3584..4096 (bytes-weighted); the whole Lyot coronagraph train with two DMs, PSF and gradient (the rest of
the hot path: MFTs, PSF accumulation, DM synthesis and adjoint) as a secondary figure; the
direct and exact-transfer-function steps (the exact one also batched); the App. B relay analogue
at 4096^2; the float64 Fresnel plane and MFT; a device-copy ceiling.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
                [--save-tune FILE | --tune-file FILE] [--copy-calibration]
Prints one JSON line.
"""

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 4096
N_D = 1024
N_LAMBDA = 21
N_ACT = 48
D_M = N_D * 25e-6
DX = D_M / N_D
Z = 1.0
OCC_M, OCC_DU = 256, 8.0 / 256
DET_M, DET_DU = 512, 0.25
LAMBDA_C = 550e-9
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense
FP64_PEAK_TFLOPS = 78.6  # vector and matrix alike
METRIC = "Fresnel planes/sec at 4096^2 c64 (fwd+adjoint, batched vs plain), %HBM roofline"

# HBM bytes per launch (fetched, written) of the sweep kernels of the timed batch from two
# rocprofv3 --pmc runs of this bench (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, averaged over
# the 1344 launches of each direction), scaled by what the counters read for a device copy of one
# 128 MiB plane in the same runs (FETCH x 2.0, WRITE x 1.0). Each entry carries the SHA-256 of the
# sources it was measured on and reads as unknown (null) once they change.
MEASURED_TRAFFIC = {
    "row_sweep": (269218249, 134217728),
    "col_sweep": (136636795, 165001379),
    "col_sweep_adj": (136488486, 167391150),
    "row_sweep_adj": (269255542, 134217728),
}
_SWEEP_SOURCES = {
    "paper_1806_06467_amd/csrc/sweeps.hip": "98e23daf76c939ad81ff8b609719321fd595eab8fd48228ec815f5a9aed09750",
    "paper_1806_06467_amd/csrc/fft_line.hpp": "66f504dc38f9cb71c51b0dd9e259e966acb90c9d9d1b256d8d7ca415edac6fae",
    "paper_1806_06467_amd/csrc/dft_small.hpp": "f079518edd36aa105b5a40ce60935e1cdb8f3c06c3c59d0fa46a65eea89b7209",
    "paper_1806_06467_amd/csrc/fr_internal.h": "02c3e065cf6306f08322cfd1ba1a1b4c9e8d4cd9567bdc661d2d3afd895ca19a",
}
TRAFFIC_SOURCES = {k: _SWEEP_SOURCES for k in MEASURED_TRAFFIC}


def measured_traffic(kernel):
    """Counter-measured HBM bytes per launch of `kernel`, or None (not measured, or measured on
    sources that have changed since)."""
    if kernel not in MEASURED_TRAFFIC:
        return None
    for rel, digest in TRAFFIC_SOURCES.get(kernel, {}).items():
        try:
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
        except OSError:
            return None
    fetch, write = MEASURED_TRAFFIC[kernel]
    return fetch + write


def sweep_bytes(n, optic_maps):
    """Algorithmic HBM bytes of one sweep of one plane: the n^2 c64 field read and written once,
    plus one read of each float n^2 map the sweep applies."""
    return 2 * n * n * 8 + optic_maps * n * n * 4


def plane_bytes(n, optic_maps=2):
    """Two sweeps per angular-spectrum step (the paraxial transfer function is separable), the
    optic maps read once (by the row sweep)."""
    return 2 * sweep_bytes(n, 0) + optic_maps * n * n * 4


def host_info():
    """CPU model, BLAS library and thread count the oracle runs with."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas, threads = "unknown", len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        libs = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if libs:
            blas = "%s %s (%s)" % (libs[0].get("internal_api"), libs[0].get("version"),
                                   libs[0].get("architecture"))
            threads = int(libs[0].get("num_threads", threads))
    except Exception:
        pass
    return model, blas, threads


def cpu_baseline(np):
    """The FP64 oracle on a bounded sample of the step: one forward and one adjoint Fresnel plane
    at 4096^2 with the same dense optic (explicit DFT matrices, four complex GEMMs per plane)."""
    import oracle
    model, blas, threads = host_info()
    rng = np.random.default_rng(7)
    u = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    amp = rng.uniform(0.99, 1.0, (N, N))
    opd = rng.normal(0.0, 10e-9, (N, N))
    t0 = time.perf_counter()
    oracle.fresnel_step(u, DX, LAMBDA_C, Z, amp=amp, opd=opd)
    oracle.fresnel_step(u, DX, LAMBDA_C, Z, amp=amp, opd=opd, adjoint=True)
    dt = time.perf_counter() - t0
    return {"value": 2.0 / dt, "unit": "Fresnel planes/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "blas": blas,
            "sample": "one forward and one adjoint fresnel_step at 4096^2 (550 nm, z = 1 m, dense "
                      "amplitude and OPD maps), FP64 oracle: explicit DFT matrices (built in the "
                      "timed region), four complex GEMMs per plane; %.1f s" % dt}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the headline Fresnel batch (for profiler runs)")
    ap.add_argument("--tune-file", default=None,
                    help="load tuned kernel choices from this file (written by --save-tune) instead "
                         "of running the autotuner, so that repeated runs launch the same kernels")
    ap.add_argument("--save-tune", default=None,
                    help="write the tuned kernel choices to this file (at the end of the run, so that "
                         "the 8192^2 train's own choices are in it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of one 4096^2 c64 plane (134217728 B read, "
                         "134217728 B written) so HBM byte counters can be scaled")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X (sharding the "
              "wavelengths over several GPUs is described in the design notes, not implemented); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1806_06467_amd import fresnel as fb
    from paper_1806_06467_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    t_wall0 = time.perf_counter()

    # autotune (untimed): sweep tiles for the plane edges, GEMM tiles (and split-K factors) for
    # the train's MFT shapes; or the choices of an earlier run
    t_tune = time.perf_counter()
    if args.tune_file:
        fb.autotune_load(args.tune_file)
    else:
        fb.autotune_fresnel(N)
        if not args.no_extras:
            for n_, m_ in ((N, OCC_M), (N_D, OCC_M), (N_D, DET_M)):
                fb.autotune_mft(n_, m_)
    tune_file = args.save_tune or os.path.join(os.environ.get("TMPDIR", "/tmp"),
                                               "fresnel_bench_tune_%d.txt" % os.getpid())
    fb.autotune_save(tune_file)
    with open(tune_file) as f:
        tuned = [l.strip() for l in f if not l.startswith("#")]
    if not args.save_tune:
        os.remove(tune_file)
    t_tune = time.perf_counter() - t_tune

    def sync():
        torch.cuda.synchronize()

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        sync()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        sync()
        return e0.elapsed_time(e1)

    def per_iteration(fn, iters):
        """ms of each of `iters` consecutive calls (events between calls)."""
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(iters + 1)]
        ev[0].record(stream)
        for i in range(iters):
            fn()
            ev[i + 1].record(stream)
        sync()
        return [ev[i].elapsed_time(ev[i + 1]) for i in range(iters)]

    def profiled(fn, calls):
        """per kernel name: [total ms, launches, planes covered] over `calls` calls, from the
        library's per-launch HIP events on the launch stream (timing tags carry the planes per
        launch)"""
        fn()
        sync()
        fb.profile_read()
        fb.profile_enable(True)
        for _ in range(calls):
            fn()
        sync()
        fb.profile_enable(False)
        agg = {}
        for k, (tot, cnt) in fb.profile_read().items():
            name, _, tag = k.partition("/")
            a = agg.setdefault(name, [0.0, 0, 0])
            a[0] += tot
            a[1] += cnt
            a[2] += cnt * (int(tag) if tag.isdigit() else 0)
        return agg

    def hbm_entry(name, nbytes, ms, extra=None):
        gbs = nbytes / (ms * 1e-3) / 1e9
        d = {"bound": "hbm", "kernel": name, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic(name), "bytes_per_launch": nbytes,
             "avg_launch_ms": ms}
        if extra:
            d.update(extra)
        return d

    # ---- headline: 42 planes at 4096^2, 21 forward + 21 adjoint, dense optic ----------------
    lams = [float(x) for x in synth.wavelengths(N_LAMBDA)]
    rng = np.random.default_rng(42)
    amp = torch.from_numpy(rng.uniform(0.99, 1.0, (N, N)).astype(np.float32)).to(dev)
    opd = torch.from_numpy(rng.normal(0.0, 10e-9, (N, N)).astype(np.float32)).to(dev)
    n_pl = 2 * N_LAMBDA
    fields = []
    for i in range(n_pl):
        g = torch.Generator(device=dev)
        g.manual_seed(1000 + i)
        fields.append(torch.randn((N, N), dtype=torch.complex64, device=dev, generator=g))
    adjs = [i >= N_LAMBDA for i in range(n_pl)]
    lam_pl = [lams[i % N_LAMBDA] for i in range(n_pl)]

    def batched(graph=True):
        fb.fresnel_step_batched(fields, DX, lam_pl, Z, amps=amp, opds=opd, adjoints=adjs, graph=graph)

    def plain():
        for i in range(n_pl):
            fb.fresnel_step(fields[i], DX, lam_pl[i], Z, amp=amp, opd=opd, adjoint=adjs[i])

    steps = args.steps
    ms_batched = timed(batched, steps, args.warmup)
    ms_per_step = ms_batched / steps
    value = n_pl * steps / (ms_batched * 1e-3)
    ms_plain = timed(plain, steps, 1)
    plain_value = n_pl * steps / (ms_plain * 1e-3)
    bytes_step = n_pl * plane_bytes(N)
    field_bytes_step = n_pl * plane_bytes(N, 0)

    def frac_of(ms_step, nbytes):
        return nbytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS

    # per-kernel durations of the same launches (the graph replays exactly these)
    agg = profiled(lambda: batched(graph=False), 3)
    # algorithmic bytes per plane of each sweep kernel: the row sweeps read the amplitude and OPD
    # maps (prologue forward, conjugate epilogue adjoint), the column sweeps move only the field
    fr_plane = {"row_sweep": sweep_bytes(N, 2), "row_sweep_adj": sweep_bytes(N, 2),
                "col_sweep": sweep_bytes(N, 0), "col_sweep_adj": sweep_bytes(N, 0)}
    sweeps = {}
    for name, (tot, cnt, planes) in agg.items():
        if name in fr_plane and cnt:
            sweeps[name] = hbm_entry(name, fr_plane[name] * planes / cnt, tot / cnt,
                                     {"ms_per_step": tot / 3, "planes_per_launch": planes / cnt})
    dominant = max(sweeps, key=lambda k: sweeps[k]["ms_per_step"])
    roofline = dict(sweeps[dominant])
    roofline["whole_plane"] = {
        "bytes_per_plane": plane_bytes(N), "field_only_bytes_per_plane": plane_bytes(N, 0),
        "frac": frac_of(ms_per_step, bytes_step), "field_only_frac": frac_of(ms_per_step, field_bytes_step),
        "roofline_planes_per_s_field_only": HBM_PEAK_GBS * 1e9 / plane_bytes(N, 0),
        "note": "two sweeps per plane, each reading and writing the field once (+ the two optic "
                "maps, read once); time per plane from the batched step"}

    # spread: 50 single steps, and the paper's style (7 runs, mean +- sigma)
    it = per_iteration(batched, 50)
    q = statistics.quantiles(it, n=4)
    runs = [timed(batched, steps, 0) / steps for _ in range(7)]
    timing = {"iterations": 50, "median_ms": statistics.median(it), "iqr_ms": [q[0], q[2]],
              "runs7_mean_ms": statistics.mean(runs), "runs7_sigma_ms": statistics.stdev(runs),
              "runs7_steps_each": steps}
    result_extra = {}

    # ---- the same 42 planes on small grids (512^2, the first configuration's padded grid), ----
    # ---- where a plane's sweeps take microseconds and the launches dominate the plain form ----
    if not args.no_extras:
        ns_ = 512
        r = np.random.default_rng(512)
        amp_s = torch.from_numpy(r.uniform(0.99, 1.0, (ns_, ns_)).astype(np.float32)).to(dev)
        opd_s = torch.from_numpy(r.normal(0.0, 10e-9, (ns_, ns_)).astype(np.float32)).to(dev)
        sfields = []
        for i in range(n_pl):
            g = torch.Generator(device=dev)
            g.manual_seed(3000 + i)
            sfields.append(torch.randn((ns_, ns_), dtype=torch.complex64, device=dev, generator=g))
        dx_s, z_s = 1e-4, 1.0

        def small_batched():
            fb.fresnel_step_batched(sfields, dx_s, lam_pl, z_s, amps=amp_s, opds=opd_s, adjoints=adjs, graph=True)

        def small_plain():
            for i in range(n_pl):
                fb.fresnel_step(sfields[i], dx_s, lam_pl[i], z_s, amp=amp_s, opd=opd_s, adjoint=adjs[i])
        s_steps = max(10, steps)
        ms_sb = timed(small_batched, s_steps, 3) / s_steps
        ms_sp = timed(small_plain, s_steps, 2) / s_steps
        result_extra["small_grid_batching"] = {
            "n": ns_, "planes_per_step": n_pl,
            "batched": {"value": n_pl / (ms_sb * 1e-3), "unit": "Fresnel planes/s", "ms_per_step": ms_sb,
                        "form": "one fresnel_step_batched_graph call (all 42 planes in one cache-sized group: "
                                "four launches)"},
            "plain": {"value": n_pl / (ms_sp * 1e-3), "unit": "Fresnel planes/s", "ms_per_step": ms_sp,
                      "form": "42 fresnel_step calls (84 launches)"},
            "batched_over_plain": ms_sp / ms_sb}
        del sfields, amp_s, opd_s

    # ---- uneven per-wavelength grids (3584..4096), forward + adjoint, bytes-weighted ---------
    if not args.no_extras:
        sizes = synth.padded_sizes(N_LAMBDA)
        maps = {}
        for n_ in sorted(set(sizes)):
            r = np.random.default_rng(n_)
            maps[n_] = (torch.from_numpy(r.uniform(0.99, 1.0, (n_, n_)).astype(np.float32)).to(dev),
                        torch.from_numpy(r.normal(0.0, 10e-9, (n_, n_)).astype(np.float32)).to(dev))
        ufields = []
        for i in range(n_pl):
            g = torch.Generator(device=dev)
            g.manual_seed(2000 + i)
            n_ = sizes[i % N_LAMBDA]
            ufields.append(torch.randn((n_, n_), dtype=torch.complex64, device=dev, generator=g))
        ua = [maps[sizes[i % N_LAMBDA]][0] for i in range(n_pl)]
        uo = [maps[sizes[i % N_LAMBDA]][1] for i in range(n_pl)]
        ubytes = sum(plane_bytes(sizes[i % N_LAMBDA]) for i in range(n_pl))

        def uneven(graph=True):
            fb.fresnel_step_batched(ufields, DX, lam_pl, Z, amps=ua, opds=uo, adjoints=adjs, graph=graph)

        def uneven_plain():
            for i in range(n_pl):
                fb.fresnel_step(ufields[i], DX, lam_pl[i], Z, amp=ua[i], opd=uo[i], adjoint=adjs[i])
        u_steps = max(1, steps // 2)
        ms_u = timed(uneven, u_steps, 2) / u_steps
        ms_up = timed(uneven_plain, u_steps, 1) / u_steps
        result_extra["uneven_grids"] = {
            "sizes": sizes, "planes_per_step": n_pl, "algorithmic_bytes_per_step": ubytes,
            "batched": {"value": n_pl / (ms_u * 1e-3), "unit": "Fresnel planes/s", "ms_per_step": ms_u,
                        "hbm_frac_bytes_weighted": frac_of(ms_u, ubytes)},
            "plain": {"value": n_pl / (ms_up * 1e-3), "unit": "Fresnel planes/s", "ms_per_step": ms_up,
                      "hbm_frac_bytes_weighted": frac_of(ms_up, ubytes)},
            "note": "the 4096^2 planes take the power-of-two sweeps, 3584, 3600, 3840 and 4032 the "
                    "register-resident mixed-radix sweeps, 3888, 3920 and 4000 the persistent ones "
                    "(in the batched form one launch per sweep for each group)"}
        del ufields, ua, uo, maps

    # ---- device-copy ceiling: 1 GiB copied (2 GiB moved), beyond the last-level cache ----------
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    ms_copy = timed(lambda: dst.copy_(src), 10, 2) / 10
    copy_gbs = 2.0 * src.numel() * 4 / (ms_copy * 1e-3) / 1e9
    del src, dst
    if args.copy_calibration:
        a = torch.randn((N, N), dtype=torch.complex64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        sync()
        del a, b

    if not args.no_extras:
        # ---- the whole coronagraph train (secondary): two DMs, PSF + gradient, 21 wavelengths --
        result_extra["train_step"] = train_step(args, fb, synth, np, torch, dev, timed, profiled, lams)
        result_extra["train_8192"] = train_8192(fb, synth, np, torch, dev, timed, profiled, not args.tune_file)
        # ---- the direct and exact-transfer-function steps, one plane per call ------------------
        z_dir = 2.0 * N * DX * DX / min(lams)

        def direct_all():
            for i in range(N_LAMBDA):
                fb.fresnel_direct(fields[i], DX, lam_pl[i], z_dir)
        ms_dr = timed(direct_all, 3, 1)
        adr = profiled(direct_all, 1)
        result_extra["direct_fresnel"] = {
            "value": 3 * N_LAMBDA / (ms_dr * 1e-3), "unit": "Fresnel planes/s", "z_m": z_dir,
            "hbm_frac_whole_plane": frac_of(ms_dr / (3 * N_LAMBDA), plane_bytes(N, 0)),
            "sweeps": {k: hbm_entry(k, sweep_bytes(N, 0), v[0] / v[1]) for k, v in adr.items()
                       if k.startswith("direct_") and v[1]}}

        def exact_all():
            for i in range(N_LAMBDA):
                fb.fresnel_step_exact(fields[i], DX, lam_pl[i], Z)

        def exact_batched():
            fb.fresnel_step_exact_batched(fields[:N_LAMBDA], DX, lam_pl[:N_LAMBDA], Z)
        ms_ex = timed(exact_all, 5, 1)
        ms_exb = timed(exact_batched, 5, 1)
        aex = profiled(exact_all, 1)
        result_extra["exact_fresnel"] = {
            "value": 5 * N_LAMBDA / (ms_ex * 1e-3), "unit": "Fresnel planes/s", "z_m": Z,
            "batched": {"value": 5 * N_LAMBDA / (ms_exb * 1e-3), "unit": "Fresnel planes/s",
                        "form": "one fresnel_step_exact_batched call for the 21 planes"},
            "hbm_frac_whole_plane": frac_of(ms_ex / (5 * N_LAMBDA), 3 * sweep_bytes(N, 0)),
            "sweeps": {k: hbm_entry(k, sweep_bytes(N, 0), v[0] / v[1]) for k, v in aex.items()
                       if k.startswith("exact_") and v[1]}}
        # ---- the App. B relay at 4096^2 (the system the paper's Fig. 2 times per wavelength):
        # aperture + primary, relay lenses, a shaped pupil, a bow-tie focal-plane mask, the focus
        d_prim, d_relay = 2.37, 0.02
        f1 = d_prim * 7.8
        f2, f3 = f1 * d_relay / d_prim, 20.0 * d_relay
        zf = [(0.0, f1), (f1 + f2, f2), (f2 + f3, f3), (2 * f3, f3), (f3, 0.0), (f3, f3), (f3, 0.0),
              (2 * f3, f3), (f3 + 0.39999923, 0.0)]
        dx_r = d_prim / (N // 4)
        pitches, transforms = fb.plan_system(N, dx_r, LAMBDA_C, d_prim / 2, [(z, f, None, None) for z, f in zf])

        def g32(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
        masks = {0: g32(synth.embed_centred(synth.pupil_amplitude(N // 4, 0.1, 0.01), N)),
                 4: g32(synth.embed_centred(synth.shaped_pupil(int(round(d_relay / pitches[4]))), N)),
                 6: g32(synth.bowtie_mask(N, LAMBDA_C * f3 / d_relay / pitches[6]))}
        r_optics = [(z, f, masks.get(i), None) for i, (z, f) in enumerate(zf)]
        r_field = torch.ones((N, N), dtype=torch.complex64, device=dev)

        def relay():
            r_field.fill_(1.0)
            fb.propagate_system(r_field, dx_r, LAMBDA_C, d_prim / 2, r_optics)
        ms_relay = timed(relay, 5, 1) / 5
        result_extra["relay_appendix_b"] = {
            "n": N, "optics": len(zf), "transforms_per_wavelength": transforms, "ms_per_wavelength": ms_relay,
            "systems_per_s": 1e3 / ms_relay,
            "context": "Fig. 2 of the paper: 90.16 s per wavelength for its App. B system at N = 4096 "
                       "(NumPy, float64, 8-core 2 GHz Xeon); this run is float32 on one MI355X "
                       "(the whole system including the field reset)"}
        del masks, r_optics, r_field
        # ---- the Fresnel plane in float64 (the paper's precision): 8 forward + 8 adjoint planes at
        # 4096^2 complex128 with float64 amplitude and OPD maps, one call each ------------------
        n64 = 8
        amp64, opd64 = amp.double(), opd.double()
        f64f = [fields[i].to(torch.complex128) for i in range(2 * n64)]

        def f64_planes():
            for i in range(2 * n64):
                fb.fresnel_step_f64(f64f[i], DX, lam_pl[i], Z, amp=amp64, opd=opd64, adjoint=i >= n64)
        ms_64 = timed(f64_planes, 2, 1) / 2
        a64 = profiled(f64_planes, 1)
        b64 = 2 * (2 * N * N * 16) + 2 * N * N * 8   # two sweeps of the c128 field, two float64 maps
        result_extra["fresnel_f64"] = {
            "value": 2 * n64 / (ms_64 * 1e-3), "unit": "Fresnel planes/s", "dtype": "c128",
            "planes_per_step": 2 * n64, "hbm_frac_whole_plane": frac_of(ms_64 / (2 * n64), b64),
            "bytes_per_plane": b64,
            "sweeps": {k: hbm_entry(k, 2 * N * N * 16 + (2 * N * N * 8 if k.startswith("row") else 0), v[0] / v[1])
                       for k, v in a64.items() if "sweep64" in k and v[1]}}
        del f64f, amp64, opd64
        # ---- the float64 MFT of the occulter plane (4096^2 -> 256^2), forward and adjoint -------
        e64 = fields[0].to(torch.complex128)
        out64 = {}

        def f64_fwd():
            out64["b"] = fb.mft_f64(e64, N_D, OCC_M, OCC_DU)

        def f64_adj():
            fb.mft_f64(out64["b"], N_D, N, OCC_DU, adjoint=True)
        f64_fwd()
        f64_flops = 8.0 * (OCC_M * N * N + OCC_M * OCC_M * N)
        f64 = {"shape": [N, OCC_M], "n_d": N_D, "du": OCC_DU, "bound": "fp64"}
        for name, fn in (("forward", f64_fwd), ("adjoint", f64_adj)):
            ms = timed(fn, 3, 1) / 3
            tf = f64_flops / (ms * 1e-3) / 1e12
            f64[name] = {"ms_per_call": ms, "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / FP64_PEAK_TFLOPS, "flops_per_call": f64_flops}
        result_extra["mft_f64_occulter"] = f64
        del e64, out64
    del fields
    t_wall = time.perf_counter() - t_wall0

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "Fresnel planes/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "fresnel_step_4096_c64_21fwd_21adj_dense_optic",
            "n": N, "dx_m": DX, "z_m": Z, "wavelengths_nm": [500, 600, N_LAMBDA],
            "planes_per_step": n_pl, "optic": "amplitude + OPD maps (4096^2 float each)",
            "form": "batched: one fresnel_step_batched_graph call per step (42 planes, recorded once, "
                    "replayed)",
        },
        "plain": {"value": plain_value, "unit": "Fresnel planes/s", "ms_per_step": ms_plain / steps,
                  "form": "42 fresnel_step calls per step, stream-ordered, no graph",
                  "hbm_frac_whole_plane": frac_of(ms_plain / steps, bytes_step)},
        "batched_over_plain": value / plain_value,
        "roofline": roofline,
        "sweep_rooflines": sweeps,
        "timing": timing,
        "hbm_copy_ceiling": {"achieved": copy_gbs, "unit": "GB/s", "frac": copy_gbs / HBM_PEAK_GBS,
                             "what": "torch device copy of 1 GiB (2 GiB moved)"},
    }
    result.update(result_extra)
    result["autotuned"] = {"choices": tuned, "seconds": t_tune, "loaded_from_file": bool(args.tune_file)}
    if args.save_tune:
        fb.autotune_save(args.save_tune)
    result["wall_s"] = t_wall
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(np)
    print(json.dumps(result), flush=True)


def train_step(args, fb, synth, np, torch, dev, timed, profiled, lams):
    """The Lyot coronagraph train of a 1024 px pupil (10 % central obscuration, four 1 % D
    spiders, power-law OPD 10 nm rms) padded 4x to 4096^2, two 48 x 48-actuator DMs (pupil and
    after the 1 m step), occulter MFT to 256^2 (3 lambda/D spot), Babinet MFT back, Lyot stop
    0.9 D, detector MFT to 512^2, 21 wavelengths; broadband PSF plus the gradient of the mean
    dark-hole contrast with respect to both DMs. Batched + graph and plain forms, the per-kernel
    breakdown, and the GEMM tiles priced against the peak of the precision they execute in."""

    def f(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    pupil = synth.pupil_amplitude(N_D, 0.1, 0.01)
    tr = fb.Train(N_D, D_M, Z, f(pupil), f(synth.lyot_stop(N_D, 0.9)), f(synth.occulter_spot(OCC_M, OCC_DU, 3.0)),
                  OCC_DU, DET_M, DET_DU, LAMBDA_C, f(synth.power_law_opd(N_D, pupil, 10e-9, -3.0, 0)),
                  n_act=N_ACT, n_dm=2)
    ns, w = [N] * N_LAMBDA, [1.0 / N_LAMBDA] * N_LAMBDA
    hg = f(np.stack([synth.dm_heights(N_ACT, 1 + k) for k in range(2)]))
    ref0 = fb.propagate_train(tr, lams, ns, w, hg, occulter=False, batched=True)
    dh = synth.dark_hole(DET_M, DET_DU, 3.0, 10.0)
    g_psf = torch.from_numpy((dh / (dh.sum() * float(ref0.max()))).astype(np.float32)).to(dev)
    psf = torch.empty((DET_M, DET_M), dtype=torch.float32, device=dev)
    gh = torch.empty_like(hg)

    def batched():
        fb.propagate_train(tr, lams, ns, w, hg, grad_psf=g_psf, batched=True, graph=True, out=psf, grad_out=gh)

    def plain():
        fb.propagate_train(tr, lams, ns, w, hg, grad_psf=g_psf, out=psf, grad_out=gh)
    k = max(2, args.steps // 2)
    ms_b = timed(batched, k, 2) / k
    ms_p = timed(plain, max(1, k // 2), 1) / max(1, k // 2)
    # the gradient in two calls (an autograd forward / backward pair): the forward keeps the
    # checkpoint, the backward runs only the adjoint chain; against one forward + gradient call
    ck = torch.empty(fb.train_ckpt_bytes(tr, ns), dtype=torch.uint8, device=dev)

    def save_then_backward():
        fb.propagate_train(tr, lams, ns, w, hg, batched=True, out=psf, ckpt=ck, phase="save")
        fb.propagate_train(tr, lams, ns, w, hg, grad_psf=g_psf, batched=True, grad_out=gh, ckpt=ck,
                           phase="backward")

    def one_call():
        fb.propagate_train(tr, lams, ns, w, hg, grad_psf=g_psf, batched=True, out=psf, grad_out=gh)

    def forward_only():
        fb.propagate_train(tr, lams, ns, w, hg, batched=True, out=psf)
    ms_two = timed(save_then_backward, k, 1) / k
    ms_one = timed(one_call, k, 1) / k
    ms_fwd = timed(forward_only, k, 1) / k
    del ck
    agg = profiled(lambda: fb.propagate_train(tr, lams, ns, w, hg, grad_psf=g_psf, batched=True, out=psf,
                                              grad_out=gh), 2)
    per_step = {name: v[0] / 2 for name, v in sorted(agg.items(), key=lambda kv: -kv[1][0])}
    gemms = {}
    for name, (tot, cnt, _) in agg.items():
        if not name.startswith("cgemm") or not cnt:
            continue
        m, n_, kk = (int(x) for x in name.split("_")[1].split("x"))
        ms = tot / cnt
        fl = 8.0 * m * n_ * kk
        tf = fl / (ms * 1e-3) / 1e12
        if name.startswith("cgemmB"):
            # the bfloat16-split tile runs on the bf16 matrix cores: 4 real products x 6 bfloat16
            # piece products x 2 M N K = 48 M N K executed flops for the 8 M N K of the method
            ex = 48.0 * m * n_ * kk / (ms * 1e-3) / 1e12
            gemms[name] = {"bound": "mfma", "dtype": "bf16 (exact pieces of f32)", "avg_launch_ms": ms,
                           "method_tflops": tf, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": tf / BF16_MFMA_PEAK_TFLOPS, "executed_tflops": ex,
                           "executed_frac": ex / BF16_MFMA_PEAK_TFLOPS}
        else:
            gemms[name] = {"bound": "mfma", "dtype": "f32", "avg_launch_ms": ms, "method_tflops": tf,
                           "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / FP32_MFMA_PEAK_TFLOPS}
    top = dict(list(per_step.items())[:12])
    return {"workload": "lyot_train_4096_21lambda_2dm_psf_and_gradient", "fresnel_planes_per_step": 2 * N_LAMBDA,
            "batched_graph": {"ms_per_step": ms_b, "fresnel_planes_per_s": 2 * N_LAMBDA / (ms_b * 1e-3)},
            "plain": {"ms_per_step": ms_p, "fresnel_planes_per_s": 2 * N_LAMBDA / (ms_p * 1e-3)},
            "gradient_two_calls": {"forward_save_plus_backward_ms": ms_two, "one_call_ms": ms_one,
                                   "forward_only_ms": ms_fwd,
                                   "note": "batched eager calls; the backward reads the forward's checkpoint "
                                           "(per wavelength the last-DM plane and the detector field)"},
            "kernels_ms_per_step": top, "gemm_rooflines": gemms,
            "checksum_psf_sum": float(psf.sum())}


def train_8192(fb, synth, np, torch, dev, timed, profiled, tune=True):
    """The large batched forward + adjoint: a 2048 px pupil (pitch 12.5 um) padded 4x to 8192^2
    (512 MiB per plane), two 64 x 64-actuator DMs 1 m apart, 8 wavelengths over 500-600 nm, the
    occulter, Lyot stop and detector of the 4096^2 train; the PSF and the gradient of the mean
    dark-hole contrast with respect to the 8192 actuators, batched + graph, plain, and in two
    calls through the caller's checkpoint (forward save, then backward)."""
    nd, n, nl, na = 2048, 8192, 8, 64
    # tuned (untimed) for its own shapes: the 8192 sweeps and the MFT GEMMs of its planes (unless
    # the choices were loaded from a file)
    t0 = time.perf_counter()
    if tune:
        fb.autotune_fresnel(n)
        for n_, m_ in ((n, OCC_M), (nd, OCC_M), (nd, DET_M)):
            fb.autotune_mft(n_, m_)
    t_tune = time.perf_counter() - t0

    def f(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    pupil = synth.pupil_amplitude(nd, 0.1, 0.01)
    tr = fb.Train(nd, nd * 12.5e-6, Z, f(pupil), f(synth.lyot_stop(nd, 0.9)),
                  f(synth.occulter_spot(OCC_M, OCC_DU, 3.0)), OCC_DU, DET_M, DET_DU, LAMBDA_C,
                  f(synth.power_law_opd(nd, pupil, 10e-9, -3.0, 0)), n_act=na, n_dm=2)
    lams8 = [float(x) for x in synth.wavelengths(nl)]
    ns, w = [n] * nl, [1.0 / nl] * nl
    hg = f(np.stack([synth.dm_heights(na, 1 + k) for k in range(2)]))
    dh = synth.dark_hole(DET_M, DET_DU, 3.0, 10.0)
    g_psf = f(dh / dh.sum())
    psf = torch.empty((DET_M, DET_M), dtype=torch.float32, device=dev)
    gh = torch.empty_like(hg)
    ck = torch.empty(fb.train_ckpt_bytes(tr, ns), dtype=torch.uint8, device=dev)

    def batched():
        fb.propagate_train(tr, lams8, ns, w, hg, grad_psf=g_psf, batched=True, graph=True, out=psf, grad_out=gh)

    def plain():
        fb.propagate_train(tr, lams8, ns, w, hg, grad_psf=g_psf, out=psf, grad_out=gh)

    def two_calls():
        fb.propagate_train(tr, lams8, ns, w, hg, batched=True, out=psf, ckpt=ck, phase="save")
        fb.propagate_train(tr, lams8, ns, w, hg, grad_psf=g_psf, batched=True, grad_out=gh, ckpt=ck,
                           phase="backward")
    ms_b = timed(batched, 2, 1) / 2
    ms_p = timed(plain, 1, 1)
    ms_two = timed(two_calls, 1, 1)
    del ck
    # per-kernel breakdown of one eager batched call (the graph replays the same launches)
    agg = profiled(lambda: fb.propagate_train(tr, lams8, ns, w, hg, grad_psf=g_psf, batched=True, out=psf,
                                              grad_out=gh), 1)
    top = {name: v[0] for name, v in sorted(agg.items(), key=lambda kv: -kv[1][0])[:10]}
    planes = 2 * nl
    return {"workload": "lyot_train_8192_8lambda_2dm_64act_psf_and_gradient", "fresnel_planes_per_step": planes,
            "batched_graph": {"ms_per_step": ms_b, "fresnel_planes_per_s": planes / (ms_b * 1e-3)},
            "plain": {"ms_per_step": ms_p, "fresnel_planes_per_s": planes / (ms_p * 1e-3)},
            "checkpointed_two_calls_ms": ms_two, "autotune_seconds": t_tune, "kernels_ms_per_step": top,
            "checksum_psf_sum": float(psf.sum())}


if __name__ == "__main__":
    main()
