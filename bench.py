#!/usr/bin/env python3
"""Benchmark: Fresnel planes/s at 4096^2 c64, forward + adjoint, batched vs plain, with the
dominant kernel's roofline fraction and the FP64 oracle timed on the host as baseline.

Step (one pass of the whole hot path): the Lyot coronagraph train of a 1024 px pupil (10 %
central obscuration, four 1 % D spiders, power-law OPD 10 nm rms) padded 4x to 4096^2, two
48 x 48-actuator DMs (one in the pupil, one after a 1 m Fresnel step), occulter MFT to 256^2
(3 lambda/D spot), Babinet MFT back, Lyot stop 0.9 D, detector MFT to 512^2, over 21
wavelengths uniform in 500-600 nm; broadband PSF plus the gradient of the mean dark-hole
(3-10 lambda/D half annulus) contrast with respect to both DMs' actuator heights. Per step:
21 forward and 21 adjoint Fresnel planes at 4096^2, the forward and adjoint MFTs, the DM
synthesis and the DM-gradient projections. All inputs resident in HBM; data synthetic.
  batched form (`value`): one propagate_train call with FR_TRAIN_BATCHED | FR_TRAIN_GRAPH
      (all wavelengths' Fresnel planes in one launch per sweep, the whole call one graph);
  plain form (reported beside it): the same call wavelength after wavelength.
Also reported: the Fresnel sweeps alone (42 planes at 4096^2 in one batched call) with their
HBM-roofline fraction.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
Prints one JSON line.
"""

import argparse
import json
import os
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

# HBM bytes per launch from two rocprofv3 --pmc runs of this bench (FETCH_SIZE, then WRITE_SIZE,
# KiB per dispatch), scaled by what the counters read for a device copy of one 128 MiB plane in
# the same runs (FETCH x 2.0, WRITE x 1.0); the entries carry the SHA-256 of the sources they
# were measured on (the GEMM kernel and the MFT code that sets up its operands), and read as
# unknown (null) once those sources change.
HERE = os.path.dirname(os.path.abspath(__file__))
MEASURED_TRAFFIC = {
    # kernel: (fetch bytes, write bytes)
    "cgemmB_4096x4096x256_s1": (2.0 * 37108.8 * 1024, 131072.0 * 1024),
    "cgemmB_4096x256x4096_s2": (2.0 * 93270.3 * 1024, 32768.0 * 1024),
}
TRAFFIC_SOURCES = {
    "paper_1806_06467_amd/csrc/mft.hip": "bfc10b5635141374e216a49597db38fc3f4e7fb412e6e860e39b274f731c50fd",
    "paper_1806_06467_amd/csrc/fr_internal.h": "5e4b00d764eb6352a0e1481967570d54e71e042c52209f5262aff17334acfb5d",
    "paper_1806_06467_amd/csrc/api.cpp": "65d43b0ed6ad9c089128aee771c1a9e554fe5701c4219e940224f7d2aaf6129f",
}


def measured_traffic(kernel):
    """Counter-measured HBM bytes per launch of `kernel`, or None (not measured, or measured on
    sources that have changed since)."""
    import hashlib
    if kernel not in MEASURED_TRAFFIC:
        return None
    for rel, digest in TRAFFIC_SOURCES.items():
        try:
            with open(os.path.join(HERE, rel), "rb") as f:
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


def train_inputs(torch, np, synth, dev):
    def f(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    pupil = synth.pupil_amplitude(N_D, 0.1, 0.01)
    opd = synth.power_law_opd(N_D, pupil, 10e-9, -3.0, 0)
    occ = synth.occulter_spot(OCC_M, OCC_DU, 3.0)
    lyot = synth.lyot_stop(N_D, 0.9)
    heights = np.stack([synth.dm_heights(N_ACT, 1 + k) for k in range(2)])
    dh = synth.dark_hole(DET_M, DET_DU, 3.0, 10.0)
    return dict(pupil=f(pupil), opd=f(opd), occ=f(occ), lyot=f(lyot), heights=f(heights),
                dh=dh, lams=[float(x) for x in synth.wavelengths(N_LAMBDA)])


def cpu_baseline(np):
    """The FP64 oracle on a bounded sample of the same step: one wavelength of the train
    (forward + gradient, which contains one forward and one adjoint Fresnel plane at 4096^2)."""
    import oracle
    from paper_1806_06467_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    pupil = synth.pupil_amplitude(N_D, 0.1, 0.01)
    geom = oracle.TrainGeometry(
        n_d=N_D, d_m=D_M, z_m=Z, occ_m=OCC_M, occ_du_c=OCC_DU, det_m=DET_M, det_du_c=DET_DU,
        lambda_c=LAMBDA_C, pupil_amp=pupil, occ_mask=synth.occulter_spot(OCC_M, OCC_DU, 3.0),
        lyot=synth.lyot_stop(N_D, 0.9), pupil_opd=synth.power_law_opd(N_D, pupil, 10e-9, -3.0, 0))
    heights = [synth.dm_heights(N_ACT, 1 + k) for k in range(2)]
    dh = synth.dark_hole(DET_M, DET_DU, 3.0, 10.0)
    lam = float(synth.wavelengths(N_LAMBDA)[N_LAMBDA // 2])
    t0 = time.perf_counter()
    fwd = oracle.train_forward(geom, lam, N, heights, True)
    oracle.train_backward(geom, lam, N, heights, fwd, dh / dh.sum())
    dt = time.perf_counter() - t0
    return {"value": 2.0 / dt, "unit": "Fresnel planes/s", "cores": int(threads), "kind": "oracle",
            "sample": "one wavelength (550 nm) of the step: train forward + gradient with two DMs "
                      "at 4096^2 (1 forward + 1 adjoint Fresnel plane and the MFTs), FP64 oracle "
                      "(explicit DFT matrices, zgemm), %.1f s" % dt}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-file", default=None,
                    help="load tuned kernel choices from this file (written by --save-tune) instead "
                         "of running the autotuner, so that repeated runs launch the same kernels")
    ap.add_argument("--save-tune", default=None, help="write the tuned kernel choices to this file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of one 4096^2 c64 plane (134217728 B read, "
                         "134217728 B written) so HBM byte counters can be scaled")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every wavelength of this workload fits one "
              "MI355X, and the multi-GPU sharding is a design note, not a run; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1806_06467_amd import fresnel as fb
    from paper_1806_06467_amd import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    # autotune (untimed): sweep tiles for the plane edge, GEMM tiles (and split-K factors) for
    # the train's MFT shapes; or the choices of an earlier run
    t_tune = time.perf_counter()
    if args.tune_file:
        fb.autotune_load(args.tune_file)
    else:
        fb.autotune_fresnel(N)
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
    inp = train_inputs(torch, np, synth, dev)
    lams = inp["lams"]
    tr = fb.Train(N_D, D_M, Z, inp["pupil"], inp["lyot"], inp["occ"], OCC_DU, DET_M, DET_DU,
                  LAMBDA_C, inp["opd"], n_act=N_ACT, n_dm=2)
    ns, w = [N] * N_LAMBDA, [1.0 / N_LAMBDA] * N_LAMBDA
    hg = inp["heights"]
    # the reference peak, held fixed in the loss (not differentiated)
    ref0 = fb.propagate_train(tr, lams, ns, w, hg, occulter=False, batched=True)
    dh = inp["dh"]
    g_psf = torch.from_numpy((dh / (dh.sum() * float(ref0.max()))).astype(np.float32)).to(dev)
    psf = torch.empty((DET_M, DET_M), dtype=torch.float32, device=dev)
    gh = torch.empty_like(hg)
    planes_per_step = 2 * N_LAMBDA  # forward + adjoint Fresnel planes

    def batched_step():
        fb.propagate_train(tr, lams, ns, w, hg, grad_psf=g_psf, batched=True, graph=True, out=psf,
                           grad_out=gh)

    def plain_step():
        fb.propagate_train(tr, lams, ns, w, hg, grad_psf=g_psf, out=psf, grad_out=gh)

    def timed(fn, steps, warmup, profile=False):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        if profile:
            fb.profile_read()
            fb.profile_enable(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        prof = None
        if profile:
            fb.profile_enable(False)
            prof = fb.profile_read()
        return e0.elapsed_time(e1), prof

    t_wall0 = time.perf_counter()
    steps = args.steps
    ms_batched, _ = timed(batched_step, steps, args.warmup)
    psf_sum = float(psf.sum())
    n_plain = max(1, steps // 4)
    ms_plain, _ = timed(plain_step, n_plain, 1)
    ms_per_step = ms_batched / steps
    value = planes_per_step * steps / (ms_batched * 1e-3)
    plain_value = planes_per_step * n_plain / (ms_plain * 1e-3)

    # per-kernel times of one step: the batched form run eagerly (the graph replays exactly
    # these launches), each launch bracketed by events
    def eager_batched():
        fb.propagate_train(tr, lams, ns, w, hg, grad_psf=g_psf, batched=True, out=psf, grad_out=gh)

    n_prof = 2
    _, prof = timed(eager_batched, n_prof, 1, profile=True)
    # per kernel name: total ms, launches, and the planes the launches covered (sweep timing
    # tags carry the planes per launch)
    agg = {}
    for k, (tot, cnt) in prof.items():
        name, _, tag = k.partition("/")
        a = agg.setdefault(name, [0.0, 0, 0])
        a[0] += tot
        a[1] += cnt
        a[2] += cnt * (int(tag) if tag.isdigit() else 0)
    kernels_ms_per_step = {k: v[0] / n_prof for k, v in sorted(agg.items(), key=lambda kv: -kv[1][0])}

    # algorithmic cost (per plane for the sweeps, per launch otherwise):
    #   forward row sweep: the pupil optic is synthesised (no field read): write the field,
    #     read the pupil DM map and the two N_D^2 pupil windows;
    #   adjoint row sweep: read + write the field, the same maps (conjugate optic);
    #   column sweeps: read + write the field and the DM map after the step;
    #   dm_grad_T: read E and B (last DM) or B, the pupil DM map and the windows (pupil DM);
    #   cgemm M x N x K: 8 M N K flops against the FP32 MFMA peak, for every tile (the
    #     bfloat16-split tile executes 48 M N K flops on the bf16 matrix cores, reported beside).
    n2, nd2 = N * N, N_D * N_D
    per_plane = {
        "row_sweep": 8 * n2 + 4 * n2 + 8 * nd2,
        "row_sweep_adj": 16 * n2 + 4 * n2 + 8 * nd2,
        "col_sweep": 16 * n2 + 4 * n2,
        "col_sweep_adj": 16 * n2 + 4 * n2,
    }
    per_launch = {"dm_grad_T": 16 * n2, "dm_grad_T_pupil": 8 * n2 + 4 * n2 + 8 * nd2}

    def roofline_of(name):
        tot, cnt, planes = agg[name]
        ms = tot / cnt
        if name in per_plane or name in per_launch:
            nbytes = per_plane[name] * planes / cnt if name in per_plane else per_launch[name]
            gbs = nbytes / (ms * 1e-3) / 1e9
            return {"bound": "hbm", "kernel": name, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": gbs / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": nbytes,
                    "avg_launch_ms": ms}
        if name.startswith("cgemmB"):
            # bfloat16-split tile: the algorithmic work is the complex GEMM's 8 M N K flops, priced
            # against the FP32 MFMA peak (the precision the result is computed to); the tile
            # executes 4 real products x 6 bfloat16 piece products x 2 M N K = 48 M N K flops on
            # the bf16 matrix cores, reported beside it against the dense bf16 peak
            m, n_, k = (int(x) for x in name.split("_")[1].split("x"))
            flops = 8.0 * m * n_ * k
            tf = flops / (ms * 1e-3) / 1e12
            tbf = 48.0 * m * n_ * k / (ms * 1e-3) / 1e12
            return {"bound": "mfma", "kernel": name, "achieved": tf, "peak": FP32_MFMA_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": tf / FP32_MFMA_PEAK_TFLOPS,
                    "traffic": measured_traffic(name), "flops_per_launch": flops, "avg_launch_ms": ms,
                    "executed_on": "bf16 MFMA, exact bfloat16 pieces of the f32 operands",
                    "executed_bf16_tflops": tbf, "executed_frac_of_bf16_peak": tbf / BF16_MFMA_PEAK_TFLOPS}
        if name.startswith("cgemm"):
            m, n_, k = (int(x) for x in name.split("_")[1].split("x"))
            flops = 8.0 * m * n_ * k
            tf = flops / (ms * 1e-3) / 1e12
            return {"bound": "mfma", "kernel": name, "achieved": tf, "peak": FP32_MFMA_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": tf / FP32_MFMA_PEAK_TFLOPS,
                    "traffic": measured_traffic(name), "flops_per_launch": flops, "avg_launch_ms": ms}
        return None

    # the dominant kernel: the largest share of the step that has a cost model
    modelled = [k for k in kernels_ms_per_step if roofline_of(k) is not None]
    roofline = roofline_of(modelled[0])
    kernel_rooflines = {k: roofline_of(k) for k in modelled[:6]}

    # the Fresnel sweeps alone: 42 planes (21 forward, 21 adjoint) of 4096^2 with a dense
    # amplitude + OPD optic in one batched call; per-launch HBM roofline of the sweep kernels
    rng = np.random.default_rng(42)
    amp = torch.from_numpy(rng.uniform(0.99, 1.0, (N, N)).astype(np.float32)).to(dev)
    opd = torch.from_numpy(rng.normal(0.0, 10e-9, (N, N)).astype(np.float32)).to(dev)
    fields = []
    for i in range(2 * N_LAMBDA):
        g = torch.Generator(device=dev)
        g.manual_seed(1000 + i)
        fields.append(torch.randn((N, N), dtype=torch.complex64, device=dev, generator=g))
    adjs = [i >= N_LAMBDA for i in range(2 * N_LAMBDA)]
    lam_pl = [lams[i % N_LAMBDA] for i in range(2 * N_LAMBDA)]
    fr_calls = 10
    ms_fr, prof_fr = timed(lambda: fb.fresnel_step_batched(fields, DX, lam_pl, Z, amps=amp, opds=opd,
                                                           adjoints=adjs), fr_calls, 2, profile=True)
    # both row sweeps apply the amplitude and OPD maps (prologue forward, conjugate epilogue
    # adjoint); the column sweeps move only the fields. Timing tags carry the planes per launch.
    fr_plane = {"row_sweep": sweep_bytes(N, 2), "row_sweep_adj": sweep_bytes(N, 2),
                "col_sweep": sweep_bytes(N, 0), "col_sweep_adj": sweep_bytes(N, 0)}
    fr_agg = {}
    for key, (tot, cnt) in prof_fr.items():
        name, _, tag = key.partition("/")
        if name in fr_plane:
            a = fr_agg.setdefault(name, [0.0, 0, 0])
            a[0] += tot
            a[1] += cnt
            a[2] += cnt * int(tag)
    fr_rl = {}
    for name, (tot, cnt, planes) in fr_agg.items():
        ms = tot / cnt
        nbytes = fr_plane[name] * planes / cnt
        gbs = nbytes / (ms * 1e-3) / 1e9
        fr_rl[name] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": nbytes, "avg_launch_ms": ms}
    # the whole Fresnel plane (both sweeps) against the two-pass model, maps included
    fr_bytes = 2 * N_LAMBDA * (2 * sweep_bytes(N, 0) + 2 * N * N * 4)
    fr_plane_frac = fr_bytes / (ms_fr / fr_calls * 1e-3) / 1e9 / HBM_PEAK_GBS
    # the direct (single-transform) Fresnel step on the forward fields, one plane per call, at
    # twice the distance beyond which its input phase is sampled; both sweeps move only the field
    z_dir = 2.0 * N * DX * DX / min(lams)
    dr_calls = 3

    def direct_all():
        for i in range(N_LAMBDA):
            fb.fresnel_direct(fields[i], DX, lam_pl[i], z_dir)
    ms_dr, prof_dr = timed(direct_all, dr_calls, 1, profile=True)
    dr_rl = {}
    for name in ("direct_rows", "direct_cols"):
        tot = sum(v[0] for k, v in prof_dr.items() if k.partition("/")[0] == name)
        cnt = sum(v[1] for k, v in prof_dr.items() if k.partition("/")[0] == name)
        if cnt:
            ms = tot / cnt
            gbs = sweep_bytes(N, 0) / (ms * 1e-3) / 1e9
            dr_rl[name] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": sweep_bytes(N, 0), "avg_launch_ms": ms}
    dr_planes = N_LAMBDA * dr_calls
    dr_frac = dr_planes * 2 * sweep_bytes(N, 0) / (ms_dr * 1e-3) / 1e9 / HBM_PEAK_GBS
    # the angular-spectrum step with the exact transfer function over the train's distance, one
    # plane per call: three sweeps, each reading and writing the whole field
    ex_calls = 3

    def exact_all():
        for i in range(N_LAMBDA):
            fb.fresnel_step_exact(fields[i], DX, lam_pl[i], Z)
    ms_ex, prof_ex = timed(exact_all, ex_calls, 1, profile=True)
    ex_rl = {}
    for name in ("exact_rows_fwd", "exact_cols", "exact_rows_inv"):
        tot = sum(v[0] for k, v in prof_ex.items() if k.partition("/")[0] == name)
        cnt = sum(v[1] for k, v in prof_ex.items() if k.partition("/")[0] == name)
        if cnt:
            ms = tot / cnt
            gbs = sweep_bytes(N, 0) / (ms * 1e-3) / 1e9
            ex_rl[name] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": sweep_bytes(N, 0), "avg_launch_ms": ms}
    ex_planes = N_LAMBDA * ex_calls
    # the float64 MFT of the occulter plane (4096^2 pupil -> 256^2 focal, n_d = 1024), forward
    # and adjoint: two complex GEMMs each, 8 (m n^2 + m^2 n) flops per call
    e64 = fields[0].to(torch.complex128)
    f64_calls = 3
    f64_out = {}

    def mft64_fwd():
        f64_out["b"] = fb.mft_f64(e64, N_D, OCC_M, OCC_DU)

    def mft64_adj():
        fb.mft_f64(f64_out["b"], N_D, N, OCC_DU, adjoint=True)
    mft64_fwd()
    ms_f64f, _ = timed(mft64_fwd, f64_calls, 1)
    ms_f64a, _ = timed(mft64_adj, f64_calls, 1)
    f64_flops = 8.0 * (OCC_M * N * N + OCC_M * OCC_M * N)
    f64_res = {}
    for name, ms in (("forward", ms_f64f), ("adjoint", ms_f64a)):
        tf = f64_flops / (ms / f64_calls * 1e-3) / 1e12
        f64_res[name] = {"ms_per_call": ms / f64_calls, "achieved": tf, "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS, "flops_per_call": f64_flops}
    del e64, f64_out
    ex_frac = ex_planes * 3 * sweep_bytes(N, 0) / (ms_ex * 1e-3) / 1e9 / HBM_PEAK_GBS
    del fields
    if args.copy_calibration:
        src = torch.randn((N, N), dtype=torch.complex64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall0

    result = {
        "metric": "Fresnel planes/sec at 4096^2 c64 (fwd+adjoint, batched vs plain), %HBM roofline",
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
            "workload": "lyot_train_4096_21lambda_2dm_psf_and_gradient",
            "n": N, "n_d": N_D, "wavelengths_nm": [500, 600, N_LAMBDA], "n_dm": 2, "n_act": N_ACT,
            "occulter": [OCC_M, OCC_DU], "detector": [DET_M, DET_DU], "z_m": Z,
            "fresnel_planes_per_step": planes_per_step,
            "form": "batched: FR_TRAIN_BATCHED | FR_TRAIN_GRAPH, one call per step",
        },
        "plain": {"value": plain_value, "unit": "Fresnel planes/s", "ms_per_step": ms_plain / n_plain},
        "roofline": roofline,
        "kernel_rooflines": kernel_rooflines,
        "kernels_ms_per_step": kernels_ms_per_step,
        "fresnel_only": {
            "value": 2 * N_LAMBDA * fr_calls / (ms_fr * 1e-3), "unit": "Fresnel planes/s",
            "planes_per_call": 2 * N_LAMBDA, "ms_per_call": ms_fr / fr_calls,
            "hbm_frac_whole_plane": fr_plane_frac,
            "roofline": fr_rl,
        },
        "direct_fresnel": {
            "value": dr_planes / (ms_dr * 1e-3), "unit": "Fresnel planes/s", "z_m": z_dir,
            "planes_per_call": 1, "hbm_frac_whole_plane": dr_frac, "roofline": dr_rl,
        },
        "mft_f64_occulter": {"shape": [N, OCC_M], "n_d": N_D, "du": OCC_DU, "bound": "fp64", **f64_res},
        "exact_fresnel": {
            "value": ex_planes / (ms_ex * 1e-3), "unit": "Fresnel planes/s", "z_m": Z,
            "planes_per_call": 1, "hbm_frac_whole_plane": ex_frac, "roofline": ex_rl,
        },
        "autotuned": {"choices": tuned, "seconds": t_tune, "loaded_from_file": bool(args.tune_file)},
        "checksum_psf_sum": psf_sum,
        "wall_s": t_wall,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(np)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
