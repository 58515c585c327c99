#!/usr/bin/env python3
"""Benchmark: Fresnel planes/s at 4096^2 c64, forward + adjoint, batched vs plain, with the
dominant kernel's HBM-roofline fraction and the FP64 oracle timed on the host as baseline.

Workload (one step): 21 wavelengths uniform over 500-600 nm, each with one forward Fresnel
plane and one adjoint plane on a dense 4096^2 complex64 field: the optic prologue (amplitude
map and power-law OPD phasor of a 1024 px pupil geometry padded 4x, dx = 25 um) then the
angular-spectrum step over z = 1 m. 42 planes per step, all resident in HBM.
  batched form (timed, `value`): one fresnel_step_batched call per step (one launch per sweep);
  plain form (reported beside it): one fresnel_step call per plane, stream-ordered.

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
DX = 25.6e-3 / N_D
Z = 1.0
HBM_PEAK_GBS = 8000.0


def plane_bytes(n, optic_reads):
    """Algorithmic HBM bytes of one Fresnel plane: two sweeps, each reading and writing the
    n^2 c64 field once, plus one read of each float optic map the plane uses."""
    return 4 * n * n * 8 + optic_reads * n * n * 4


def sweep_bytes(n, optic_maps_in_this_sweep):
    return 2 * n * n * 8 + optic_maps_in_this_sweep * n * n * 4


def build_inputs(torch, np, synth, dev):
    lams = synth.wavelengths(N_LAMBDA)
    pupil = synth.pupil_amplitude(N_D, 0.1, 0.01)
    opd_p = synth.power_law_opd(N_D, pupil, 10e-9, -3.0, 0)
    off = (N - N_D) // 2
    rng = np.random.default_rng(42)
    amp = rng.uniform(0.99, 1.0, (N, N)).astype(np.float32)       # dense optic amplitude
    amp[off:off + N_D, off:off + N_D] *= pupil.astype(np.float32)
    opd = np.zeros((N, N), np.float32)
    opd[off:off + N_D, off:off + N_D] = opd_p
    amp_t = torch.from_numpy(amp).to(dev)
    opd_t = torch.from_numpy(opd).to(dev)
    fields = []
    for i in range(2 * N_LAMBDA):
        g = torch.Generator(device=dev)
        g.manual_seed(1000 + i)
        fields.append(torch.randn((N, N), dtype=torch.complex64, device=dev, generator=g))
    return lams, amp_t, opd_t, fields


def cpu_baseline(np):
    """The FP64 oracle on a bounded sample: one forward + one adjoint 4096^2 Fresnel plane."""
    import oracle
    from paper_1806_06467_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(7)
    field = synth.random_field(N, 99)
    amp = rng.uniform(0.99, 1.0, (N, N))
    opd = rng.normal(0.0, 10e-9, (N, N))
    t0 = time.perf_counter()
    out = oracle.fresnel_step(field, DX, 550e-9, Z, amp=amp, opd=opd)
    out = oracle.fresnel_step(out, DX, 550e-9, Z, amp=amp, opd=opd, adjoint=True)
    dt = time.perf_counter() - t0
    return {"value": 2.0 / dt, "unit": "Fresnel planes/s", "cores": int(threads), "kind": "oracle",
            "sample": "1 forward + 1 adjoint Fresnel plane at 4096^2 with amplitude+OPD optic, "
                      "FP64 oracle (explicit DFT matrices, zgemm), %.1f s" % dt}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    lams, amp, opd, fields = build_inputs(torch, np, synth, dev)
    n_pl = len(fields)
    adjs = [i >= N_LAMBDA for i in range(n_pl)]
    lam_pl = [float(lams[i % N_LAMBDA]) for i in range(n_pl)]

    def batched_step():
        fb.fresnel_step_batched(fields, DX, lam_pl, Z, amps=amp, opds=opd, adjoints=adjs)

    def plain_step():
        for i in range(n_pl):
            fb.fresnel_step(fields[i], DX, lam_pl[i], Z, amp=amp, opd=opd, adjoint=adjs[i])

    stream = torch.cuda.current_stream(dev)
    if args.copy_calibration:
        dst = torch.empty_like(fields[0])
        for _ in range(3):
            dst.copy_(fields[0])
        torch.cuda.synchronize()
        del dst

    def timed(fn, steps, profile=False):
        for _ in range(args.warmup):
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
    ms_batched, prof = timed(batched_step, args.steps, profile=True)
    ms_plain, prof_plain = timed(plain_step, max(1, args.steps // 2), profile=True)
    t_wall = time.perf_counter() - t_wall0

    steps = args.steps
    ms_per_step = ms_batched / steps
    planes_per_s = n_pl * steps / (ms_batched * 1e-3)
    plain_planes_per_s = n_pl * max(1, steps // 2) / (ms_plain * 1e-3)

    # roofline of the dominant kernel. Each sweep launch covers the 21 planes of one direction
    # (forward planes: rows then columns; adjoint planes: columns then rows). Both row launches
    # apply the optic (prologue forward, conjugate epilogue adjoint), so a row launch reads the
    # amplitude and OPD maps of its planes once; a column launch moves only the fields.
    per_launch = {"row_sweep": N_LAMBDA * sweep_bytes(N, 2), "col_sweep": N_LAMBDA * sweep_bytes(N, 0)}
    kern = {k.split("/")[0]: v for k, v in prof.items() if k.split("/")[0] in per_launch}
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms = kern[dom][0] / kern[dom][1]
    bytes_launch = per_launch[dom]
    achieved = bytes_launch / (dom_ms * 1e-3) / 1e9
    total_bytes_step = N_LAMBDA * plane_bytes(N, 2) * 2

    result = {
        "metric": "Fresnel planes/sec at 4096^2 c64 (fwd+adjoint, batched vs plain), %HBM roofline",
        "value": planes_per_s,
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
            "workload": "fresnel_planes_4096_fwd_adj_21lambda",
            "n": N, "planes_per_step": n_pl, "wavelengths_nm": [500, 600, N_LAMBDA],
            "dx_m": DX, "z_m": Z, "optic": "amplitude + OPD phasor per plane",
            "form": "batched (one launch per sweep per step)",
        },
        "plain": {"value": plain_planes_per_s, "unit": "Fresnel planes/s",
                  "ms_per_plane": ms_plain / (n_pl * max(1, steps // 2)),
                  "kernels_ms_per_plane": {k: v[0] / v[1] for k, v in prof_plain.items()}},
        "hbm_fraction_whole_plane": (total_bytes_step / (ms_per_step * 1e-3)) / (HBM_PEAK_GBS * 1e9),
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "bytes_per_launch": bytes_launch, "avg_launch_ms": dom_ms,
        },
        "kernels_ms_per_launch": {k: v[0] / v[1] for k, v in prof.items()},
        "wall_s": t_wall,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(np)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
