"""Throughput benchmark of the forward wave-equation operator on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--tti]

Workload (default): 3D isotropic acoustic, 256^3 grid, h = 10 m, two-layer
velocity 1500/2500 m/s, space order 8, 40-point damping layer, 15 Hz Ricker
source, 256 x 256 receiver plane with trilinear interpolation, FP32.  A
"step" is one time step of the whole path: stencil update with fused source
injection, then receiver interpolation.  The default K = 1000 is the
workload's full time axis.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line with the throughput in GPts/s (grid points x steps / s),
the HBM roofline of the dominant stencil kernel (algorithmic bytes per launch
over its average launch time, from HIP events around every launch in the
timed region) and the FP64 oracle timed on the host cores on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=40, help="oracle steps of the bounded CPU sample")
    ap.add_argument("--tti", action="store_true", help="also time the 512^3 TTI so=12 operator")
    return ap.parse_args()


def time_shot(prob, steps, warmup, device):
    """Warm up, reset to the zero initial state, then time `steps` time steps."""
    import torch

    from paper_1807_03032_amd import fdw

    shot = fdw.Shot(prob, device)
    stream = torch.cuda.current_stream(device)
    if warmup > 0:
        shot.apply(0, min(warmup, prob.nt) - 1)
    torch.cuda.synchronize(device)
    for t in shot.wave.values():
        t.zero_()
    shot.rec_data.zero_()
    fdw.fdw_operator_set_timing(shot.op, True)
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    lo = 0
    while lo < steps:
        hi = min(lo + prob.nt, steps) - 1 - lo
        shot.apply(0, hi, stream.cuda_stream)
        lo += hi + 1
    torch.cuda.synchronize(device)
    wall = time.perf_counter() - t0
    kms, launches = fdw.fdw_operator_kernel_time(shot.op)
    desc, alg_bytes = fdw.fdw_operator_describe(shot.op)
    tr = shot.traces()
    f = shot.fields(steps - 1) if steps <= prob.nt else None
    shot.close()
    return wall, kms, launches, desc, alg_bytes, tr, f


def parity_vs_stored(name, prob, steps, tr, f):
    """Relative L2 of sampled outputs against the stored oracle values (full runs only)."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", f"full_{name}.npz")
    if steps != prob.nt or not os.path.exists(path) or f is None:
        return None
    z = np.load(path)
    out = {}
    for nm, (lv_prev, lv_cur) in f.items():
        for tag, a in (("prev", lv_prev), ("cur", lv_cur)):
            ref = z[f"{nm}_{tag}_val"]
            got = a.reshape(-1)[z[f"{nm}_{tag}_idx"]]
            out[f"{nm}_{tag}"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    ref = z["rec_val"]
    out["rec"] = float(np.linalg.norm(tr[:, z["rec_idx"]] - ref) / np.linalg.norm(ref))
    return out


def cpu_baseline(prob, nsteps):
    import oracle

    g = oracle.Grid(prob.shape, prob.extent, prob.origin, so=prob.so, dt=prob.dt, nbl=prob.nbl, vmax=prob.vmax,
                    rc=prob.rc)
    t0 = time.perf_counter()
    if prob.kind == "iso":
        oracle.iso_run(g, prob.fields["m"], prob.nt, src_coords=prob.src_coords, src=prob.src,
                       rec_coords=prob.rec_coords, time_m=0, time_M=nsteps - 1)
    else:
        f = prob.fields
        oracle.tti_run(g, f["m"], f["eps"], f["delta"], f["theta"], f.get("phi"), prob.nt,
                       src_coords=prob.src_coords, src=prob.src, rec_coords=prob.rec_coords, time_m=0,
                       time_M=nsteps - 1)
    wall = time.perf_counter() - t0
    return {"value": prob.npoints * nsteps / wall / 1e9, "unit": "GPts/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle, full {'x'.join(map(str, prob.shape))} grid, first {nsteps} of {prob.nt} steps "
                      f"({wall:.1f} s wall)"}


def roofline(prob, kms, launches, alg_bytes):
    if launches <= 0 or kms <= 0:
        return None
    avg_s = kms / launches / 1e3
    per_launch = alg_bytes * prob.npoints
    achieved = per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel_avg_us": round(avg_s * 1e6, 2), "bytes_per_point": alg_bytes}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_1807_03032_amd import fdw
    from paper_1807_03032_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no ROCm GPU visible"}))
        sys.exit(2)
    fdw.load()
    dev = torch.device("cuda:0")
    prob = W.config_3d_iso_256(nt=max(1000, args.steps) if args.steps > 1000 else 1000)
    steps, warmup = args.steps, args.warmup
    wall, kms, launches, desc, alg_bytes, tr, f = time_shot(prob, steps, warmup, dev)
    value = prob.npoints * steps / wall / 1e9
    line = {
        "metric": "GPts/s (iso so=8, FP32)",
        "value": round(value, 3),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(wall * 1e3 / steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D isotropic acoustic 256^3, h=10 m, v 1500/2500 m/s two-layer, so=8, nbl=40, "
                               "15 Hz Ricker source, 256x256 receiver plane (trilinear), 1000 steps",
                   "grid": list(prob.shape), "space_order": prob.so, "nt": prob.nt, "kernel": desc},
        "roofline": roofline(prob, kms, launches, alg_bytes),
    }
    par = parity_vs_stored("3d_iso_256", prob, steps, tr, f)
    if par is not None:
        line["parity_rel_l2_sampled"] = par
    if args.tti:
        pt = W.config_3d_tti_512()
        w2, k2, l2, d2, b2, tr2, f2 = time_shot(pt, pt.nt, 20, dev)
        line["tti"] = {"workload": "3D TTI 512^3, h=12.5 m, so=12, nbl=40, 800 steps", "kernel": d2,
                       "value": round(pt.npoints * pt.nt / w2 / 1e9, 3), "unit": "GPts/s",
                       "roofline": roofline(pt, k2, l2, b2)}
        p2 = parity_vs_stored("3d_tti_512", pt, pt.nt, tr2, f2)
        if p2 is not None:
            line["tti"]["parity_rel_l2_sampled"] = p2
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
