"""Throughput benchmark of the forward wave-equation operators on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-tti] [--no-iso512] [--no-serve] [--no-attainable]

Headline workload: 3D isotropic acoustic, 256^3 grid, h = 10 m, two-layer
velocity 1500/2500 m/s, space order 8, 40-point damping layer, 15 Hz Ricker
source, 256 x 256 receiver plane with trilinear interpolation, FP32.  A
"step" is one time step of the whole path: stencil update with fused source
injection, then receiver interpolation.  The default K = 1000 is the
workload's full time axis.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line with the throughput in GPts/s (grid points x steps / s),
the HBM roofline of the dominant stencil kernel (algorithmic bytes per launch
over its average launch time, from HIP events around every launch in the
timed region; also as a fraction of the attainable bandwidth measured by the
library's triad probe in the same run) and the FP64 oracle timed on the host
cores on a bounded sample of the same workload.  The same line carries, by
default, K steps of the 512^3 TTI so = 12 workload (`tti`), K steps of the
isotropic so = 8 workload at 512^3 (`iso512`, working set beyond the
Infinity Cache), the copy/triad probe rates (`attainable`) and the served
shot stream (`serve`: p50/p99 latency, aggregate GPts/s, burst against
sequential plain solves).
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
    ap.add_argument("--cpu-steps", type=int, default=400, help="oracle steps of the bounded CPU sample")
    ap.add_argument("--no-tti", action="store_true", help="skip the 512^3 TTI so=12 leg")
    ap.add_argument("--no-iso512", action="store_true", help="skip the 512^3 isotropic so=8 leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the served shot-stream leg")
    ap.add_argument("--no-attainable", action="store_true", help="skip the copy/triad bandwidth probe")
    ap.add_argument("--serve-extra", action="store_true",
                    help="also run the same-shape fused bursts (2D 401^2 and LDS-resident 101^2 shots)")
    ap.add_argument("--tti-n", type=int, default=512, help="grid points per axis of the TTI leg (512: the workload)")
    ap.add_argument("--tti-steps", type=int, default=0, help="steps of the TTI leg (0: the workload's 800)")
    ap.add_argument("--nslots", type=int, default=2, choices=(2, 3),
                    help="wavefield storage of the isotropic workload: 2 = in-place leapfrog (default), "
                         "3 = modulo-3 buffer u[t %% 3]")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time one gradient (forward with checkpoints + recomputation + adjoint + imaging) "
                         "on the 320^3 so=8 1500-step workload")
    ap.add_argument("--serve", action="store_true",
                    help="no effect: the served shot stream (Poisson arrivals, mixed sizes, kinds and orders; "
                         "p50/p99 latency and aggregate GPts/s against sequential per-shot solves) runs by "
                         "default, --no-serve skips it")
    ap.add_argument("--serve-count", type=int, default=24)
    ap.add_argument("--serve-rate", type=float, default=3.0, help="mean request arrivals per second")
    ap.add_argument("--serve-streams", type=int, default=4, help="server streams (buckets advance concurrently)")
    ap.add_argument("--serve-chunk-us", type=float, default=20000, help="server chunk length target (us)")
    ap.add_argument("--tb2d", action="store_true",
                    help="also time the 2D temporal blocking (steps per launch on LDS patches) against one "
                         "launch per step on a 2D 8001^2 so=8 grid")
    ap.add_argument("--save-every", type=int, default=0,
                    help="also time the isotropic workload while saving every k-th level (snapshots)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (counter calibration under rocprofv3 --pmc)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE counter CSVs into profiles/traffic.json")
    return ap.parse_args()


def time_shot(prob, steps, warmup, device, nslots=3, timing_every=50):
    """Warm up, reset to the zero initial state, then time `steps` time steps."""
    import torch

    from paper_1807_03032_amd import fdw

    shot = fdw.Shot(prob, device, nslots=nslots)
    stream = torch.cuda.current_stream(device)
    if warmup > 0:
        shot.apply(0, min(warmup, prob.nt) - 1)
    torch.cuda.synchronize(device)
    for t in shot.wave.values():
        t.zero_()
    shot.rec_data.zero_()
    # HIP events around runs of `timing_every` consecutive stencil launches
    # (every launch covered; the events' own few microseconds spread over a run)
    fdw.fdw_operator_set_timing(shot.op, timing_every)
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


def snapshot_leg(prob, every, device):
    """The isotropic workload with every `every`-th level saved into a device
    buffer (subsampled saving fused into the stencil kernel)."""
    import torch

    from paper_1807_03032_amd import fdw

    shot = fdw.Shot(prob, device, nslots=2)
    try:
        nlev = prob.nt // every + 1
        buf = torch.empty(nlev * shot.lay.elems_per_slot, dtype=torch.float32, device=device)
        fdw.fdw_operator_set_save(shot.op, buf.data_ptr(), nlev, every, 0)
        shot.apply(0, 19)
        torch.cuda.synchronize(device)
        t0 = time.perf_counter()
        shot.apply(0, prob.nt - 1)
        torch.cuda.synchronize(device)
        wall = time.perf_counter() - t0
    finally:
        shot.close()
    return {"every": every, "levels": nlev, "buffer_gib": round(nlev * shot.lay.elems_per_slot * 4 / 2 ** 30, 2),
            "value": round(prob.npoints * prob.nt / wall / 1e9, 3), "unit": "GPts/s",
            "ms_per_step": round(wall * 1e3 / prob.nt, 5)}


def tb2d_leg(device, n=8001, so=8, nt=200):
    """2D isotropic n^2, so, nt steps, two-slot storage: temporal blocking
    (several steps per launch, FDW_TB=1) against one launch per step."""
    import torch

    from paper_1807_03032_amd import fdw
    from paper_1807_03032_amd import workloads as W

    prob = W.small_problem("iso", (n, n), so, nt=nt, seed=5, nsrc=1, nrec=n, nbl=40)
    out = {"workload": f"2D isotropic {n}^2, so={so}, {nt} steps, 1 source, {n} receivers, two-slot storage"}
    for label, env in (("temporal_blocking", "1"), ("per_step", "0")):
        os.environ["FDW_TB"] = env
        shot = fdw.Shot(prob, device, nslots=2)
        try:
            shot.apply(0, 9)
            torch.cuda.synchronize(device)
            fdw.fdw_operator_set_timing(shot.op, 10)
            t0 = time.perf_counter()
            shot.apply(0, nt - 1)
            torch.cuda.synchronize(device)
            wall = time.perf_counter() - t0
            kms, launches = fdw.fdw_operator_kernel_time(shot.op)
            desc = fdw.fdw_operator_describe(shot.op)[0]
        finally:
            shot.close()
        out[label] = {"kernel": desc, "value": round(prob.npoints * nt / wall / 1e9, 2), "unit": "GPts/s",
                      "ms_per_step": round(wall * 1e3 / nt, 4), "launches": launches,
                      "kernel_avg_us": round(kms * 1e3 / max(launches, 1), 2)}
    os.environ.pop("FDW_TB", None)
    out["speedup"] = round(out["temporal_blocking"]["value"] / out["per_step"]["value"], 2)
    return out


def run_server(reqs, arrivals, chunk_us=20000, nstreams=4):
    """Serve requests arriving at the given times (seconds from the start; all
    zero = one burst).  Returns per-request latencies, the makespan and stats."""
    from paper_1807_03032_amd import fdw

    sv = fdw.Server(budget_bytes=0, chunk_target_us=chunk_us, nstreams=nstreams)
    try:
        t0 = sv.stats()["now"]
        order = sorted(range(len(reqs)), key=lambda i: arrivals[i])
        k, tickets, lat, done_at = 0, {}, {}, []
        while len(lat) < len(reqs):
            now = sv.stats()["now"] - t0
            while k < len(order) and arrivals[order[k]] <= now:
                i = order[k]
                tickets[i] = sv.submit(reqs[i])
                k += 1
            q, r = sv.progress()
            for i, tk in tickets.items():
                if i in lat:
                    continue
                inf = sv.info(tk)
                if inf.state == fdw.FDW_SHOT_DONE:
                    lat[i] = inf.t_done - inf.t_submit
                    done_at.append(inf.t_done - t0)
                    sv.release(tk)
            if q == 0 and r == 0 and k < len(order):
                time.sleep(max(0.0, min(arrivals[order[k]] - now, 0.01)))
            else:
                time.sleep(2e-4)
        st = sv.stats()
        return lat, max(done_at), st
    finally:
        sv.close()


def serve_leg(device, count, rate, seed=7, nstreams=4, chunk_us=20000):
    """Served shot stream: Poisson arrivals (rate per second) of requests with
    grids from 2D 201^2 to 3D 400^3, orders 4-16, 500-2000 steps, iso or TTI;
    then the same requests as one burst, and as sequential per-shot solves."""
    import numpy as np
    import torch

    from paper_1807_03032_amd import fdw
    from paper_1807_03032_amd import workloads as W

    t_gen = time.perf_counter()
    stream = W.serve_stream(count=count, seed=seed, rate_hz=rate)
    t_gen = time.perf_counter() - t_gen
    reqs = [p for _, p in stream]
    arrivals = [a for a, _ in stream]
    work = sum(p.npoints * p.nt for p in reqs)
    # warm-up: one small request of each kind through the server (kernel loading)
    run_server([W.serve_problem(k, nd, n, 8, 20, seed=1) for k in ("iso", "tti") for nd, n in ((2, 201), (3, 48))],
               [0.0] * 4)
    lat, span, st = run_server(reqs, arrivals, chunk_us=chunk_us, nstreams=nstreams)
    lat_b, span_b, st_b = run_server(reqs, [0.0] * len(reqs), chunk_us=chunk_us, nstreams=nstreams)
    # sequential plain per-shot solves (set-up, all steps, traces), back to back
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    for p in reqs:
        shot = fdw.Shot(p, device, nslots=2)
        shot.apply(0, p.nt - 1)
        shot.traces()
        shot.close()
    torch.cuda.synchronize(device)
    seq = time.perf_counter() - t0
    lv = np.array([lat[i] for i in range(len(reqs))])
    mix = {}
    for p in reqs:
        key = f"{p.kind}{p.ndim}d"
        mix[key] = mix.get(key, 0) + 1
    return {
        "workload": f"{count} requests, Poisson arrivals at {rate}/s, grids 2D 201^2..801^2 and 3D 100^3..400^3, "
                    f"so in {{4,8,12,16}}, 500-2000 steps, iso/TTI (seed {seed})",
        "mix": mix, "gpoint_steps": round(work / 1e9, 2),
        "latency_p50_s": round(float(np.percentile(lv, 50)), 4),
        "latency_p99_s": round(float(np.percentile(lv, 99)), 4),
        "aggregate_gpts_poisson": round(work / span / 1e9, 2),
        "aggregate_gpts_burst": round(work / span_b / 1e9, 2),
        "sequential_gpts": round(work / seq / 1e9, 2),
        "burst_vs_sequential": round(seq / span_b, 3),
        "burst_latency_p50_s": round(float(np.percentile(list(lat_b.values()), 50)), 4),
        "chunks": st["chunks"], "graph_builds": st["graph_builds"], "graph_launches": st["graph_launches"],
        "host_admit_s": round(st["admit_seconds"], 3), "host_launch_s": round(st["launch_seconds"], 3),
        "burst_host_admit_s": round(st_b["admit_seconds"], 3), "burst_makespan_s": round(span_b, 3),
        "sequential_s": round(seq, 3),
        "model_generation_s": round(t_gen, 1),
        "server_streams": nstreams, "chunk_target_us": chunk_us,
    }


def fused_burst_leg(device, count=32, n=401, so=8, nt=1000):
    """Same-shape burst: `count` isotropic 2D n^2 shots (different sources)
    served as one bucket (fused launches, replayed graphs) against sequential
    per-shot solves."""
    import torch

    from paper_1807_03032_amd import fdw
    from paper_1807_03032_amd import workloads as W

    cache = {}
    reqs = [W.serve_problem("iso", 2, n, so, nt, seed=100 + i, model_cache=cache) for i in range(count)]
    run_server(reqs[:2], [0.0, 0.0])
    work = sum(p.npoints * p.nt for p in reqs)
    lat, span, st = run_server(reqs, [0.0] * count)
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    for p in reqs:
        shot = fdw.Shot(p, device, nslots=2)
        shot.apply(0, p.nt - 1)
        shot.traces()
        shot.close()
    torch.cuda.synchronize(device)
    seq = time.perf_counter() - t0
    return {"workload": f"{count} isotropic 2D {n}^2 so={so} shots of {nt} steps, one burst",
            "served_gpts": round(work / span / 1e9, 2), "sequential_gpts": round(work / seq / 1e9, 2),
            "speedup": round(seq / span, 2), "chunks": st["chunks"], "graph_launches": st["graph_launches"],
            "host_admit_s": round(st["admit_seconds"], 3), "makespan_s": round(span, 4), "sequential_s": round(seq, 4)}


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


def adjoint_leg(device):
    """One full-waveform gradient on the 320^3 workload: observed data from the
    true model, then forward at the background model, residual, and the
    adjoint-state gradient, twice: keeping the imaging factors of all 1500
    steps in HBM when they fit (no recomputation), and with checkpoints every
    50 steps (segments recomputed).  Also the FP32 adjoint dot-product test on
    this geometry."""
    import torch

    from paper_1807_03032_amd import workloads as W
    from paper_1807_03032_amd.modeling import IsoModeling

    prob, m_true = W.config_3d_iso_adjoint_320()
    n = prob.npoints * prob.nt
    out = {"workload": "3D isotropic 320^3, h=10 m, so=8, nbl=40, 1500 steps, smooth background + 5% perturbation, "
                       "320x320 receivers"}
    d_obs = resid = None
    for label, K in (("", None), ("_checkpointed", 50)):
        md = IsoModeling(prob.shape, prob.extent, prob.origin, prob.so, prob.dt, prob.nt, prob.nbl, prob.vmax,
                         prob.src_coords, prob.rec_coords, device=device, checkpoint_every=K, rc=prob.rc)
        try:
            if d_obs is None:
                md.set_m(m_true)
                d_obs = md.forward(prob.src, checkpoints=False)
            md.set_m(prob.fields["m"])
            torch.cuda.synchronize(device)
            t0 = time.perf_counter()
            resid = md.forward(prob.src, checkpoints=True) - d_obs
            torch.cuda.synchronize(device)
            t1 = time.perf_counter()
            g = md.gradient(resid)
            torch.cuda.synchronize(device)
            t2 = time.perf_counter()
            out[f"checkpoint_every{label}"] = md.K
            out[f"forward_s{label}"] = round(t1 - t0, 4)
            out[f"gradient_s{label}"] = round(t2 - t1, 4)
            out[f"gradient_GPts_per_s{label}"] = round(n / (t2 - t0) / 1e9, 3)
            if not label:
                # dot test on this geometry: <F q, d> vs <q, F^T d> with d = the residual
                ftd = md.adjoint(resid)
                fq = md.forward(prob.src, checkpoints=False)
                lhs = float(torch.sum(fq.double() * resid.double()))
                rhs = float(torch.sum(torch.as_tensor(prob.src, device=device).double() * ftd.double()))
                out["dot_test_rel"] = abs(lhs - rhs) / abs(lhs)
                g_first = g
            else:
                out["grad_rel_diff_vs_checkpointed"] = float(
                    torch.linalg.norm((g - g_first).double()) / torch.linalg.norm(g_first.double()))
            out[f"grad_norm{label}"] = float(torch.linalg.norm(g.double()))
        finally:
            md.close()
            del md
            torch.cuda.empty_cache()
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


# ---------------------------------------------------------------------------
# Measured HBM traffic of the dominant kernels.  FETCH_SIZE / WRITE_SIZE are
# read per dispatch with rocprofv3 --pmc (one counter per run) and scaled by
# what the same counter reads for a plain device copy of known size run in the
# same process.  The summary is keyed by the operator description and a hash
# of the kernel sources, so a changed kernel reports traffic = null.
# ---------------------------------------------------------------------------
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {
    "iso": ["fdw_device.h", "fdw_stream2.h", "fdw_iso_op.h", "fdw_iso.hip", "fdw_internal.h"],
    "tti": ["fdw_device.h", "fdw_tti.hip", "fdw_internal.h"],
}
CALIB_BYTES = 256 * 1024 * 1024


def source_hash(kind):
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_1807_03032_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def calib_copy(device):
    """Plain streaming kernel of known size: b = -a over 256 MiB (reads and
    writes 256 MiB each); its distinctive name (neg_kernel) identifies it in
    the counter CSVs."""
    import torch

    a = torch.ones(CALIB_BYTES // 4, device=device)
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize(device)


def summarize_traffic(fetch_csv, write_csv):
    """Median KiB per dispatch of every fdw kernel, scaled by the copy calibration."""
    import csv
    import statistics

    def per_dispatch(path):
        agg = {}
        for r in csv.DictReader(open(path)):
            k = int(r["Dispatch_Id"])
            agg.setdefault(k, [r["Kernel_Name"], 0.0])
            agg[k][1] += float(r["Counter_Value"])
        return agg

    out = {}
    fetch, write = per_dispatch(fetch_csv), per_dispatch(write_csv)
    # calibration: the median reading of the 256 MiB neg_kernel dispatches
    def cal(agg):
        vals = [v for n, v in agg.values() if "neg_kernel" in n]
        return statistics.median(vals)

    factors = {"fetch": (CALIB_BYTES / 1024.0) / cal(fetch), "write": (CALIB_BYTES / 1024.0) / cal(write)}
    for counter, agg in (("fetch", fetch), ("write", write)):
        kern = {}
        for n, v in agg.values():
            if "fdw::" in n:
                kern.setdefault(n, []).append(v)
        for n, vals in kern.items():
            e = out.setdefault(n, {})
            e[f"{counter}_kib_median"] = statistics.median(vals)
            e[f"{counter}_factor"] = round(factors[counter], 4)
            e[f"{counter}_bytes"] = statistics.median(vals) * 1024.0 * factors[counter]
            e["dispatches"] = len(vals)
    return out


def iso_kernel_match(desc):
    """Kernel-name fragments of the isotropic operator described by desc: the
    streaming kernel's template arguments <R, NY, PF, NQ, NP, BY> follow from
    its tile, wavefront count and prefetch distance, its operator type from
    the pointwise loads' hint (one-thread-per-point kernels otherwise)."""
    import re

    m = re.search(r"tile=64x(\d+) \((\d+) waves\).*prefetch=(\d+).* R=(\d+)", desc)
    if not m:
        return ["iso_naive"]
    ty, by, pf, r = (int(v) for v in m.groups())
    op = "IsoOpNTu" if "pointwise=nt(u" in desc else "IsoOpNT" if "pointwise=nt" in desc else "IsoOp"
    return [f"<{r}, {ty // by}, {pf}, 1, 2, {by}, fdw::{op}>"]


def load_traffic(kind, desc):
    """Measured bytes per launch of this operator's kernels, or None."""
    try:
        db = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    e = db.get(desc)
    if not e or e.get("source_hash") != source_hash(kind):
        return None
    return e.get("bytes_per_launch")


def roofline(prob, kms, launches, alg_bytes, traffic=None, attainable=None):
    if launches <= 0 or kms <= 0:
        return None
    avg_s = kms / launches / 1e3
    per_launch = alg_bytes * prob.npoints
    achieved = per_launch / avg_s / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": round(traffic) if traffic is not None else None,
           "algorithmic_bytes": round(per_launch),
           "kernel_avg_us": round(avg_s * 1e6, 2), "bytes_per_point": alg_bytes}
    if attainable:
        out["attainable"] = round(attainable, 1)
        out["frac_attainable"] = round(achieved / attainable, 4)
    return out


def attainable_bandwidth(device, mib=1024, reps=20):
    """HBM bandwidth of the library's copy and triad probes (the paper's
    STREAM-triad convention for the attainable peak) on arrays of `mib` MiB,
    far beyond the 256 MB Infinity Cache: best per-launch rate over `reps`
    launches, each bracketed by events on the launch stream."""
    import torch

    from paper_1807_03032_amd import fdw

    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, device=device)
    b = torch.full((n,), 0.5, device=device)
    c = torch.empty(n, device=device)
    st = torch.cuda.current_stream(device)
    out = {"array_mib": mib}
    for kind, name, nbytes in ((0, "copy", 8 * n), (1, "triad", 12 * n)):
        for _ in range(3):
            fdw.fdw_bandwidth_probe(kind, c.data_ptr(), a.data_ptr(), b.data_ptr(), 3.0, n, st.cuda_stream)
        best = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fdw.fdw_bandwidth_probe(kind, c.data_ptr(), a.data_ptr(), b.data_ptr(), 3.0, n, st.cuda_stream)
            e1.record(st)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out[f"{name}_gbs"] = round(nbytes / (best * 1e-3) / 1e9, 1)
    expect = 1.0 + 3.0 * 0.5
    assert float(c[0]) == expect and float(c[-1]) == expect, "triad probe result"
    del a, b, c
    torch.cuda.empty_cache()
    out["attainable_gbs"] = out["triad_gbs"]
    return out


def main():
    args = parse()
    if args.traffic_from:
        ops = json.load(open(args.traffic_from[0] + ".ops.json")) if os.path.exists(
            args.traffic_from[0] + ".ops.json") else None
        kern = summarize_traffic(*args.traffic_from)
        print(json.dumps(kern, indent=1))
        if ops:
            db = json.load(open(TRAFFIC_JSON)) if os.path.exists(TRAFFIC_JSON) else {}
            for op in ops:
                names = [n for n in kern if any(s in n for s in op["kernel_match"])]
                tot = sum(kern[n]["fetch_bytes"] + kern[n]["write_bytes"] for n in names)
                db[op["desc"]] = {"source_hash": op["source_hash"], "kernels": {n: kern[n] for n in names},
                                  "bytes_per_launch": tot, "fetch_csv": os.path.basename(args.traffic_from[0]),
                                  "write_csv": os.path.basename(args.traffic_from[1])}
            os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
            json.dump(db, open(TRAFFIC_JSON, "w"), indent=1, sort_keys=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the operators run on one GPU per process; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_1807_03032_amd import fdw
    from paper_1807_03032_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no ROCm GPU visible"}))
        sys.exit(2)
    fdw.load()
    dev = torch.device("cuda:0")
    if args.calib_copy:
        calib_copy(dev)
    steps, warmup = args.steps, args.warmup
    att = None if args.no_attainable else attainable_bandwidth(dev)
    att_gbs = att["attainable_gbs"] if att else None
    prob = W.config_3d_iso_256(nt=max(1000, args.steps) if args.steps > 1000 else 1000)
    wall, kms, launches, desc, alg_bytes, tr, f = time_shot(prob, steps, warmup, dev, args.nslots)
    desc = f"{desc} slots={args.nslots}"
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
                   "grid": list(prob.shape), "space_order": prob.so, "nt": prob.nt, "kernel": desc,
                   "wavefield_storage": "in-place leapfrog, 2 slots" if args.nslots == 2 else "modulo-3 buffer"},
        "roofline": roofline(prob, kms, launches, alg_bytes, load_traffic("iso", desc), att_gbs),
    }
    ops_seen = [{"desc": desc, "source_hash": source_hash("iso"), "kernel_match": iso_kernel_match(desc)}]
    par = parity_vs_stored("3d_iso_256", prob, steps, tr, f)
    if par is not None:
        line["parity_rel_l2_sampled"] = par
    del tr, f
    if att:
        line["attainable"] = att
    if not args.no_iso512:
        # working set far beyond the 256 MB Infinity Cache: the off-cache rate
        p5 = W.config_3d_iso_256(nt=max(1000, steps), n=512)
        w5, k5, l5, d5, b5, _, _ = time_shot(p5, steps, warmup, dev, 2)
        d5 = f"{d5} slots=2"
        line["iso512"] = {"workload": "3D isotropic acoustic 512^3, h=10 m, v 1500/2500 m/s two-layer, so=8, nbl=40, "
                                      "15 Hz Ricker source, 512x512 receiver plane",
                          "kernel": d5, "steps": steps, "value": round(p5.npoints * steps / w5 / 1e9, 3),
                          "unit": "GPts/s", "ms_per_step": round(w5 * 1e3 / steps, 5),
                          "roofline": roofline(p5, k5, l5, b5, load_traffic("iso", d5), att_gbs)}
        ops_seen.append({"desc": d5, "source_hash": source_hash("iso"), "kernel_match": iso_kernel_match(d5)})
        del p5
    if not args.no_tti:
        tsteps = args.tti_steps or steps
        pt = W.config_3d_tti_512(nt=max(800, tsteps), n=args.tti_n)
        w2, k2, l2, d2, b2, tr2, f2 = time_shot(pt, tsteps, min(warmup, 20), dev)
        line["tti"] = {"workload": f"3D TTI {args.tti_n}^3, h=12.5 m, so=12, nbl=40, 800 steps, smooth random "
                                   f"v/eps/delta/theta/phi", "kernel": d2, "steps": tsteps,
                       "value": round(pt.npoints * tsteps / w2 / 1e9, 3), "unit": "GPts/s",
                       "ms_per_step": round(w2 * 1e3 / tsteps, 5),
                       "roofline": roofline(pt, k2, l2, b2, load_traffic("tti", d2), att_gbs)}
        ops_seen.append({"desc": d2, "source_hash": source_hash("tti"), "kernel_match": ["TtiS1Op", "TtiS2Op", "tti_naive"]})
        p2 = parity_vs_stored("3d_tti_512", pt, tsteps, tr2, f2) if (args.tti_n, pt.nt, tsteps) == (512, 800, 800) \
            else None
        if p2 is not None:
            line["tti"]["parity_rel_l2_sampled"] = p2
        del pt, tr2, f2
    if args.adjoint:
        line["adjoint"] = adjoint_leg(dev)
    if args.save_every > 0:
        line["snapshots"] = snapshot_leg(prob, args.save_every, dev)
    if args.tb2d:
        line["tb2d"] = tb2d_leg(dev)
    if not args.no_serve:
        line["serve"] = serve_leg(dev, args.serve_count, args.serve_rate, nstreams=args.serve_streams,
                                  chunk_us=args.serve_chunk_us)
    if args.serve_extra:
        line["serve_fused_burst"] = fused_burst_leg(dev)
        # grids that fit in LDS: one workgroup per shot, whole range in one launch
        line["serve_fused_burst_lds"] = fused_burst_leg(dev, count=64, n=101, so=4, nt=500)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_steps)
    if os.environ.get("FDW_BENCH_OPS_OUT"):
        json.dump(ops_seen, open(os.environ["FDW_BENCH_OPS_OUT"], "w"))
    print(json.dumps(line), flush=True)

if __name__ == "__main__":
    main()
