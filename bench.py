"""Benchmark of the RPA chi0 hot path on one MI355X.

A step is one pass of the whole hot path on the 24^3 workload (16 Gaussian wells,
N_s = 16, N_r = 64, 8 Gauss-Legendre frequencies, COCG tol 1e-8): rpa_energy over all
frequencies (subspace iteration stopping at a relative energy change of 1e-8, at most 50
iterations per frequency) and then rpa_energy_backward (one chi0 block-apply per
frequency).  By default the frequencies are batched (every frequency starts from V0 and all
frequencies still iterating share one COCG launch per subspace iteration) in FP64;
--freq-mode warm runs Algorithm 1's warm-started sequence instead.  Inputs are synthetic,
seeded and resident in HBM before the timed region.

Printed: one JSON line with the metric (chi0 block-applies per second over the timed
steps), time-to-E_c, the roofline of the dominant kernel (batched COCG) measured with
HIP events on its own stream, the same path with complex64 state and float64 reliable
updates (one warm-up, one timed step: "compare"), and the CPU oracle timed on a bounded
sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per grid point per COCG iteration: read and write x, r, p
ALG_BYTES = {"fp64": 96.0, "mixed": 48.0}


def host_driven_bytes(precond, block, shape):
    """Algorithmic HBM bytes per point and system-iteration of the host-driven solvers: the
    step (q = A p; with the x and r updates for single systems: 128 B) and its direction update
    (r^T z and p: 64 B), or the block kernels (q = A p 32 B, alpha step 128 B, beta step 80 B);
    the preconditioner adds 32 B per pass, 3 fused passes for axes <= 32, else 7."""
    b = 240.0 if block >= 2 else 192.0
    if precond:
        b += 32.0 * (3 if max(shape) <= 32 else 7)
    return b


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1, help="workload index (0..4)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--freq-mode", default="independent", choices=["warm", "independent"],
                    help="warm: frequencies in sequence, each started from the previous one's "
                         "subspace (Algorithm 1); independent: every frequency from V0, all "
                         "frequencies batched into one chi0 launch per subspace iteration")
    ap.add_argument("--sq-order", type=int, default=0,
                    help="energy by Gauss spectral quadrature of this order (0: Rayleigh-Ritz)")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ec-tol", type=float, default=1e-8)
    ap.add_argument("--precond", action="store_true",
                    help="Sternheimer solves by COCG with the Kronecker shifted-Laplacian "
                         "preconditioner (FP64)")
    ap.add_argument("--block", type=int, default=0,
                    help="block COCG width (2..8; 0: single systems), with --precond "
                         "preconditioned (FP64)")
    ap.add_argument("--max-systems", type=int, default=0,
                    help="cap on COCG systems per launch (0: the library's memory budget)")
    ap.add_argument("--max-subspace", type=int, default=50)
    ap.add_argument("--compare", default="other", choices=["none", "other"],
                    help="other: after the timed steps, also time one step (after one warm-up) "
                         "of the same path in the other precision")
    return ap.parse_args()


def cocg_traffic(workload, precision, point_iters_per_launch):
    """HBM bytes per COCG launch from the committed FETCH_SIZE / WRITE_SIZE measurement
    (bytes per point-iteration, copy-kernel scaled) times this run's point-iterations per
    launch; None when the kernel sources changed since the counters were taken."""
    from paper_2504_01816_amd import profiling

    path = os.path.join(ROOT, "profiles", "cocg_wg_traffic.json")
    if not os.path.exists(path):
        return None, None
    sha = profiling.kernel_source_hash()
    for e in json.load(open(path))["entries"]:
        if e["precision"] == precision and e["workload"] == workload and e["kernel_source_sha256"] == sha:
            return e["bytes_per_point_iter"] * point_iters_per_launch, e["bytes_per_point_iter"]
    return None, None


def cpu_baseline(wl):
    """Oracle (as written, single BLAS thread) on two trial vectors at every frequency."""
    from threadpoolctl import threadpool_limits

    from oracle import chi0 as ochi0
    from oracle import coulomb as ocoul

    c = wl.cells[0]
    nr = wl.n_r[0]
    pick = list(range(len(wl.omegas)))
    nv = 2
    V = wl.V0[0][:nv].T.copy()
    times = []
    with threadpool_limits(1):
        for m in pick:
            t0 = time.perf_counter()
            U = ocoul.nu_apply(V, c.shape, c.h, 1)
            D, _, _ = ochi0.chi0_apply(U, c.vloc, c.psi.T, c.eps, float(wl.omegas[m]), c.shape, c.h,
                                       wl.cocg_tol, 5000)
            ocoul.nu_apply(D, c.shape, c.h, 1)
            times.append((time.perf_counter() - t0) / nv)
    per_apply = nr * float(np.mean(times))
    return {"value": 1.0 / per_apply, "unit": "chi0 block-applies/s", "cores": 1,
            "kind": "oracle",
            "sample": "%d of %d trial vectors (%d of %d Sternheimer systems, nu^1/2 both sides) "
                      "at each of the %d frequencies; block-apply time = %d x mean per-vector "
                      "time %.2f s" % (nv, nr, nv * c.n_occ, c.n_occ * nr, len(pick), nr,
                                       float(np.mean(times)))}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only; --gpus %d is not supported (sharding the "
              "Sternheimer systems across GPUs is described in the design notes, not "
              "implemented)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2504_01816_amd import api, synth
    from paper_2504_01816_amd import lib as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    t0 = time.perf_counter()
    # the 48^3 and larger inputs get their ground states on the GPU (untimed)
    wl = synth.workload(args.config, device=dev if args.config in (2, 3, 4) else None)
    print("[bench] workload %s generated in %.1f s" % (wl.name, time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    cells = [api.device_cell(c, dev) for c in wl.cells]
    V0 = [torch.tensor(v, device=dev) for v in wl.V0]
    prec = L.RPA_FP64 if args.precision == "fp64" else L.RPA_MIXED
    opts = dict(precision=prec, cocg_tol=wl.cocg_tol, subspace_iters=args.max_subspace,
                ec_tol=args.ec_tol, sq_order=args.sq_order, max_systems=args.max_systems,
                flags=L.RPA_FLAG_PRECOND if args.precond else 0, cocg_block=args.block,
                freq_mode=L.RPA_WARM if args.freq_mode == "warm" else L.RPA_INDEPENDENT)
    if wl.subspace_iters > 0:
        opts.update(subspace_iters=wl.subspace_iters, ec_tol=0.0)

    def step(opts=opts):
        st = {"fwd_s": 0.0, "bwd_s": 0.0, "applies": 0, "cocg_ms": 0.0, "point_iters": 0.0,
              "launches": 0, "iters": None, "E": None}
        torch.cuda.synchronize()
        a = time.perf_counter()
        res = api.rpa_energy(cells, wl.n_r, wl.omegas, wl.weights, V0, opts,
                             save=not args.no_backward)
        torch.cuda.synchronize()
        b = time.perf_counter()
        st["fwd_s"] = b - a
        for k in ("chi0_applies",):
            st["applies"] += res["stats"][k]
        st["cocg_ms"] += res["stats"]["cocg_kernel_ms"]
        st["point_iters"] += res["stats"]["cocg_point_iters"]
        st["launches"] += res["stats"]["cocg_launches"]
        st["iters"] = res["iters"].tolist()
        st["E"] = res["E_c"].tolist()
        if not args.no_backward:
            for ci, c in enumerate(cells):
                g, rc, s2 = api.rpa_energy_backward(c, wl.omegas, wl.weights, res["Vsave"][ci],
                                                    res["Csave"][ci], 1.0, opts)
                st["applies"] += s2["chi0_applies"]
                st["cocg_ms"] += s2["cocg_kernel_ms"]
                st["point_iters"] += s2["cocg_point_iters"]
                st["launches"] += s2["cocg_launches"]
            torch.cuda.synchronize()
            st["bwd_s"] = time.perf_counter() - b
        return st

    for w in range(args.warmup):
        s = step()
        print("[bench] warmup %d: %.2f s fwd, %.2f s bwd, subspace iters %s" %
              (w, s["fwd_s"], s["bwd_s"], s["iters"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T0 = time.perf_counter()
    steps = []
    for k in range(args.steps):
        s = step()
        steps.append(s)
        print("[bench] step %d: %.2f s fwd, %.2f s bwd, applies %d, E_c %s" %
              (k, s["fwd_s"], s["bwd_s"], s["applies"], s["E"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - T0
    applies = sum(s["applies"] for s in steps)
    cocg_ms = sum(s["cocg_ms"] for s in steps)
    pit = sum(s["point_iters"] for s in steps)
    launches = sum(s["launches"] for s in steps)
    alg_pp = ALG_BYTES[args.precision]
    if args.precond or args.block >= 2:
        alg_pp = host_driven_bytes(args.precond, args.block, wl.cells[0].shape)
    alg = alg_pp * pit
    achieved = alg / (cocg_ms * 1e-3) / 1e9 if cocg_ms > 0 else 0.0
    avg_ms = cocg_ms / max(1, launches)
    timing = "HIP events on the launch stream"
    if len(cells) > 1:
        # cells run concurrently: their launches overlap, so the summed launch time overstates
        # the COCG time; the forward wall time bounds it from above instead
        fwd = sum(s["fwd_s"] for s in steps)
        achieved = alg / fwd / 1e9
        timing = "forward wall time (concurrent cells)"
    traffic, tb = cocg_traffic(wl.name, args.precision, pit / max(1, launches))
    kernel = "cocg_wg (batched COCG, one workgroup per system)"
    if args.precond or args.block >= 2:
        # the host-driven solvers: a launch is a whole solve of several kernels, and the
        # counters were taken on the plain kernel
        kernel = ("host-driven %s (all kernels of a solve)" %
                  ("block COCG" if args.block >= 2 else "preconditioned COCG"))
        traffic, tb = None, None
    out = {
        "metric": "chi0 block-applies/s and time-to-E_c, FP32-refined batched vs FP64, 1 GPU",
        "value": applies / T,
        "unit": "chi0 block-applies/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * T / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128" if args.precision == "fp64" else "c64+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.cells[0].shape), "h": wl.cells[0].h,
                   "n_occ": wl.cells[0].n_occ, "n_r": wl.n_r[0], "n_freq": len(wl.omegas),
                   "cocg_tol": wl.cocg_tol, "ec_tol": opts["ec_tol"],
                   "backward": not args.no_backward, "precision": args.precision,
                   "freq_mode": args.freq_mode, "sq_order": args.sq_order,
                   "precond": bool(args.precond), "cocg_block": args.block},
        "time_to_ec_s": float(np.mean([s["fwd_s"] for s in steps])),
        "backward_s": float(np.mean([s["bwd_s"] for s in steps])),
        "E_c": steps[-1]["E"],
        "subspace_iters": steps[-1]["iters"],
        "chi0_applies_per_step": applies / args.steps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel,
                     "launches": launches, "avg_launch_ms": avg_ms,
                     "traffic_bytes_per_point_iter": tb,
                     "traffic_GBs": (traffic / (avg_ms * 1e-3) / 1e9) if traffic else None,
                     "alg_bytes_per_point_iter": alg_pp,
                     "cocg_share_of_step": cocg_ms * 1e-3 / T, "timing": timing},
    }
    if args.compare == "other":
        # the metric's comparison: the same path and inputs in the other precision (complex64
        # state with float64 reliable updates against complex128); a preconditioned run is
        # compared with the plain FP64 solver instead, and so is a block COCG run
        if args.precond or args.block >= 2:
            other = "fp64"
            o2 = dict(opts, flags=0, cocg_block=0)
        else:
            other = "mixed" if args.precision == "fp64" else "fp64"
            o2 = dict(opts, precision=L.RPA_MIXED if other == "mixed" else L.RPA_FP64)
        step(o2)
        torch.cuda.synchronize()
        t = time.perf_counter()
        s2 = step(o2)
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        out["compare"] = {
            "precision": other, "precond": False,
            "chi0_block_applies_per_s": s2["applies"] / t,
            "time_to_ec_s": s2["fwd_s"], "backward_s": s2["bwd_s"],
            "E_c": s2["E"], "subspace_iters": s2["iters"],
            "E_c_rel_diff": [abs(a - b) / abs(b) for a, b in zip(s2["E"], steps[-1]["E"])],
            "cocg_alg_GBs": ALG_BYTES[other] * s2["point_iters"] / (s2["cocg_ms"] * 1e-3) / 1e9,
            "time_to_ec_ratio_vs_main": s2["fwd_s"] / out["time_to_ec_s"],
        }
        print("[bench] compare %s: %.2f s fwd, %.2f applies/s, E_c %s" % (
            other, s2["fwd_s"], out["compare"]["chi0_block_applies_per_s"], s2["E"]),
            file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(wl)
        print("[bench] cpu baseline %.1f s" % (time.perf_counter() - t), file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
