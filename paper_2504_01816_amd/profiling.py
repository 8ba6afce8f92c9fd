"""Workloads and summaries for hardware-counter profiling of the COCG kernel.

Subcommands (run under rocprofv3, one counter set per run):

  copy       a plain device copy of a known size (torch's copy kernel), used to scale the
             FETCH_SIZE / WRITE_SIZE counters to bytes
  apply      one chi0 block-apply at each frequency of a workload; prints the COCG kernel's
             point-iterations and launch count as JSON (stderr)
  summarize  reduce a rocprofv3 counter CSV to per-kernel means (markdown on stdout)
  kstats     a rocprofv3 --stats kernel summary as a markdown table
  gaps       kernel time and idle time between dispatches of a traced subspace run (what a HIP
             graph of the small launches could save)
  krange     mean duration of a range of one kernel's dispatches in a kernel trace (a bench
             run's timed region)
  traffic    combine the FETCH_SIZE and WRITE_SIZE summaries of the copy and the apply runs
             into HBM bytes per point-iteration of the COCG kernel (JSON read by bench.py)

Example:
  rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o copy -- \
      python -m paper_2504_01816_amd.profiling copy --mib 1024
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/cocg_kernel.h", "csrc/cocg.hip", "csrc/cocg_f64.hip", "csrc/cocg_mixed.hip")


def kernel_source_hash():
    """SHA-256 over the COCG kernel's sources: counters taken on other sources are stale."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def cmd_copy(args):
    import torch

    n = args.mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0")   # no fill kernel in the trace
    dst = torch.empty_like(src)
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "reps": args.reps}), file=sys.stderr)


def _workload(args):
    from . import synth
    return synth.workload(args.config, device="cuda:0" if args.gen_device else None)


def cmd_apply(args):
    import torch

    from . import api, synth
    from . import lib as L

    wl = _workload(args)
    c = wl.cells[0]
    if args.box:
        # the isolated-box counterpart of the workload's cell: same grid, spacing and
        # occupied count, 16 seeded wells inside a Dirichlet box
        c = synth.box_cell(c.shape, c.h, 16, c.n_occ, 101)
    dc = api.device_cell(c, "cuda:0")
    nvec = args.nvec or wl.n_r[0]
    X = api.rpa_apply_coulomb(dc, torch.tensor(wl.V0[0][:nvec], device="cuda:0"), 1)
    prec = L.RPA_FP64 if args.precision == "fp64" else L.RPA_MIXED
    opts = dict(precision=prec, cocg_tol=wl.cocg_tol, flags=L.RPA_FLAG_PRECOND if args.precond else 0,
                cocg_block=args.block)
    if args.refine_tol > 0:
        opts["refine_tol"] = args.refine_tol
    if args.mixed_min_omega >= 0:
        opts["mixed_min_omega"] = args.mixed_min_omega
    tot = {"cocg_point_iters": 0.0, "cocg_launches": 0, "cocg_kernel_ms": 0.0, "cocg_iters_total": 0}
    idx = range(len(wl.omegas)) if args.omega_index < 0 else [args.omega_index]
    if args.warmup:
        # one untimed apply first (module load, launch-shape selection); not for counter runs,
        # whose per-point figures divide by the timed applies' point-iterations
        api.rpa_apply_chi0(dc, float(wl.omegas[idx[0]]), X, opts)
    for m in idx:
        _, _, st = api.rpa_apply_chi0(dc, float(wl.omegas[m]), X, opts)
        print("omega %.4g: %.2f ms, iterations %d (max %d), reliable updates %d" % (
            wl.omegas[m], st["cocg_kernel_ms"], st["cocg_iters_total"], st["cocg_iters_max"],
            st["refinements"]), file=sys.stderr)
        for k in tot:
            tot[k] += st[k]
    torch.cuda.synchronize()
    tot.update(workload=wl.name, precision=args.precision, nvec=nvec, omegas=list(idx),
               precond=bool(args.precond), block=args.block, box=bool(args.box))
    print(json.dumps(tot), file=sys.stderr)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(tot, f)


def cmd_subspace(args):
    """One (or --iters) subspace iteration step(s) at one frequency: every stage of the path
    (two nu^1/2 applications, projector, COCG, Delta rho, projection, energy, Cholesky-QR)."""
    import torch

    from . import api
    from . import lib as L

    wl = _workload(args)
    c = wl.cells[0]
    dc = api.device_cell(c, "cuda:0")
    prec = L.RPA_FP64 if args.precision == "fp64" else L.RPA_MIXED
    Q, _ = torch.linalg.qr(torch.tensor(wl.V0[0], device="cuda:0").T)   # orthonormal start
    V = Q.T.contiguous()
    m = args.omega_index
    r = api.rpa_subspace_iter(dc, float(wl.omegas[m]), float(wl.weights[m]), V,
                              dict(precision=prec, cocg_tol=wl.cocg_tol, subspace_iters=args.iters,
                                   ec_tol=0.0), want_ritz=False, want_saved=False)
    torch.cuda.synchronize()
    out = dict(workload=wl.name, precision=args.precision, omega=float(wl.omegas[m]),
               iters=args.iters, E=r["E"], nd=c.nd, n=list(c.shape), ns=c.n_occ, nr=wl.n_r[0],
               stats=r["stats"])
    print(json.dumps(out), file=sys.stderr)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f)


# stage of the path -> (substrings of the kernel names, separated by |; flops of one subspace
# step)
def _stage_flops(nd, n, ns, nr):
    return [
        ("projector coefficients c = dV Psi^T (psi_n u_j)", "gemm_coeff|PsiT",
         2.0 * nd * ns * ns * nr),
        ("projected right-hand sides b' = b - Psi c (HBM-bound: writes the COCG start vectors)",
         "CoeffT", 2.0 * nd * ns * ns * nr),
        ("nu^1/2 Kronecker transforms (2 applications x 6 passes; HBM-bound, n/8 flop/B)", "Axis",
         2 * sum(4.0 * a * nd * nr for a in n)),
        ("projection C = V^T R and Gram M = R^T R", "ColT", 2 * 2.0 * nd * nr * nr),
        ("Cholesky-QR rotation V = R L^-T", "SmallT", 2.0 * nd * nr * nr),
    ]


def cmd_stages(args):
    """Per-stage kernel time and achieved FLOP/s of a traced `subspace` run (FP64 MFMA peak
    78.6 TFLOP/s for the GEMM stages)."""
    info = json.load(open(args.run))
    fn = args.trace
    if os.path.isdir(fn):
        fn = sorted(glob.glob(os.path.join(fn, "**", "*kernel_trace.csv"), recursive=True))[0]
    rows = list(csv.DictReader(open(fn)))
    dur = {}
    for r in rows:
        d = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9
        dur.setdefault(r["Kernel_Name"], []).append(d)
    it = info["iters"]
    print("| stage | kernels matched | dispatches | time ms | flop | TFLOP/s | of 78.6 |")
    print("|---|---|---|---|---|---|---|")
    for name, key, fl in _stage_flops(info["nd"], info["n"], info["ns"], info["nr"]):
        ks = [k for k in dur if any(part in k for part in key.split("|"))]
        t = sum(sum(dur[k]) for k in ks)
        nds = sum(len(dur[k]) for k in ks)
        f = fl * it
        print("| %s | `%s` | %d | %.3f | %.3g | %.2f | %.1f%% |" % (
            name, key.replace("|", "`, `"), nds, t * 1e3, f, f / t / 1e12 if t else 0,
            100 * f / t / 78.6e12 if t else 0))
    for key, label in (("cocg_wg", "COCG"), ("drho", "Delta rho"), ("reduce_parts", "split-K reductions"),
                       ("energy_kernel", "energy (Cholesky of I - C)"), ("chol_inv", "Cholesky + inverse")):
        ks = [k for k in dur if key in k]
        t = sum(sum(dur[k]) for k in ks)
        print("| %s | `%s` | %d | %.3f | | | |" % (label, key, sum(len(dur[k]) for k in ks), t * 1e3))


def cmd_gaps(args):
    """Launch overhead of a traced `subspace` run: per dispatch the kernel time and the idle
    time since the previous kernel ended, summed for the COCG kernel and for everything else
    (the ~30 small launches of a subspace iteration around it).  The idle time outside the COCG
    kernel bounds what capturing those launches in a HIP graph could save."""
    fn = args.trace
    if os.path.isdir(fn):
        fn = sorted(glob.glob(os.path.join(fn, "**", "*kernel_trace.csv"), recursive=True))[0]
    rows = sorted(csv.DictReader(open(fn)), key=lambda r: int(r["Start_Timestamp"]))
    if args.skip:
        rows = rows[args.skip:]
    k_cocg = k_other = gap_other = 0.0
    n_other = 0
    prev_end = None
    for r in rows:
        a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        d = (b - a) * 1e-6
        gap = max(0.0, (a - prev_end) * 1e-6) if prev_end is not None else 0.0
        if "cocg_wg" in r["Kernel_Name"]:
            k_cocg += d
        else:
            k_other += d
            gap_other += gap
            n_other += 1
        prev_end = b if prev_end is None else max(prev_end, b)
    span = (int(rows[-1]["End_Timestamp"]) - int(rows[0]["Start_Timestamp"])) * 1e-6
    print("| quantity | ms |")
    print("|---|---|")
    print("| span of the traced dispatches | %.3f |" % span)
    print("| COCG kernel time | %.3f |" % k_cocg)
    print("| other kernels (%d dispatches) | %.3f |" % (n_other, k_other))
    print("| idle time before the other kernels (launch gaps and host synchronisations) | %.3f |"
          % gap_other)
    print("| idle share of the span | %.2f%% |" % (100.0 * gap_other / span))


def cmd_krange(args):
    """Mean duration of one kernel's dispatches number a .. b-1 (in dispatch order) in a kernel
    trace: the dispatches of a bench run's timed region (bench.py prints their range), to set
    beside the bench's own HIP-event timing of the same launches.  With --also, further
    (kernel, first, last) ranges join the selection (a timed region that spans two kernels),
    and a last row gives the mean over all of them."""
    fn = args.trace
    if os.path.isdir(fn):
        fn = sorted(glob.glob(os.path.join(fn, "**", "*kernel_trace.csv"), recursive=True))[0]
    trace = list(csv.DictReader(open(fn)))
    ranges = [(args.match, args.first, args.last)] + [(m, int(a), int(b)) for m, a, b in args.also]
    print("| kernel | dispatches in the trace | selected | mean ms | min ms | max ms |")
    print("|---|---|---|---|---|---|")
    every = []
    for match, first, last in ranges:
        rows = sorted((r for r in trace if match in r["Kernel_Name"]),
                      key=lambda r: int(r["Start_Timestamp"]))
        sel = rows[first:last]
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6 for r in sel]
        every += d
        names = sorted(set(r["Kernel_Name"] for r in sel))
        print("| `%s` | %d | %d .. %d | %.3f | %.3f | %.3f |" % (
            short(names[0] if names else match, 90), len(rows), first, last - 1,
            sum(d) / max(1, len(d)), min(d) if d else 0.0, max(d) if d else 0.0))
    if len(ranges) > 1:
        print("| all %d selected dispatches | | | %.3f | %.3f | %.3f |" % (
            len(every), sum(every) / max(1, len(every)), min(every) if every else 0.0,
            max(every) if every else 0.0))


def read_counters(path):
    """Rows of a rocprofv3 counter_collection CSV as (kernel, counter, value) per dispatch."""
    rows = []
    for fn in sorted(glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
                     if os.path.isdir(path) else [path]):
        with open(fn) as f:
            for r in csv.DictReader(f):
                rows.append((r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]),
                             r.get("Dispatch_Id", "")))
    return rows


def per_kernel_means(rows):
    acc = {}
    for k, c, v, d in rows:
        key = (k, c)
        s = acc.setdefault(key, {"sum": 0.0, "dispatches": set()})
        s["sum"] += v
        s["dispatches"].add(d)
    return {key: (s["sum"] / max(1, len(s["dispatches"])), len(s["dispatches"]), s["sum"])
            for key, s in acc.items()}


def short(name, n=70):
    name = name.replace("rpa::cocg::", "").replace("HIP_vector_type", "vec")
    return name if len(name) <= n else name[: n - 3] + "..."


def cmd_summarize(args):
    means = per_kernel_means(read_counters(args.csv))
    print("| kernel | counter | dispatches | mean per dispatch | total |")
    print("|---|---|---|---|---|")
    for (k, c), (m, n, t) in sorted(means.items(), key=lambda kv: -kv[1][2]):
        if args.match and args.match not in k:
            continue
        print("| `%s` | %s | %d | %.6g | %.6g |" % (short(k), c, n, m, t))


def cmd_kstats(args):
    """Markdown table of a rocprofv3 --stats kernel summary (kernel_stats.csv)."""
    fn = args.csv
    if os.path.isdir(fn):
        fn = sorted(glob.glob(os.path.join(fn, "**", "*kernel_stats.csv"), recursive=True))[0]
    with open(fn) as f:
        rows = list(csv.DictReader(f))
    print("| kernel | calls | total ms | average ms | min ms | max ms | share |")
    print("|---|---|---|---|---|---|---|")
    for r in rows[: args.top]:
        print("| `%s` | %s | %.3f | %.4f | %.4f | %.4f | %.2f%% |" % (
            short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6, float(r["MaxNs"]) / 1e6,
            float(r["Percentage"])))


def _total(rows, match, counter):
    return sum(v for k, c, v, _ in rows if match in k and c == counter)


def cmd_traffic(args):
    """Bytes per COCG point-iteration from FETCH_SIZE / WRITE_SIZE (KiB), each scaled so that
    the copy kernel of known size reads (writes) exactly its size."""
    out = {"kernel_source_sha256": kernel_source_hash(), "precision": args.precision}
    stats = json.load(open(args.apply_stats))
    copy_bytes = float(args.copy_mib << 20) * args.copy_reps
    for counter, copy_csv, apply_csv in (("FETCH_SIZE", args.copy_fetch, args.apply_fetch),
                                         ("WRITE_SIZE", args.copy_write, args.apply_write)):
        crow = read_counters(copy_csv)
        cval = sum(v for k, c, v, _ in crow if c == counter and "cocg" not in k)
        factor = copy_bytes / (cval * 1024.0) if cval > 0 else float("nan")
        aval = _total(read_counters(apply_csv), "cocg_wg", counter)
        out[counter.lower() + "_copy_factor"] = factor
        out[counter.lower() + "_bytes_per_point_iter"] = aval * 1024.0 * factor / stats["cocg_point_iters"]
    out["bytes_per_point_iter"] = (out["fetch_size_bytes_per_point_iter"]
                                   + out["write_size_bytes_per_point_iter"])
    out["apply_stats"] = stats
    out["workload"] = stats["workload"]
    print(json.dumps(out, indent=1))
    if args.write:
        # one entry per (precision, workload): replace that entry, keep the others
        doc = {"kernel": "cocg_wg", "entries": []}
        if os.path.exists(args.write):
            with open(args.write) as f:
                old = json.load(f)
            if isinstance(old, dict) and isinstance(old.get("entries"), list):
                doc = old
        doc["entries"] = [e for e in doc["entries"]
                          if (e.get("precision"), e.get("workload")) != (out["precision"],
                                                                        out["workload"])]
        doc["entries"].append(out)
        with open(args.write, "w") as f:
            json.dump(doc, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=4)
    a = sub.add_parser("apply")
    a.add_argument("--gen-device", action="store_true", help="ground states computed on the GPU")
    a.add_argument("--config", type=int, default=1)
    a.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    a.add_argument("--omega-index", type=int, default=-1, help="-1: every frequency")
    a.add_argument("--nvec", type=int, default=0)
    a.add_argument("--out", default="")
    a.add_argument("--warmup", action="store_true", help="one untimed apply first")
    a.add_argument("--precond", action="store_true",
                   help="preconditioned COCG (Kronecker shifted-Laplacian preconditioner)")
    a.add_argument("--block", type=int, default=0,
                   help="block COCG width (options.cocg_block; 0: single systems)")
    a.add_argument("--refine-tol", type=float, default=0.0,
                   help="mixed: refine_tol (0: the library default)")
    a.add_argument("--mixed-min-omega", type=float, default=-1.0,
                   help="mixed: options.mixed_min_omega (negative: the library default; 0: "
                        "complex64 at every frequency)")
    a.add_argument("--box", action="store_true",
                   help="an isolated (Dirichlet) box of the workload's grid instead of its cell")
    ss = sub.add_parser("subspace")
    ss.add_argument("--gen-device", action="store_true")
    ss.add_argument("--config", type=int, default=2)
    ss.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ss.add_argument("--omega-index", type=int, default=0)
    ss.add_argument("--iters", type=int, default=1)
    ss.add_argument("--out", default="")
    st = sub.add_parser("stages")
    st.add_argument("trace")
    st.add_argument("--run", required=True, help="JSON written by `subspace --out`")
    kr = sub.add_parser("krange")
    kr.add_argument("trace")
    kr.add_argument("--match", required=True, help="substring of the kernel name")
    kr.add_argument("--first", type=int, required=True)
    kr.add_argument("--last", type=int, required=True)
    kr.add_argument("--also", nargs=3, action="append", default=[],
                    metavar=("MATCH", "FIRST", "LAST"), help="a further kernel range")
    gp = sub.add_parser("gaps")
    gp.add_argument("trace")
    gp.add_argument("--skip", type=int, default=0, help="leading dispatches to drop (set-up)")
    s = sub.add_parser("summarize")
    s.add_argument("csv")
    s.add_argument("--match", default="")
    k = sub.add_parser("kstats")
    k.add_argument("csv")
    k.add_argument("--top", type=int, default=25)
    t = sub.add_parser("traffic")
    t.add_argument("--precision", default="fp64")
    t.add_argument("--copy-mib", type=int, default=1024)
    t.add_argument("--copy-reps", type=int, default=4)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--apply-fetch", required=True)
    t.add_argument("--apply-write", required=True)
    t.add_argument("--apply-stats", required=True)
    t.add_argument("--write", default="")
    args = ap.parse_args()
    {"copy": cmd_copy, "apply": cmd_apply, "subspace": cmd_subspace, "stages": cmd_stages,
     "summarize": cmd_summarize, "kstats": cmd_kstats, "traffic": cmd_traffic,
     "gaps": cmd_gaps, "krange": cmd_krange}[args.cmd](args)


if __name__ == "__main__":
    main()
