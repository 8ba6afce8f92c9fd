"""Launch-shape autotuner for the batched COCG kernel.

For one workload and precision it times one chi0 block-apply per candidate shape
(columns per thread C, z-planes per step Z, launch-bound bucket, row slabs per plane) using
the COCG kernel's own HIP-event time reported in rpa_stats, and writes the fastest shape per
(precision, grid) to a tuning file that the library reads (RPA_TUNE_FILE, default
cocg_shapes.txt next to the shared library).

Usage: python -m paper_2504_01816_amd.autotune --config 1 [--precision fp64|mixed]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TUNE_FILE = os.path.join(HERE, "cocg_shapes.txt")


def candidates(n0, n1, n2, whole=True):
    """(C, Z, bsmax, bs, occ, nslab): for the whole plane (nslab = 1) and for row slabs of
    at least 12 rows (one column per thread, at least 12 n0 threads), the tightest block and
    the block rounded up to whole 4-wave groups (one wave per SIMD per group, so the four
    SIMDs get equal work)."""
    out = []
    splits = [(C, 1) for C in (1, 2, 3)] if whole else []
    splits += [(1, ns) for ns in range(2, n1 // 12 + 1) if n1 % ns == 0]
    for C, nslab in splits:
        P = n0 * (n1 // nslab)
        bs0 = ((P + C - 1) // C + 63) // 64 * 64
        for bs in sorted({bs0, (bs0 + 255) // 256 * 256}):
            if nslab > 1 and bs < 12 * n0:
                continue
            for BM in (512, 768, 1024):
                lower = {512: 0, 768: 512, 1024: 768}[BM]
                if not (lower < bs <= BM):
                    continue
                for Z in ((1, 2) if nslab > 1 else (1, 2, 4)):
                    if n2 % Z == 0 and (Z <= 2 or C <= 2):
                        out.append((C, Z, BM, bs, 0, nslab))
    return out


def time_shape(api, cell, omega, X, opts, shape):
    os.environ["RPA_COCG_SHAPE"] = "%d,%d,%d,%d,%d,%d" % shape
    try:
        out, rc, st = api.rpa_apply_chi0(cell, omega, X, opts)
    except RuntimeError as e:
        return None, str(e)
    finally:
        del os.environ["RPA_COCG_SHAPE"]
    return st, None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--omega-index", type=int, default=4)
    ap.add_argument("--nvec", type=int, default=0, help="trial vectors (0 = N_r)")
    ap.add_argument("--cell", type=int, default=0, help="cell of a several-cell workload")
    ap.add_argument("--write", default="", help="tuning file to record the best shape in")
    ap.add_argument("--gen-device", action="store_true", help="ground states computed on the GPU")
    ap.add_argument("--slabs-only", action="store_true",
                    help="only row-slab shapes (large planes, whose whole-plane shapes spill)")
    args = ap.parse_args()
    import torch

    from . import api, synth
    from . import lib as L

    wl = synth.workload(args.config, device="cuda:0" if args.gen_device else None)
    c = wl.cells[args.cell]
    dc = api.device_cell(c, "cuda:0")
    nvec = args.nvec or wl.n_r[args.cell]
    X = torch.tensor(wl.V0[args.cell][:nvec], device="cuda:0")
    X = api.rpa_apply_coulomb(dc, X, 1)
    omega = float(wl.omegas[min(args.omega_index, len(wl.omegas) - 1)])
    prec = L.RPA_FP64 if args.precision == "fp64" else L.RPA_MIXED
    opts = dict(precision=prec, cocg_tol=wl.cocg_tol)
    bpp = 96.0 if args.precision == "fp64" else 48.0
    rows = []
    api.rpa_apply_chi0(dc, omega, X, opts)               # warm-up with the default shape
    for shape in candidates(*c.shape, whole=not args.slabs_only):
        st, err = time_shape(api, dc, omega, X, opts, shape)
        if st is None:
            print("shape C=%d Z=%d bsmax=%d bs=%d occ=%d nslab=%d: %s" % (shape + (err,)),
                  flush=True)
            continue
        gbs = bpp * st["cocg_point_iters"] / (st["cocg_kernel_ms"] * 1e-3) / 1e9
        rows.append(dict(C=shape[0], Z=shape[1], bsmax=shape[2], bs=shape[3], occ=shape[4],
                         nslab=shape[5], ms=st["cocg_kernel_ms"], alg_GBs=gbs,
                         iters=st["cocg_iters_total"]))
        print("shape C=%d Z=%d bsmax=%4d bs=%4d occ=%d nslab=%d: %8.2f ms  %7.1f GB/s "
              "algorithmic  iters %d" % (shape + (st["cocg_kernel_ms"], gbs, st["cocg_iters_total"])),
              flush=True)
    _, _, st0 = api.rpa_apply_chi0(dc, omega, X, opts)
    print("default choice: %.2f ms" % st0["cocg_kernel_ms"], flush=True)
    if rows:
        best = min(rows, key=lambda r: r["ms"])
        print(json.dumps({"workload": wl.name, "precision": args.precision, "omega": omega,
                          "best": best}), flush=True)
        if args.write:
            key = "%s %d %d %d" % (args.precision, *c.shape)
            lines = []
            if os.path.exists(args.write):
                lines = [l for l in open(args.write) if not l.startswith(key + " ")]
            lines.append("%s %d %d %d %d %d %d\n" % (key, best["C"], best["Z"], best["bsmax"],
                                                      best["bs"], best["occ"], best["nslab"]))
            open(args.write, "w").writelines(lines)


if __name__ == "__main__":
    sys.exit(main())
