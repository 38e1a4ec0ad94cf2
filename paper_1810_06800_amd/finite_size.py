"""Thresholds over an (L, k) grid on the batched engine, with the paper's
finite-size extrapolations (Sec. II.A, Eqs. 9-10, Table I).

For each k and each ratio L/k, ``samples`` independent runs give
p_c = n_wrap_any * k / L^2 and p_j = n_jam * k / L^2 (mean and standard error
of the mean).  The infinite-lattice values are then read off straight-line
fits: p_c(L) against (L/k)^(-1/nu) with nu = 4/3 (Eq. 9) and p_j(L) against
1/L (Eq. 10), each extrapolated to zero.  Every run goes through the
library's kernels; only the means and the fits are host arithmetic.

    python -m paper_1810_06800_amd.finite_size --k 1,2,4,8 --ratios 16,32,64 --samples 256
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

NU = 4.0 / 3.0


def mean_sem(values):
    n = len(values)
    m = sum(values) / n
    if n < 2:
        return m, float("nan")
    var = sum((v - m) ** 2 for v in values) / (n - 1)
    return m, math.sqrt(var / n)


def line_fit(xs, ys, ws=None):
    """Weighted least squares y = a + b*x: (a, b, standard error of a)."""
    ws = ws or [1.0] * len(xs)
    sw = sum(ws)
    sx = sum(w * x for w, x in zip(ws, xs))
    sy = sum(w * y for w, y in zip(ws, ys))
    sxx = sum(w * x * x for w, x in zip(ws, xs))
    sxy = sum(w * x * y for w, x, y in zip(ws, xs, ys))
    det = sw * sxx - sx * sx
    if det == 0:
        raise ValueError("degenerate fit")
    b = (sw * sxy - sx * sy) / det
    a = (sy - b * sx) / sw
    return a, b, math.sqrt(sxx / det)


def extrapolate(points, key: str):
    """Infinite-lattice value of p_c (key 'pc', Eq. 9) or p_j ('pj', Eq. 10)
    from [(L, k, mean, sem)], weights 1/sem^2."""
    xs, ys, ws = [], [], []
    for L, k, m, e in points:
        xs.append((L / k) ** (-1.0 / NU) if key == "pc" else 1.0 / L)
        ys.append(m)
        # a cell with no spread (p_j = 1 at k = 1) is exact: give it all the weight
        ws.append(1.0 / (e * e) if e == e and e > 0 else 1e12)
    if len(xs) < 2:
        return None
    a, b, ea = line_fit(xs, ys, ws)
    return {"value": a, "stderr": ea, "slope": b}


def run_grid(ctx, ks, ratios, samples: int, seed: int = 7, log=None, keep: bool = False):
    """Runs every (k, L = r*k) cell as one batch; returns the table (with
    keep=True each row also holds the cell's descriptors and raw results)."""
    rows = []
    for k in ks:
        for r in ratios:
            L = r * k
            if L > 32768:
                continue
            descs = [(L, k, seed + 1000003 * k + r, s, 0) for s in range(samples)]
            t0 = time.perf_counter()
            res = ctx.run(descs)
            dt = time.perf_counter() - t0
            bad = [x for x in res if x["status"] != 0]
            if bad:
                raise RuntimeError(f"({L}, {k}): {len(bad)} runs failed")
            pc = [x["n_wrap_any"] * k / (L * L) for x in res]
            pj = [x["n_jam"] * k / (L * L) for x in res]
            pcm, pce = mean_sem(pc)
            pjm, pje = mean_sem(pj)
            dep = sum(x["n_jam"] for x in res)
            rows.append({"k": k, "L": L, "samples": samples, "pc": pcm, "pc_sem": pce, "pj": pjm,
                         "pj_sem": pje, "seconds": dt, "deposits_per_s": dep / dt})
            if keep:
                rows[-1]["descs"] = descs
                rows[-1]["results"] = res
            if log:
                log(f"k={k} L={L}: p_c {pcm:.4f} +- {pce:.4f}  p_j {pjm:.4f} +- {pje:.4f}  ({dt:.2f} s)")
    return rows


def fits(rows):
    out = {}
    for k in sorted({r["k"] for r in rows}):
        cell = [r for r in rows if r["k"] == k]
        out[k] = {
            "pc_inf": extrapolate([(r["L"], k, r["pc"], r["pc_sem"]) for r in cell], "pc"),
            "pj_inf": extrapolate([(r["L"], k, r["pj"], r["pj_sem"]) for r in cell], "pj"),
        }
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1810_06800_amd.finite_size")
    ap.add_argument("--k", default="1,2,4,8,16,32,64")
    ap.add_argument("--ratios", default="16,32,64")
    ap.add_argument("--samples", type=int, default=256)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    from . import rsa

    ctx = rsa.Context(0)
    rows = run_grid(ctx, [int(v) for v in a.k.split(",")], [int(v) for v in a.ratios.split(",")],
                    a.samples, a.seed, log=lambda m: print(m, flush=True))
    ctx.close()
    out = {"rows": rows, "fits": fits(rows)}
    for k, f in out["fits"].items():
        pc, pj = f["pc_inf"], f["pj_inf"]
        if pc and pj:
            print(f"k={k}: p_c(inf) {pc['value']:.4f} +- {pc['stderr']:.4f}, "
                  f"p_j(inf) {pj['value']:.4f} +- {pj['stderr']:.4f}", flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    sys.exit(main())
