"""Write tests/golden/c4_reference.npz: exact (P1) optima of a sample of the
4800 x 2100 cross-and-bouquet workload (300 subjects x 7 columns, 2048 test
vectors with a per-instance corruption fraction U[0, 0.5]).

Calls only the oracle: the split linear program of Sec. III-A solved by
HiGHS (``oracle.p1_lp``) on the materialised matrix [B, I], and the FP64
optimality report (``oracle.kkt_report``, LP duality of Sec. III-A / V-B),
which must certify every stored optimum: relative primal residual, dual
infeasibility and sign disagreement <= 1e-9, relative duality gap <= 1e-8
(the solver's 1e-10 feasibility tolerances leave gaps of a few 1e-9 on
these 4800-row problems; the goldens are used at 1e-4 and 1e-3).  The sample is chosen from
the generator's corruption fractions alone: the five most corrupted
instances of the batch (above 48 %), two near 35 % and one near 10 %.

Usage: python tests/golden/make_c4_reference.py [--procs 8]
(8 to 14 minutes of one core per instance; each instance's result is kept
in a part file until all are done).
"""
import argparse
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import p1_lp, full_matrix, kkt_report  # noqa: E402
from workloads.generators import cab_dictionary, cab_instances, _rng  # noqa: E402

M, CLASSES, PER, N, CFG = 4800, 300, 7, 2048, 4
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_reference.npz")


def fractions():
    """Corruption fraction of every instance, drawn as cab_instances draws it."""
    ps = np.empty(N)
    for j in range(N):
        r = _rng(CFG, 1, j)
        r.integers(CLASSES)
        r.dirichlet(np.ones(PER))
        ps[j] = r.uniform(0.0, 0.5)
    return ps


def sample(ps):
    order = np.argsort(-ps)
    pick = list(order[:5])
    for target in (0.35, 0.35, 0.10):
        for j in np.argsort(np.abs(ps - target)):
            if j not in pick:
                pick.append(int(j))
                break
    return [int(j) for j in pick]


def solve_one(j):
    part = OUT.replace(".npz", f".part{j}.npz")
    if os.path.exists(part):
        d = np.load(part)
        return j, d["w"], d["y"], dict(zip(("primal", "dual_inf", "sign", "gap"), d["kkt"]))
    t = time.time()
    B = cab_dictionary(M, CLASSES, PER, cfg=CFG)
    b, _, x0, _ = cab_instances(B, 1, PER, frac="uneven", cfg=CFG, first=j)
    Af = full_matrix(B, "cab")
    w, y = p1_lp(Af, b[:, 0])
    rep = kkt_report(Af, b[:, 0].astype(np.float64), w, y)
    print(f"instance {j}: {time.time() - t:.0f} s, kkt {rep}", flush=True)
    np.savez(part, w=w, y=y, kkt=np.array([rep["primal"], rep["dual_inf"], rep["sign"], rep["gap"]]))
    return j, w, y, rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    ps = fractions()
    idx = sample(ps)
    print("instances", idx, "fractions", np.round(ps[idx], 3).tolist(), flush=True)
    with Pool(args.procs) as pool:
        res = sorted(pool.map(solve_one, idx), key=lambda t: idx.index(t[0]))
    W = np.stack([r[1] for r in res], axis=1)
    rep = np.array([[r[3]["primal"], r[3]["dual_inf"], r[3]["sign"], r[3]["gap"]] for r in res])
    assert np.all(rep[:, :3] <= 1e-9) and np.all(rep[:, 3] <= 1e-8), rep
    np.savez_compressed(OUT, idx=np.array(idx), frac=ps[idx], w=W, kkt=rep)
    for j in idx:
        os.remove(OUT.replace(".npz", f".part{j}.npz"))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
