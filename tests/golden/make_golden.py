"""Write the stored expected values of the full-length parity tests from the FP64 CPU oracle.

Only the oracle and the seeded input generators are called.  Each output file
holds, for one workload run for its full step count, the concentrations
C1, C2, C3 at a seeded sample of nodes and the sum of each field over all
nodes, written with 17 significant digits.

    python tests/golden/make_golden.py [spinodal2d] [spinodal3d] [batched] [adjoint]

Run times on 8 shared cores: spinodal2d ~50 min, spinodal3d ~6.5 h, batched ~30 min
(each domain also with FP32-storage rounding, one step at a time), adjoint ~1 min.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))  # tests/: the FP32-storage model of the oracle

import oracle  # noqa: E402
from paper_1511_02155_amd import inputs  # noqa: E402

KEYS = ("lattice", "nx", "ny", "nz", "walls_y", "kappa", "alpha", "tau_f", "tau_g", "tau_k", "gamma_phi", "gamma_psi")
NSAMPLE = 512


def sample_nodes(N, seed, n=NSAMPLE):
    """Seeded sample of node indices (first and last node always included)."""
    idx = np.random.default_rng(seed).choice(N, size=min(n, N) - 2, replace=False)
    return np.unique(np.concatenate([[0, N - 1], idx]))


def run(w, C, h, steps):
    p = oracle.Params(**{k: w[k] for k in KEYS})
    pop = oracle.init_equilibrium(p, C, None, h)
    oracle.step(p, pop, steps, h)
    return p, oracle.fields(p, pop, h)


def write(name, header, F, nodes, extra=None):
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        for line in header:
            fh.write(f"# {line}\n")
        fh.write("# written by tests/golden/make_golden.py from the FP64 CPU oracle\n")
        for k, v in (extra or {}).items():
            fh.write(f"scalar {k} {float(v)!r}\n")
        for f in ("C1", "C2", "C3"):
            fh.write(f"sum {f} {float(F[f].sum())!r}\n")
        for n in nodes:
            fh.write(f"node {int(n)} {float(F['C1'][n])!r} {float(F['C2'][n])!r} {float(F['C3'][n])!r}\n")
    print("wrote", path, flush=True)


def spinodal2d():
    w = inputs.spinodal_2d(1024, 10000)
    p, F = run(w, w["C"](), None, w["steps"])
    write("spinodal_2d_1024_10000.txt",
          ["D2Q9 1024x1024 periodic spinodal decomposition (Sec. V.C phase separation), 10000 steps",
           "C1, C2 = 1/3 + U(-0.01, 0.01) (seed 2), kappa = (0.01, 0.015, 0.02), alpha = 1, tau = 1, M = 0.1"],
          F, sample_nodes(p.N, 102))


def spinodal3d():
    w = inputs.spinodal_3d(256, 2000)
    p, F = run(w, w["C"](), None, w["steps"])
    write("spinodal_3d_256_2000.txt",
          ["D3Q19 256^3 periodic spinodal decomposition (Sec. V.C phase separation), 2000 steps",
           "C1, C2 = 1/3 + U(-0.01, 0.01) (seed 3), kappa = 0.01, alpha = 1, tau = 0.8, M = 0.05"],
          F, sample_nodes(p.N, 103))


def batched_picks(doms):
    sizes = [d["nx"] * d["ny"] for d in doms]
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes))}
    pick |= set(int(i) for i in np.random.default_rng(104).choice(len(doms), 2, replace=False))
    return sorted(pick)


def batched():
    """Each picked domain twice: the FP64 oracle, and the FP64 oracle whose stored state is rounded as FP32
    storage rounds it after every step (the state an FP32-storage run holds, up to its own arithmetic).  The
    second file also records the largest difference between the two over all nodes (the storage floor)."""
    from storage32 import run_fp32_storage

    doms = inputs.batched_walls()
    for i in batched_picks(doms):
        d = doms[i]
        head = [f"domain {i} of the 512-domain walled D2Q9 batch (seed 4): {d['nx']}x{d['ny']}, 5000 steps",
                f"kappa = {tuple(float(k) for k in d['kappa'])}, h = {tuple(float(v) for v in d['h'][0][:, 0])} "
                "on both walls, tau = 1, M = 0.1, alpha = 1"]
        nodes = sample_nodes(d["nx"] * d["ny"], 105 + i, 256)
        p, F = run(d, d["C"], d["h"], d["steps"])
        write(f"batched_domain{i:03d}_5000.txt", head, F, nodes)
        pop = oracle.init_equilibrium(p, d["C"], None, d["h"])
        run_fp32_storage(oracle, p, pop, d["steps"], d["h"])
        G = oracle.fields(p, pop, d["h"])
        floor = {f"floor_{f}": float(np.abs(G[f] - F[f]).max()) for f in ("C1", "C2", "C3")}
        write(f"batched_domain{i:03d}_5000_storage32.txt",
              head + ["state rounded to FP32 after every step (populations relative to w_i, 0, 1/3 for f, g, k_0)",
                      "scalar floor_Cm = max over all nodes of |C_m(rounded run) - C_m(FP64 run)|"],
              G, nodes, extra=floor)


def adjoint():
    w = inputs.adjoint_drop_512()
    p, F = run(w, w["C"], w["h"], w["steps"])
    L = float(((F["C1"] - w["target"]) ** 2).sum())
    write("adjoint_drop_512_forward_2000.txt",
          ["D2Q9 512x512 walled sessile drop of the gradient problem, forward run of 2000 steps",
           "per-node h on the lower wall U[-0.01, 0.01] (seed 5), target drop (seed 6), kappa = 0.01, tau = 1, M = 0.1",
           "scalar loss = sum over nodes of (C1 - C1_target)^2 after the run"],
          F, sample_nodes(p.N, 106), extra={"loss": L})


if __name__ == "__main__":
    todo = sys.argv[1:] or ["batched", "adjoint", "spinodal2d", "spinodal3d"]
    oracle.build()
    for t in todo:
        t0 = time.time()
        globals()[t]()
        print(f"{t}: {time.time() - t0:.0f} s", flush=True)
