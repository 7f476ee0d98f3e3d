"""Training sets for the rank predictor: ranks the solver itself measures.

Boundaries come from the seeded random-star generator (the batch workload's
recipe); each group of boundaries is compressed in one batched context at one
ID tolerance, and the context's box table (features and measured ranks of
every compressed box) is collected.  Training and inference then run on the
GPU through the C-ABI (symhss_predictor_train / _predict); nothing here does
arithmetic of the solver or of the network.
"""

from __future__ import annotations

import numpy as np

from . import binding


def measured_boxes(boundaries, media, tol: float, leaf: int = 128, n_proxy: int = 64):
    """Compress the boundaries at `tol`; return (features, ranks) of every box."""
    s = binding.Solver(0)
    try:
        s.assemble_batch(boundaries, media, leaf=leaf, tol=tol, n_proxy=n_proxy)
        s.compress()
        feat, rank, _ = s.box_table()
    finally:
        s.close()
    return feat, rank.astype(np.float32)


def training_set(seeds=range(1000, 1100), tols=(1e-6, 1e-8, 1e-10, 1e-12), leaf: int = 128,
                 group: int = 25):
    """Solver-measured samples from one random star per seed (the batch
    generator's recipe), seed i compressed at tols[i % len(tols)]."""
    import workloads
    by_tol = {t: [] for t in tols}
    for i, sd in enumerate(seeds):
        wl = workloads.config3_batch(seed=sd, count=1, leaf=leaf)[0]
        by_tol[tols[i % len(tols)]].append(wl)
    feats, ranks = [], []
    for t, wls in by_tol.items():
        for g in range(0, len(wls), group):
            chunk = wls[g:g + group]
            f, r = measured_boxes([w.boundary() for w in chunk], [(w.k0, w.k1, w.eps0, w.eps1) for w in chunk],
                                  tol=t, leaf=leaf)
            feats.append(f)
            ranks.append(r)
    return np.concatenate(feats), np.concatenate(ranks)
