"""Seeded choice of the primitives whose gradients are checked one by one at
the benchmark size (the 200-primitive subset of the training-step workload).
Test infrastructure: it only reads the oracle's projection."""
import numpy as np

# (min tiles, max tiles, how many): every size class of the frame, with the
# large primitives (tens to hundreds of tiles, the longest transmittance
# chains and the most per-wavefront atomic adds) represented on purpose
STRATA = ((1, 1, 30), (2, 4, 70), (5, 9, 36), (10, 49, 40), (50, 199, 20), (200, 400, 4))


def stratified_primitives(pr, seed: int, strata=STRATA):
    """Visible, well-conditioned primitives drawn without replacement from
    each tile-count class (fewer where a class has fewer members).  Returns
    an int64 array, class by class."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vis = pr.visible.numpy() & ~pr.fragile_prim
    out = []
    for lo, hi, n in strata:
        pool = np.nonzero(vis & (pr.tiles >= lo) & (pr.tiles <= hi))[0]
        if len(pool):
            out.append(np.sort(rng.choice(pool, size=min(n, len(pool)), replace=False)))
    return np.concatenate(out).astype(np.int64)
