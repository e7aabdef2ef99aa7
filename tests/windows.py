"""Windows of seeded initial fields for the full-size parity checks (index bookkeeping only, no
numerical method code).

A node's state after k steps depends on the initial fields within a fixed distance of it (the
pull reaches one spacing per step, the derivative stencils of the double distribution one or
two more per collision). The oracle therefore runs on a window of the initial fields around the
checked nodes and reproduces them exactly, even though the window's own edges are wrong (they
wrap, or act as walls, in the oracle); the margins below are chosen larger than that distance.
"""
import numpy as np


def periodic_box(a, centre, radius, lead=0):
    """Sub-array of `a` on a box of side 2 radius + 1 around `centre` (one index per spatial
    axis, the last len(centre) axes of `a`), with periodic wrap; `lead` leading axes (components)
    are kept whole."""
    idx = []
    for ax, c in enumerate(centre):
        n = a.shape[lead + ax]
        idx.append([(c + d) % n for d in range(-radius, radius + 1)])
    return a[(Ellipsis,) + np.ix_(*idx)] if lead else a[np.ix_(*idx)]


def rows(a, lo, hi, axis=-2):
    """Rows lo..hi-1 of `a` along `axis` (no wrap)."""
    sl = [slice(None)] * a.ndim
    sl[axis] = slice(lo, hi)
    return a[tuple(sl)]


def wall_blocks(a, depth, axis=-2):
    """The first and the last `depth` rows along `axis`, stacked: a window whose two ends are
    the lattice's real walls (the junction in the middle is far from both)."""
    n = a.shape[axis]
    return np.concatenate([rows(a, 0, depth, axis), rows(a, n - depth, n, axis)], axis=axis)
