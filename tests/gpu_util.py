"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import numpy as np

from paper_2404_02950_amd import shamr


def decompose(M: int, cuts=None):
    """Boxes tiling [0, M)^3; ``cuts`` = per-axis lists of interior cut positions."""
    if cuts is None:
        return [(0, 0, 0, M - 1, M - 1, M - 1)]
    edges = [[0] + list(c) + [M] for c in cuts]
    out = []
    for z0, z1 in zip(edges[2][:-1], edges[2][1:]):
        for y0, y1 in zip(edges[1][:-1], edges[1][1:]):
            for x0, x1 in zip(edges[0][:-1], edges[0][1:]):
                out.append((x0, y0, z0, x1 - 1, y1 - 1, z1 - 1))
    return out


def single_level(U0, L=None, boxes=None, prec=shamr.SH_F64, cfl=0.25, eta0=0.1, lam=1.0, alpha=2.0, beta=2):
    """A GPU hierarchy holding one periodic level initialised with the dense state U0."""
    M = U0.shape[-1]
    h = shamr.Hierarchy(M, float(M) if L is None else L, cfl, eta0, lam, alpha, beta, max_level=0, prec=prec)
    h.set_layout(0, boxes if boxes is not None else decompose(M))
    h.write_dense(0, U0)
    h.fill_ghosts(0)
    return h


def assert_bitwise(a, b, what=""):
    """Equal bit for bit, NaN positions included."""
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, what
    same = (a == b) | (np.isnan(a) & np.isnan(b))
    if not same.all():
        i = np.argwhere(~same)[0]
        raise AssertionError(f"{what}: {np.count_nonzero(~same)} values differ, first at {tuple(i)}: "
                             f"{a[tuple(i)]!r} vs {b[tuple(i)]!r}")
