"""The aggregation chain on the device (pairwise passes as matching rounds,
Galerkin products per coarse row) against the host chain and the oracle:
the same aggregates and the same coarse matrices, bit for bit.  A block
pattern that is not structurally symmetric takes the host chain."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_08594_amd import msp, synth

pytestmark = pytest.mark.gpu


def announce(*a):
    print("[case]", *a, flush=True)


def assert_same_hierarchy(a, b):
    assert a.nlevels == b.nlevels
    for l in range(b.nlevels):
        x, y = a.level(l), b.level(l)
        assert x["n"] == y["n"], f"level {l} size"
        assert np.array_equal(x["row_ptr"], y["row_ptr"]), f"level {l} row_ptr"
        assert np.array_equal(x["col_ind"], y["col_ind"]), f"level {l} col_ind"
        assert np.array_equal(x["val"], y["val"]), f"level {l} values"
        if l < b.nlevels - 1:
            assert np.array_equal(x["agg"], y["agg"]), f"level {l} aggregates"


CHAIN_CASES = [
    # equal permeability everywhere: equal strengths, every tie rule in play
    ("uniform16x16x8b3", lambda: synth.lognormal_grid(16, 16, 8, 3, 1, 0.0, 1.0, "corners2"), 64),
    ("grid40x40x12b4", lambda: synth.lognormal_grid(40, 40, 12, 4, 10, 1.5, 0.1, "lateral4"),
     1000),
    ("grid33x17x5b2", lambda: synth.lognormal_grid(33, 17, 5, 2, 9, 1.5, 1.0, "corners2"), 150),
    ("layered24x60x25b4-stall", lambda: synth.layered_grid(24, 60, 25, 4, 0), 100),
    ("cfg1-64x64x32b4", lambda: synth.config(1), 10000),
]


@pytest.mark.parametrize("name,mk,mc", CHAIN_CASES, ids=[c[0] for c in CHAIN_CASES])
def test_device_chain_equals_host_chain(name, mk, mc):
    sys_ = mk()
    announce(name, f"n={sys_.n} b={sys_.b} max_coarse={mc}")
    d = msp.Solver(max_coarse=mc)
    h = msp.Solver(max_coarse=mc, host_chain=True)
    d.setup(sys_)
    h.setup(sys_)
    assert d.nlevels >= 2
    assert_same_hierarchy(d, h)
    # and the solve that follows is the same
    xd, infd = d.solve(sys_.rhs, rtol=1e-6)
    xh, infh = h.solve(sys_.rhs, rtol=1e-6)
    assert infd["iterations"] == infh["iterations"]
    assert np.array_equal(xd.cpu().numpy(), xh.cpu().numpy())
    d.close()
    h.close()


def _drop_block(sys_, row):
    """The same system without the first off-diagonal block of `row` (the
    block pattern is then not structurally symmetric)."""
    rp, ci = sys_.row_ptr.astype(np.int64), sys_.col_ind
    k = next(k for k in range(rp[row], rp[row + 1]) if ci[k] != row)
    keep = np.ones(len(ci), dtype=bool)
    keep[k] = False
    rp2 = rp.copy()
    rp2[row + 1:] -= 1
    ci2 = ci[keep]
    rows = np.repeat(np.arange(sys_.n), np.diff(rp2))
    return dataclasses.replace(sys_, name=sys_.name + "-asym", row_ptr=rp2.astype(np.int32),
                               col_ind=ci2, vals=sys_.vals[keep],
                               diag_pos=np.nonzero(ci2 == rows)[0])


def test_asymmetric_pattern_takes_the_host_chain():
    sys_ = _drop_block(synth.lognormal_grid(20, 18, 9, 3, 5, 1.5, 0.1, "lateral4"), 57)
    announce(sys_.name, f"n={sys_.n} nnzb={sys_.nnzb}")
    d = msp.Solver(max_coarse=200)
    h = msp.Solver(max_coarse=200, host_chain=True)
    o = O.OracleSolver(max_coarse=200)
    d.setup(sys_)
    h.setup(sys_)
    o.setup(sys_)
    assert_same_hierarchy(d, h)
    assert_same_hierarchy(d, o)
    d.close()
    h.close()
    o.close()


def test_reuse_and_regeneration_keep_the_device_chain_exact():
    """Two systems of different size through one context: each regeneration
    builds its own chain (work arrays sized for the new level 0)."""
    d = msp.Solver(max_coarse=100)
    h = msp.Solver(max_coarse=100, host_chain=True)
    for sys_ in (synth.lognormal_grid(30, 20, 10, 3, 3, 1.5, 0.1, "lateral4"),
                 synth.lognormal_grid(12, 12, 6, 4, 4, 1.0, 1.0, "corners2")):
        announce(sys_.name, f"n={sys_.n}")
        d.setup(sys_)
        h.setup(sys_)
        assert_same_hierarchy(d, h)
    d.close()
    h.close()
