"""The list build's bin layout and stencil row table (host logic, no GPU).

For random cells (triclinic, thin, partly open) and cutoffs from 12 to 50 A,
every pair within the list cutoff found by brute force must fall into a bin
offset the build visits: within the stencil reach and, when the stencil has
a row table, inside its row's span; every pair within the R_cn list cutoff
must fall into one of the rows listed first.  Atoms are binned the way the
binning kernel does it (fractional coordinates, wrapped on periodic axes,
clamped into the edge bins otherwise), so a trimming that drops a bin which
can hold a pair fails here.
"""

import itertools

import numpy as np
import pytest

from paper_2310_05279_amd import d3


def _bins(pos, cell, pbc, nb):
    hinv = np.linalg.inv(cell)
    s = pos @ hinv
    wrapped = pos.copy()
    b = np.zeros(pos.shape, np.int64)
    for k in range(3):
        if pbc[k]:
            f = np.floor(s[:, k])
            wrapped -= f[:, None] * cell[k][None, :]
            q = np.floor((s[:, k] - f) * nb[k])
        else:
            q = np.floor(s[:, k] * nb[k])
        b[:, k] = np.clip(q, 0, nb[k] - 1)
    return wrapped, b


def _check(cell, pbc, rlist, rcn, pos):
    n = pos.shape[0]
    plan = d3.d3_bin_plan(cell, pbc, rlist, rcn, n)
    nb, reach, rows, ncn = plan["nb"], plan["reach"], plan["rows"], plan["ncnrows"]
    # row spans indexed by (d1, d2); rows the table leaves out keep lo > hi
    lo_t = np.full((2 * reach[1] + 1, 2 * reach[2] + 1), 1 << 30)
    hi_t = np.full_like(lo_t, -(1 << 30))
    idx_t = np.full_like(lo_t, 1 << 30)
    for i, (d1, d2, lo, hi) in enumerate(rows):
        lo_t[d1 + reach[1], d2 + reach[2]] = lo
        hi_t[d1 + reach[1], d2 + reach[2]] = hi
        idx_t[d1 + reach[1], d2 + reach[2]] = i
    wrapped, b = _bins(pos, np.asarray(cell), pbc, nb)
    timg = [int(np.ceil(reach[k] / nb[k])) + 1 if pbc[k] else 0 for k in range(3)]
    checked = 0
    for t in itertools.product(*[range(-m, m + 1) for m in timg]):
        T = np.asarray(t, dtype=np.float64) @ np.asarray(cell)
        d = wrapped[None, :, :] + T[None, None, :] - wrapped[:, None, :]
        r2 = np.einsum("ijk,ijk->ij", d, d)
        ii, jj = np.nonzero(r2 < rlist * rlist)
        if not any(t):
            keep = ii != jj
            ii, jj = ii[keep], jj[keep]
        if ii.size == 0:
            continue
        off = b[jj] + np.asarray(t)[None, :] * nb[None, :] - b[ii]
        assert np.all(np.abs(off) <= reach[None, :]), "pair outside the stencil reach"
        if len(rows):
            inc = r2[ii, jj] < rcn * rcn
            r1, r2i = off[:, 1] + reach[1], off[:, 2] + reach[2]
            assert np.all((lo_t[r1, r2i] <= off[:, 0]) & (off[:, 0] <= hi_t[r1, r2i])), \
                "pair in a trimmed bin"
            assert np.all(idx_t[r1, r2i][inc] < ncn), "R_cn pair in a row after the R_cn rows"
        checked += ii.size
    return plan, checked


@pytest.mark.parametrize("rlist", [12.0, 20.0, 30.0, 50.0])
def test_orthorhombic_periodic(rlist):
    rng = np.random.default_rng(int(rlist))
    L = np.array([20.5, 19.0, 21.3])  # 0.035 atoms per A^3
    cell = np.diag(L)
    n = 300
    pos = rng.uniform(0, 1, (n, 3)) * L
    plan, checked = _check(cell, (1, 1, 1), rlist, rlist / 2, pos)
    assert checked > n
    if rlist >= 20.0:
        assert len(plan["rows"]) > 0 and plan["ncnrows"] < len(plan["rows"])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_triclinic_periodic_long(seed):
    rng = np.random.default_rng(seed)
    cell = np.array([[30.0, 0.0, 0.0], [9.0, 27.0, 0.0], [-5.0, 6.0, 29.0]])
    cell += rng.normal(scale=1.0, size=(3, 3))
    pos = rng.uniform(-0.2, 1.2, (250, 3)) @ cell  # some atoms outside the cell
    plan, checked = _check(cell, (1, 1, 1), 30.0, 15.0, pos)
    assert len(plan["rows"]) > 0 and checked > 0


@pytest.mark.parametrize("pbc", [(1, 1, 0), (1, 0, 1), (0, 1, 1), (0, 0, 1)])
def test_open_axes_long(pbc):
    """Along an open axis atoms may lie outside the cell and join its edge
    bins; the table must not trim along that axis."""
    rng = np.random.default_rng(sum(pbc) * 7 + pbc[0])
    cell = np.array([[26.0, 0.0, 0.0], [6.0, 24.0, 0.0], [2.0, -3.0, 22.0]])
    s = rng.uniform(0, 1, (260, 3))
    for k in range(3):
        if not pbc[k]:
            s[:, k] = rng.uniform(-0.4, 1.4, s.shape[0])
    pos = s @ cell
    plan, checked = _check(cell, pbc, 25.0, 12.5, pos)
    assert checked > 0


def test_thin_cell_short_cutoff():
    """A cell thinner than the cutoff along one axis: several images of every
    atom, bins wider than R/3 along that axis."""
    rng = np.random.default_rng(9)
    cell = np.array([[18.0, 0.0, 0.0], [3.0, 17.0, 0.0], [0.0, 1.0, 5.5]])
    pos = rng.uniform(0, 1, (120, 3)) @ cell
    plan, checked = _check(cell, (1, 1, 1), 13.0, 7.0, pos)
    assert checked > 0


def test_bin_plan_rejects_bad_arguments():
    with pytest.raises(d3.D3Error):
        d3.d3_bin_plan(np.eye(3) * 10, (1, 1, 1), 5.0, 6.0, 10)   # rcn > rlist
    with pytest.raises(d3.D3Error):
        d3.d3_bin_plan(np.zeros((3, 3)), (1, 1, 1), 12.0, 6.0, 10)  # singular cell
