"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Plain FP64 gates: |dE|/atom <= 1e-6 eV, max |dF| <= 1e-5 eV/A; the virial
is held to 1e-9 relative (it is FP64 throughout).  Precision form:
max |dF| <= 1e-4 eV/A, errors of E and W reported.
"""

import numpy as np
import pytest

import synth
from oracle import d3_oracle as O
from oracle import d3_ref as R

pytestmark = pytest.mark.gpu

TAB = synth.make_table()


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


def run_gpu(system, mode="plain", skin=0.0, table=TAB, prm=None, calc_out=False):
    torch = _torch()
    from paper_2310_05279_amd import d3
    calc = d3.D3(table, mode=mode, skin=skin, **(prm or {}))
    calc.build(system["pos"], system["types"], system["cell"], system["pbc"])
    out = calc.compute()
    cn = calc.coordination()
    torch.cuda.synchronize()
    calc.status()
    res = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    res["energy"] = float(res["energy"][0])
    res["cn"] = cn.cpu().numpy()
    res["stats"] = calc.stats()
    if calc_out:
        return res, calc
    calc.close()
    return res


def compare(gpu, ref, n, tol_e=1e-6, tol_f=1e-5, tol_w_rel=1e-9, label=""):
    de = abs(gpu["energy"] - ref["energy"]) / max(n, 1)
    df = np.abs(gpu["forces"] - ref["forces"]).max() if n else 0.0
    wscale = max(np.abs(ref["virial"]).max(), 1e-30)
    dw = np.abs(gpu["virial"] - ref["virial"]).max()
    dae = np.abs(gpu["atom_energy"] - ref["atom_energy"]).max() if n else 0.0
    dcn = np.abs(gpu["cn"] - ref["cn"]).max() if n else 0.0
    print("%s |dE|/atom=%.2e max|dF|=%.2e max|dW|=%.2e (rel %.2e) max|dU_i|=%.2e max|dCN|=%.2e"
          % (label, de, df, dw, dw / wscale, dae, dcn), flush=True)
    assert de <= tol_e
    assert df <= tol_f
    assert dw <= tol_w_rel * wscale + 1e-14
    assert dae <= tol_e
    return de, df, dw


def test_bilayer_graphene_144_plain():
    """6x6 AB bilayer (144 atoms): several images of each atom within R_pot."""
    g = synth.bilayer_graphene()
    ref = O.d3(g["pos"], g["types"], g["cell"], g["pbc"], TAB)
    gpu = run_gpu(g)
    compare(gpu, ref, 144, label="graphene144")
    assert np.abs(gpu["cn"] - ref["cn"]).max() < 1e-12


def test_mof_3000_plain():
    """3000-atom MOF-like cube: many 64-entry tiles per atom, ragged tails."""
    m = synth.mof_like(3000, seed=31)
    ref = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], TAB)
    gpu = run_gpu(m)
    compare(gpu, ref, 3000, label="mof3000")
    assert np.abs(gpu["cn"] - ref["cn"]).max() < 1e-12
    assert gpu["stats"]["max_pot"] > 64 * 4


@pytest.mark.parametrize("case", ["mof3000", "graphene144"])
def test_invariances_relabel_translate_rotate(case):
    """The GPU path under a relabelling of the atoms, a translation (atoms
    leave the cell and are wrapped along its periodic axes) and a rotation
    of cell and positions together (no lattice vector then lies along a
    coordinate axis): the energy is unchanged, forces and site energies are
    relabelled or rotated with the atoms, the virial becomes R W R^T.  The
    inputs differ from the original ones by their own rounding, so the
    bounds are rounding-sized: 1e-12 relative for E and W, 1e-9 eV/A for
    forces (every force is also within the oracle gates of the original)."""
    s = synth.mof_like(3000, seed=31) if case == "mof3000" else synth.bilayer_graphene()
    n = s["pos"].shape[0]
    base = run_gpu(s)
    rng = np.random.default_rng(17)
    perm = rng.permutation(n)
    shift = np.array([3.7, -11.2, 25.3])
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    R = q * np.sign(np.linalg.det(q))  # a proper rotation
    variants = {
        "relabel": (dict(s, pos=s["pos"][perm], types=s["types"][perm]), perm, np.eye(3)),
        "translate": (dict(s, pos=s["pos"] + shift), np.arange(n), np.eye(3)),
        "rotate": (dict(s, pos=s["pos"] @ R.T, cell=s["cell"] @ R.T), np.arange(n), R),
    }
    for name, (sv, idx, rot) in variants.items():
        g = run_gpu(sv)
        de = abs(g["energy"] - base["energy"])
        df = np.abs(g["forces"] - base["forces"][idx] @ rot.T).max()
        du = np.abs(g["atom_energy"] - base["atom_energy"][idx]).max()
        dw = np.abs(g["virial"].reshape(3, 3) - rot @ base["virial"].reshape(3, 3) @ rot.T).max()
        wsc = np.abs(base["virial"]).max()
        print("%s %s: |dE|=%.2e max|dF|=%.2e max|dU_i|=%.2e max|dW|/|W|=%.2e"
              % (case, name, de, df, du, dw / wsc), flush=True)
        assert de <= 1e-12 * abs(base["energy"])
        assert df <= 1e-9 and du <= 1e-12 * np.abs(base["atom_energy"]).max()
        assert dw <= 1e-12 * wsc


def test_tiny_triclinic_cell_many_images():
    """Four atoms in a skewed cell far smaller than R_pot: every atom sees
    hundreds of images of every atom, itself included."""
    cell = np.array([[5.0, 0.0, 0.0], [2.0, 4.6, 0.0], [0.5, 0.7, 5.3]])
    s = np.random.default_rng(2).uniform(0, 1, (4, 3))
    sys_ = {"pos": s @ cell, "types": np.array([0, 1, 2, 4], np.int32), "cell": cell,
            "pbc": np.array([1, 1, 1], np.int32)}
    ref = O.d3(sys_["pos"], sys_["types"], cell, sys_["pbc"], TAB)
    gpu = run_gpu(sys_)
    compare(gpu, ref, 4, label="tiny")


def test_mixed_open_and_periodic_axes_and_unwrapped_positions():
    """Slab periodic in-plane, open along z, with atoms displaced by lattice
    vectors (outside the cell) and atoms outside the cell along the open
    axis: same result as the oracle."""
    m = synth.mof_like(600, seed=8)
    cell = m["cell"].copy()
    pbc = np.array([1, 1, 0], np.int32)
    pos = m["pos"].copy()
    rng = np.random.default_rng(4)
    pos += rng.integers(-2, 3, (600, 1)) * cell[0] + rng.integers(-1, 2, (600, 1)) * cell[1]
    pos[:20, 2] += 3.0 * cell[2, 2] / 4.0  # some beyond the open face
    sys_ = {"pos": pos, "types": m["types"], "cell": cell, "pbc": pbc}
    ref = R.d3(pos, m["types"], cell, pbc, TAB)
    gpu = run_gpu(sys_)
    compare(gpu, ref, 600, label="slab")


def _random_cell_case(seed):
    """A small random cell: skewed lattice vectors of 4-16 A, any mix of
    periodic and open axes, 3-40 atoms of random elements (some outside the
    cell), cutoffs from 5 to 30 A with R_cn from R_pot/4 to R_pot."""
    rng = np.random.default_rng(1000 + seed)
    while True:
        cell = np.diag(rng.uniform(4.0, 16.0, 3)) + rng.uniform(-3.0, 3.0, (3, 3)) * \
            (1 - np.eye(3))
        if abs(np.linalg.det(cell)) > 0.2 * np.prod(np.linalg.norm(cell, axis=1)):
            break
    pbc = rng.integers(0, 2, 3).astype(np.int32)
    n = int(rng.integers(3, 41))
    for _ in range(1000):
        pos = rng.uniform(-0.3, 1.3, (n, 3)) @ cell
        if n < 2 or O.entries(pos, cell, pbc, 0.9)[0].size == 0:
            break
    types = rng.integers(0, 5, n).astype(np.int32)
    r_pot = float(rng.uniform(5.0, 30.0))
    r_cn = float(rng.uniform(0.25, 1.0)) * r_pot
    return {"pos": pos, "types": types, "cell": cell, "pbc": pbc}, dict(r_pot=r_pot, r_cn=r_cn)


@pytest.mark.parametrize("seed", range(16))
def test_random_small_cells(seed):
    """Random small cells against the NumPy oracle in the plain and the
    precision forms: shallow and deep stencils, with and without row tables,
    open axes with atoms beyond their faces, many images."""
    s, prm = _random_cell_case(seed)
    n = s["pos"].shape[0]
    print("random cell %d: n=%d pbc=%s r_pot=%.2f r_cn=%.2f" % (seed, n, s["pbc"], prm["r_pot"],
                                                             prm["r_cn"]), flush=True)
    ref = O.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB, O.Params(**prm))
    gpu = run_gpu(s, prm=prm)
    compare(gpu, ref, n, label="random-%d" % seed)
    gpu = run_gpu(s, mode="prec", prm=prm)
    compare(gpu, ref, n, tol_e=1e-6, tol_f=1e-4, tol_w_rel=1e-5, label="random-prec-%d" % seed)


def test_finite_cluster_no_pbc():
    c = synth.cluster(80, 7.0, seed=5)
    cell = np.eye(3) * 14.0
    sys_ = {"pos": c["pos"] + 7.0, "types": c["types"], "cell": cell,
            "pbc": np.array([0, 0, 0], np.int32)}
    ref = O.d3(sys_["pos"], c["types"], None, (0, 0, 0), TAB)
    gpu = run_gpu(sys_)
    compare(gpu, ref, 80, label="cluster")
    # a finite cluster: the virial is sum_i r_i (x) F_i
    assert np.abs(gpu["virial"] - sys_["pos"].T @ gpu["forces"]).max() < 1e-10


def test_one_context_through_changing_systems():
    """One context built in turn for systems that differ in size, cell,
    periodicity and image count, so that every buffer grows and shrinks and
    the lists, image table and bin layout are re-sized each time: the 144-atom
    bilayer, a 3 000-atom cube, four atoms in a skewed cell smaller than R_pot
    (hundreds of images), an empty system, a slab open along z with atoms
    outside the cell, and a free cluster.  Each against the oracle; then the
    first system again, bit for bit its first result."""
    torch = _torch()
    from paper_2310_05279_amd import d3
    tiny_cell = np.array([[5.0, 0.0, 0.0], [2.0, 4.6, 0.0], [0.5, 0.7, 5.3]])
    m600 = synth.mof_like(600, seed=8)
    slab_pos = m600["pos"].copy()
    slab_pos[:20, 2] += 0.75 * m600["cell"][2, 2]
    c80 = synth.cluster(80, 7.0, seed=5)
    seq = [
        ("bilayer 144", synth.bilayer_graphene()),
        ("cube 3000", synth.mof_like(3000, seed=31)),
        ("tiny skewed", {"pos": np.random.default_rng(2).uniform(0, 1, (4, 3)) @ tiny_cell,
                         "types": np.array([0, 1, 2, 4], np.int32), "cell": tiny_cell,
                         "pbc": np.array([1, 1, 1], np.int32)}),
        ("empty", {"pos": np.zeros((0, 3)), "types": np.zeros(0, np.int32),
                   "cell": np.eye(3) * 10.0, "pbc": np.array([1, 1, 1], np.int32)}),
        ("slab 600", {"pos": slab_pos, "types": m600["types"], "cell": m600["cell"],
                      "pbc": np.array([1, 1, 0], np.int32)}),
        ("cluster 80", {"pos": c80["pos"] + 7.0, "types": c80["types"],
                        "cell": np.eye(3) * 14.0, "pbc": np.array([0, 0, 0], np.int32)}),
    ]
    calc = d3.D3(TAB)

    def run(sys_):
        calc.build(sys_["pos"], sys_["types"], sys_["cell"], sys_["pbc"])
        out = calc.compute()
        torch.cuda.synchronize()
        calc.status()
        res = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
        res["energy"] = float(res["energy"][0])
        res["cn"] = calc.coordination().cpu().numpy() if sys_["pos"].shape[0] else np.zeros(0)
        return res

    first = None
    for label, sys_ in seq:
        n = sys_["pos"].shape[0]
        print("one context: %s" % label, flush=True)
        got = run(sys_)
        if n == 0:
            assert got["energy"] == 0.0 and np.all(got["virial"] == 0.0)
            continue
        pbc = sys_["pbc"]
        ref = R.d3(sys_["pos"], sys_["types"], None if not np.any(pbc) else sys_["cell"],
                   pbc, TAB)
        compare(got, ref, n, label=label)
        if first is None:
            first = got
    again = run(seq[0][1])
    for k in ("forces", "virial", "atom_energy", "cn"):
        assert np.array_equal(again[k], first[k]), k
    assert again["energy"] == first["energy"]
    calc.close()


@pytest.mark.parametrize("mode,skin", [("plain", 0.0), ("plain", 1.0), ("prec", 1.0)])
def test_cutoff_boundaries_are_strict(mode, skin):
    """Isolated pairs at exactly R_pot = 12 A, one ulp inside it, exactly
    R_cn = 6 A and one ulp inside it (the first atom of each pair at x = 0, so
    the displacements are those values exactly in FP64): the
    strict FP64 tests r^2 < R^2 of the passes leave out the pairs at the
    cutoffs and keep the ones just inside, as the oracle does, also when the
    lists (R + skin) hold them and in the precision form."""
    xs = [12.0, np.nextafter(12.0, 0.0), 6.0, np.nextafter(6.0, 0.0)]
    pos = []
    for k, x in enumerate(xs):
        pos += [[0.0, 5.0 + 30.0 * k, 5.0], [x, 5.0 + 30.0 * k, 5.0]]
    s_ = {"pos": np.array(pos), "types": np.ones(8, np.int32), "cell": np.diag([30.0, 120.0, 10.0]),
          "pbc": np.array([0, 0, 0], np.int32)}
    ref = O.d3(s_["pos"], s_["types"], None, (0, 0, 0), TAB)
    gpu = run_gpu(s_, mode=mode, skin=skin)
    print("%s skin %.1f: U=%s CN=%s" % (mode, skin, gpu["atom_energy"], gpu["cn"]), flush=True)
    assert np.all(gpu["atom_energy"][:2] == 0.0) and np.all(ref["atom_energy"][:2] == 0.0)
    assert np.all(gpu["atom_energy"][2:] < 0.0) and np.all(ref["atom_energy"][2:] < 0.0)
    assert np.all(gpu["cn"][:6] == 0.0) and np.all(ref["cn"][:6] == 0.0)
    assert np.all(gpu["cn"][6:] > 0.0) and np.all(ref["cn"][6:] > 0.0)
    tol = 1e-6 if mode == "prec" else 1e-13
    assert abs(gpu["energy"] - ref["energy"]) <= tol * abs(ref["energy"])


def test_two_contexts_on_two_streams():
    """Two contexts, each driven on a stream of its own (default priority),
    with their builds and evaluations interleaved and no synchronisation
    between them, then a second round with D3_REBUILD: every result bit for
    bit what the same system gives alone on the default stream."""
    torch = _torch()
    from paper_2310_05279_amd import d3
    sa = synth.mof_like(3000, seed=31)
    sb = synth.bilayer_graphene(20, 20, seed=7)
    want = {"a": run_gpu(sa), "b": run_gpu(sb)}
    calc = {"a": d3.D3(TAB), "b": d3.D3(TAB)}
    sys_ = {"a": sa, "b": sb}
    st = {"a": torch.cuda.Stream(), "b": torch.cuda.Stream()}
    got = {"a": [], "b": []}
    for k in ("a", "b"):
        with torch.cuda.stream(st[k]):
            calc[k].build(sys_[k]["pos"], sys_[k]["types"], sys_[k]["cell"], sys_[k]["pbc"])
    for flags in (0, d3.D3_REBUILD):
        for k in ("a", "b"):
            with torch.cuda.stream(st[k]):
                got[k].append(calc[k].compute(flags=flags))
    torch.cuda.synchronize()
    for k in ("a", "b"):
        calc[k].status()
        for out in got[k]:
            for key in ("forces", "virial", "atom_energy"):
                assert np.array_equal(out[key].cpu().numpy(), want[k][key]), (k, key)
            assert float(out["energy"].cpu()[0]) == want[k]["energy"]
        calc[k].close()


def test_single_reference_table():
    """K_e = 1 for every element (C6 constant): the chain term vanishes."""
    tab1 = synth.make_table(force_k=1)
    m = synth.mof_like(800, seed=12)
    ref = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], tab1)
    gpu = run_gpu(m, table=tab1)
    compare(gpu, ref, 800, label="k1")


def test_twelve_element_table():
    """A 12-element table, beyond the eight elements whose C6 table the
    dispersion pass stages in LDS: parity on a random periodic cell."""
    tab12 = synth.make_table(seed=77, n_elem=12)
    m = synth.mof_like(900, seed=13)
    types = np.random.default_rng(12).integers(0, 12, 900).astype(np.int32)
    s = {"pos": m["pos"], "types": types, "cell": m["cell"], "pbc": m["pbc"]}
    ref = R.d3(s["pos"], types, s["cell"], s["pbc"], tab12)
    gpu = run_gpu(s, table=tab12)
    compare(gpu, ref, 900, label="12 elements")


def test_dense_cell_long_cutoffs():
    """R_pot = 30 A and R_cn = 10 A on a dense 1 500-atom cell smaller than
    the cutoff: lists exceed 9 000 entries, images reach two cells out and
    the list build's stencil reaches 10 bins each way."""
    m = synth.mof_like(1500, density=0.08, seed=14)
    prm = dict(r_pot=30.0, r_cn=10.0)
    ref = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], TAB, **prm)
    gpu = run_gpu(m, prm=prm)
    print("dense: list stats %s" % gpu["stats"], flush=True)
    assert gpu["stats"]["max_pot"] > 8000
    compare(gpu, ref, 1500, label="dense")


def test_dense_block_in_vacuum_large_bins():
    """The dense 1 500-atom block in the middle of an 84 A periodic cube:
    the mean density is low, so the list build keeps bins of R_list / 3 =
    10 A, and the block's bins hold ~80 atoms each (two groups of 64 per
    wave)."""
    b = synth.mof_like(1500, density=0.08, seed=14)
    side = b["cell"][0, 0]
    L = 84.0
    pos = np.mod(b["pos"], side) + 0.5 * (L - side)
    s = {"pos": pos, "types": b["types"], "cell": np.diag([L, L, L]),
         "pbc": np.array([1, 1, 1], np.int32)}
    prm = dict(r_pot=30.0, r_cn=10.0)
    ref = R.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB, **prm)
    gpu = run_gpu(s, prm=prm)
    print("block: list stats %s" % gpu["stats"], flush=True)
    assert gpu["stats"]["bins"] == 512
    compare(gpu, ref, 1500, label="block")


@pytest.mark.parametrize("mode", ["plain", "prec"])
def test_long_cutoffs_50_25(mode):
    """R_pot = 50 A and R_cn = 25 A (the long-cutoff regime): ~21 000
    entries per atom, a 27-bin stencil of narrow bins, images two cells out
    of a 2 000-atom MOF-like cube."""
    m = synth.mof_like(2000, seed=50)
    prm = dict(r_pot=50.0, r_cn=25.0)
    print("long cutoffs", mode, flush=True)
    ref = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], TAB, **prm)
    gpu = run_gpu(m, mode=mode, prm=prm)
    print("long: list stats %s" % gpu["stats"], flush=True)
    assert gpu["stats"]["max_pot"] > 20000
    if mode == "plain":
        compare(gpu, ref, 2000, label="long")
    else:
        compare(gpu, ref, 2000, tol_e=1e-6, tol_f=1e-4, tol_w_rel=1e-5, label="long-prec")


def test_long_cutoffs_open_axis():
    """R_pot = 30 A and R_cn = 15 A on a 12 x 12 AB bilayer (periodic in
    plane, open along z): a deep stencil whose row table must leave the
    open axis unbounded (atoms outside the cell join its edge bins)."""
    g = synth.bilayer_graphene(12, 12, seed=12)
    g = dict(g)
    g["pos"] = g["pos"] + np.array([0.0, 0.0, -12.0])  # the lower layer lies below the cell
    prm = dict(r_pot=30.0, r_cn=15.0)
    ref = R.d3(g["pos"], g["types"], g["cell"], g["pbc"], TAB, **prm)
    gpu = run_gpu(g, prm=prm)
    print("open-axis long: list stats %s" % gpu["stats"], flush=True)
    compare(gpu, ref, g["pos"].shape[0], label="open-long")


def test_mof_24000_plain_config2():
    """The 24 000-atom MOF-like cell: full comparison with the C oracle."""
    m = synth.mof_like(24000)
    ref = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], TAB)
    gpu = run_gpu(m)
    compare(gpu, ref, 24000, label="mof24k")
    assert np.abs(gpu["cn"] - ref["cn"]).max() < 1e-12


@pytest.mark.parametrize("case", ["graphene", "mof", "tiny"])
def test_precision_form(case):
    """FP32 pair arithmetic with FP64 cutoffs, weights and accumulation
    (the tiny triclinic cell takes the path with images outside LDS)."""
    if case == "graphene":
        s = synth.bilayer_graphene(12, 12, seed=3)
        ref = R.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB)
    elif case == "tiny":
        cell = np.array([[5.0, 0.0, 0.0], [2.0, 4.6, 0.0], [0.5, 0.7, 5.3]])
        frac = np.random.default_rng(2).uniform(0, 1, (4, 3))
        s = {"pos": frac @ cell, "types": np.array([0, 1, 2, 4], np.int32), "cell": cell,
             "pbc": np.array([1, 1, 1], np.int32)}
        ref = O.d3(s["pos"], s["types"], cell, s["pbc"], TAB)
    else:
        s = synth.mof_like(3000, seed=31)
        ref = R.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB)
    n = s["pos"].shape[0]
    gpu = run_gpu(s, mode="prec")
    de, df, dw = compare(gpu, ref, n, tol_e=1e-6, tol_f=1e-4, tol_w_rel=1e-5,
                         label="prec-" + case)


def _tiny_cell():
    cell = np.array([[5.0, 0.0, 0.0], [2.0, 4.6, 0.0], [0.5, 0.7, 5.3]])
    s = np.random.default_rng(2).uniform(0, 1, (4, 3))
    return {"pos": s @ cell, "types": np.array([0, 1, 2, 4], np.int32), "cell": cell,
            "pbc": np.array([1, 1, 1], np.int32)}


@pytest.mark.parametrize("case", ["graphene", "mof", "tiny", "twelve_elements"])
def test_literal_eq3_mode(case):
    """C6 from Eq. 3 as printed (K_i K_j Gaussian weights per pair, mode
    "literal") meets the plain FP64 gates against the oracle, and agrees
    with the factorised default to rounding: energy, forces, virial and
    the per-atom virial."""
    import torch
    table = TAB
    if case == "graphene":
        s, oracle = synth.bilayer_graphene(), O
    elif case == "mof":
        s, oracle = synth.mof_like(3000, seed=31), R
    elif case == "tiny":
        s, oracle = _tiny_cell(), O
    else:
        table = synth.make_table(seed=77, n_elem=12)
        m = synth.mof_like(900, seed=13)
        types = np.random.default_rng(12).integers(0, 12, 900).astype(np.int32)
        s = {"pos": m["pos"], "types": types, "cell": m["cell"], "pbc": m["pbc"]}
        oracle = R
    n = s["pos"].shape[0]
    print("literal case", case, n, flush=True)
    ref = oracle.d3(s["pos"], s["types"], s["cell"], s["pbc"], table)
    lit, calc = run_gpu(s, mode="literal", table=table, calc_out=True)
    compare(lit, ref, n, label="literal " + case)
    assert np.abs(lit["cn"] - ref["cn"]).max() < 1e-12
    fac = run_gpu(s, mode="plain", table=table)
    scale_f = max(np.abs(fac["forces"]).max(), 1e-30)
    assert abs(lit["energy"] - fac["energy"]) <= 1e-12 * abs(fac["energy"])
    assert np.abs(lit["forces"] - fac["forces"]).max() <= 1e-11 * scale_f
    assert np.abs(lit["virial"] - fac["virial"]).max() <= 1e-11 * np.abs(fac["virial"]).max()
    vel = torch.as_tensor(np.random.default_rng(5).normal(scale=0.01, size=(n, 3)), device="cuda")
    out = calc.compute(atom_virial=True, velocities=vel)
    torch.cuda.synchronize()
    W = out["atom_virial"].cpu().numpy()
    assert np.abs(W - ref["atom_virial"]).max() <= 1e-9 * np.abs(ref["atom_virial"]).max()
    assert np.abs(W.sum(0) - lit["virial"]).max() <= 1e-11 * np.abs(lit["virial"]).max()
    calc.close()


def test_deterministic_and_accumulate():
    torch = _torch()
    from paper_2310_05279_amd import d3
    m = synth.mof_like(2000, seed=3)
    calc = d3.D3(TAB)
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    a = calc.compute()
    b = calc.compute()
    torch.cuda.synchronize()
    for k in ("energy", "forces", "virial", "atom_energy"):
        assert torch.equal(a[k], b[k]), k
    # rebuild from scratch: same bits
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    c = calc.compute()
    torch.cuda.synchronize()
    for k in ("energy", "forces", "virial", "atom_energy"):
        assert torch.equal(a[k], c[k]), k
    # D3_ACCUMULATE adds onto existing outputs (Eq. 9 style)
    out = {k: v.clone() for k, v in a.items()}
    calc.compute(out=out, flags=d3.D3_ACCUMULATE)
    torch.cuda.synchronize()
    for k in ("energy", "forces", "virial", "atom_energy"):
        assert torch.allclose(out[k], 2 * a[k], rtol=1e-15, atol=0), k
    calc.status()
    calc.close()


def test_skin_reuse_stale_and_auto_rebuild():
    """Lists built with a 1 A skin stay exact while atoms move < 0.5 A;
    a larger move is flagged; D3_AUTO_REBUILD rebuilds and is exact."""
    torch = _torch()
    from paper_2310_05279_amd import d3
    m = synth.mof_like(1500, seed=21)
    calc = d3.D3(TAB, skin=1.0)
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    rng = np.random.default_rng(0)
    d = rng.normal(size=m["pos"].shape)
    d *= (0.45 * rng.uniform(size=(len(d), 1))) / np.linalg.norm(d, axis=1, keepdims=True)
    p1 = m["pos"] + d
    out = calc.compute(pos=p1)
    torch.cuda.synchronize()
    calc.status()
    ref = R.d3(p1, m["types"], m["cell"], m["pbc"], TAB)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    g["energy"] = float(g["energy"][0])
    g["cn"] = ref["cn"]
    compare(g, ref, 1500, label="skin-reuse")
    p2 = p1.copy()
    p2[7] += np.array([0.7, 0.0, 0.0])
    calc.compute(pos=p2)
    torch.cuda.synchronize()
    with pytest.raises(d3.D3Error) as ei:
        calc.status()
    assert ei.value.code == d3.D3_ERR_STALE
    out = calc.compute(pos=p2, flags=d3.D3_AUTO_REBUILD)
    torch.cuda.synchronize()
    calc.status()
    ref = R.d3(p2, m["types"], m["cell"], m["pbc"], TAB)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    g["energy"] = float(g["energy"][0])
    g["cn"] = ref["cn"]
    compare(g, ref, 1500, label="auto-rebuild")
    calc.close()


def test_stale_threshold_is_half_the_skin():
    """The lists stay valid while no atom has moved more than skin/2 from
    its build position: one atom moved by exactly 0.5 A (skin 1 A; its x in
    [16, 31.5) A, so x + 0.5 is exact) is not reported stale and the result
    matches the oracle; one ulp of x further is reported stale."""
    torch = _torch()
    from paper_2310_05279_amd import d3
    m = synth.mof_like(1500, seed=21)
    k = int(np.nonzero((m["pos"][:, 0] >= 16.0) & (m["pos"][:, 0] < 31.0))[0][0])
    calc = d3.D3(TAB, skin=1.0)
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    p1 = m["pos"].copy()
    p1[k, 0] += 0.5
    assert p1[k, 0] - m["pos"][k, 0] == 0.5
    out = calc.compute(pos=p1)
    torch.cuda.synchronize()
    calc.status()  # not stale
    ref = R.d3(p1, m["types"], m["cell"], m["pbc"], TAB)
    g = {key: v.cpu().numpy() for key, v in out.items()}
    g["energy"] = float(g["energy"][0])
    g["cn"] = ref["cn"]
    compare(g, ref, 1500, label="moved by skin/2")
    p2 = p1.copy()
    p2[k, 0] = np.nextafter(p1[k, 0], 100.0)
    assert p2[k, 0] - m["pos"][k, 0] > 0.5
    calc.compute(pos=p2)
    torch.cuda.synchronize()
    with pytest.raises(d3.D3Error) as ei:
        calc.status()
    assert ei.value.code == d3.D3_ERR_STALE
    calc.close()


def test_rebuild_flag():
    """D3_REBUILD rebuilds the lists from the given positions before the
    evaluation: after large moves it gives bit for bit what a fresh build
    and evaluation give, alone or together with the other flags, and the
    build counts as one (no position update follows it)."""
    import torch
    from paper_2310_05279_amd import d3
    m = synth.mof_like(2000, seed=41)
    n = m["pos"].shape[0]
    calc = d3.D3(TAB, skin=0.5)
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    rng = np.random.default_rng(3)
    for rep, flags in enumerate((d3.D3_REBUILD, d3.D3_REBUILD | d3.D3_AUTO_REBUILD)):
        pos = m["pos"] + rng.uniform(-0.6, 0.6, size=(n, 3))  # beyond half the skin
        got = calc.compute(pos, flags=flags, atom_virial=rep == 1)
        ref = d3.D3(TAB, skin=0.5)
        ref.build(pos, m["types"], m["cell"], m["pbc"])
        exp = ref.compute(pos, atom_virial=rep == 1)
        torch.cuda.synchronize()
        calc.status()
        for k in exp:
            if exp[k] is not None:
                assert torch.equal(got[k], exp[k]), "flags %d: %s differs" % (flags, k)
        ref.close()
        print("rebuild flag %d: bitwise equal to a fresh build" % flags, flush=True)
    r = R.d3(pos, m["types"], m["cell"], m["pbc"], TAB)
    assert abs(float(got["energy"].cpu()[0]) - r["energy"]) / n <= 1e-6
    got.pop("atom_virial", None)
    acc = calc.compute(pos, flags=d3.D3_REBUILD | d3.D3_ACCUMULATE, out=got)
    torch.cuda.synchronize()
    assert torch.allclose(acc["forces"], 2 * exp["forces"], rtol=1e-14, atol=0)
    calc.close()


def test_mode_switch_on_one_context():
    """Switching the mode of one context between evaluations (plain,
    precision, literal, plain, with and without per-atom virials) gives,
    bit for bit, what a fresh context in each mode gives."""
    import torch
    from paper_2310_05279_amd import d3
    m = synth.mof_like(1200, seed=17)
    calc = d3.D3(TAB)
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    for mode in ("plain", "prec", "literal", "plain", "prec"):
        calc.set_mode(mode)
        for av in (False, True):
            got = calc.compute(atom_virial=av)
            ref = d3.D3(TAB, mode=mode)
            ref.build(m["pos"], m["types"], m["cell"], m["pbc"])
            exp = ref.compute(atom_virial=av)
            torch.cuda.synchronize()
            calc.status()
            for k in exp:
                if exp[k] is not None:
                    assert torch.equal(got[k], exp[k]), "%s (atom_virial=%s): %s" % (mode, av, k)
            ref.close()
        print("mode %s after a switch: bitwise equal to a fresh context" % mode, flush=True)
    calc.close()


def test_bad_species_reported_and_contained():
    torch = _torch()
    from paper_2310_05279_amd import d3
    m = synth.mof_like(500, seed=2)
    t = m["types"].copy()
    t[10] = 9
    calc = d3.D3(TAB)
    calc.build(m["pos"], t, m["cell"], m["pbc"])
    calc.compute()
    torch.cuda.synchronize()
    with pytest.raises(d3.D3Error) as ei:
        calc.status()
    assert ei.value.code == d3.D3_ERR_SPECIES
    calc.close()


def test_empty_and_single_atom():
    torch = _torch()
    from paper_2310_05279_amd import d3
    calc = d3.D3(TAB)
    calc.build(np.zeros((0, 3)), np.zeros(0, np.int32), np.eye(3) * 10, (1, 1, 1))
    out = calc.compute()
    torch.cuda.synchronize()
    assert out["energy"].item() == 0.0 and torch.all(out["virial"] == 0)
    one = {"pos": np.array([[1.0, 2.0, 3.0]]), "types": np.array([2], np.int32),
           "cell": np.eye(3) * 4.0, "pbc": np.array([1, 1, 1], np.int32)}
    ref = O.d3(one["pos"], one["types"], one["cell"], one["pbc"], TAB)
    gpu = run_gpu(one)
    compare(gpu, ref, 1, label="one-atom")
    assert np.abs(gpu["forces"]).max() < 1e-14
    calc.close()


def test_list_encoding_limit():
    """A list entry packs (atom, image) into 32 bits: a system whose atom
    count and periodic images do not fit is refused on the host before any
    device work, and the context stays usable."""
    _torch()
    from paper_2310_05279_amd import d3
    calc = d3.D3(TAB, r_pot=60.0, r_cn=6.0)
    # 60 A over a 10 A cube: 2 bins and 13 images per axis, 2197 images, 12 bits
    n = (1 << (32 - 12)) + 1
    pos = np.random.default_rng(0).uniform(0.0, 10.0, (n, 3))
    with pytest.raises(d3.D3Error) as ei:
        calc.build(pos, np.zeros(n, np.int32), np.eye(3) * 10.0, (1, 1, 1))
    assert ei.value.code == d3.D3_ERR_CELL
    assert "32-bit" in str(ei.value)
    s = synth.bilayer_graphene()
    calc.build(s["pos"], s["types"], s["cell"], s["pbc"])
    out = calc.compute()
    ref = R.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB, r_pot=60.0, r_cn=6.0)
    assert abs(float(out["energy"].cpu()[0]) - ref["energy"]) <= 1e-6 * s["pos"].shape[0]
    calc.close()


def test_state_errors():
    _torch()
    from paper_2310_05279_amd import d3
    calc = d3.D3(TAB)
    e = __import__("torch").zeros(1, dtype=__import__("torch").float64, device="cuda")
    with pytest.raises(d3.D3Error) as ei:
        d3.d3_energy_forces_virial(calc.ctx, None, e)
    assert ei.value.code == d3.D3_ERR_STATE
    with pytest.raises(d3.D3Error) as ei:
        calc.build(np.zeros((2, 3)), np.zeros(2, np.int32), np.zeros((3, 3)), (1, 1, 1))
    assert ei.value.code == d3.D3_ERR_CELL
    calc.close()


_FULL_REF = {}


def _full_case(case):
    """The full-size cell and the oracle's cell-list evaluation of all of it
    (computed once per cell and shared by the plain and precision tests)."""
    if case not in _FULL_REF:
        if case == "mof1M":
            s = synth.mof_like(1_000_000)
        else:
            s = synth.bilayer_graphene(250, 500, seed=500000)
        ref = R.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB, cells=True)
        _FULL_REF.clear()
        _FULL_REF[case] = (s, ref)
    return _FULL_REF[case]


@pytest.mark.parametrize("case,mode", [("graphene500k", "plain"), ("graphene500k", "prec"),
                                       ("mof1M", "plain"), ("mof1M", "prec")])
def test_full_size_against_cell_list_oracle(case, mode):
    """Full-size cells (the 10^6-atom MOF-like cube and the 500 000-atom
    bilayer) in the plain and precision forms, in the launch shape the bench
    times, against the C oracle's cell-list evaluation of the whole cell:
    every force, every site energy and CN, the energy and the virial.  Plain
    gates: |dE|/atom <= 1e-6 eV, max |dF| <= 1e-5 eV/A, virial 1e-9
    relative; precision form: max |dF| <= 1e-4 eV/A, with |dE|/atom <= 1e-6
    eV and the virial to 1e-6 relative (errors printed)."""
    print("case", case, mode, flush=True)
    s, ref = _full_case(case)
    n = s["pos"].shape[0]
    gpu = run_gpu(s, mode=mode)
    de = abs(gpu["energy"] - ref["energy"]) / n
    df = np.abs(gpu["forces"] - ref["forces"]).max()
    du = np.abs(gpu["atom_energy"] - ref["atom_energy"]).max()
    dcn = np.abs(gpu["cn"] - ref["cn"]).max()
    wsc = np.abs(ref["virial"]).max()
    dw = np.abs(gpu["virial"] - ref["virial"]).max()
    print("%s %s (%d entries/atom): |dE|/atom=%.2e max|dF|=%.2e max|dU_i|=%.2e max|dCN|=%.2e "
          "max|dW|=%.2e (rel %.2e)" % (case, mode, ref["n_entries"] // n, de, df, du, dcn, dw,
                                       dw / wsc), flush=True)
    assert de <= 1e-6 and du <= 1e-6
    if mode == "plain":
        assert df <= 1e-5 and dcn <= 1e-12 and dw <= 1e-9 * wsc
    else:
        assert df <= 1e-4 and dcn <= 1e-5 and dw <= 1e-6 * wsc


@pytest.mark.parametrize("mode", ["plain", "prec"])
def test_supercell_beyond_32_bit_list_offsets(mode):
    """A 4 x 2 x 2 supercell of the 10^6-atom MOF-like cube (1.6e7 atoms,
    lists at 13 A: ~5.9e9 entries, so list offsets and the summed lengths
    pass 2^32) against the oracle's cell-list evaluation of the base cube:
    periodicity fixes every copy of an atom to the base atom's force, site
    energy and CN, and the energy and virial to 16 times the base cell's.
    Every atom is checked, with the full-size gates of the plain and
    precision forms.  The copies are replicas only up to rounding, which
    bounds the plain form's CN check (see ``cn_tol``)."""
    print("supercell", mode, flush=True)
    s, ref = _full_case("mof1M")
    n = s["pos"].shape[0]
    reps = (4, 2, 2)
    L = s["cell"]
    shifts = [i * L[0] + j * L[1] + k * L[2]
              for i in range(reps[0]) for j in range(reps[1]) for k in range(reps[2])]
    sup = {"pos": np.concatenate([s["pos"] + t for t in shifts]),
           "types": np.tile(s["types"], len(shifts)),
           "cell": L * np.array(reps, dtype=np.float64)[:, None], "pbc": s["pbc"]}
    m = len(shifts) * n
    gpu = run_gpu(sup, mode=mode, skin=1.0)
    st = gpu["stats"]
    assert st["mean_pot"] * m > 2.0 ** 32 and st["max_pot"] * m > 2.0 ** 32
    df = du = dcn = 0.0
    for c in range(len(shifts)):
        sl = slice(c * n, (c + 1) * n)
        df = max(df, float(np.abs(gpu["forces"][sl] - ref["forces"]).max()))
        du = max(du, float(np.abs(gpu["atom_energy"][sl] - ref["atom_energy"]).max()))
        dcn = max(dcn, float(np.abs(gpu["cn"][sl] - ref["cn"]).max()))
    de = abs(gpu["energy"] - len(shifts) * ref["energy"]) / m
    wsc = len(shifts) * np.abs(ref["virial"]).max()
    dw = np.abs(gpu["virial"] - len(shifts) * ref["virial"]).max()
    print("supercell %s: %d atoms, %.3g entries: |dE|/atom=%.2e max|dF|=%.2e max|dU_i|=%.2e "
          "max|dCN|=%.2e max|dW|=%.2e (rel %.2e)"
          % (mode, m, st["mean_pot"] * m, de, df, du, dcn, dw, dw / wsc), flush=True)
    # a tiled coordinate is rounded to half an ulp u of the largest magnitude
    # (an image-shifted coordinate, below twice the longest cell edge), and so
    # are the image shift and difference that form a displacement: each
    # component may differ from the base cell's by 2u, a length by 2 sqrt(3) u.
    # Eq. 4's counting function changes by at most 4 R_s / r^2 per Angstrom
    # (R_s the largest covalent-radius sum, r >= the 1 A minimum separation)
    u = float(np.spacing(2.0 * np.abs(sup["cell"]).sum(axis=1).max()))
    slope = 4.0 * (2.0 * TAB["rcov"].max()) / 1.0 ** 2
    cn_tol = st["max_cn"] * slope * 2.0 * np.sqrt(3.0) * u
    print("CN bound from the tiling's rounding: %.2e" % cn_tol, flush=True)
    assert de <= 1e-6 and du <= 1e-6
    if mode == "plain":
        assert df <= 1e-5 and dcn <= cn_tol and dw <= 1e-9 * wsc
    else:
        assert df <= 1e-4 and dcn <= 1e-5 and dw <= 1e-6 * wsc


@pytest.mark.parametrize("mode", ["plain", "prec"])
def test_two_bin_units_sparse_skewed_cell(mode):
    """A large periodic bulk cell builds its lists in units of two
    neighbouring bins (from 100 000 bins on): a sparse (0.004 A^-3) sheared
    cell of 36 000 atoms with 47 x 47 x 48 bins (an odd count along the first
    lattice vector, so every row ends in a single-bin unit) and a 1 A skin,
    against the oracle's cell-list evaluation of the whole cell."""
    m = synth.mof_like(36000, density=0.004, seed=77)
    shear = np.array([[1.0, 0.0, 0.0], [0.12, 1.0, 0.0], [-0.08, 0.1, 1.0]])
    s = {"pos": m["pos"] @ shear, "types": m["types"], "cell": m["cell"] @ shear,
         "pbc": m["pbc"]}
    ref = R.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB, cells=True)
    gpu = run_gpu(s, mode=mode, skin=1.0)
    assert gpu["stats"]["bins"] >= 100000
    if mode == "plain":
        compare(gpu, ref, 36000, label="two-bin units plain")
    else:
        compare(gpu, ref, 36000, tol_f=1e-4, tol_w_rel=1e-6, label="two-bin units prec")


def test_capacity_overflow_reported_bounded_and_regrown():
    """List overflow: lists sized (with a 1 A skin) for a sparse cell
    overflow when its atoms are drawn together into the middle of the cell
    and rebuilt with D3_REBUILD, which neither sizes the lists nor
    synchronises.  d3_status reports CAPACITY; the build's writes stayed
    within the lists (the evaluation in the same call ran on the truncated
    lists and the context stays usable); an evaluation without a rebuild
    flag is then refused with CAPACITY; D3_AUTO_REBUILD sizes the lists
    again and the result matches the oracle."""
    torch = _torch()
    from paper_2310_05279_amd import d3
    m = synth.mof_like(3000, density=0.02, seed=71)
    n = m["pos"].shape[0]
    calc = d3.D3(TAB, skin=1.0)
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    cap0 = calc.stats()["max_pot"]
    mid = 0.5 * m["cell"].sum(axis=0)
    pos = mid + 0.6 * (m["pos"] - mid)  # about 4.6 times the density
    calc.compute(pos, flags=d3.D3_REBUILD)
    torch.cuda.synchronize()
    with pytest.raises(d3.D3Error) as ei:
        calc.status()
    assert ei.value.code == d3.D3_ERR_CAPACITY
    with pytest.raises(d3.D3Error) as ei:
        calc.compute(pos)
    assert ei.value.code == d3.D3_ERR_CAPACITY
    out = calc.compute(pos, flags=d3.D3_AUTO_REBUILD)
    cn = calc.coordination(pos)
    torch.cuda.synchronize()
    calc.status()
    st = calc.stats()
    print("overflow: list max %d before, %d after regrowing" % (cap0, st["max_pot"]), flush=True)
    assert st["max_pot"] > 2 * cap0
    ref = R.d3(pos, m["types"], m["cell"], m["pbc"], TAB)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    g["energy"] = float(g["energy"][0])
    g["cn"] = cn.cpu().numpy()
    compare(g, ref, n, label="after regrow")
    calc.close()


def test_nonfinite_position_reported_and_contained():
    """A NaN coordinate is reported by d3_status as INVALID_ARG; the atom is
    left out of every list, so the other atoms get exactly the results of
    the cell without it, and the context stays usable for a clean build."""
    torch = _torch()
    from paper_2310_05279_amd import d3
    m = synth.mof_like(800, seed=72)
    n = m["pos"].shape[0]
    bad = m["pos"].copy()
    bad[5, 1] = np.nan
    calc = d3.D3(TAB)
    calc.build(bad, m["types"], m["cell"], m["pbc"])
    out = calc.compute()
    torch.cuda.synchronize()
    with pytest.raises(d3.D3Error) as ei:
        calc.status()
    assert ei.value.code == d3.D3_ERR_INVALID_ARG
    assert "non-finite" in str(ei.value)
    keep = np.arange(n) != 5
    ref = R.d3(m["pos"][keep], m["types"][keep], m["cell"], m["pbc"], TAB)
    f = out["forces"].cpu().numpy()
    assert np.all(np.isfinite(f))
    assert np.abs(f[keep] - ref["forces"]).max() <= 1e-5
    assert abs(float(out["energy"].cpu()[0]) - ref["energy"]) <= 1e-6 * n
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    out = calc.compute()
    cn = calc.coordination()
    torch.cuda.synchronize()
    calc.status()
    ref = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], TAB)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    g["energy"] = float(g["energy"][0])
    g["cn"] = cn.cpu().numpy()
    compare(g, ref, n, label="after a clean build")
    calc.close()
