"""GPU parity of the D3 variants the paper sets aside (Sec. II A, before
Eq. 1) and that are built here as the D3 reference the paper cites defines
them: zero damping of the two-body term and the three-body
(Axilrod-Teller-Muto) term, alone and together, in the plain, precision
and literal forms, through the C ABI, against the FP64 oracles.

Gates as for Eq. 2: plain and literal |dE|/atom <= 1e-6 eV, max |dF| <=
1e-5 eV/A, virial to 1e-9 relative; precision form max |dF| <= 1e-4 eV/A
(energy and virial errors printed)."""

import numpy as np
import pytest

import synth
from oracle import d3_oracle as O
from oracle import d3_ref as R

pytestmark = pytest.mark.gpu

TAB = synth.make_table()
ZERO = dict(damping="zero", s6=1.0, s8=0.722, rs6=1.217, rs8=1.0)
VARIANTS = {"zero": dict(ZERO), "atm": dict(s9=1.0), "zero_atm": dict(ZERO, s9=1.0)}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


def _gpu(s, mode="plain", atom_virial=False, **prm):
    torch = _torch()
    from paper_2310_05279_amd import d3
    calc = d3.D3(TAB, mode=mode, **prm)
    calc.build(s["pos"], s["types"], s["cell"], s["pbc"])
    out = calc.compute(atom_virial=atom_virial)
    torch.cuda.synchronize()
    calc.status()
    res = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    res["energy"] = float(res["energy"][0])
    calc.close()
    return res


def _check(got, ref, n, mode, label):
    de = abs(got["energy"] - ref["energy"]) / n
    df = np.abs(got["forces"] - ref["forces"]).max()
    du = np.abs(got["atom_energy"] - ref["atom_energy"]).max()
    wsc = np.abs(ref["virial"]).max()
    dw = np.abs(got["virial"] - ref["virial"]).max()
    print("%s %s: |dE|/atom=%.2e max|dF|=%.2e max|dU_i|=%.2e max|dW|=%.2e (rel %.2e)"
          % (label, mode, de, df, du, dw, dw / wsc), flush=True)
    assert de <= 1e-6 and du <= 1e-6
    if mode == "prec":
        assert df <= 1e-4 and dw <= 1e-6 * wsc
    else:
        assert df <= 1e-5 and dw <= 1e-9 * wsc


def _small_cell(seed):
    rng = np.random.default_rng(300 + seed)
    cell = np.diag(rng.uniform(7.0, 11.0, 3))
    cell[1, 0] = rng.uniform(-2, 2)
    cell[2, :2] = rng.uniform(-2, 2, 2)
    n = int(rng.integers(6, 40))
    pbc = [(1, 1, 1), (1, 1, 0), (1, 0, 1), (1, 1, 1)][seed % 4]
    return {"pos": rng.uniform(-0.1, 1.1, (n, 3)) @ cell,
            "types": rng.integers(0, 5, n).astype(np.int32), "cell": cell, "pbc": np.array(pbc)}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("mode", ["plain", "prec", "literal"])
def test_variants_small_cells(variant, mode):
    """Small skewed cells (images within every cutoff, open axes, atoms
    beyond the faces) with R_pot 10 A, R_cn = r_atm 5 A."""
    kw = dict(VARIANTS[variant], r_pot=10.0, r_cn=5.0, r_atm=5.0)
    for seed in range(4):
        s = _small_cell(seed)
        ref = O.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB, O.Params(**kw))
        got = _gpu(s, mode=mode, **kw)
        _check(got, ref, s["pos"].shape[0], mode, "%s seed %d" % (variant, seed))


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_variants_image_triangles_and_cluster(variant):
    """Edge cases of the three-body term: a one-atom triclinic cell, whose
    triangles are all made of the atom's own periodic images, a two-atom
    cell, and a 40-atom cluster with no periodic axis."""
    cell1 = np.array([[3.6, 0.0, 0.0], [0.9, 3.4, 0.0], [0.4, -0.6, 3.9]])
    one = {"pos": np.array([[0.3, 0.2, 0.1]]), "types": np.array([4], np.int32), "cell": cell1,
           "pbc": np.array([1, 1, 1])}
    two = {"pos": np.array([[0.3, 0.2, 0.1], [1.9, 1.6, 2.2]]), "types": np.array([1, 3], np.int32),
           "cell": cell1 * 1.3, "pbc": np.array([1, 1, 1])}
    rng = np.random.default_rng(41)
    pts = []
    while len(pts) < 40:
        p = rng.uniform(0, 9.0, 3)
        if all(np.linalg.norm(p - q) > 1.2 for q in pts):
            pts.append(p)
    clu = {"pos": np.array(pts), "types": rng.integers(0, 5, 40).astype(np.int32),
           "cell": np.eye(3) * 10.0, "pbc": np.array([0, 0, 0])}
    kw = dict(VARIANTS[variant], r_pot=10.0, r_cn=6.0, r_atm=6.0)
    for s, label in ((one, "one-atom cell"), (two, "two-atom cell"), (clu, "cluster")):
        ref = O.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB, O.Params(**kw))
        got = _gpu(s, **kw)
        _check(got, ref, s["pos"].shape[0], "plain", "%s %s" % (variant, label))


def test_atm_side_at_r_atm_is_left_out():
    """An isolated 3-4-5 triangle (its longest side exactly 5 A in FP64):
    with r_atm = 5 A the strict test leaves the triangle out, so the
    three-body term changes nothing, bit for bit; with r_atm one ulp above
    5 A it is in, as in the oracle."""
    s = {"pos": np.array([[0.0, 0.0, 2.0], [3.0, 0.0, 2.0], [0.0, 4.0, 2.0]]),
         "types": np.array([1, 3, 4], np.int32), "cell": np.eye(3) * 10.0,
         "pbc": np.array([0, 0, 0])}
    base = _gpu(s)
    out = _gpu(s, s9=1.0, r_atm=5.0)
    for k in ("forces", "atom_energy", "virial"):
        assert np.array_equal(out[k], base[k]), k
    assert out["energy"] == base["energy"]
    r_in = float(np.nextafter(5.0, 6.0))
    got = _gpu(s, s9=1.0, r_atm=r_in)
    ref = O.d3(s["pos"], s["types"], None, (0, 0, 0), TAB, O.Params(s9=1.0, r_atm=r_in))
    ref0 = O.d3(s["pos"], s["types"], None, (0, 0, 0), TAB, O.Params(s9=1.0, r_atm=5.0))
    print("3-4-5 triangle: E(two-body)=%.12e, E(r_atm=5)=%.12e, E(r_atm=5+ulp)=%.12e (oracle %.12e)"
          % (base["energy"], out["energy"], got["energy"], ref["energy"]), flush=True)
    assert ref0["energy"] == pytest.approx(base["energy"], rel=1e-14)
    assert got["energy"] != base["energy"]
    _check(got, ref, 3, "plain", "3-4-5 triangle")


@pytest.mark.parametrize("variant", sorted(VARIANTS))
def test_variants_bilayer(variant):
    """The 144-atom bilayer at the workload's cutoffs (12 / 6 A, r_atm 6 A)."""
    g = synth.bilayer_graphene()
    kw = dict(VARIANTS[variant], r_pot=12.0, r_cn=6.0, r_atm=6.0)
    ref = O.d3(g["pos"], g["types"], g["cell"], g["pbc"], TAB, O.Params(**kw))
    _check(_gpu(g, **kw), ref, 144, "plain", "bilayer " + variant)


@pytest.mark.parametrize("variant,mode", [("zero", "plain"), ("atm", "plain"),
                                          ("zero_atm", "plain"), ("zero", "prec"),
                                          ("atm", "prec"), ("zero_atm", "prec")])
def test_variants_mof_24000(variant, mode):
    """The 24 000-atom MOF-like cell at 12 / 6 A (r_atm 6 A) against the C
    oracle's cell-list evaluation of the whole cell."""
    m = synth.mof_like(24000)
    kw = dict(VARIANTS[variant], r_pot=12.0, r_cn=6.0, r_atm=6.0)
    print("mof 24000", variant, mode, flush=True)
    ref = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], TAB, cells=True, **kw)
    _check(_gpu(m, mode=mode, **kw), ref, 24000, mode, "mof24000 " + variant)


def test_variants_full_size_mof1M():
    """Zero damping and the three-body term together on the 10^6-atom cell in
    the launch shape the bench times (lists in two-bin units, the three-body
    pass over every atom), against the C oracle's cell-list evaluation of the
    whole cell: every force and site energy, E and W, plain gates."""
    m = synth.mof_like(1_000_000)
    kw = dict(VARIANTS["zero_atm"], r_pot=12.0, r_cn=6.0, r_atm=6.0)
    print("mof 10^6 zero+atm", flush=True)
    ref = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], TAB, cells=True, **kw)
    _check(_gpu(m, **kw), ref, 1_000_000, "plain", "mof1M zero_atm")


@pytest.mark.parametrize("mode", ["plain", "prec"])
def test_atm_long_lists(mode):
    """The three-body term over R_cn lists several 64-entry blocks long
    (R_cn 9.5 A with a 1 A skin: ~190 entries per atom, pairs within and
    across blocks) and r_atm below R_cn (7.5 A), so that blocks also hold
    entries beyond r_atm; against the C oracle."""
    m = synth.mof_like(1500, seed=33)
    kw = dict(s9=1.0, r_pot=12.0, r_cn=9.5, r_atm=7.5)
    ref = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], TAB, cells=True, **kw)
    _check(_gpu(m, mode=mode, skin=1.0, **kw), ref, 1500, mode, "atm long lists")


@pytest.mark.parametrize("mode", ["plain", "literal"])
def test_variants_twelve_elements(mode):
    """Zero damping and the three-body term with a 12-element table, beyond
    the eight elements whose C6 table the passes stage in LDS (the table is
    read from global memory), against the C oracle."""
    tab12 = synth.make_table(seed=77, n_elem=12)
    m = synth.mof_like(900, seed=13)
    types = np.random.default_rng(12).integers(0, 12, 900).astype(np.int32)
    kw = dict(VARIANTS["zero_atm"], r_pot=12.0, r_cn=6.0, r_atm=6.0)
    ref = R.d3(m["pos"], types, m["cell"], m["pbc"], tab12, **kw)
    torch = _torch()
    from paper_2310_05279_amd import d3
    calc = d3.D3(tab12, mode=mode, **kw)
    calc.build(m["pos"], types, m["cell"], m["pbc"])
    out = calc.compute()
    torch.cuda.synchronize()
    calc.status()
    got = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    got["energy"] = float(got["energy"][0])
    calc.close()
    _check(got, ref, 900, mode, "12 elements zero_atm")


@pytest.mark.parametrize("seed", range(8))
def test_variants_random_cells(seed):
    """Both variants on random small cells: skewed lattice vectors of
    5-14 A, any mix of periodic and open axes, 3-30 atoms (some outside the
    cell), R_pot 5-20 A, R_cn from R_pot/4 to R_pot, r_atm from R_cn/2 to
    R_cn (at most 8 A)."""
    rng = np.random.default_rng(2000 + seed)
    while True:
        cell = np.diag(rng.uniform(5.0, 14.0, 3)) + rng.uniform(-2.5, 2.5, (3, 3)) * \
            (1 - np.eye(3))
        if abs(np.linalg.det(cell)) > 0.2 * np.prod(np.linalg.norm(cell, axis=1)):
            break
    pbc = rng.integers(0, 2, 3).astype(np.int32)
    n = int(rng.integers(3, 31))
    for _ in range(1000):
        pos = rng.uniform(-0.3, 1.3, (n, 3)) @ cell
        if O.entries(pos, cell, pbc, 0.9)[0].size == 0:
            break
    types = rng.integers(0, 5, n).astype(np.int32)
    r_pot = float(rng.uniform(5.0, 20.0))
    r_cn = float(rng.uniform(0.25, 1.0)) * r_pot
    r_atm = min(float(rng.uniform(0.5, 1.0)) * r_cn, 8.0)
    kw = dict(VARIANTS["zero_atm"], r_pot=r_pot, r_cn=r_cn, r_atm=r_atm)
    s = {"pos": pos, "types": types, "cell": cell, "pbc": pbc}
    ref = R.d3(pos, types, cell, pbc, TAB, **kw)
    _check(_gpu(s, **kw), ref, n, "plain", "random cell %d (pbc %s, %d atoms, %.1f/%.1f/%.1f A)"
           % (seed, pbc.tolist(), n, r_pot, r_cn, r_atm))


def test_atm_per_atom_virial():
    """Per-atom virials with the three-body term (a third of each
    triangle's virial per vertex) against the oracle, and their sum rule."""
    s = synth.mof_like(600, seed=17)
    kw = dict(s9=1.0, r_pot=12.0, r_cn=6.0, r_atm=6.0)
    ref = O.d3(s["pos"], s["types"], s["cell"], s["pbc"], TAB, O.Params(**kw))
    got = _gpu(s, atom_virial=True, **kw)
    sc = np.abs(ref["atom_virial"]).max()
    dv = np.abs(got["atom_virial"] - ref["atom_virial"]).max()
    print("atm per-atom virial: max|dW_i| = %.2e (rel %.2e)" % (dv, dv / sc), flush=True)
    assert dv <= 1e-9 * sc
    assert np.abs(got["atom_virial"].sum(0) - got["virial"]).max() <= 1e-9 * np.abs(got["virial"]).max()


def test_variant_argument_checks():
    """The surrogate pass implements Becke-Johnson damping only: zero
    damping in that mode is refused at evaluation; a three-body cutoff
    beyond R_cn is refused at creation."""
    _torch()
    from paper_2310_05279_amd import d3
    with pytest.raises(d3.D3Error) as ei:
        d3.D3(TAB, s9=1.0, r_cn=6.0, r_atm=7.0)
    assert ei.value.code == d3.D3_ERR_INVALID_ARG
    calc = d3.D3(TAB, mode="surrogate", **ZERO)
    d3.d3_c6_surrogate_init(calc.ctx, 1)
    w = d3.d3_c6_surrogate_get_weights(calc.ctx)
    d3.d3_c6_surrogate_set_weights(calc.ctx, w)
    g = synth.bilayer_graphene()
    calc.build(g["pos"], g["types"], g["cell"], g["pbc"])
    with pytest.raises(d3.D3Error) as ei:
        calc.compute()
    assert ei.value.code == d3.D3_ERR_INVALID_ARG
    calc.close()


def test_md_with_variants_matches_oracle_integrator():
    """Velocity-Verlet NVE with zero damping and the three-body term: 12
    steps of a hot 800-atom cell (lists rebuilt on the way) against the
    NumPy integrator driven by the C oracle with the same variants."""
    torch = _torch()
    from paper_2310_05279_amd import d3
    from oracle import md_oracle
    m = synth.mof_like(800, seed=18)
    vel, mass = synth.maxwell_velocities(m["types"], 300.0, seed=301)
    vel = vel * 10.0
    kw = dict(VARIANTS["zero_atm"], r_pot=12.0, r_cn=6.0, r_atm=6.0)
    calc = d3.D3(TAB, skin=1.0, **kw)
    calc.build(m["pos"], m["types"], m["cell"], m["pbc"])
    p = torch.as_tensor(m["pos"], device="cuda").clone()
    v = torch.as_tensor(vel, device="cuda").clone()
    ms = torch.as_tensor(mass, device="cuda")
    thermo, rebuilds = d3.d3_md_nve(calc.ctx, 12, 1.0, p, v, ms, every=4)
    rp, rv, rth = md_oracle.run(m["pos"], vel, mass, m["types"], m["cell"], m["pbc"], TAB, 12,
                                1.0, **kw)
    dp = np.abs(p.cpu().numpy() - rp).max()
    dv = np.abs(v.cpu().numpy() - rv).max()
    print("md zero+atm: rebuilds=%d max|dx|=%.2e max|dv|=%.2e" % (rebuilds, dp, dv), flush=True)
    assert rebuilds >= 1
    assert dp < 1e-9 and dv < 1e-10
    assert thermo[:, 0] == pytest.approx(rth[::4, 0], rel=1e-9)
    calc.close()
