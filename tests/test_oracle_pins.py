"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics, independent of the oracle's own code path.

Each test names the part of the method it pins (Ying & Fan, Sec. II A,
Eqs. 1-7) and what would break it.
"""

import os

import numpy as np
import pytest

import synth
from oracle import d3_oracle as O
from oracle import d3_ref as R

HARTREE_EV = 27.211386245988
BOHR_ANG = 0.529177210903
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table(**kw):
    return synth.make_table(**kw)


def _dimer(za, zb, r):
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    return pos, np.array([za, zb], dtype=np.int32)


def _free_energy(pos, types, tab, prm):
    return O.energy_only(pos, types, None, (0, 0, 0), tab, prm)


# --------------------------------------------------------------- Eq. 4 ----

def test_counting_function_is_half_at_covalent_sum():
    """Eq. 4: the counting function is exactly 1/2 at r = Rcov_i + Rcov_j,
    so a dimer at that distance has n_1 = n_2 = 1/2 (catches a wrong sign,
    a swapped ratio or a wrong radius sum)."""
    tab = _table()
    for za, zb in [(0, 1), (1, 1), (2, 4), (3, 0)]:
        r = tab["rcov"][za] + tab["rcov"][zb]
        pos, types = _dimer(za, zb, r)
        res = O.d3(pos, types, None, (0, 0, 0), tab, O.Params(r_cn=6.0))
        assert res["cn"] == pytest.approx([0.5, 0.5], abs=1e-15)


def test_cn_dimer_closed_form_and_cutoff():
    """Eq. 4 dimer closed form 1/(1+exp(-16(Rs/r-1))), and n = 0 once the
    pair lies beyond R_cn (hard cutoff)."""
    tab = _table()
    for r in [0.9, 1.3, 2.2, 4.0, 5.99]:
        pos, types = _dimer(1, 3, r)
        rs = tab["rcov"][1] + tab["rcov"][3]
        want = 1.0 / (1.0 + np.exp(-16.0 * (rs / r - 1.0)))
        res = O.d3(pos, types, None, (0, 0, 0), tab, O.Params(r_cn=6.0))
        assert res["cn"] == pytest.approx([want, want], rel=1e-14)
    pos, types = _dimer(1, 3, 6.01)
    res = O.d3(pos, types, None, (0, 0, 0), tab, O.Params(r_cn=6.0))
    assert np.all(res["cn"] == 0.0)


def test_cn_simple_cubic_shells():
    """Eq. 4 summed over lattice images: in a simple-cubic crystal with
    lattice constant a and R_cn between sqrt(3)a and 2a, n = 6 f(a) +
    12 f(sqrt2 a) + 8 f(sqrt3 a) (coordination shells 6, 12, 8)."""
    tab = _table()
    a = 1.5
    lat = synth.simple_lattice("sc", a, element=1)
    rs = 2.0 * tab["rcov"][1]

    def f(r):
        return 1.0 / (1.0 + np.exp(-16.0 * (rs / r - 1.0)))

    want = 6 * f(a) + 12 * f(np.sqrt(2) * a) + 8 * f(np.sqrt(3) * a)
    res = O.d3(lat["pos"], lat["types"], lat["cell"], lat["pbc"], tab,
               O.Params(r_cn=2.8, r_pot=2.8))
    assert res["cn"][0] == pytest.approx(want, rel=1e-14)


# --------------------------------------------------------------- Eq. 3 ----

def test_c6_single_reference_is_the_reference():
    """Eq. 3 with one reference point per element: C6 = C6ref for any CN
    and dC6/dn = 0."""
    tab = O.convert_table(_table(force_k=1))
    zi = np.array([0, 1, 4, 2, 3])
    zj = np.array([4, 1, 0, 3, 3])
    ni = np.array([0.0, 1.3, 7.5, 30.0, 2.0])
    nj = np.array([5.0, 0.1, 2.2, 0.0, 60.0])
    c6, di, dj = O.c6_eq3(zi, zj, ni, nj, tab)
    raw = _table(force_k=1)["c6_ref"][zi, zj, 0, 0] * HARTREE_EV * BOHR_ANG ** 6
    assert c6 == pytest.approx(raw, rel=1e-14)
    assert np.abs(di).max() <= 1e-13 * raw.max()
    assert np.abs(dj).max() <= 1e-13 * raw.max()


def test_c6_two_reference_logistic_closed_form():
    """Eq. 3 with K_i = 2 and K_j = 1 reduces to a logistic blend:
    C6 = C1 + (C2 - C1) s(8 (r2 - r1)(n_i - (r1 + r2)/2)), s the logistic
    function, because the two Gaussian weights differ by
    exp(-4 (r2 - r1)(2 n_i - r1 - r2)).  Its n_i-derivative follows."""
    raw = _table()
    e = int(np.nonzero(raw["n_ref"] == 2)[0][0])
    f = int(np.nonzero(raw["n_ref"] == 1)[0][0])
    tab = O.convert_table(raw)
    r1, r2 = tab["cn_ref"][e, 0], tab["cn_ref"][e, 1]
    c1, c2 = tab["c6"][e, f, 0, 0], tab["c6"][e, f, 1, 0]
    ni = np.linspace(-1.0, 6.0, 57)
    z = 8.0 * (r2 - r1) * (ni - 0.5 * (r1 + r2))
    s = 1.0 / (1.0 + np.exp(-z))
    want = c1 + (c2 - c1) * s
    dwant = (c2 - c1) * s * (1.0 - s) * 8.0 * (r2 - r1)
    c6, di, dj = O.c6_eq3(np.full(ni.size, e), np.full(ni.size, f), ni,
                          np.full(ni.size, 2.5), tab)
    assert c6 == pytest.approx(want, rel=1e-13)
    assert di == pytest.approx(dwant, rel=1e-9, abs=1e-12 * abs(c2 - c1))
    # K_j = 1: no dependence on n_j (zero up to rounding)
    assert np.abs(dj).max() <= 1e-13 * max(c1, c2)


def test_c6_limits_at_separated_references():
    """Eq. 3 at a reference point far (>= 3 CN units) from every other
    reference returns that reference's C6 to within exp(-36)."""
    raw = _table(force_k=2)
    raw["cn_ref"][:, 0] = 0.0
    raw["cn_ref"][:, 1] = 3.5
    tab = O.convert_table(raw)
    for a, na in ((0, 0.0), (1, 3.5)):
        for b, nb in ((0, 0.0), (1, 3.5)):
            c6, _, _ = O.c6_eq3(np.array([1]), np.array([4]), np.array([na]),
                                np.array([nb]), tab)
            assert c6[0] == pytest.approx(tab["c6"][1, 4, a, b], rel=1e-15)


def test_c6_symmetry_and_derivatives():
    """C6_ef(n_i, n_j) = C6_fe(n_j, n_i) (the table is symmetric), and the
    analytic CN derivatives agree with central differences of C6."""
    tab = O.convert_table(_table())
    rng = np.random.default_rng(5)
    zi = rng.integers(0, 5, 200)
    zj = rng.integers(0, 5, 200)
    ni = rng.uniform(0, 5, 200)
    nj = rng.uniform(0, 5, 200)
    a, dai, daj = O.c6_eq3(zi, zj, ni, nj, tab)
    b, dbi, dbj = O.c6_eq3(zj, zi, nj, ni, tab)
    assert a == pytest.approx(b, rel=1e-13)
    assert dai == pytest.approx(dbj, rel=1e-11, abs=1e-9)
    h = 1e-6
    p, _, _ = O.c6_eq3(zi, zj, ni + h, nj, tab)
    m, _, _ = O.c6_eq3(zi, zj, ni - h, nj, tab)
    assert dai == pytest.approx((p - m) / (2 * h), rel=1e-6, abs=1e-5)
    p, _, _ = O.c6_eq3(zi, zj, ni, nj + h, tab)
    m, _, _ = O.c6_eq3(zi, zj, ni, nj - h, tab)
    assert daj == pytest.approx((p - m) / (2 * h), rel=1e-6, abs=1e-5)


def test_c6_no_underflow_far_from_references():
    """Eq. 3 stays finite (and equals the nearest reference blend) when the
    CN is so far from every reference that every raw Gaussian underflows."""
    tab = O.convert_table(_table())
    c6, di, dj = O.c6_eq3(np.array([0]), np.array([4]), np.array([40.0]),
                          np.array([35.0]), tab)
    assert np.isfinite(c6).all() and np.isfinite(di).all()
    k0 = tab["n_ref"][0] - 1
    k4 = tab["n_ref"][4] - 1
    # largest reference CN dominates; the tie breaks only if refs coincide
    assert c6[0] == pytest.approx(tab["c6"][0, 4, k0, k4], rel=1e-6)


# --------------------------------------------------------- Eqs. 1-2 -------

def test_dimer_energy_closed_form():
    """Eqs. 1-2 for a single-reference dimer: E(r) = -s6 C6/(r^6 + Rd^6)
    - s8 C6 R0^2/(r^8 + Rd^8) with R0^2 = 3 r2r4_i r2r4_j bohr^2 and
    Rd = a1 R0 + a2; the two site energies are equal halves."""
    raw = _table(force_k=1)
    prm = O.Params(r_pot=12.0, r_cn=6.0)
    for za, zb in [(0, 4), (1, 1), (2, 3)]:
        c6 = raw["c6_ref"][za, zb, 0, 0] * HARTREE_EV * BOHR_ANG ** 6
        r0 = np.sqrt(3.0 * raw["r2r4"][za] * raw["r2r4"][zb]) * BOHR_ANG
        rd = prm.a1 * r0 + prm.a2
        for r in [1.0, 2.5, 4.4, 8.0, 11.9]:
            pos, types = _dimer(za, zb, r)
            res = O.d3(pos, types, None, (0, 0, 0), raw, prm)
            want = -(prm.s6 * c6 / (r ** 6 + rd ** 6) +
                     prm.s8 * c6 * r0 ** 2 / (r ** 8 + rd ** 8))
            assert res["energy"] == pytest.approx(want, rel=1e-13)
            assert res["atom_energy"] == pytest.approx([want / 2, want / 2],
                                                       rel=1e-13)
            dE = (prm.s6 * c6 * 6 * r ** 5 / (r ** 6 + rd ** 6) ** 2 +
                  prm.s8 * c6 * r0 ** 2 * 8 * r ** 7 / (r ** 8 + rd ** 8) ** 2)
            # atom 2 sits at +x: F_2 = -dE/dr, F_1 = +dE/dr
            assert res["forces"][1, 0] == pytest.approx(-dE, rel=1e-12)
            assert res["forces"][0, 0] == pytest.approx(dE, rel=1e-12)
        pos, types = _dimer(za, zb, 12.0001)
        assert O.d3(pos, types, None, (0, 0, 0), raw, prm)["energy"] == 0.0


def test_damping_limits():
    """Eq. 2 limits: s8 = 0 keeps only the C6 term; a1 = a2 = 0 gives the
    undamped -C6/r^6 - C8/r^8; far away the C6 tail dominates."""
    raw = _table(force_k=1)
    c6 = raw["c6_ref"][1, 1, 0, 0] * HARTREE_EV * BOHR_ANG ** 6
    r0sq = 3.0 * raw["r2r4"][1] ** 2 * BOHR_ANG ** 2
    pos, types = _dimer(1, 1, 3.0)
    e = O.d3(pos, types, None, (0, 0, 0), raw,
             O.Params(a1=0.0, a2=0.0, s8=0.0))["energy"]
    assert e == pytest.approx(-c6 / 3.0 ** 6, rel=1e-14)
    e = O.d3(pos, types, None, (0, 0, 0), raw,
             O.Params(a1=0.0, a2=0.0, s8=1.0))["energy"]
    assert e == pytest.approx(-c6 / 3.0 ** 6 - c6 * r0sq / 3.0 ** 8, rel=1e-14)
    pos, types = _dimer(1, 1, 400.0)
    e = O.d3(pos, types, None, (0, 0, 0), raw, O.Params(r_pot=500.0))["energy"]
    assert e == pytest.approx(-c6 / 400.0 ** 6, rel=1e-6)


def _golden_lattice():
    rows = []
    with open(os.path.join(GOLDEN, "lattice_sums.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, a6, tol = line.split()
                rows.append((k, float(a6), float(tol)))
    return rows


@pytest.mark.parametrize("kind,a6,tol", _golden_lattice())
def test_lattice_sum_constants(kind, a6, tol):
    """Eqs. 1-2 summed over periodic images reproduce the classic lattice
    sums: with one reference (constant C6), s8 = 0 and no damping, the
    energy per atom of a cubic crystal is -1/2 C6 A6 / d_nn^6 (A6 from the
    golden file) once the cutoff tail, 2 pi rho/(3 R^3) per atom in the
    continuum limit, is added back."""
    raw = _table(force_k=1)
    c6 = raw["c6_ref"][1, 1, 0, 0] * HARTREE_EV * BOHR_ANG ** 6
    a = 4.0
    lat = synth.simple_lattice(kind, a, element=1)
    dnn = {"sc": a, "bcc": a * np.sqrt(3) / 2, "fcc": a / np.sqrt(2)}[kind]
    rcut = 30.0 * a
    nat = lat["pos"].shape[0]
    rho = nat / a ** 3
    res = R.d3(lat["pos"], lat["types"], lat["cell"], lat["pbc"], raw,
               s6=1.0, a1=0.0, s8=0.0, a2=0.0, r_pot=rcut, r_cn=0.5)
    tail = 0.5 * c6 * 4.0 * np.pi * rho / (3.0 * rcut ** 3)
    e_atom = res["energy"] / nat - tail
    want = -0.5 * c6 * a6 / dnn ** 6
    assert e_atom == pytest.approx(want, rel=tol)


# ----------------------------------------------------- Eqs. 5-7 -----------

def _fd_forces(pos, types, cell, pbc, tab, prm, h=1e-5, atoms=None):
    atoms = range(pos.shape[0]) if atoms is None else atoms
    out = {}
    for a in atoms:
        f = np.zeros(3)
        for k in range(3):
            p = pos.copy()
            p[a, k] += h
            ep = O.energy_only(p, types, cell, pbc, tab, prm)
            p[a, k] -= 2 * h
            em = O.energy_only(p, types, cell, pbc, tab, prm)
            f[k] = -(ep - em) / (2 * h)
        out[a] = f
    return out


def _min_gap_to_cutoffs(pos, cell, pbc, prm):
    i, j, d = O.entries(pos, cell, pbc, max(prm.r_pot, prm.r_cn) + 0.5)
    r = np.linalg.norm(d, axis=1)
    return min(np.abs(r - prm.r_pot).min(), np.abs(r - prm.r_cn).min())


def test_forces_match_finite_differences_cluster():
    """Forces are -grad E including the chain term through the CNs (the
    many-body remark after Eq. 4): central differences on a cluster whose
    diameter is below both cutoffs (no cutoff crossings)."""
    tab = _table()
    c = synth.cluster(24, 4.0, seed=11)
    prm = O.Params(r_pot=12.0, r_cn=9.0)
    res = O.d3(c["pos"], c["types"], None, (0, 0, 0), tab, prm)
    fd = _fd_forces(c["pos"], c["types"], None, (0, 0, 0), tab, prm)
    scale = np.abs(res["forces"]).max()
    for a, f in fd.items():
        assert f == pytest.approx(res["forces"][a], abs=1e-8 + 1e-7 * scale)


def test_forces_match_finite_differences_periodic_triclinic():
    """Same pin in a small triclinic periodic cell where several images of
    one atom lie inside R_pot (self-image entries included); the geometry
    keeps every entry more than 1e-3 A from either cutoff."""
    tab = _table()
    rng = np.random.default_rng(3)
    cell = np.array([[7.0, 0.0, 0.0], [2.1, 6.5, 0.0], [1.0, -1.4, 7.5]])
    pos = None
    for _ in range(100):
        s = rng.uniform(0, 1, (10, 3))
        p = s @ cell
        ii, jj, d = O.entries(p, cell, (1, 1, 1), 1.2)
        if len(ii) == 0:
            prm = O.Params(r_pot=9.0, r_cn=4.5)
            if _min_gap_to_cutoffs(p, cell, (1, 1, 1), prm) > 1e-3:
                pos = p
                break
    assert pos is not None
    types = rng.integers(0, 5, 10).astype(np.int32)
    res = O.d3(pos, types, cell, (1, 1, 1), tab, prm)
    fd = _fd_forces(pos, types, cell, (1, 1, 1), tab, prm)
    scale = np.abs(res["forces"]).max()
    for a, f in fd.items():
        assert f == pytest.approx(res["forces"][a], abs=1e-8 + 1e-7 * scale)
    assert np.abs(res["forces"].sum(0)).max() < 1e-12 * max(1.0, scale) * 10


def _strained(pos, cell, eps):
    F = np.eye(3) + eps
    return pos @ F.T, cell @ F.T


def test_virial_matches_strain_derivative():
    """Eq. 7 summed over atoms equals -dE/d(strain): central differences of
    E under a homogeneous deformation r -> (1 + eps) r of positions and
    lattice vectors, per tensor component, in a periodic triclinic cell."""
    tab = _table()
    rng = np.random.default_rng(8)
    cell = np.array([[8.0, 0.0, 0.0], [1.5, 7.2, 0.0], [-0.8, 1.1, 8.4]])
    prm = O.Params(r_pot=8.5, r_cn=4.0)
    for _ in range(200):
        s = rng.uniform(0, 1, (12, 3))
        pos = s @ cell
        ii, jj, d = O.entries(pos, cell, (1, 1, 1), 1.2)
        if len(ii) == 0 and _min_gap_to_cutoffs(pos, cell, (1, 1, 1), prm) > 2e-3:
            break
    types = rng.integers(0, 5, 12).astype(np.int32)
    res = O.d3(pos, types, cell, (1, 1, 1), tab, prm)
    h = 1e-6
    W = res["virial"]
    assert W == pytest.approx(W.T, abs=1e-13 * np.abs(W).max())
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            p1, c1 = _strained(pos, cell, e)
            p2, c2 = _strained(pos, cell, -e)
            ep = O.energy_only(p1, types, c1, (1, 1, 1), tab, prm)
            em = O.energy_only(p2, types, c2, (1, 1, 1), tab, prm)
            assert -(ep - em) / (2 * h) == pytest.approx(
                W[a, b], abs=1e-7 * np.abs(W).max())


def test_virial_equals_r_cross_f_for_cluster():
    """For a finite cluster the virial is sum_i r_i (x) F_i."""
    tab = _table()
    c = synth.cluster(30, 5.0, seed=2)
    res = O.d3(c["pos"], c["types"], None, (0, 0, 0), tab, O.Params())
    assert res["virial"] == pytest.approx(c["pos"].T @ res["forces"],
                                          abs=1e-13)


# ----------------------------------------- Eqs. 7-8 per atom -------------

def _site_energies(pos, types, tab, prm):
    return O.d3(pos, types, None, (0, 0, 0), tab, prm)["atom_energy"]


def test_atom_virial_is_eq7_by_finite_differences():
    """Eq. 7 as printed, W_i = sum_j r_ij (x) dU_j/dr_ji, with dU_j/dr_ji
    taken by central differences of the site energy U_j (Eq. 2) while atom
    i alone moves.  With one reference point per element C6 does not
    depend on the coordination numbers, so U_j depends on r_i only through
    r_ji and the formula is exact (catches a transposed product, a missing
    half or a sign)."""
    tab = _table(force_k=1)
    c = synth.cluster(8, 3.5, seed=21)
    prm = O.Params(r_pot=12.0, r_cn=9.0)
    pos, types = c["pos"], c["types"]
    res = O.d3(pos, types, None, (0, 0, 0), tab, prm)
    n, h = pos.shape[0], 1e-5
    dU = np.zeros((n, n, 3))  # dU[j, i, :] = dU_j / dr_i
    for i in range(n):
        for k in range(3):
            p = pos.copy()
            p[i, k] += h
            up = _site_energies(p, types, tab, prm)
            p[i, k] -= 2 * h
            um = _site_energies(p, types, tab, prm)
            dU[:, i, k] = (up - um) / (2 * h)
    scale = np.abs(res["atom_virial"]).max()
    for i in range(n):
        w = np.zeros((3, 3))
        for j in range(n):
            if j != i:
                w += np.outer(pos[j] - pos[i], dU[j, i])
        assert np.abs(w - res["atom_virial"][i]).max() < 1e-7 * scale


def test_heat_current_is_eq8_by_directional_differences():
    """Eq. 8, J_i = W_i . v_i: for the same single-reference cluster,
    J_i = sum_j r_ij (dU_j/dr_ji . v_i), the derivative of U_j along v_i
    taken by central differences (catches W^T v in place of W v for a
    non-symmetric tensor and a wrong velocity index)."""
    tab = _table(force_k=1)
    c = synth.cluster(7, 3.5, seed=22)
    prm = O.Params(r_pot=12.0, r_cn=9.0)
    pos, types = c["pos"], c["types"]
    vel = np.random.default_rng(4).normal(size=pos.shape)
    res = O.d3(pos, types, None, (0, 0, 0), tab, prm)
    J = O.heat_current(res["atom_virial"], vel)
    h = 1e-5
    for i in range(pos.shape[0]):
        p = pos.copy()
        p[i] += h * vel[i]
        up = _site_energies(p, types, tab, prm)
        p[i] -= 2 * h * vel[i]
        um = _site_energies(p, types, tab, prm)
        du = (up - um) / (2 * h)
        ji = sum((pos[j] - pos[i]) * du[j] for j in range(pos.shape[0]) if j != i)
        assert np.abs(ji - J[i]).max() < 1e-7 * np.abs(J).max()


def test_atom_virials_sum_to_strain_derivative():
    """With coordination-dependent C6 (several reference points) the
    per-atom virials of a periodic triclinic cell sum to -dE/d(strain),
    taken by central differences of E under homogeneous strain, and each is
    a symmetric tensor."""
    tab = _table()
    rng = np.random.default_rng(18)
    cell = np.array([[7.6, 0.0, 0.0], [1.2, 7.0, 0.0], [-0.6, 0.9, 8.1]])
    prm = O.Params(r_pot=8.0, r_cn=4.0)
    for _ in range(200):
        pos = rng.uniform(0, 1, (11, 3)) @ cell
        ii, jj, d = O.entries(pos, cell, (1, 1, 1), 1.2)
        if len(ii) == 0 and _min_gap_to_cutoffs(pos, cell, (1, 1, 1), prm) > 2e-3:
            break
    types = rng.integers(0, 5, 11).astype(np.int32)
    res = O.d3(pos, types, cell, (1, 1, 1), tab, prm)
    av = res["atom_virial"]
    scale = np.abs(av).max()
    assert np.abs(av - av.transpose(0, 2, 1)).max() < 1e-14 * scale
    tot = av.sum(0)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            p1, c1 = _strained(pos, cell, e)
            p2, c2 = _strained(pos, cell, -e)
            ep = O.energy_only(p1, types, c1, (1, 1, 1), tab, prm)
            em = O.energy_only(p2, types, c2, (1, 1, 1), tab, prm)
            assert -(ep - em) / (2 * h) == pytest.approx(tot[a, b], abs=1e-7 * np.abs(tot).max())


def test_atom_virial_splits_each_pair_evenly():
    """A heteronuclear dimer inside R_cn, with CN-dependent C6: G_1 != G_2,
    yet both atoms carry the same virial, half of the total (the chain term
    (G_1 + G_2) f'(r) is shared evenly, not given to one atom)."""
    tab = _table(force_k=(3, 4, 2, 5, 3))
    pos, types = _dimer(1, 4, 2.3)
    res = O.d3(pos, types, None, (0, 0, 0), tab, O.Params())
    assert abs(res["dedn"][0] - res["dedn"][1]) > 1e-6 * np.abs(res["dedn"]).max()
    av = res["atom_virial"]
    assert np.abs(av[0] - av[1]).max() < 1e-14 * np.abs(av).max()
    assert np.abs(av[0] + av[1] - res["virial"]).max() < 1e-14 * np.abs(av).max()
    # the virial of a dimer is the outer product of the bond with the force
    w = np.outer(pos[1] - pos[0], res["forces"][1])
    assert np.abs(av.sum(0) - w).max() < 1e-13 * np.abs(w).max()


# ------------------------------------------------------ invariances -------

def test_invariances_translation_rotation_permutation():
    """E, W invariant and F covariant under rigid translation (with atoms
    leaving the cell), rotation of cell and positions, and relabelling of
    the atoms; sum of forces is zero."""
    tab = _table()
    m = synth.mof_like(300, seed=4)
    cell, pbc = m["cell"], m["pbc"]
    prm = O.Params(r_pot=9.0, r_cn=5.0)
    ref = O.d3(m["pos"], m["types"], cell, pbc, tab, prm)
    assert np.abs(ref["forces"].sum(0)).max() < 1e-11
    t = O.d3(m["pos"] + np.array([3.3, -17.0, 41.0]), m["types"], cell, pbc,
             tab, prm)
    assert t["energy"] == pytest.approx(ref["energy"], rel=1e-12)
    assert t["forces"] == pytest.approx(ref["forces"], abs=1e-11)
    th = 0.7
    rot = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0],
                    [0, 0, 1.0]]) @ np.array([[1, 0, 0], [0, np.cos(0.3), -np.sin(0.3)],
                                              [0, np.sin(0.3), np.cos(0.3)]])
    r = O.d3(m["pos"] @ rot.T, m["types"], cell @ rot.T, pbc, tab, prm)
    assert r["energy"] == pytest.approx(ref["energy"], rel=1e-12)
    assert r["forces"] == pytest.approx(ref["forces"] @ rot.T, abs=1e-11)
    assert r["virial"] == pytest.approx(rot @ ref["virial"] @ rot.T, abs=1e-10)
    perm = np.random.default_rng(1).permutation(300)
    p = O.d3(m["pos"][perm], m["types"][perm], cell, pbc, tab, prm)
    assert p["energy"] == pytest.approx(ref["energy"], rel=1e-12)
    assert p["forces"] == pytest.approx(ref["forces"][perm], abs=1e-12)


def test_supercell_replication():
    """Replicating a periodic cell 2x2 in-plane leaves the energy per atom,
    the virial per atom and the force on each copy of an atom unchanged
    (images handled consistently, cutoff wider than the small cell)."""
    tab = _table()
    g = synth.bilayer_graphene(3, 3, seed=9)
    cell = g["cell"]
    reps = []
    for ia in range(2):
        for ib in range(2):
            reps.append(g["pos"] + ia * cell[0] + ib * cell[1])
    pos2 = np.concatenate(reps)
    cell2 = cell.copy()
    cell2[0] *= 2
    cell2[1] *= 2
    t2 = np.tile(g["types"], 4)
    a = R.d3(g["pos"], g["types"], cell, g["pbc"], tab)
    b = R.d3(pos2, t2, cell2, g["pbc"], tab)
    n = g["pos"].shape[0]
    assert b["energy"] / (4 * n) == pytest.approx(a["energy"] / n, rel=1e-12)
    assert b["virial"] / 4 == pytest.approx(a["virial"], rel=1e-11, abs=1e-14)
    for k in range(4):
        assert b["forces"][k * n:(k + 1) * n] == pytest.approx(a["forces"],
                                                               abs=1e-14)


def test_perfect_ab_bilayer_symmetry():
    """A perfect AB bilayer has no in-plane forces (every atom sits on a
    site of threefold symmetry) and an in-plane isotropic virial."""
    tab = _table()
    g = synth.bilayer_graphene(6, 6, jitter=0.0)
    res = R.d3(g["pos"], g["types"], g["cell"], g["pbc"], tab)
    assert np.abs(res["forces"][:, :2]).max() < 1e-14
    W = res["virial"]
    assert W[0, 0] == pytest.approx(W[1, 1], rel=1e-12)
    assert abs(W[0, 1]) < 1e-12 * abs(W[0, 0])
    # the two layers attract: equal and opposite z forces
    fz = res["forces"][:, 2]
    z = g["pos"][:, 2]
    top = z > z.mean()
    assert fz[top].sum() == pytest.approx(-fz[~top].sum(), rel=1e-12)
    assert fz[top].sum() < 0.0


def test_single_atom_cells():
    """One atom in a large box has no entries (E = 0); one atom in a small
    periodic box interacts with its own images: E < 0 and zero force."""
    tab = _table()
    big = np.eye(3) * 30.0
    r = O.d3(np.array([[1.0, 2.0, 3.0]]), np.array([2]), big, (1, 1, 1), tab)
    assert r["energy"] == 0.0 and np.all(r["forces"] == 0.0)
    small = np.eye(3) * 4.0
    r = O.d3(np.array([[1.0, 2.0, 3.0]]), np.array([2]), small, (1, 1, 1), tab)
    assert r["energy"] < 0.0 and np.abs(r["forces"]).max() < 1e-15
    assert r["cn"][0] > 0.0


# ------------------------------------------------------ oracle<->oracle ---

def test_c_oracle_matches_numpy_oracle():
    """The C oracle (used at larger sizes and for the CPU baseline) agrees
    with the NumPy oracle on graphene, a MOF-like cube and a tiny
    triclinic cell with many images."""
    tab = _table()
    cases = [synth.bilayer_graphene(), synth.mof_like(500, seed=5)]
    cell = np.array([[5.0, 0.0, 0.0], [2.0, 4.6, 0.0], [0.5, 0.7, 5.3]])
    s = np.random.default_rng(2).uniform(0, 1, (4, 3))
    cases.append({"pos": s @ cell, "types": np.array([0, 1, 2, 4], np.int32),
                  "cell": cell, "pbc": np.array([1, 1, 1])})
    for c in cases:
        a = O.d3(c["pos"], c["types"], c["cell"], c["pbc"], tab)
        b = R.d3(c["pos"], c["types"], c["cell"], c["pbc"], tab)
        assert b["energy"] == pytest.approx(a["energy"], rel=1e-12)
        for k in ("forces", "virial", "atom_energy", "atom_virial", "cn", "dedn"):
            sc = max(np.abs(a[k]).max(), 1e-30)
            # dE/dn sums terms of both signs: looser relative bound
            tol = 1e-10 if k == "dedn" else 1e-12
            assert np.abs(a[k] - b[k]).max() <= tol * sc, k


def _random_cell(rng, lo, hi, skew):
    """A random triclinic cell: rows a, b, c with lengths in [lo, hi] and
    off-diagonal parts up to skew times the diagonal."""
    cell = np.diag(rng.uniform(lo, hi, 3))
    cell[1, 0] = skew * rng.uniform(-1, 1) * cell[1, 1]
    cell[2, 0] = skew * rng.uniform(-1, 1) * cell[2, 2]
    cell[2, 1] = skew * rng.uniform(-1, 1) * cell[2, 2]
    return cell


def _brute_vs_cells(c, tab, **prm):
    a = R.d3(c["pos"], c["types"], c["cell"], c["pbc"], tab, **prm)
    b = R.d3(c["pos"], c["types"], c["cell"], c["pbc"], tab, cells=True, **prm)
    assert b["n_entries"] == a["n_entries"]
    assert b["energy"] == pytest.approx(a["energy"], rel=1e-12, abs=1e-300)
    for k in ("forces", "virial", "atom_energy", "atom_virial", "cn", "dedn"):
        # forces that cancel by symmetry (one atom and its images) are
        # rounding noise: scale them by the energy, eV per Angstrom
        sc = max(np.abs(a[k]).max(), abs(a["energy"]), 1e-30)
        tol = 1e-10 if k == "dedn" else 1e-12
        assert np.abs(a[k] - b[k]).max() <= tol * sc, k
    return a


@pytest.mark.parametrize("seed", range(6))
def test_cell_list_mode_matches_brute_force_small_cells(seed):
    """The oracle's cell-list mode (used for the 10^5-10^6-atom cells)
    finds exactly the entries of the brute-force mode and gives the same
    results, on tiny skewed cells whose lattice planes lie closer than the
    cutoffs (several images of one atom, and the same bin visited with
    different images), with atoms outside the cell, and with open axes.  A
    stencil one bin too short, a wrong image of a wrapped bin or a missed
    self-image would change the entry count."""
    rng = np.random.default_rng(100 + seed)
    tab = _table()
    cell = _random_cell(rng, 4.0, 9.0, 0.4)
    n = int(rng.integers(1, 9))
    pbc = [(1, 1, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 0, 0), (0, 0, 0)][seed]
    s = rng.uniform(-0.3, 1.3, (n, 3))
    c = {"pos": s @ cell, "types": rng.integers(0, 5, n).astype(np.int32), "cell": cell,
         "pbc": np.array(pbc)}
    a = _brute_vs_cells(c, tab, r_pot=12.0, r_cn=6.0)
    if sum(pbc) == 3 and n > 1:
        assert a["n_entries"] > 20 * n  # many images per atom


def test_cell_list_mode_matches_brute_force_mid_cells():
    """Cells between two and three cutoffs wide (two bins per axis: both
    neighbouring offsets reach the other bin, with different images),
    unequal cutoffs and a cutoff above the box, on a MOF-like cube and on
    the bilayer."""
    tab = _table()
    m = synth.mof_like(700, seed=9)  # L = 25.96 A
    _brute_vs_cells(m, tab, r_pot=12.0, r_cn=6.0)
    _brute_vs_cells(m, tab, r_pot=9.0, r_cn=9.5)
    g = synth.bilayer_graphene()
    _brute_vs_cells(g, tab, r_pot=16.0, r_cn=5.0)


def test_sampled_mode_matches_full():
    """The per-atom neighbourhood evaluation used at 10^5-10^6 atoms gives
    the same force, site energy, CN and dE/dn as the full evaluation."""
    tab = _table()
    m = synth.mof_like(900, seed=6)
    full = R.d3(m["pos"], m["types"], m["cell"], m["pbc"], tab)
    idx = [0, 11, 450, 899]
    s = O.sampled(m["pos"], m["types"], m["cell"], m["pbc"], tab, idx)
    sc = np.abs(full["forces"]).max()
    assert np.abs(s["forces"] - full["forces"][idx]).max() < 1e-12 * sc
    assert s["atom_energy"] == pytest.approx(full["atom_energy"][idx], rel=1e-11)
    assert s["cn"] == pytest.approx(full["cn"][idx], rel=1e-12)
    assert s["dedn"] == pytest.approx(full["dedn"][idx], rel=1e-10, abs=1e-14)
    sw = np.abs(full["atom_virial"]).max()
    assert np.abs(s["atom_virial"] - full["atom_virial"][idx]).max() < 1e-11 * sw


# ------------------------------------------------- surrogate network ------

def test_mlp_oracle_gradient_matches_finite_differences():
    """The backpropagated loss gradient of the surrogate network equals
    central differences of its loss, parameter by parameter."""
    from oracle import mlp_oracle as M
    rng = np.random.default_rng(0)
    theta = rng.normal(0.0, 0.4, M.N_PARAMS)
    x = rng.uniform(-1, 1, (17, 2))
    t = rng.normal(size=(17, 3))
    loss, g = M.loss_and_grad(theta, x, t)
    h = 1e-6
    idx = np.concatenate([np.arange(0, 64, 7), np.arange(64, 96, 5), np.arange(96, 1120, 97),
                          np.arange(1120, 1152, 9), np.arange(1152, 1251, 11)])
    for q in idx:
        tp = theta.copy()
        tp[q] += h
        tm = theta.copy()
        tm[q] -= h
        fd = (M.loss_and_grad(tp, x, t)[0] - M.loss_and_grad(tm, x, t)[0]) / (2 * h)
        assert g[q] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_mlp_oracle_closed_forms():
    """Networks with a closed-form output: biases only give y = b3; a
    constant hidden layer gives y = silu(c) W3 column sums; silu(0) = 0 and
    silu(z) -> z for large z."""
    from oracle import mlp_oracle as M
    p = M.unpack(np.zeros(M.N_PARAMS)).copy()
    p = {k: v.copy() for k, v in p.items()}
    p["b3"][:] = [0.5, -1.0, 2.0]
    y, _ = M.forward(M.pack(p), np.array([[0.3, -0.7], [1.0, 1.0]]))
    assert np.all(y == np.array([0.5, -1.0, 2.0]))
    p["b2"][:] = 1.3
    p["W3"][:, 0] = 1.0 / 32
    p["W3"][:, 1] = 0.0
    p["W3"][:, 2] = -2.0 / 32
    y, _ = M.forward(M.pack(p), np.array([[0.1, 0.2]]))
    s = 1.3 / (1.0 + np.exp(-1.3))
    assert y[0] == pytest.approx([0.5 + s, -1.0, 2.0 - 2.0 * s], rel=1e-14)
    assert M.silu(np.array([0.0]))[0] == 0.0
    assert M.silu(np.array([40.0]))[0] == pytest.approx(40.0, rel=1e-15)


def test_adam_first_steps_closed_form():
    """Adam (one update per step, step counted from 1) against its closed
    form for the first two steps, from zero moments: with gradient g1 then
    g2 the bias-corrected moments are g1, g1^2 after step 1 and
    (b1 g1 + g2)/(1 + b1), (b2 g1^2 + g2^2)/(1 + b2) after step 2, so the
    updates are -lr g1/(|g1| + eps) and -lr m2/(sqrt(v2) + eps).  A bias
    correction from step 0, swapped betas or a missing square root fail
    this."""
    from oracle import mlp_oracle as M
    rng = np.random.default_rng(4)
    theta = rng.normal(size=40)
    g1 = rng.normal(size=40)
    g2 = rng.normal(size=40) * rng.uniform(0.1, 3.0, 40)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    z = np.zeros(40)
    t1, m, v = M.adam_step(theta, g1, z, z, 1, lr)
    assert t1 - theta == pytest.approx(-lr * g1 / (np.abs(g1) + eps), rel=1e-12)
    t2, m, v = M.adam_step(t1, g2, m, v, 2, lr)
    mh = (b1 * g1 + g2) / (1 + b1)
    vh = (b2 * g1 * g1 + g2 * g2) / (1 + b2)
    assert t2 - t1 == pytest.approx(-lr * mh / (np.sqrt(vh) + eps), rel=1e-10)
    # a constant gradient moves every parameter by lr per step (eps aside)
    t3, m3, v3 = M.adam_step(theta, g1, z, z, 1, lr)
    t4, _, _ = M.adam_step(t3, g1, m3, v3, 2, lr)
    assert t4 - t3 == pytest.approx(-lr * np.sign(g1), rel=1e-6)


def test_cosine_step_size_endpoints():
    """The cosine schedule starts at lr0, ends at lr1, passes their mean
    half way and is symmetric about it (a sine in place of the cosine, or a
    period of total/2, fails this)."""
    from oracle import mlp_oracle as M
    lr0, lr1, T = 5e-3, 1e-6, 400
    assert M.cosine_step_size(0, T, lr0, lr1) == pytest.approx(lr0, rel=1e-15)
    assert M.cosine_step_size(T, T, lr0, lr1) == pytest.approx(lr1, rel=1e-12)
    assert M.cosine_step_size(T // 2, T, lr0, lr1) == pytest.approx(0.5 * (lr0 + lr1), rel=1e-14)
    a = M.cosine_step_size(100, T, lr0, lr1) - 0.5 * (lr0 + lr1)
    b = M.cosine_step_size(300, T, lr0, lr1) - 0.5 * (lr0 + lr1)
    assert a == pytest.approx(-b, rel=1e-12) and a > 0


# ----------------------------------------------- velocity-Verlet driver ----

def test_md_oracle_energy_conservation_and_reversibility():
    """The NVE reference integrator on a free 8-atom cluster with cutoffs
    beyond its diameter (so E is smooth): the total-energy error of velocity
    Verlet shrinks as dt^2 and stays far below the potential-energy swing
    (catches a unit mismatch between the force-to-acceleration and the
    kinetic-energy constants, or a dropped half-kick), and reversing the
    velocities retraces the trajectory to rounding (catches a kick that uses
    the wrong force)."""
    from oracle import md_oracle as MD
    tab = _table()
    c = synth.cluster(8, 2.5, dmin=1.5, seed=11)
    vel = np.random.default_rng(5).normal(scale=0.01, size=(8, 3))
    mass = np.asarray(synth.MASSES_AMU)[c["types"]]
    prm = dict(r_pot=40.0, r_cn=40.0)
    err = []
    for dt, n in ((1.0, 200), (0.5, 400)):
        p, v, th = MD.run(c["pos"], vel, mass, c["types"], None, (0, 0, 0), tab, n, dt, **prm)
        et = th[:, 0] + th[:, 1]
        err.append(np.abs(et - et[0]).max())
        swing = th[:, 0].max() - th[:, 0].min()
    assert np.abs(p - c["pos"]).max() > 1.0          # the atoms really moved
    assert 3.5 < err[0] / err[1] < 4.5
    assert err[1] < 1e-3 * swing
    p, v, _ = MD.run(c["pos"], vel, mass, c["types"], None, (0, 0, 0), tab, 200, 1.0, **prm)
    p2, v2, _ = MD.run(p, -v, mass, c["types"], None, (0, 0, 0), tab, 200, 1.0, **prm)
    assert np.abs(p2 - c["pos"]).max() < 1e-12
    assert np.abs(v2 + vel).max() < 1e-14


# ------------------------------------- zero damping and the ATM term ------
# Both are the D3 variants the paper names and sets aside (Sec. II A, the
# paragraph before Eq. 1); their definitions follow the D3 reference the
# paper cites (Grimme et al., J. Chem. Phys. 132, 154104 (2010)).

def _c6_r0(raw, za, zb):
    c6 = raw["c6_ref"][za, zb, 0, 0] * HARTREE_EV * BOHR_ANG ** 6
    r0 = np.sqrt(3.0 * raw["r2r4"][za] * raw["r2r4"][zb]) * BOHR_ANG
    return c6, r0


def test_zero_damping_dimer_closed_form():
    """Zero damping on a single-reference dimer: E(r) = -s6 C6 f6 / r^6
    - s8 C6 R0^2 f8 / r^8 with f_n = 1 / (1 + 6 (r / (s_r,n R0))^-alpha_n),
    alpha = 14, 16.  At r = s_r,6 R0 the C6 term is damped to exactly 1/7,
    at r = s_r,8 R0 the C8 term; far away both dampings go to 1.  A swapped
    alpha, a missing factor 6 or R0 in place of s_r R0 fails one of these;
    the force is -dE/dr of the closed form."""
    raw = _table(force_k=1)
    for za, zb in [(0, 4), (1, 1), (2, 3)]:
        c6, r0 = _c6_r0(raw, za, zb)
        prm6 = O.Params(damping="zero", s6=1.0, s8=0.0, rs6=1.217, r_pot=30.0)
        r = 1.217 * r0
        res = O.d3(*_dimer(za, zb, r), None, (0, 0, 0), raw, prm6)
        assert res["energy"] == pytest.approx(-c6 / r ** 6 / 7.0, rel=1e-13)
        prm8 = O.Params(damping="zero", s6=0.0, s8=0.722, rs8=1.0, r_pot=30.0)
        r = r0
        res = O.d3(*_dimer(za, zb, r), None, (0, 0, 0), raw, prm8)
        assert res["energy"] == pytest.approx(-0.722 * c6 * r0 ** 2 / r ** 8 / 7.0, rel=1e-13)
        prm = O.Params(damping="zero", s6=1.0, s8=0.722, rs6=1.217, rs8=1.0, r_pot=30.0)
        for r in (1.5, 3.0, 5.5, 9.0):
            res = O.d3(*_dimer(za, zb, r), None, (0, 0, 0), raw, prm)

            def e_of(x):
                f6 = 1.0 / (1.0 + 6.0 * (x / (1.217 * r0)) ** -14)
                f8 = 1.0 / (1.0 + 6.0 * (x / r0) ** -16)
                return -c6 * f6 / x ** 6 - 0.722 * c6 * r0 ** 2 * f8 / x ** 8
            assert res["energy"] == pytest.approx(e_of(r), rel=1e-13)
            h = 1e-6 * r
            dE = (e_of(r + h) - e_of(r - h)) / (2 * h)
            assert res["forces"][1, 0] == pytest.approx(-dE, rel=1e-7)
        far = O.d3(*_dimer(za, zb, 28.0), None, (0, 0, 0), raw, prm)
        assert far["energy"] == pytest.approx(-c6 / 28.0 ** 6 - 0.722 * c6 * r0 ** 2 / 28.0 ** 8,
                                              rel=1e-9)


def _atm_energy(pos, types, raw, **kw):
    """Three-body part alone: E(s9) - E(s9 = 0) on a free cluster."""
    on = O.d3(pos, types, None, (0, 0, 0), raw, O.Params(s9=1.0, **kw))
    off = O.d3(pos, types, None, (0, 0, 0), raw, O.Params(s9=0.0, **kw))
    return on, off


@pytest.mark.parametrize("shape", ["equilateral", "collinear", "right"])
def test_atm_triangle_closed_forms(shape):
    """The ATM term of one homonuclear triangle (single reference, so every
    C6 is the reference value): E = C6^(3/2) (1 + 3 cos A cos B cos C)
    / (r_AB r_BC r_CA)^3 f3, f3 = 1 / (1 + 6 (rbar / (4/3 R0))^-16).  The
    angle factor is 11/8 for an equilateral triangle (repulsive), -2 for a
    collinear A-B-C with AB = BC, and 1 with a right angle; at rbar = 4/3 R0
    the damping is exactly 1/7.  The site energies are thirds of E and the
    total force is zero."""
    raw = _table(force_k=1)
    z = 1
    c6, r0 = _c6_r0(raw, z, z)
    types = np.array([z, z, z], np.int32)
    for rbar in (4.0 / 3.0 * r0, 5.0):
        if shape == "equilateral":
            s = rbar
            pos = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * np.sqrt(3) / 2, 0]])
            sides, factor = (s, s, s), 11.0 / 8.0
        elif shape == "collinear":
            s = rbar / 2 ** (1 / 3)
            pos = np.array([[0, 0, 0], [s, 0, 0], [2 * s, 0, 0]])
            sides, factor = (s, s, 2 * s), -2.0
        else:
            s = rbar / 2 ** (1 / 6)
            pos = np.array([[0, 0, 0], [s, 0, 0], [0, s, 0]])
            sides, factor = (s, s, s * np.sqrt(2)), 1.0
        on, off = _atm_energy(pos, types, raw, r_pot=15.0, r_cn=15.0, r_atm=15.0)
        prod = sides[0] * sides[1] * sides[2]
        f3 = 1.0 / (1.0 + 6.0 * (prod ** (1 / 3) / (4.0 / 3.0 * r0)) ** -16)
        want = c6 ** 1.5 * factor / prod ** 3 * f3
        if rbar == 4.0 / 3.0 * r0:
            assert f3 == pytest.approx(1.0 / 7.0, rel=1e-14)
        assert on["energy"] - off["energy"] == pytest.approx(want, rel=1e-12)
        assert on["atom_energy"] - off["atom_energy"] == pytest.approx([want / 3] * 3, rel=1e-12)
        assert np.abs(on["forces"].sum(0)).max() < 1e-12 * np.abs(on["forces"]).max()
    if shape == "equilateral":
        assert want > 0.0


def test_atm_counts_each_triangle_once():
    """Four atoms on a regular tetrahedron: the three-body energy is exactly
    four equilateral-triangle terms, whichever vertex finds them; with the
    cutoff below the edge it vanishes."""
    raw = _table(force_k=1)
    z = 2
    c6, r0 = _c6_r0(raw, z, z)
    s = 4.0
    pos = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) * s / np.sqrt(8)
    types = np.full(4, z, np.int32)
    on, off = _atm_energy(pos, types, raw, r_pot=10.0, r_cn=10.0, r_atm=10.0)
    f3 = 1.0 / (1.0 + 6.0 * (s / (4.0 / 3.0 * r0)) ** -16)
    assert on["energy"] - off["energy"] == pytest.approx(4 * c6 ** 1.5 * 11 / 8 / s ** 9 * f3,
                                                         rel=1e-12)
    short, off2 = _atm_energy(pos, types, raw, r_pot=10.0, r_cn=10.0, r_atm=3.99)
    assert short["energy"] == off2["energy"]


def _variant_params(**kw):
    base = dict(damping="zero", s6=1.0, s8=0.722, rs6=1.217, rs8=1.0, s9=1.0)
    base.update(kw)
    return O.Params(**base)


@pytest.mark.parametrize("damping", ["bj", "zero"])
def test_atm_and_zero_damping_forces_are_the_gradient(damping):
    """Forces with the three-body term (and either damping) against central
    differences of the energy, on a cluster whose diameter lies within every
    cutoff (so E is smooth) and whose coordination numbers vary, so the
    chain term of the three-body coefficient through dE/dn is exercised."""
    raw = _table()
    c = synth.cluster(9, 2.6, dmin=1.3, seed=14)
    prm = _variant_params(damping=damping, r_pot=20.0, r_cn=20.0, r_atm=20.0)
    res = O.d3(c["pos"], c["types"], None, (0, 0, 0), raw, prm)
    h = 1e-5
    for k in (0, 4, 8):
        for ax in range(3):
            p = c["pos"].copy()
            p[k, ax] += h
            ep = O.energy_only(p, c["types"], None, (0, 0, 0), raw, prm)
            p[k, ax] -= 2 * h
            em = O.energy_only(p, c["types"], None, (0, 0, 0), raw, prm)
            assert res["forces"][k, ax] == pytest.approx(-(ep - em) / (2 * h), abs=2e-8)
    assert np.abs(res["forces"].sum(0)).max() < 1e-12


def test_atm_virial_is_the_strain_derivative():
    """With the three-body term on a small triclinic periodic cell (images
    inside every cutoff): W = -dE/d(strain) by central differences of a
    homogeneous strain of cell and positions, and sum_i W_i = W."""
    raw = _table()
    cell = np.array([[7.0, 0.0, 0.0], [1.2, 6.5, 0.0], [0.4, -0.8, 7.4]])
    s = np.random.default_rng(9).uniform(0, 1, (5, 3))
    pos = s @ cell
    types = np.array([0, 1, 2, 3, 4], np.int32)
    prm = _variant_params(damping="bj", r_pot=9.0, r_cn=6.0, r_atm=6.0)
    res = O.d3(pos, types, cell, (1, 1, 1), raw, prm)
    h = 1e-6
    for a, b in [(0, 0), (1, 1), (0, 1), (2, 0), (1, 2)]:
        eps = np.zeros((3, 3))
        eps[a, b] = eps[b, a] = h if a != b else h
        def strained(sign):
            m = np.eye(3) + sign * eps
            return O.energy_only(pos @ m.T, types, cell @ m.T, (1, 1, 1), raw, prm)
        de = (strained(1) - strained(-1)) / (2 * h)
        want = -de if a == b else -de / 2
        assert res["virial"][a, b] == pytest.approx(want, rel=1e-6, abs=1e-9)
    assert np.abs(res["atom_virial"].sum(0) - res["virial"]).max() < 1e-12 * np.abs(res["virial"]).max()


def test_variants_off_reduce_to_eq2():
    """s9 = 0 with BJ damping is exactly the two-body Eq. 2 evaluation."""
    raw = _table()
    m = synth.mof_like(300, seed=8)
    a = O.d3(m["pos"], m["types"], m["cell"], m["pbc"], raw)
    b = O.d3(m["pos"], m["types"], m["cell"], m["pbc"], raw, O.Params(s9=0.0, r_atm=6.0))
    for k in ("energy", "forces", "virial", "atom_energy", "dedn"):
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_c_oracle_variants_match_numpy_oracle():
    """The C oracle's zero damping and three-body term (both enumerations)
    agree with the NumPy oracle on a skewed periodic cell with images
    inside the cutoffs, a MOF-like cube and the bilayer."""
    raw = _table()
    cell = np.array([[7.0, 0.0, 0.0], [1.2, 6.5, 0.0], [0.4, -0.8, 7.4]])
    s = np.random.default_rng(9).uniform(0, 1, (5, 3))
    cases = [{"pos": s @ cell, "types": np.array([0, 1, 2, 3, 4], np.int32), "cell": cell,
              "pbc": np.array([1, 1, 1])}, synth.mof_like(400, seed=12), synth.bilayer_graphene()]
    for c in cases:
        for damping, s8 in (("bj", 0.7875), ("zero", 0.722)):
            kw = dict(damping=damping, s8=s8, s9=1.0, r_pot=10.0, r_cn=5.0, r_atm=5.0)
            a = O.d3(c["pos"], c["types"], c["cell"], c["pbc"], raw, O.Params(**kw))
            for cells in (False, True):
                b = R.d3(c["pos"], c["types"], c["cell"], c["pbc"], raw, cells=cells, **kw)
                assert b["energy"] == pytest.approx(a["energy"], rel=1e-12)
                for k in ("forces", "virial", "atom_energy", "atom_virial", "dedn"):
                    sc = max(np.abs(a[k]).max(), abs(a["energy"]))
                    tol = 1e-10 if k == "dedn" else 1e-12
                    assert np.abs(a[k] - b[k]).max() <= tol * sc, (damping, cells, k)
