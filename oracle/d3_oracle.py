"""Plain FP64 NumPy oracle for D3 with Becke-Johnson damping.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the
product path may import this module.

What it computes, and where each step comes from (Ying & Fan, "Combining
the D3 dispersion correction with the neuroevolution machine-learned
potential", Sec. II A):

* entries: every ordered pair (i, j, T) of an atom i and an image j + T of
  atom j (T a lattice translation, zero on open axes) with (j, T) != (i, 0)
  and |r_j + T - r_i| below the cutoff.  Found by brute force over all j
  and all translations that can reach the cutoff.  Cutoffs are hard: an
  entry counts iff r^2 < R^2.
* coordination number, Eq. 4: n_i = sum over entries with r < R_cn of
  1 / (1 + exp(-16 ((Rcov_i + Rcov_j) / r - 1))).
* C6, Eq. 3: the Gaussian-weighted (exponent -4) average of the reference
  C6 values over all reference-CN pairs (a, b), evaluated per entry exactly
  as printed.  All exponents of one entry are shifted by their maximum
  first; the shift cancels between numerator and denominator and keeps
  both sums representable.
* C8 = C6 R0^2 and R0 the geometric mean of the per-species parameters
  (text after Eq. 2).  The per-species parameter is sqrt(3) * r2r4, so
  R0^2 = 3 r2r4_i r2r4_j (bohr^2), the usual BJ convention.
* site energy, Eq. 2: U_i = -1/2 sum_j [s6 C6/(r^6 + Rd^6) + s8 C8/(r^8 + Rd^8)]
  with Rd = a1 R0 + a2, over entries with r < R_pot; total energy Eq. 1.
* forces: the exact negative gradient of the total energy.  Eqs. 5-6
  state the many-body force through dU_i/dr_ij; because C6 depends on the
  coordination numbers (the "two-body" term is really many-body, text
  after Eq. 4), the gradient has a direct part at fixed C6 and a chain
  part through dE/dn_k.
* virial, Eq. 7 summed over atoms: W = -dE/d(strain), which for a finite
  cluster equals sum_i r_i (x) F_i (eV).
* per-atom virial, Eq. 7: W_i = sum over the entries (i, j, T) of i of the
  entry's term of W, -1/2 [phi'(r) 1(r < R_pot) + (G_i + G_j) f'(r)
  1(r < R_cn)] r (x) r / r.  Each unordered pair's term is split half and
  half between its two atoms, so sum_i W_i = W exactly.  For the direct
  part this is Eq. 7 as printed (r_ij (x) dU_j/dr_ji at fixed C6); the
  paper's formula assumes U_j depends on its own neighbour vectors only,
  which D3's coordination numbers break, and the chain part is given the
  same half-and-half split.
* per-atom heat current, Eq. 8: J_i = W_i v_i.

Units: Angstrom and eV.  The table arrives in Hartree*bohr^6 (C6) and bohr
(r2r4) and is converted here with CODATA 2018 constants.

Parity: pinned (closed forms, lattice sums, finite differences and
invariances in the test suite; see the oracle pin tests).
"""

import numpy as np

HARTREE_EV = 27.211386245988
BOHR_ANG = 0.529177210903
MAX_REF = 5


class Params:
    """Damping parameters and cutoffs (a2 and cutoffs in Angstrom).

    damping="bj" is Eq. 2 (Becke-Johnson).  damping="zero" is the other D3
    damping the paper names and sets aside (Sec. II A, before Eq. 1), in its
    definition by Grimme et al. (J. Chem. Phys. 132, 154104 (2010), the D3
    reference the paper cites): each term -s_n C_n / r^n is multiplied by
    f_n = 1 / (1 + 6 (r / (s_r,n R0))^(-alpha_n)), alpha_6 = 14,
    alpha_8 = 16, with s_r,6 = rs6 and s_r,8 = rs8.

    s9 != 0 adds the three-body Axilrod-Teller-Muto term of the same
    reference (the paper also sets it aside) over triples whose three
    distances are below r_atm (see atm_terms)."""

    def __init__(self, s6=1.0, a1=0.4289, s8=0.7875, a2=4.4407,
                 r_pot=12.0, r_cn=6.0, damping="bj", rs6=1.217, rs8=1.0,
                 s9=0.0, r_atm=None):
        self.s6, self.a1, self.s8, self.a2 = s6, a1, s8, a2
        self.r_pot, self.r_cn = r_pot, r_cn
        assert damping in ("bj", "zero")
        self.damping, self.rs6, self.rs8 = damping, rs6, rs8
        self.s9 = s9
        self.r_atm = r_cn if r_atm is None else r_atm


def convert_table(table):
    """Per-element-pair constants in eV/Angstrom units."""
    n_ref = np.asarray(table["n_ref"], dtype=np.int64)
    cn_ref = np.asarray(table["cn_ref"], dtype=np.float64)
    c6 = np.asarray(table["c6_ref"], dtype=np.float64) * HARTREE_EV * BOHR_ANG ** 6
    r2r4 = np.asarray(table["r2r4"], dtype=np.float64)
    r0sq = 3.0 * np.outer(r2r4, r2r4) * BOHR_ANG ** 2
    return {"n_ref": n_ref, "cn_ref": cn_ref, "c6": c6,
            "rcov": np.asarray(table["rcov"], dtype=np.float64), "r0sq": r0sq}


def translations(cell, pbc, rmax, pos=None):
    """All lattice translations n0 a + n1 b + n2 c that can bring an image of
    one atom within rmax of another: on a periodic axis k, |n_k| <=
    ceil(rmax/h_k + spread_k), where h_k is the distance between lattice
    planes k and spread_k the extent of the atoms' fractional coordinate k
    (below 1 for wrapped atoms); zero on open axes."""
    cell = np.asarray(cell, dtype=np.float64)
    vol = abs(np.linalg.det(cell))
    if pos is not None and len(pos):
        s = np.asarray(pos, dtype=np.float64) @ np.linalg.inv(cell)
        spread = s.max(axis=0) - s.min(axis=0)
    else:
        spread = np.ones(3)
    reach = []
    for k in range(3):
        if not pbc[k]:
            reach.append(0)
            continue
        cr = np.cross(cell[(k + 1) % 3], cell[(k + 2) % 3])
        h = vol / np.linalg.norm(cr)
        reach.append(int(np.ceil(rmax / h + spread[k])))
    rng = [np.arange(-m, m + 1) for m in reach]
    n = np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, 3)
    return n, n.astype(np.float64) @ cell


def entries(pos, cell, pbc, rcut, rows=None):
    """Brute-force entry list.  Returns (i, j, d) with d = r_j + T - r_i for
    every (i, j, T) with (j,T) != (i,0) and |d|^2 < rcut^2.  ``rows``
    restricts i to a subset (others are still candidates for j)."""
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    if cell is None:
        cell = np.eye(3)
        pbc = (0, 0, 0)
    nvec, tvec = translations(cell, pbc, rcut, pos)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    rc2 = rcut * rcut
    out_i, out_j, out_d = [], [], []
    chunk = max(1, 4_000_000 // max(1, n * len(tvec)))
    for s in range(0, len(rows), chunk):
        ii = rows[s:s + chunk]
        for t, T in zip(nvec, tvec):
            d = pos[None, :, :] + T[None, None, :] - pos[ii][:, None, :]
            r2 = np.einsum("abk,abk->ab", d, d)
            m = r2 < rc2
            if not np.any(t):
                m[np.arange(len(ii)), ii] = False
            a, b = np.nonzero(m)
            out_i.append(ii[a])
            out_j.append(b)
            out_d.append(d[a, b])
    if not out_i:
        return (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3)))
    return (np.concatenate(out_i).astype(np.int64),
            np.concatenate(out_j).astype(np.int64),
            np.concatenate(out_d, axis=0))


def counting(r, rs):
    """Eq. 4 counting function and its r-derivative."""
    e = np.exp(-16.0 * (rs / r - 1.0))
    f = 1.0 / (1.0 + e)
    df = -16.0 * rs * e / (r * r * (1.0 + e) ** 2)
    return f, df


def coordination(n_atoms, types, tab, i, j, d, r_cn):
    """Eq. 4 summed over entries with r < R_cn."""
    r2 = np.einsum("ek,ek->e", d, d)
    m = r2 < r_cn * r_cn
    r = np.sqrt(r2[m])
    rs = tab["rcov"][types[i[m]]] + tab["rcov"][types[j[m]]]
    f, _ = counting(r, rs)
    return np.bincount(i[m], weights=f, minlength=n_atoms)


def c6_eq3(zi, zj, ni, nj, tab):
    """Eq. 3 per entry, with its derivatives wrt n_i and n_j.

    Exponent of pair (a,b): x_ab = -4[(n_i - ref_ia)^2 + (n_j - ref_jb)^2];
    C6 = sum_ab C_ab e^{x_ab} / sum_ab e^{x_ab} (after subtracting max x_ab).
    """
    zi = np.asarray(zi)
    zj = np.asarray(zj)
    ni = np.asarray(ni, dtype=np.float64)
    nj = np.asarray(nj, dtype=np.float64)
    ki = tab["n_ref"][zi]
    kj = tab["n_ref"][zj]
    ref_i = tab["cn_ref"][zi]                       # (E,5)
    ref_j = tab["cn_ref"][zj]
    valid = (np.arange(MAX_REF)[None, :, None] < ki[:, None, None]) & \
            (np.arange(MAX_REF)[None, None, :] < kj[:, None, None])
    di = ni[:, None] - ref_i                        # (E,5)
    dj = nj[:, None] - ref_j
    x = -4.0 * (di[:, :, None] ** 2 + dj[:, None, :] ** 2)
    x = np.where(valid, x, -np.inf)
    x = x - x.max(axis=(1, 2), keepdims=True)
    L = np.exp(x)                                   # zero where invalid
    C = tab["c6"][zi, zj]                           # (E,5,5)
    Z = L.sum(axis=(1, 2))
    S = (C * L).sum(axis=(1, 2))
    c6 = S / Z
    dxi = np.where(valid, -8.0 * di[:, :, None], 0.0)
    dxj = np.where(valid, -8.0 * dj[:, None, :], 0.0)
    dc6_dni = ((C * L * dxi).sum(axis=(1, 2)) - c6 * (L * dxi).sum(axis=(1, 2))) / Z
    dc6_dnj = ((C * L * dxj).sum(axis=(1, 2)) - c6 * (L * dxj).sum(axis=(1, 2))) / Z
    return c6, dc6_dni, dc6_dnj


ZERO_ALPHA6 = 14.0
ZERO_ALPHA8 = 16.0


def _zero_term(r2, c, s, sr, r0, n, alpha):
    """One zero-damped term -s C f(r) / r^n, f = 1 / (1 + 6 (r/(sr R0))^-alpha):
    its value, its r-derivative divided by r, and f / r^n."""
    r = np.sqrt(r2)
    q = (r / (sr * r0)) ** (-alpha)
    f = 1.0 / (1.0 + 6.0 * q)
    rn = r2 ** (n // 2)
    e = -s * c * f / rn
    # d/dr [f / r^n] = f' / r^n - n f / r^(n+1), with f' = 6 alpha q f^2 / r
    de_r = -s * c * (6.0 * alpha * q * f * f - n * f) / (rn * r2)
    return e, de_r, f / rn


def pair_terms(r2, zi, zj, c6, tab, prm):
    """Pair energy phi (both halves), d phi/dr divided by r, and
    d phi / d C6, at fixed C6: Eq. 2 (Becke-Johnson damping), or zero
    damping (see Params)."""
    r0sq = tab["r0sq"][zi, zj]
    if prm.damping == "zero":
        r0 = np.sqrt(r0sq)
        e6, d6, g6 = _zero_term(r2, c6, prm.s6, prm.rs6, r0, 6, ZERO_ALPHA6)
        e8, d8, g8 = _zero_term(r2, c6 * r0sq, prm.s8, prm.rs8, r0, 8, ZERO_ALPHA8)
        return e6 + e8, d6 + d8, -(prm.s6 * g6 + prm.s8 * r0sq * g8)
    rd = prm.a1 * np.sqrt(r0sq) + prm.a2
    r6 = r2 ** 3
    r8 = r2 ** 4
    rd6 = rd ** 6
    rd8 = rd ** 8
    t6 = 1.0 / (r6 + rd6)
    t8 = 1.0 / (r8 + rd8)
    c8 = c6 * r0sq
    phi = -(prm.s6 * c6 * t6 + prm.s8 * c8 * t8)
    # d/dr [-C/(r^k + Rd^k)] = C k r^(k-1) / (r^k + Rd^k)^2 ; divide by r
    dphi_r = prm.s6 * c6 * 6.0 * r2 * r2 * t6 * t6 + \
        prm.s8 * c8 * 8.0 * r6 * t8 * t8
    dphi_dc6 = -(prm.s6 * t6 + prm.s8 * r0sq * t8)
    return phi, dphi_r, dphi_dc6


ATM_SR3 = 4.0 / 3.0
ATM_ALPHA = 16.0


def atm_triple(a, b, c, r0ab, r0bc, r0ca, prm):
    """Geometry and damping of the three-body term of one triangle with
    squared sides a = r_AB^2, b = r_BC^2, c = r_CA^2 (arrays):
      g = (1 + 3 cos(A) cos(B) cos(C)) / (r_AB r_BC r_CA)^3 * f3,
    where the cosine product is (a + c - b)(a + b - c)(b + c - a) / (8 abc)
    (law of cosines) and f3 = 1 / (1 + 6 (rbar / (4/3 R0bar))^-16), rbar and
    R0bar the geometric means of the three sides and of the three pair radii.
    Returns g and its derivatives dg/da, dg/db, dg/dc."""
    u = a * b * c
    P = (a + c - b) * (a + b - c) * (b + c - a)
    dP = ((a + b - c) * (b + c - a) + (a + c - b) * (b + c - a) - (a + c - b) * (a + b - c),
          (a + c - b) * (b + c - a) - (a + b - c) * (b + c - a) + (a + c - b) * (a + b - c),
          (a + b - c) * (b + c - a) - (a + c - b) * (b + c - a) + (a + c - b) * (a + b - c))
    du = (b * c, a * c, a * b)
    ang = 1.0 + 3.0 * P / (8.0 * u)
    k0 = (ATM_SR3 ** 3 * r0ab * r0bc * r0ca) ** (ATM_ALPHA / 3.0)   # (sr3 R0bar)^16
    q = k0 * u ** (-ATM_ALPHA / 6.0)                                # (rbar/(sr3 R0bar))^-16
    f3 = 1.0 / (1.0 + 6.0 * q)
    g = ang * u ** -1.5 * f3
    out = []
    for k in range(3):
        dang = 3.0 / 8.0 * (dP[k] * u - P * du[k]) / (u * u)
        du15 = -1.5 * u ** -2.5 * du[k]
        df3 = 6.0 * f3 * f3 * q * (ATM_ALPHA / 6.0) * du[k] / u
        out.append(dang * u ** -1.5 * f3 + ang * du15 * f3 + ang * u ** -1.5 * df3)
    return g, out[0], out[1], out[2]


def atm_terms(n, types, tab, prm, i, j, d, cn, c6_fn=None):
    """The three-body (Axilrod-Teller-Muto) term of D3 (Grimme et al. 2010),
    which the paper sets aside: over every triangle of atom images whose
    three sides are below r_atm,
      E_ABC = s9 sqrt(C6_AB C6_BC C6_CA) (1 + 3 cos A cos B cos C)
              / (r_AB r_BC r_CA)^3 f3,
    with each C6 from Eq. 3 at the atoms' coordination numbers (positive
    for an equilateral triangle: the triple-dipole repulsion).  Atom A
    finds each triangle it belongs to as a pair of its own entries (B, C)
    within r_atm whose third side is also below r_atm; each of the three
    atoms takes a third of E_ABC (site energy and per-atom virial), its own
    force and its own dE/dn.  Returns site energies, dE/dn, forces, the
    virial and the per-atom virials."""
    if c6_fn is None:
        def c6_fn(zi, zj, ni, nj):
            return c6_eq3(zi, zj, ni, nj, tab)
    r2 = np.einsum("ek,ek->e", d, d)
    ra2 = prm.r_atm * prm.r_atm
    m = r2 < ra2
    i, j, d = i[m], j[m], d[m]
    order = np.argsort(i, kind="stable")
    i, j, d = i[order], j[order], d[order]
    starts = np.searchsorted(i, np.arange(n + 1))
    atom_e = np.zeros(n)
    dedn = np.zeros(n)
    forces = np.zeros((n, 3))
    atom_vir = np.zeros((n, 3, 3))
    r0 = np.sqrt(tab["r0sq"])
    for A in range(n):
        s0, s1 = starts[A], starts[A + 1]
        k = s1 - s0
        if k < 2:
            continue
        e1, e2 = np.triu_indices(k, 1)
        dab, dac = d[s0 + e1], d[s0 + e2]
        dbc = dac - dab
        a = np.einsum("ek,ek->e", dab, dab)
        c = np.einsum("ek,ek->e", dac, dac)
        b = np.einsum("ek,ek->e", dbc, dbc)
        keep = b < ra2
        e1, e2, dab, dac, dbc, a, b, c = (x[keep] for x in (e1, e2, dab, dac, dbc, a, b, c))
        if e1.size == 0:
            continue
        B, C = j[s0 + e1], j[s0 + e2]
        zA = np.full(B.size, types[A])
        zB, zC = types[B], types[C]
        nA = np.full(B.size, cn[A])
        cab, dab_dnA, _ = c6_fn(zA, zB, nA, cn[B])
        cac, dac_dnA, _ = c6_fn(zA, zC, nA, cn[C])
        cbc, _, _ = c6_fn(zB, zC, cn[B], cn[C])
        g, ga, gb, gc = atm_triple(a, b, c, r0[zA, zB], r0[zB, zC], r0[zC, zA], prm)
        cc = prm.s9 * np.sqrt(cab * cbc * cac)
        E = cc * g
        atom_e[A] = E.sum() / 3.0
        dedn[A] = (0.5 * E * (dab_dnA / cab + dac_dnA / cac)).sum()
        # a = |d_AB|^2 and c = |d_AC|^2 depend on r_A: dE/dr_A = -2 E_a d_AB - 2 E_c d_AC
        forces[A] = 2.0 * ((cc * ga)[:, None] * dab + (cc * gc)[:, None] * dac).sum(0)
        # W = -dE/d(strain) = -2 sum over the three sides of dE/d(side^2) side (x) side
        w = -2.0 * (np.einsum("e,ea,eb->ab", cc * ga, dab, dab) +
                    np.einsum("e,ea,eb->ab", cc * gb, dbc, dbc) +
                    np.einsum("e,ea,eb->ab", cc * gc, dac, dac))
        atom_vir[A] = w / 3.0
    return atom_e, dedn, forces, atom_vir.sum(0), atom_vir


def d3(pos, types, cell, pbc, table, prm=None, c6_fn=None):
    """Full FP64 evaluation.  Returns dict with energy, forces (N,3),
    virial (3,3), atom_energy (N), cn (N), dE/dn (N).

    c6_fn(zi, zj, ni, nj) -> (C6, dC6/dn_i, dC6/dn_j), arrays over the
    dispersion entries, replaces Eq. 3 when given (in eV A^6); the rest of
    the evaluation is unchanged.  It lets a test feed another C6 model, such
    as the learned surrogate, through the same Eqs. 1-7."""
    prm = prm or Params()
    tab = convert_table(table)
    pos = np.asarray(pos, dtype=np.float64)
    types = np.asarray(types, dtype=np.int64)
    n = pos.shape[0]
    i, j, d = entries(pos, cell, pbc, max(prm.r_pot, prm.r_cn, prm.r_atm))
    return _evaluate(n, types, tab, prm, i, j, d, c6_fn=c6_fn)


def _evaluate(n, types, tab, prm, i, j, d, cn=None, c6_fn=None):
    r2 = np.einsum("ek,ek->e", d, d)
    if cn is None:
        cn = coordination(n, types, tab, i, j, d, prm.r_cn)
    # dispersion entries
    mp = r2 < prm.r_pot * prm.r_pot
    ip, jp, dp, r2p = i[mp], j[mp], d[mp], r2[mp]
    zi, zj = types[ip], types[jp]
    if c6_fn is None:
        c6, dci, _ = c6_eq3(zi, zj, cn[ip], cn[jp], tab)
    else:
        c6, dci, _ = c6_fn(zi, zj, cn[ip], cn[jp])
    phi, dphi_r, dphi_dc6 = pair_terms(r2p, zi, zj, c6, tab, prm)
    atom_e = 0.5 * np.bincount(ip, weights=phi, minlength=n)
    dedn = np.bincount(ip, weights=dphi_dc6 * dci, minlength=n)
    forces = np.zeros((n, 3))
    for k in range(3):
        forces[:, k] += np.bincount(ip, weights=dphi_r * dp[:, k], minlength=n)
    vir = -0.5 * np.einsum("e,ea,eb->ab", dphi_r, dp, dp)
    atom_vir3 = 0.0
    if prm.s9 != 0.0:
        ue3, g3, f3, w3, atom_vir3 = atm_terms(n, types, tab, prm, i, j, d, cn, c6_fn)
        atom_e = atom_e + ue3
        dedn = dedn + g3
        forces += f3
        vir = vir + w3
    # chain entries through the coordination numbers
    mc = r2 < prm.r_cn * prm.r_cn
    ic, jc, dc, r2c = i[mc], j[mc], d[mc], r2[mc]
    rc = np.sqrt(r2c)
    rs = tab["rcov"][types[ic]] + tab["rcov"][types[jc]]
    _, df = counting(rc, rs)
    coef = (dedn[ic] + dedn[jc]) * df / rc
    for k in range(3):
        forces[:, k] += np.bincount(ic, weights=coef * dc[:, k], minlength=n)
    vir += -0.5 * np.einsum("e,ea,eb->ab", coef, dc, dc)
    # Eq. 7 per atom: every entry's term goes to the atom that owns it
    atom_vir = np.zeros((n, 3, 3))
    for a in range(3):
        for b in range(3):
            atom_vir[:, a, b] = -0.5 * (
                np.bincount(ip, weights=dphi_r * dp[:, a] * dp[:, b], minlength=n) +
                np.bincount(ic, weights=coef * dc[:, a] * dc[:, b], minlength=n))
    atom_vir = atom_vir + atom_vir3
    return {"energy": float(atom_e.sum()), "forces": forces, "virial": vir,
            "atom_energy": atom_e, "atom_virial": atom_vir, "cn": cn, "dedn": dedn}


def heat_current(atom_virial, vel):
    """Eq. 8: J_i = W_i v_i for per-atom virials (N,3,3) and velocities
    (N,3)."""
    return np.einsum("iab,ib->ia", np.asarray(atom_virial), np.asarray(vel, dtype=np.float64))


def energy_only(pos, types, cell, pbc, table, prm=None):
    """Total energy alone (used by finite-difference pins)."""
    prm = prm or Params()
    tab = convert_table(table)
    pos = np.asarray(pos, dtype=np.float64)
    types = np.asarray(types, dtype=np.int64)
    n = pos.shape[0]
    i, j, d = entries(pos, cell, pbc, max(prm.r_pot, prm.r_cn, prm.r_atm))
    r2 = np.einsum("ek,ek->e", d, d)
    cn = coordination(n, types, tab, i, j, d, prm.r_cn)
    mp = r2 < prm.r_pot * prm.r_pot
    zi, zj = types[i[mp]], types[j[mp]]
    c6, _, _ = c6_eq3(zi, zj, cn[i[mp]], cn[j[mp]], tab)
    phi, _, _ = pair_terms(r2[mp], zi, zj, c6, tab, prm)
    e = 0.5 * phi.sum()
    if prm.s9 != 0.0:
        e += atm_terms(n, types, tab, prm, i, j, d, cn)[0].sum()
    return e


def sampled(pos, types, cell, pbc, table, idx, prm=None, c6_fn=None):
    """Forces, site energies, per-atom virials, coordination numbers and
    dE/dn of the atoms ``idx`` of a large cell, each computed from its own
    neighbourhood.

    The force on k depends on n_j for j within R_pot of k and on dE/dn_j for
    j within R_cn of k; dE/dn_j depends on n_l for l within R_pot of j, and
    n_l on atoms within R_cn of l.  So every quantity needed for atom k is
    fixed by the images within R_pot + 2 R_cn of k, and the full definition
    restricted to that ball gives the exact result.  c6_fn: as in d3()."""
    prm = prm or Params()
    if prm.s9 != 0.0:
        raise NotImplementedError("the sampled mode covers the two-body terms only")
    tab = convert_table(table)
    if c6_fn is None:
        def c6_fn(zi, zj, ni, nj):
            return c6_eq3(zi, zj, ni, nj, tab)
    pos = np.asarray(pos, dtype=np.float64)
    types = np.asarray(types, dtype=np.int64)
    rbig = prm.r_pot + 2.0 * prm.r_cn + 1e-6
    nvec, tvec = translations(cell, pbc, rbig, pos)
    res = {"forces": [], "atom_energy": [], "atom_virial": [], "cn": [], "dedn": []}
    for k in np.asarray(idx):
        loc_pos, loc_atom = [], []
        for T in tvec:
            d = pos + T - pos[k]
            r2 = np.einsum("ak,ak->a", d, d)
            m = np.nonzero(r2 < rbig * rbig)[0]
            loc_pos.append(d[m])
            loc_atom.append(m)
        lp = np.concatenate(loc_pos)
        la = np.concatenate(loc_atom)
        lt = types[la]
        dist = np.sqrt(np.einsum("ak,ak->a", lp, lp))
        me = int(np.nonzero((la == k) & (dist == 0.0))[0][0])
        nl = lp.shape[0]
        # n for local images within R_pot + R_cn of k (all their CN
        # neighbours lie inside the ball)
        need_n = np.nonzero(dist < prm.r_pot + prm.r_cn + 1e-9)[0]
        cn = np.full(nl, np.nan)
        for a in need_n:
            dd = lp - lp[a]
            rr = np.einsum("ak,ak->a", dd, dd)
            m = rr < prm.r_cn * prm.r_cn
            m[a] = False
            f, _ = counting(np.sqrt(rr[m]), tab["rcov"][lt[a]] + tab["rcov"][lt[m]])
            cn[a] = f.sum()
        # dE/dn for local images within R_cn of k
        need_g = np.nonzero(dist < prm.r_cn + 1e-9)[0]
        g = np.full(nl, np.nan)
        for a in need_g:
            dd = lp - lp[a]
            rr = np.einsum("ak,ak->a", dd, dd)
            m = rr < prm.r_pot * prm.r_pot
            m[a] = False
            zi = np.full(int(m.sum()), lt[a])
            c6, dci, _ = c6_fn(zi, lt[m], np.full(zi.size, cn[a]), cn[m])
            _, _, dphi_dc6 = pair_terms(rr[m], zi, lt[m], c6, tab, prm)
            g[a] = (dphi_dc6 * dci).sum()
        # force and site energy of k
        dd = lp - lp[me]
        rr = np.einsum("ak,ak->a", dd, dd)
        m = rr < prm.r_pot * prm.r_pot
        m[me] = False
        zi = np.full(int(m.sum()), lt[me])
        c6, _, _ = c6_fn(zi, lt[m], np.full(zi.size, cn[me]), cn[m])
        phi, dphi_r, _ = pair_terms(rr[m], zi, lt[m], c6, tab, prm)
        f = (dphi_r[:, None] * dd[m]).sum(0)
        w = -0.5 * np.einsum("e,ea,eb->ab", dphi_r, dd[m], dd[m])
        mc = rr < prm.r_cn * prm.r_cn
        mc[me] = False
        rc = np.sqrt(rr[mc])
        _, df = counting(rc, tab["rcov"][lt[me]] + tab["rcov"][lt[mc]])
        coef = (g[me] + g[mc]) * df / rc
        f += (coef[:, None] * dd[mc]).sum(0)
        w += -0.5 * np.einsum("e,ea,eb->ab", coef, dd[mc], dd[mc])
        res["forces"].append(f)
        res["atom_virial"].append(w)
        res["atom_energy"].append(0.5 * phi.sum())
        res["cn"].append(cn[me])
        res["dedn"].append(g[me])
    return {k: np.asarray(v) for k, v in res.items()}
