"""Seeded synthetic D3 reference table.

The real D3 parameter set (per-element reference coordination numbers,
the C6 reference grid, covalent radii and the r2/r4 expectation ratios for
94 elements) is only mentioned by the paper (Sec. II A, the sentence after
Eq. 4 and the C6 definition, Eq. 3) and is not available here.  This module
draws a stand-in with the same shapes:

* elements H, C, N, O, Zn (indices 0..4);
* K_e reference points per element, K_e uniform on {1..5};
* reference coordination numbers uniform on [0, 4);
* C6 reference values log-uniform on [2, 500] in Hartree*bohr^6, symmetric
  under swapping the two atoms: C6ref[f][e][b][a] == C6ref[e][f][a][b];
* effective covalent radii in Angstrom (fixed, chosen once; any scaling of
  the bare radii is already folded in);
* r2r4 (square root of the <r^4>/<r^2> ratio that sets C8/C6) in bohr,
  uniform on [2, 5).

Values are in the units D3 tables are published in; converting them to
eV and Angstrom is left to each consumer.
"""

import numpy as np

ELEMENTS = ("H", "C", "N", "O", "Zn")
MAX_REF = 5
# effective covalent radii (Angstrom), fixed by hand for the synthetic table
RCOV_EFF_ANG = np.array([0.43, 1.00, 0.95, 0.84, 1.57], dtype=np.float64)
MASSES_AMU = np.array([1.008, 12.011, 14.007, 15.999, 65.38], dtype=np.float64)


def make_table(seed=2310, n_elem=5, k_min=1, k_max=5, cn_hi=4.0,
               c6_lo=2.0, c6_hi=500.0, rcov=None, force_k=None):
    """Draw a synthetic D3 table.

    Returns a dict with numpy arrays:
      n_ref  int32[n_elem]            number of reference points K_e
      cn_ref f64[n_elem, MAX_REF]     reference CNs (unused slots = 0)
      c6_ref f64[n_elem, n_elem, MAX_REF, MAX_REF]  Hartree*bohr^6
      rcov   f64[n_elem]              Angstrom
      r2r4   f64[n_elem]              bohr
    ``force_k`` (int or sequence) overrides K_e, e.g. force_k=1 gives the
    single-reference special case.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if force_k is None:
        n_ref = rng.integers(k_min, k_max + 1, size=n_elem).astype(np.int32)
    else:
        n_ref = np.broadcast_to(np.asarray(force_k, dtype=np.int32),
                                (n_elem,)).copy()
        rng.integers(k_min, k_max + 1, size=n_elem)  # keep the stream aligned
    cn_ref = np.zeros((n_elem, MAX_REF), dtype=np.float64)
    for e in range(n_elem):
        cn_ref[e, :n_ref[e]] = np.sort(rng.uniform(0.0, cn_hi, size=n_ref[e]))
    c6 = np.zeros((n_elem, n_elem, MAX_REF, MAX_REF), dtype=np.float64)
    lo, hi = np.log(c6_lo), np.log(c6_hi)
    for e in range(n_elem):
        for f in range(e, n_elem):
            for a in range(n_ref[e]):
                for b in range(n_ref[f]):
                    if e == f and b < a:
                        continue
                    v = float(np.exp(rng.uniform(lo, hi)))
                    c6[e, f, a, b] = v
                    c6[f, e, b, a] = v
    if rcov is None:
        rcov = RCOV_EFF_ANG[:n_elem] if n_elem <= len(RCOV_EFF_ANG) else \
            rng.uniform(0.4, 1.6, size=n_elem)
    r2r4 = rng.uniform(2.0, 5.0, size=n_elem)
    return {
        "n_ref": n_ref,
        "cn_ref": cn_ref,
        "c6_ref": c6,
        "rcov": np.asarray(rcov, dtype=np.float64).copy(),
        "r2r4": r2r4.astype(np.float64),
        "seed": seed,
    }
