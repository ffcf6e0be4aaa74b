"""Seeded synthetic periodic cells.

The paper's structures (the bilayer-graphene data set and the MOF-5, ZIF-8
and HKUST-1 cells of Sec. II B-D) are not available, so these generators
stand in for them with the same shapes, densities and compositions:

* ``bilayer_graphene``: AB (Bernal) stacked bilayer on a hexagonal
  supercell, a = 2.46 A, interlayer 3.4 A, vacuum along z (Sec. II C uses
  AB bilayers at 3.4 A; Table I times a 40 000-atom bilayer).
* ``mof_like``: cubic periodic cell of H, C, N, O, Zn atoms at a fixed
  number density, with positions drawn by random sequential addition under
  a hard minimum separation.
* ``cluster`` and ``simple_lattice``: small test geometries.

Every array is a plain numpy array; cells are 3x3 with the lattice vectors
as rows (r = s @ cell for fractional s).  Positions are Angstrom.
"""

import os
import tempfile

import numpy as np
from scipy.spatial import cKDTree

from .table import MASSES_AMU

_CACHE_DIR = os.environ.get("D3_SYNTH_CACHE",
                            os.path.join(tempfile.gettempdir(), "d3synth_cache"))


def _rng(*key):
    return np.random.Generator(np.random.PCG64(list(key)))


def _cached(name, builder):
    path = os.path.join(_CACHE_DIR, name + ".npz")
    if os.path.exists(path):
        try:
            with np.load(path, allow_pickle=False) as z:
                return {k: z[k] for k in z.files}
        except Exception:
            pass
    out = builder()
    try:
        os.makedirs(_CACHE_DIR, exist_ok=True)
        tmp = path + ".%d.tmp.npz" % os.getpid()
        np.savez(tmp, **out)
        os.replace(tmp, path)
    except OSError:
        pass
    return out


def bilayer_graphene(nx=6, ny=6, a=2.46, d=3.4, vacuum=20.0, jitter=0.01,
                     seed=1, z0=None, shift=(1.0 / 3.0, 1.0 / 3.0)):
    """AB-stacked bilayer graphene on an nx x ny hexagonal supercell.

    Lattice: A1 = nx*a*(1,0,0), A2 = ny*a*(1/2, sqrt(3)/2, 0),
    A3 = (0, 0, d + vacuum).  Layer 1 holds the basis (0,0) and (1/3,1/3)
    of the primitive cell; layer 2 is layer 1 displaced by ``shift`` (in
    primitive fractional units; (1/3,1/3) gives AB stacking, (0,0) AA) and
    by d along z.  Every coordinate then gets N(0, jitter^2) noise.
    Returns dict(pos, types, cell, pbc); all atoms are carbon (element 1).
    pbc is (1, 1, 0): periodic in-plane, open along z.
    """
    a1 = np.array([a, 0.0, 0.0])
    a2 = np.array([0.5 * a, 0.5 * np.sqrt(3.0) * a, 0.0])
    c = d + vacuum
    if z0 is None:
        z0 = 0.5 * (c - d)
    basis1 = [(0.0, 0.0), (1.0 / 3.0, 1.0 / 3.0)]
    basis2 = [(b0 + shift[0], b1 + shift[1]) for (b0, b1) in basis1]
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ix = ix.ravel().astype(np.float64)
    iy = iy.ravel().astype(np.float64)
    pos = []
    for layer, basis in ((0, basis1), (1, basis2)):
        for (b0, b1) in basis:
            f0 = (ix + b0) % nx
            f1 = (iy + b1) % ny
            p = f0[:, None] * a1[None, :] + f1[:, None] * a2[None, :]
            p[:, 2] = z0 + layer * d
            pos.append(p)
    # order: cell index major, then (layer, basis)
    pos = np.stack(pos, axis=1).reshape(-1, 3)
    if jitter > 0.0:
        pos = pos + _rng(seed, 0).normal(0.0, jitter, size=pos.shape)
    cell = np.array([nx * a1, ny * a2, [0.0, 0.0, c]], dtype=np.float64)
    types = np.full(pos.shape[0], 1, dtype=np.int32)
    return {"pos": pos.astype(np.float64), "types": types, "cell": cell,
            "pbc": np.array([1, 1, 0], dtype=np.int32)}


def mof_counts(n, ratios=(4, 6, 1, 2, 1)):
    """Element counts for n atoms by the largest-remainder rule."""
    r = np.asarray(ratios, dtype=np.float64)
    exact = n * r / r.sum()
    base = np.floor(exact).astype(np.int64)
    rem = exact - base
    short = n - int(base.sum())
    order = np.argsort(-rem, kind="stable")
    base[order[:short]] += 1
    return base


def _rsa_positions(n, box, dmin, rng):
    """Uniform positions in a periodic cube with pairwise image distance
    >= dmin, accepted in index order (a parallel form of random sequential
    addition: a pending point is accepted when it clashes neither with an
    accepted point nor with a pending point of lower index; rejected points
    are redrawn)."""
    pos = rng.uniform(0.0, box, size=(n, 3))
    accepted = np.zeros(n, dtype=bool)
    for _ in range(1000):
        pending = ~accepted
        if not pending.any():
            return pos
        tree = cKDTree(np.mod(pos, box), boxsize=box)
        pairs = tree.query_pairs(r=dmin, output_type="ndarray")
        bad = np.zeros(n, dtype=bool)
        if pairs.size:
            p, q = pairs[:, 0], pairs[:, 1]
            lo, hi = np.minimum(p, q), np.maximum(p, q)
            # hi clashes with lo; hi is rejected if it is pending and lo is
            # accepted or pending with a lower index (always true: lo < hi)
            m = pending[hi]
            bad[hi[m]] = True
            # lo pending clashing with an accepted hi must also go
            m2 = pending[lo] & accepted[hi]
            bad[lo[m2]] = True
        newly = pending & ~bad
        accepted |= newly
        redo = np.nonzero(pending & bad)[0]
        if redo.size:
            pos[redo] = rng.uniform(0.0, box, size=(redo.size, 3))
    raise RuntimeError("random sequential addition did not converge")


def mof_like(n=24000, density=0.04, ratios=(4, 6, 1, 2, 1), dmin=1.0,
             seed=None, cache=True):
    """MOF-like periodic cube: n atoms of H, C, N, O, Zn in ``ratios`` at
    ``density`` atoms/A^3, minimum image separation ``dmin``.

    Element labels are a seeded permutation of the count vector; positions
    come from ``_rsa_positions``.  Seed defaults to n.
    """
    if seed is None:
        seed = n

    def build():
        box = (n / density) ** (1.0 / 3.0)
        counts = mof_counts(n, ratios)
        labels = np.repeat(np.arange(len(ratios), dtype=np.int32), counts)
        labels = _rng(seed, 1).permutation(labels).astype(np.int32)
        pos = _rsa_positions(n, box, dmin, _rng(seed, 0))
        cell = np.eye(3) * box
        return {"pos": pos.astype(np.float64), "types": labels,
                "cell": cell, "pbc": np.array([1, 1, 1], dtype=np.int32)}

    if not cache or n < 5000:
        return build()
    key = "mof_n%d_rho%g_d%g_s%d_r%s" % (n, density, dmin, seed,
                                         "-".join(str(int(x)) for x in ratios))
    return _cached(key, build)


def cluster(n, radius, n_elem=5, dmin=1.2, seed=0, center=(0.0, 0.0, 0.0)):
    """Random finite cluster: n points uniform in a ball of ``radius`` with
    pairwise distance >= dmin (rejection), random element labels."""
    rng = _rng(seed, 7)
    pts = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > 200000:
            raise RuntimeError("cluster: could not place points")
        p = rng.uniform(-radius, radius, size=3)
        if p @ p > radius * radius:
            continue
        if pts and np.min(np.linalg.norm(np.asarray(pts) - p, axis=1)) < dmin:
            continue
        pts.append(p)
    pos = np.asarray(pts) + np.asarray(center)[None, :]
    types = rng.integers(0, n_elem, size=n).astype(np.int32)
    return {"pos": pos, "types": types}


def simple_lattice(kind, a, reps=1, element=1):
    """Conventional cubic cell of an sc/bcc/fcc lattice, ``reps`` times
    along each axis; fully periodic."""
    basis = {
        "sc": [(0, 0, 0)],
        "bcc": [(0, 0, 0), (0.5, 0.5, 0.5)],
        "fcc": [(0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5), (0, 0.5, 0.5)],
    }[kind]
    pts = []
    for i in range(reps):
        for j in range(reps):
            for k in range(reps):
                for b in basis:
                    pts.append(((i + b[0]) * a, (j + b[1]) * a, (k + b[2]) * a))
    pos = np.asarray(pts, dtype=np.float64)
    return {"pos": pos, "types": np.full(len(pts), element, dtype=np.int32),
            "cell": np.eye(3) * a * reps,
            "pbc": np.array([1, 1, 1], dtype=np.int32)}


def maxwell_velocities(types, temperature=300.0, seed=300, masses=None):
    """Maxwell-Boltzmann velocities in Angstrom/fs for atoms of ``types``
    at ``temperature`` K: the centre-of-mass velocity is removed and the
    result is rescaled to exactly ``temperature`` over 3N-3 degrees of
    freedom.  Returns (vel (N,3), mass (N,) amu)."""
    if masses is None:
        masses = MASSES_AMU
    m = np.asarray(masses, dtype=np.float64)[np.asarray(types)]
    kb_ev = 8.617333262e-5            # eV/K
    ev_per_amu_a2_fs2 = 103.642691    # 1 amu*A^2/fs^2 in eV
    rng = _rng(seed, 3)
    sig = np.sqrt(kb_ev * temperature / (m * ev_per_amu_a2_fs2))
    v = rng.normal(size=(m.size, 3)) * sig[:, None]
    v -= (m[:, None] * v).sum(0) / m.sum()
    ke = 0.5 * (m[:, None] * v * v).sum() * ev_per_amu_a2_fs2
    dof = 3 * m.size - 3
    t_now = 2.0 * ke / (dof * kb_ev)
    v *= np.sqrt(temperature / t_now)
    return v, m
