"""ctypes wrapper of the plain C FP64 oracle (oracle/d3_ref.c).

TEST INFRASTRUCTURE ONLY: see the package docstring.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "d3_ref.c")
_LIB = os.path.join(_HERE, "libd3ref.so")
_lib = None


def build(force=False):
    """Compile the C oracle with gcc -O2 -fopenmp."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".%d.tmp" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        lib.d3ref_evaluate_mode.restype = ctypes.c_long
        lib.d3ref_evaluate_mode.argtypes = [I, P, P, P, P, I, P, P, P, P, P,
                                            D, D, D, D, D, D, I, D, D, D, D, I, I, I,
                                            P, P, P, P, P, P, P]
        lib.d3ref_threads.restype = I
        lib.d3ref_threads_for.restype = I
        lib.d3ref_threads_for.argtypes = [I]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def threads(n_threads=0):
    """OpenMP threads an evaluation with n_threads uses (0: all)."""
    return _load().d3ref_threads_for(int(n_threads))


def d3(pos, types, cell, pbc, table, s6=1.0, a1=0.4289, s8=0.7875, a2=4.4407,
       r_pot=12.0, r_cn=6.0, n_threads=0, cells=False, n_eval=None, damping="bj",
       rs6=1.217, rs8=1.0, s9=0.0, r_atm=None):
    """Full FP64 evaluation; returns the same dict layout as
    d3_oracle.d3 plus the number of dispersion entries.  cells=False finds
    the entries by brute force over every atom and lattice translation;
    cells=True from cell lists (the same entries, in O(n) time and memory:
    the mode for large cells).  n_threads=0 uses every OpenMP thread.
    n_eval (cell-list mode, timing only): run each pass for the first n_eval
    atoms alone, the work of n_eval atoms of the cell; the results are then
    not the cell's.  damping="zero" and s9 (three-body term within r_atm,
    default r_cn) select the variants, as in d3_oracle.Params."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    types = np.ascontiguousarray(types, dtype=np.int32)
    cellp = None if cell is None else np.ascontiguousarray(cell, dtype=np.float64)
    pbcp = None if cell is None else np.ascontiguousarray(pbc, dtype=np.int32)
    n_ref = np.ascontiguousarray(table["n_ref"], dtype=np.int32)
    ne = n_ref.shape[0]
    cn_ref = np.ascontiguousarray(table["cn_ref"], dtype=np.float64)
    c6 = np.ascontiguousarray(table["c6_ref"], dtype=np.float64)
    rcov = np.ascontiguousarray(table["rcov"], dtype=np.float64)
    r2r4 = np.ascontiguousarray(table["r2r4"], dtype=np.float64)
    energy = np.zeros(1)
    forces = np.zeros((n, 3))
    virial = np.zeros((3, 3))
    ae = np.zeros(n)
    cn = np.zeros(n)
    g = np.zeros(n)
    av = np.zeros((n, 3, 3))
    if cells and cellp is None:
        raise ValueError("the cell-list mode needs a cell")
    total = lib.d3ref_evaluate_mode(
        n, _ptr(pos), _ptr(types), _ptr(cellp), _ptr(pbcp), ne, _ptr(n_ref),
        _ptr(cn_ref), _ptr(c6), _ptr(rcov), _ptr(r2r4), s6, a1, s8, a2,
        r_pot, r_cn, 1 if damping == "zero" else 0, rs6, rs8, s9,
        r_cn if r_atm is None else r_atm, int(n_threads), 1 if cells else 0,
        n if n_eval is None else int(n_eval), _ptr(energy), _ptr(forces),
        _ptr(virial), _ptr(ae), _ptr(cn), _ptr(g), _ptr(av))
    if total < 0:
        raise MemoryError("d3ref_evaluate failed")
    return {"energy": float(energy[0]), "forces": forces, "virial": virial,
            "atom_energy": ae, "atom_virial": av, "cn": cn, "dedn": g,
            "n_entries": int(total)}
