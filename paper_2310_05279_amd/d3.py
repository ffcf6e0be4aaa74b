"""ctypes binding of the C ABI in include/d3.h.

Argument marshalling only: every step of the computation runs in the HIP
library libd3.so.  Functions keep the C names and raise D3Error on a
non-zero status.  Device buffers are torch tensors on the current HIP
device; streams are torch streams (their ``cuda_stream`` handle).

If libd3.so is missing the import fails loudly: there is no fallback.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libd3.so")

D3_OK = 0
D3_ERR_INVALID_ARG = -1
D3_ERR_HIP = -2
D3_ERR_CAPACITY = -3
D3_ERR_STALE = -4
D3_ERR_CELL = -5
D3_ERR_STATE = -6
D3_ERR_NOT_TRAINED = -7
D3_ERR_SPECIES = -8

D3_MODE_PLAIN_F64 = 0
D3_MODE_PREC_F32 = 1
D3_MODE_SURROGATE = 2
D3_MODE_LITERAL = 3
MODES = {"plain": 0, "prec": 1, "surrogate": 2, "literal": 3}

D3_ACCUMULATE = 1
D3_AUTO_REBUILD = 2
D3_REBUILD = 4
D3_MAX_REF = 5
D3_MAX_ELEM = 16
D3_MLP_PARAMS = 1251

_c_d = ctypes.c_double
_c_i32 = ctypes.c_int32
_c_i64 = ctypes.c_int64
_c_u32 = ctypes.c_uint32
_c_u64 = ctypes.c_uint64
_vp = ctypes.c_void_p


D3_DAMP_BJ = 0
D3_DAMP_ZERO = 1
DAMPINGS = {"bj": 0, "zero": 1}


class d3_params(ctypes.Structure):
    _fields_ = [("s6", _c_d), ("a1", _c_d), ("s8", _c_d), ("a2", _c_d),
                ("r_pot", _c_d), ("r_cn", _c_d), ("skin", _c_d),
                ("mode", _c_i32), ("damping", _c_i32), ("rs6", _c_d), ("rs8", _c_d),
                ("s9", _c_d), ("r_atm", _c_d)]


class d3_table(ctypes.Structure):
    _fields_ = [("n_elem", _c_i32), ("n_ref", _vp), ("cn_ref", _vp),
                ("c6_ref", _vp), ("rcov", _vp), ("r2r4", _vp)]


class d3_train_cfg(ctypes.Structure):
    _fields_ = [("n_samples", _c_i64), ("epochs", _c_i32), ("batch", _c_i32),
                ("lr", _c_d), ("lr_final", _c_d), ("seed", _c_u64),
                ("cn_hi", _c_d)]


class d3_outputs(ctypes.Structure):
    _fields_ = [("energy", _vp), ("forces", _vp), ("virial", _vp),
                ("atom_energy", _vp), ("atom_virial", _vp), ("velocities", _vp),
                ("heat_current", _vp)]


class D3Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("d3 error %d: %s" % (code, msg))
        self.code = code


_SIGS = {
    "d3_create": (_c_i32, [ctypes.POINTER(d3_params), ctypes.POINTER(d3_table),
                           ctypes.POINTER(_vp)]),
    "d3_destroy": (None, [_vp]),
    "d3_last_error": (ctypes.c_char_p, []),
    "d3_set_mode": (_c_i32, [_vp, _c_i32]),
    "d3_build_neighbors": (_c_i32, [_vp, _c_i64, _vp, _vp, _vp, _vp, _vp]),
    "d3_coordination": (_c_i32, [_vp, _vp, _vp, _vp]),
    "d3_build_positions": (_c_i32, [_vp, _vp, _vp]),
    "d3_energy_forces_virial": (_c_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _c_u32, _vp]),
    "d3_evaluate": (_c_i32, [_vp, _vp, ctypes.POINTER(d3_outputs), _c_u32, _vp]),
    "d3_status": (_c_i32, [_vp]),
    "d3_bin_plan": (_c_i32, [_vp, _vp, _c_d, _c_d, _c_i64, _vp, _vp, _vp, _vp, _vp, _c_i32]),
    "d3_list_stats": (_c_i32, [_vp, _vp]),
    "d3_set_timing": (_c_i32, [_vp, _c_i32]),
    "d3_get_timing": (_c_i32, [_vp, _vp, _vp]),
    "d3_c6_surrogate_init": (_c_i32, [_vp, _c_u64]),
    "d3_c6_surrogate_train": (_c_i32, [_vp, ctypes.POINTER(d3_train_cfg), _vp, _vp]),
    "d3_c6_surrogate_eval": (_c_i32, [_vp, _c_i64, _vp, _vp, _vp, _vp, _vp, _c_i32, _vp]),
    "d3_c6_exact_eval": (_c_i32, [_vp, _c_i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "d3_c6_surrogate_bytes": (_c_i64, [_vp]),
    "d3_c6_surrogate_get_weights": (_c_i32, [_vp, _vp, _c_i64]),
    "d3_c6_surrogate_set_weights": (_c_i32, [_vp, _vp, _c_i64]),
    "d3_c6_surrogate_grad": (_c_i32, [_vp, _c_i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "d3_c6_surrogate_adam_step": (_c_i32, [_vp, _c_i64, _vp, _vp, _vp, _c_i64, _c_i64, _c_d,
                                           _c_d, _vp]),
    "d3_md_nve": (_c_i32, [_vp, _c_i64, _c_d, _vp, _vp, _vp, _c_i32, _vp, _vp, _vp]),
    "d3_energy_forces_virial_noalloc": (_c_i32, [ctypes.POINTER(d3_params),
                                                 ctypes.POINTER(d3_table), _c_i64, _vp, _vp,
                                                 _vp, _vp, _vp, _vp, _vp, _vp, _c_u32, _vp]),
}

EXPORTS = tuple(_SIGS)
_lib = None


def lib():
    """Load libd3.so (once).  Raises OSError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError("libd3.so not built at %s (run paper_2310_05279_amd/build.py)"
                          % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != D3_OK:
        msg = lib().d3_last_error()
        raise D3Error(code, msg.decode() if msg else "")
    return code


def _ptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------ raw calls --

def make_params(s6=1.0, a1=0.4289, s8=0.7875, a2=4.4407, r_pot=12.0, r_cn=6.0,
                skin=0.0, mode=D3_MODE_PLAIN_F64, damping=D3_DAMP_BJ, rs6=1.217, rs8=1.0,
                s9=0.0, r_atm=None):
    return d3_params(s6, a1, s8, a2, r_pot, r_cn, skin, int(mode),
                     int(DAMPINGS.get(damping, damping)), rs6, rs8, s9,
                     r_cn if r_atm is None else r_atm)


class _Table:
    """Keeps the numpy arrays alive while a d3_table points into them."""

    def __init__(self, table):
        self.n_ref = np.ascontiguousarray(table["n_ref"], dtype=np.int32)
        self.cn_ref = np.ascontiguousarray(table["cn_ref"], dtype=np.float64)
        self.c6_ref = np.ascontiguousarray(table["c6_ref"], dtype=np.float64)
        self.rcov = np.ascontiguousarray(table["rcov"], dtype=np.float64)
        self.r2r4 = np.ascontiguousarray(table["r2r4"], dtype=np.float64)
        self.c = d3_table(self.n_ref.shape[0], self.n_ref.ctypes.data,
                          self.cn_ref.ctypes.data, self.c6_ref.ctypes.data,
                          self.rcov.ctypes.data, self.r2r4.ctypes.data)


def d3_create(params, table):
    t = _Table(table)
    out = _vp()
    _check(lib().d3_create(ctypes.byref(params), ctypes.byref(t.c), ctypes.byref(out)))
    return out


def d3_destroy(ctx):
    lib().d3_destroy(ctx)


def d3_set_mode(ctx, mode):
    _check(lib().d3_set_mode(ctx, int(mode)))


def d3_build_neighbors(ctx, pos, types, cell, pbc, stream=None):
    cell = np.ascontiguousarray(cell, dtype=np.float64).reshape(9)
    pbc = np.ascontiguousarray(pbc, dtype=np.int32).reshape(3)
    n = int(pos.shape[0]) if pos is not None else 0
    _check(lib().d3_build_neighbors(ctx, n, _ptr(pos), _ptr(types),
                                    cell.ctypes.data, pbc.ctypes.data,
                                    _stream(stream)))


def d3_build_positions(ctx, pos_out, stream=None):
    _check(lib().d3_build_positions(ctx, _ptr(pos_out), _stream(stream)))


def d3_coordination(ctx, pos, cn_out=None, stream=None):
    _check(lib().d3_coordination(ctx, _ptr(pos), _ptr(cn_out), _stream(stream)))


def d3_energy_forces_virial(ctx, pos, energy, forces=None, virial=None,
                            atom_energy=None, flags=0, stream=None):
    _check(lib().d3_energy_forces_virial(ctx, _ptr(pos), _ptr(energy), _ptr(forces),
                                         _ptr(virial), _ptr(atom_energy), int(flags),
                                         _stream(stream)))


def d3_evaluate(ctx, pos, energy, forces=None, virial=None, atom_energy=None,
                atom_virial=None, velocities=None, heat_current=None, flags=0, stream=None):
    def p(t):
        return t.data_ptr() if t is not None else None
    out = d3_outputs(p(energy), p(forces), p(virial), p(atom_energy), p(atom_virial),
                     p(velocities), p(heat_current))
    _check(lib().d3_evaluate(ctx, _ptr(pos), ctypes.byref(out), int(flags), _stream(stream)))


D3_NOALLOC_MAX_ATOMS = 4096


def d3_energy_forces_virial_noalloc(params, table, pos, types, cell, pbc, energy, forces=None,
                                    virial=None, atom_energy=None, flags=0, stream=None):
    """One evaluation with no context and no allocation (the static-scratch
    entry point); device tensors in, synchronises before returning."""
    t = _Table(table)
    cell = np.ascontiguousarray(cell, dtype=np.float64).reshape(9)
    pbc = np.ascontiguousarray(pbc, dtype=np.int32).reshape(3)
    n = int(pos.shape[0]) if pos is not None else 0
    _check(lib().d3_energy_forces_virial_noalloc(
        ctypes.byref(params), ctypes.byref(t.c), n, _ptr(pos), _ptr(types), cell.ctypes.data,
        pbc.ctypes.data, _ptr(energy), _ptr(forces), _ptr(virial), _ptr(atom_energy),
        int(flags), _stream(stream)))


def d3_bin_plan(cell, pbc, rlist, rcn, n, max_rows=8192):
    """Host-side bin layout of a build: bins, stencil reach and row table."""
    cell = np.ascontiguousarray(cell, dtype=np.float64).reshape(9)
    pbc = np.ascontiguousarray(pbc, dtype=np.int32).reshape(3)
    nb = np.zeros(3, np.int32)
    reach = np.zeros(3, np.int32)
    nrows = ctypes.c_int32()
    ncn = ctypes.c_int32()
    rows = np.zeros((max_rows, 4), np.int32)
    _check(lib().d3_bin_plan(cell.ctypes.data, pbc.ctypes.data, float(rlist), float(rcn),
                             int(n), nb.ctypes.data, reach.ctypes.data, ctypes.byref(nrows),
                             ctypes.byref(ncn), rows.ctypes.data, int(max_rows)))
    return {"nb": nb, "reach": reach, "rows": rows[:min(nrows.value, max_rows)],
            "ncnrows": ncn.value}


def d3_status(ctx):
    _check(lib().d3_status(ctx))


def d3_list_stats(ctx):
    out = np.zeros(6)
    _check(lib().d3_list_stats(ctx, out.ctypes.data))
    return {"max_pot": out[0], "mean_pot": out[1], "max_cn": out[2],
            "mean_cn": out[3], "bins": out[4], "images": out[5]}


PHASES = ("sort", "update", "cn", "pair", "chain", "list", "atm")


def d3_set_timing(ctx, enable):
    _check(lib().d3_set_timing(ctx, int(bool(enable))))


def d3_get_timing(ctx):
    ms = np.zeros(len(PHASES))
    calls = np.zeros(len(PHASES), dtype=np.int64)
    _check(lib().d3_get_timing(ctx, ms.ctypes.data, calls.ctypes.data))
    return {p: (float(ms[k]), int(calls[k])) for k, p in enumerate(PHASES)}


def d3_c6_surrogate_init(ctx, seed):
    _check(lib().d3_c6_surrogate_init(ctx, int(seed)))


def d3_c6_surrogate_train(ctx, n_samples=1_000_000, epochs=40, batch=256,
                          lr=3e-3, lr_final=1e-5, seed=4, cn_hi=6.0, stream=None):
    cfg = d3_train_cfg(int(n_samples), int(epochs), int(batch), float(lr),
                       float(lr_final), int(seed), float(cn_hi))
    loss = np.zeros(1)
    _check(lib().d3_c6_surrogate_train(ctx, ctypes.byref(cfg), loss.ctypes.data,
                                       _stream(stream)))
    return float(loss[0])


def d3_c6_surrogate_eval(ctx, elem_i, elem_j, cn_i, cn_j, out, precision=1, stream=None):
    _check(lib().d3_c6_surrogate_eval(ctx, int(elem_i.shape[0]), _ptr(elem_i), _ptr(elem_j),
                                      _ptr(cn_i), _ptr(cn_j), _ptr(out), int(precision),
                                      _stream(stream)))


def d3_c6_exact_eval(ctx, elem_i, elem_j, cn_i, cn_j, out, stream=None):
    _check(lib().d3_c6_exact_eval(ctx, int(elem_i.shape[0]), _ptr(elem_i), _ptr(elem_j),
                                  _ptr(cn_i), _ptr(cn_j), _ptr(out), _stream(stream)))


def d3_c6_surrogate_bytes(ctx):
    return int(lib().d3_c6_surrogate_bytes(ctx))


def d3_c6_surrogate_get_weights(ctx):
    nb = d3_c6_surrogate_bytes(ctx)
    buf = np.zeros(nb // 4, dtype=np.float32)
    _check(lib().d3_c6_surrogate_get_weights(ctx, buf.ctypes.data, nb))
    return buf


def d3_c6_surrogate_set_weights(ctx, buf):
    buf = np.ascontiguousarray(buf, dtype=np.float32)
    _check(lib().d3_c6_surrogate_set_weights(ctx, buf.ctypes.data, buf.nbytes))


def d3_c6_surrogate_grad(ctx, pair, x, y, grads, loss, stream=None):
    _check(lib().d3_c6_surrogate_grad(ctx, int(pair.shape[0]), _ptr(pair), _ptr(x), _ptr(y),
                                      _ptr(grads), _ptr(loss), _stream(stream)))


def d3_c6_surrogate_adam_step(ctx, pair, x, y, step, total_steps, lr, lr_final, stream=None):
    _check(lib().d3_c6_surrogate_adam_step(ctx, int(pair.shape[0]), _ptr(pair), _ptr(x), _ptr(y),
                                           int(step), int(total_steps), float(lr),
                                           float(lr_final), _stream(stream)))


def d3_md_nve(ctx, n_steps, dt, pos, vel, mass, every=0, stream=None):
    n_rec = (n_steps // every + 1) if every > 0 else 0
    thermo = np.zeros((max(n_rec, 1), 3))
    rebuilds = np.zeros(1, dtype=np.int64)
    _check(lib().d3_md_nve(ctx, int(n_steps), float(dt), _ptr(pos), _ptr(vel), _ptr(mass),
                           int(every), thermo.ctypes.data if every > 0 else None,
                           rebuilds.ctypes.data, _stream(stream)))
    return thermo[:n_rec], int(rebuilds[0])


# ------------------------------------------------------- convenience ----

class D3:
    """Owns one context.  ``build`` takes numpy or torch inputs; ``compute``
    returns torch tensors on the current device."""

    def __init__(self, table, mode="plain", skin=0.0, **prm):
        import torch
        self.torch = torch
        self.params = make_params(skin=skin, mode=MODES.get(mode, mode), **prm)
        self.ctx = d3_create(self.params, table)
        self.n = 0
        self.dev = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if self.ctx:
            d3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.dev, dtype=dtype).contiguous()
        return t.as_tensor(np.asarray(a), dtype=dtype, device=self.dev).contiguous()

    def set_mode(self, mode):
        d3_set_mode(self.ctx, MODES.get(mode, mode))

    def build(self, pos, types, cell, pbc=(1, 1, 1), stream=None):
        self.pos = self._dev(pos, self.torch.float64)
        self.types = self._dev(types, self.torch.int32)
        self.n = int(self.pos.shape[0])
        d3_build_neighbors(self.ctx, self.pos, self.types, cell, pbc, stream)

    def compute(self, pos=None, atom_energy=True, flags=0, stream=None, out=None,
                atom_virial=False, velocities=None):
        """Energy, forces, virial and site energies; with atom_virial=True also
        the per-atom virials (n,3,3), and given velocities (n,3) also the
        per-atom heat currents (n,3)."""
        t = self.torch
        p = self.pos if pos is None else self._dev(pos, t.float64)
        if out is None:
            out = {"energy": t.zeros(1, dtype=t.float64, device=self.dev),
                   "forces": t.zeros((self.n, 3), dtype=t.float64, device=self.dev),
                   "virial": t.zeros((3, 3), dtype=t.float64, device=self.dev),
                   "atom_energy": (t.zeros(self.n, dtype=t.float64, device=self.dev)
                                   if atom_energy else None)}
            if atom_virial:
                out["atom_virial"] = t.zeros((self.n, 3, 3), dtype=t.float64, device=self.dev)
            if velocities is not None:
                out["heat_current"] = t.zeros((self.n, 3), dtype=t.float64, device=self.dev)
        v = None if velocities is None else self._dev(velocities, t.float64)
        if out.get("atom_virial") is None and out.get("heat_current") is None:
            d3_energy_forces_virial(self.ctx, p, out["energy"], out["forces"], out["virial"],
                                    out["atom_energy"], flags, stream)
        else:
            d3_evaluate(self.ctx, p, out["energy"], out["forces"], out["virial"],
                        out["atom_energy"], out.get("atom_virial"), v, out.get("heat_current"),
                        flags, stream)
        return out

    def coordination(self, pos=None, stream=None):
        t = self.torch
        p = self.pos if pos is None else self._dev(pos, t.float64)
        cn = t.zeros(self.n, dtype=t.float64, device=self.dev)
        d3_coordination(self.ctx, p, cn, stream)
        return cn

    def status(self):
        d3_status(self.ctx)

    def stats(self):
        return d3_list_stats(self.ctx)
