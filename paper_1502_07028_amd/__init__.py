"""Python binding of libtca.so, the MI355X (gfx950) HIP implementation of the
parallelized traveling cluster approximation (arXiv:1502.07028).

Argument marshalling only: every step of the Monte Carlo hot path runs in the
library's HIP kernels.  The functions carry the C names of ``include/tca.h``.
Importing this module raises if the HIP library has not been built
(``python -m paper_1502_07028_amd.build``); there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtca.so")

TCA_ABI_VERSION = 2
TCA_OK, TCA_E_INVAL, TCA_E_NOMEM, TCA_E_DEVICE, TCA_E_UNSUPPORTED = 0, -1, -2, -3, -4
TCA_FP64, TCA_MIXED = 0, 1
TCA_INIT_RANDOM, TCA_INIT_FERRO, TCA_INIT_NEEL, TCA_INIT_USER = 0, 1, 2, 3
TCA_FLAG_PROFILE, TCA_FLAG_NO_GRAPH, TCA_FLAG_NO_AUTOTUNE, TCA_FLAG_EXACT_METROPOLIS = 1, 2, 4, 8

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python -m paper_1502_07028_amd.build)")
_lib = ctypes.CDLL(LIB_PATH)


class tca_params(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_int32), ("L", ctypes.c_int32), ("Lc", ctypes.c_int32),
                ("n_classes", ctypes.c_int32), ("Lc_classes", ctypes.c_int32 * 4),
                ("t", ctypes.c_double), ("JH", ctypes.c_double), ("JAF", ctypes.c_double),
                ("mu", ctypes.c_double), ("seed", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("init", ctypes.c_int32), ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class tca_update_record(ctypes.Structure):
    _fields_ = [("site", ctypes.c_int32), ("Lc", ctypes.c_int16), ("accept", ctypes.c_uint8),
                ("flags", ctypes.c_uint8), ("dF", ctypes.c_double), ("dE", ctypes.c_double),
                ("u", ctypes.c_double), ("dS_f", ctypes.c_float), ("dS_r", ctypes.c_float)]


class tca_sweep_stats(ctypes.Structure):
    _fields_ = [("updates", ctypes.c_int64), ("accepted", ctypes.c_int64),
                ("near_threshold", ctypes.c_int64), ("elapsed_ms", ctypes.c_double),
                ("reduce_ms", ctypes.c_double), ("eig_ms", ctypes.c_double),
                ("decide_ms", ctypes.c_double), ("reduce_launches", ctypes.c_int64),
                ("eig_launches", ctypes.c_int64), ("decide_launches", ctypes.c_int64),
                ("stage1_passed", ctypes.c_int64), ("surrogate_ms", ctypes.c_double),
                ("surrogate_launches", ctypes.c_int64)]


RECORD_DTYPE = np.dtype([("site", "<i4"), ("Lc", "<i2"), ("accept", "u1"), ("flags", "u1"),
                         ("dF", "<f8"), ("dE", "<f8"), ("u", "<f8"), ("dS_f", "<f4"),
                         ("dS_r", "<f4")])
assert RECORD_DTYPE.itemsize == ctypes.sizeof(tca_update_record)

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)
_F = ctypes.POINTER(ctypes.c_float)
_L = ctypes.POINTER(ctypes.c_int64)
_SIGS = {
    "tca_init_lattice": [ctypes.POINTER(tca_params), _D, _P, ctypes.POINTER(_P)],
    "tca_sweep": [_P, _D, ctypes.c_int32, _P, ctypes.POINTER(tca_sweep_stats)],
    "tca_cluster_eigvals": [_P, _I, _I, _D, ctypes.c_int32, _D, ctypes.c_int32],
    "tca_observables": [_P, _D, _D, _D],
    "tca_set_state": [_P, _D, ctypes.c_uint64],
    "tca_get_sweep_counter": [_P, ctypes.POINTER(ctypes.c_uint64)],
    "tca_heevals_batched": [_D, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                            ctypes.c_double, _D, _D],
    "tca_heevals_batched_dev": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_double, ctypes.c_double, _P, _P, _P],
    "tca_destroy": [_P],
    "tca_abi_sizes": [_I],
    "tca_surrogate_create": [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, _P,
                             ctypes.POINTER(_P)],
    "tca_surrogate_destroy": [_P],
    "tca_surrogate_info": [_P, _L, _I, _L],
    "tca_surrogate_save": [_P, _F],
    "tca_surrogate_load": [_P, _F],
    "tca_surrogate_collect": [_P, _P, _D, ctypes.c_int32, ctypes.POINTER(tca_sweep_stats)],
    "tca_surrogate_add_rows": [_P, _F, _F, ctypes.c_int64],
    "tca_surrogate_get_rows": [_P, ctypes.c_int64, ctypes.c_int64, _F, _F],
    "tca_surrogate_train": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_double,
                            _D, _D, _D],
    "tca_surrogate_grad": [_P, _F, _F, ctypes.c_int32, _F, _D],
    "tca_surrogate_adam_step": [_P, _F, ctypes.c_float],
    "tca_surrogate_eval": [_P, _F, ctypes.c_int32, ctypes.c_int32, _F],
    "tca_attach_surrogate": [_P, _P],
    "tca_tuning_report": [_P, ctypes.c_char_p, ctypes.c_int32],
    "tca_reducer_variants": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _I,
                             ctypes.POINTER(ctypes.c_char_p)],
    "tca_select_reducer_variant": [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.tca_strerror.argtypes = [ctypes.c_int]
_lib.tca_strerror.restype = ctypes.c_char_p
_lib.tca_last_error.argtypes = []
_lib.tca_last_error.restype = ctypes.c_char_p


class TCAError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.tca_last_error().decode() or _lib.tca_strerror(status).decode()
        super().__init__(f"{where}: {_lib.tca_strerror(status).decode()} ({status}): {msg}")


def _check(status, where):
    if status != TCA_OK:
        raise TCAError(status, where)


def _dptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _fptr(a):
    return a.ctypes.data_as(_F) if a is not None else None


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _stats(st):
    return {k: getattr(st, k) for k, _ in tca_sweep_stats._fields_}


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def tca_abi_sizes():
    out = np.zeros(3, dtype=np.int32)
    _check(_lib.tca_abi_sizes(out.ctypes.data_as(_I)), "tca_abi_sizes")
    return tuple(int(x) for x in out)


def make_params(L, Lc=8, t=1.0, JH=8.0, JAF=0.0, mu=0.0, seed=1, precision=TCA_FP64,
                init=TCA_INIT_RANDOM, Lc_classes=(), flags=0):
    p = tca_params()
    p.abi_version = TCA_ABI_VERSION
    p.L, p.Lc = int(L), int(Lc)
    p.n_classes = len(Lc_classes)
    for k, v in enumerate(Lc_classes):
        p.Lc_classes[k] = int(v)
    p.t, p.JH, p.JAF, p.mu = float(t), float(JH), float(JAF), float(mu)
    p.seed = int(seed)
    p.precision, p.init = int(precision), int(init)
    p.flags = int(flags)
    return p


def tca_init_lattice(params, spins=None, stream=None):
    """Create a context; returns an opaque handle (int).  ``stream`` is a raw
    hipStream_t (e.g. ``torch.cuda.current_stream().cuda_stream``) or None."""
    sp = None if spins is None else _f64(spins, (-1, 3))
    h = _P()
    _check(_lib.tca_init_lattice(ctypes.byref(params), _dptr(sp), stream, ctypes.byref(h)),
           "tca_init_lattice")
    return h.value


def tca_tuning_report(ctx):
    buf = ctypes.create_string_buffer(4096)
    _check(_lib.tca_tuning_report(ctx, buf, len(buf)), "tca_tuning_report")
    return buf.value.decode()


def tca_reducer_variants(n, precision=TCA_FP64):
    """Names of the reducer variants for dimension n at a precision."""
    cnt = ctypes.c_int32()
    _check(_lib.tca_reducer_variants(int(n), int(precision), 0, ctypes.byref(cnt), None),
           "tca_reducer_variants")
    out = []
    for v in range(cnt.value):
        nm = ctypes.c_char_p()
        _check(_lib.tca_reducer_variants(int(n), int(precision), v, ctypes.byref(cnt),
                                         ctypes.byref(nm)), "tca_reducer_variants")
        out.append(nm.value.decode())
    return out


def tca_select_reducer_variant(n, precision, variant):
    _check(_lib.tca_select_reducer_variant(int(n), int(precision), int(variant)),
           "tca_select_reducer_variant")


def tca_destroy(ctx):
    _check(_lib.tca_destroy(ctx), "tca_destroy")


def tca_sweep(ctx, T, nsweeps=None, log=False, N=None):
    """Run sweeps at temperatures T (array, one per sweep).  Returns
    (records or None, stats dict)."""
    T = _f64(np.atleast_1d(T))
    ns = len(T) if nsweeps is None else int(nsweeps)
    recs = None
    if log:
        if N is None:
            raise ValueError("N (lattice sites) is needed to size the log")
        recs = np.zeros(ns * N, dtype=RECORD_DTYPE)
    st = tca_sweep_stats()
    _check(_lib.tca_sweep(ctx, _dptr(T), ns, recs.ctypes.data if recs is not None else None,
                          ctypes.byref(st)), "tca_sweep")
    return recs, _stats(st)


def tca_cluster_eigvals(ctx, sites, Lc=None, proposed=None, ld=None):
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    n = len(sites)
    lcs = None if Lc is None else np.ascontiguousarray(np.broadcast_to(Lc, (n,)), dtype=np.int32)
    if ld is None:
        ld = 2 * int(np.max(lcs)) ** 2 if lcs is not None else 200
    prop = None if proposed is None else _f64(proposed, (n, 3))
    out = np.full((n, ld), np.nan)
    _check(_lib.tca_cluster_eigvals(ctx, sites.ctypes.data_as(_I),
                                    lcs.ctypes.data_as(_I) if lcs is not None else None,
                                    _dptr(prop), n, _dptr(out), ld), "tca_cluster_eigvals")
    return out


def tca_observables(ctx, L):
    N = L * L
    spins = np.zeros((N, 3))
    sq = np.zeros((L, L))
    m = np.zeros(3)
    _check(_lib.tca_observables(ctx, _dptr(spins), _dptr(sq), _dptr(m)), "tca_observables")
    return spins, sq, m


def tca_set_state(ctx, spins, sweep_counter):
    sp = _f64(spins, (-1, 3))
    _check(_lib.tca_set_state(ctx, _dptr(sp), int(sweep_counter)), "tca_set_state")


def tca_get_sweep_counter(ctx):
    v = ctypes.c_uint64()
    _check(_lib.tca_get_sweep_counter(ctx, ctypes.byref(v)), "tca_get_sweep_counter")
    return v.value


def tca_heevals_batched(A, precision=TCA_FP64, T=None, mu=0.0):
    """A: (batch, n, n) complex Hermitian.  Returns (eigenvalues (batch, n),
    free energies (batch,) or None)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    batch, n, _ = A.shape
    w = np.zeros((batch, n))
    F = np.zeros(batch) if T is not None else None
    Ad = A.view(np.float64)
    _check(_lib.tca_heevals_batched(_dptr(Ad), n, batch, precision,
                                    float(T) if T is not None else 1.0, float(mu), _dptr(w),
                                    _dptr(F)), "tca_heevals_batched")
    return w, F


def tca_heevals_batched_dev(A_ptr, n, batch, precision, T, mu, w_ptr, F_ptr, stream):
    """Device-pointer variant (raw addresses, e.g. tensor.data_ptr())."""
    _check(_lib.tca_heevals_batched_dev(A_ptr, n, batch, precision, float(T), float(mu),
                                        w_ptr, F_ptr, stream), "tca_heevals_batched_dev")


class Lattice:
    """Owning wrapper of one tca_ctx."""

    def __init__(self, L, Lc=8, stream=None, spins=None, **kw):
        if spins is not None:
            kw["init"] = TCA_INIT_USER
        self.L, self.N = int(L), int(L) * int(L)
        self.params = make_params(L, Lc, **kw)
        self.ctx = tca_init_lattice(self.params, spins, stream)

    def sweep(self, T, log=False):
        return tca_sweep(self.ctx, T, log=log, N=self.N)

    def tuning_report(self):
        return tca_tuning_report(self.ctx)

    def attach(self, surrogate):
        """Use a Surrogate as the first stage of delayed acceptance (None: plain)."""
        tca_attach_surrogate(self.ctx, surrogate.handle if surrogate is not None else None)
        self._sg = surrogate

    def eigvals(self, sites, Lc=None, proposed=None):
        return tca_cluster_eigvals(self.ctx, sites, Lc, proposed)

    def observables(self):
        return tca_observables(self.ctx, self.L)

    def spins(self):
        return self.observables()[0]

    def set_state(self, spins, sweep_counter):
        tca_set_state(self.ctx, spins, sweep_counter)

    @property
    def sweep_counter(self):
        return tca_get_sweep_counter(self.ctx)

    def close(self):
        if self.ctx:
            tca_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- surrogate
def tca_surrogate_create(Lc, hidden=256, seed=1, capacity=0, stream=None):
    h = _P()
    _check(_lib.tca_surrogate_create(int(Lc), int(hidden), int(seed), int(capacity), stream,
                                     ctypes.byref(h)), "tca_surrogate_create")
    return h.value


def tca_surrogate_destroy(sg):
    _check(_lib.tca_surrogate_destroy(sg), "tca_surrogate_destroy")


def tca_surrogate_info(sg):
    n, k, r = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(_lib.tca_surrogate_info(sg, ctypes.byref(n), ctypes.byref(k), ctypes.byref(r)),
           "tca_surrogate_info")
    return n.value, k.value, r.value


def tca_surrogate_save(sg):
    n = tca_surrogate_info(sg)[0]
    out = np.zeros(n, dtype=np.float32)
    _check(_lib.tca_surrogate_save(sg, _fptr(out)), "tca_surrogate_save")
    return out


def tca_surrogate_load(sg, params):
    v = _f32(params).ravel()
    if v.size != tca_surrogate_info(sg)[0]:
        raise ValueError("parameter vector has the wrong length")
    _check(_lib.tca_surrogate_load(sg, _fptr(v)), "tca_surrogate_load")


def tca_surrogate_collect(sg, ctx, T):
    T = _f64(np.atleast_1d(T))
    st = tca_sweep_stats()
    _check(_lib.tca_surrogate_collect(sg, ctx, _dptr(T), len(T), ctypes.byref(st)),
           "tca_surrogate_collect")
    return _stats(st)


def tca_surrogate_add_rows(sg, X, y):
    n_in = tca_surrogate_info(sg)[1]
    X = _f32(X, (-1, n_in))
    y = _f32(y).ravel()
    if len(y) != len(X):
        raise ValueError("X and y row counts differ")
    _check(_lib.tca_surrogate_add_rows(sg, _fptr(X), _fptr(y), len(y)), "tca_surrogate_add_rows")


def tca_surrogate_get_rows(sg, r0, rows):
    n_in = tca_surrogate_info(sg)[1]
    X = np.zeros((int(rows), n_in), dtype=np.float32)
    y = np.zeros(int(rows), dtype=np.float32)
    _check(_lib.tca_surrogate_get_rows(sg, int(r0), int(rows), _fptr(X), _fptr(y)),
           "tca_surrogate_get_rows")
    return X, y


def tca_surrogate_train(sg, steps, batch=1024, lr=1e-3, holdout=0.1):
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_lib.tca_surrogate_train(sg, int(steps), int(batch), float(lr), float(holdout),
                                    ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "tca_surrogate_train")
    return dict(train_mse=a.value, holdout_rmse_fp32=b.value, holdout_rmse_bf16=c.value)


def tca_surrogate_grad(sg, X, y):
    n, n_in, _ = tca_surrogate_info(sg)
    X = _f32(X, (-1, n_in))
    y = _f32(y).ravel()
    g = np.zeros(n, dtype=np.float32)
    loss = ctypes.c_double()
    _check(_lib.tca_surrogate_grad(sg, _fptr(X), _fptr(y), len(y), _fptr(g), ctypes.byref(loss)),
           "tca_surrogate_grad")
    return loss.value, g


def tca_surrogate_adam_step(sg, grad, lr):
    g = _f32(grad).ravel()
    _check(_lib.tca_surrogate_adam_step(sg, _fptr(g), float(lr)), "tca_surrogate_adam_step")


def tca_surrogate_eval(sg, X, bf16=True):
    n_in = tca_surrogate_info(sg)[1]
    X = _f32(X, (-1, n_in))
    out = np.zeros(len(X), dtype=np.float32)
    _check(_lib.tca_surrogate_eval(sg, _fptr(X), len(X), int(bool(bf16)), _fptr(out)),
           "tca_surrogate_eval")
    return out


def tca_attach_surrogate(ctx, sg):
    _check(_lib.tca_attach_surrogate(ctx, sg), "tca_attach_surrogate")


class Surrogate:
    """Owning wrapper of one tca_surrogate (the learned first stage)."""

    def __init__(self, Lc, hidden=256, seed=1, capacity=0, stream=None):
        self.handle = tca_surrogate_create(Lc, hidden, seed, capacity, stream)
        self.Lc, self.hidden = int(Lc), int(hidden)

    @property
    def n_params(self):
        return tca_surrogate_info(self.handle)[0]

    @property
    def n_in(self):
        return tca_surrogate_info(self.handle)[1]

    @property
    def rows(self):
        return tca_surrogate_info(self.handle)[2]

    def params(self):
        return tca_surrogate_save(self.handle)

    def load(self, params):
        tca_surrogate_load(self.handle, params)

    def collect(self, lattice, T):
        return tca_surrogate_collect(self.handle, lattice.ctx, T)

    def add_rows(self, X, y):
        tca_surrogate_add_rows(self.handle, X, y)

    def get_rows(self, r0, rows):
        return tca_surrogate_get_rows(self.handle, r0, rows)

    def train(self, steps, batch=1024, lr=1e-3, holdout=0.1):
        return tca_surrogate_train(self.handle, steps, batch, lr, holdout)

    def grad(self, X, y):
        return tca_surrogate_grad(self.handle, X, y)

    def adam_step(self, grad, lr):
        tca_surrogate_adam_step(self.handle, grad, lr)

    def eval(self, X, bf16=True):
        return tca_surrogate_eval(self.handle, X, bf16)

    def close(self):
        if self.handle:
            tca_surrogate_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
