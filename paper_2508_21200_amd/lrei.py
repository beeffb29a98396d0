"""Thin ctypes binding of liblrei.so (the C ABI declared in include/lrei.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  If the library is missing the import fails loudly; there is no
CPU fallback.  Arrays may be numpy arrays (host) or torch tensors on a ROCm
device (their data_ptr() is passed with the *_is_device flag).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrei.so")

LREI_OK = 0
LREI_E_INVALID = 1
LREI_E_NOTCONVERGED = 3
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_NOTCONVERGED", 4: "E_DEVICE",
                5: "E_STATE", 6: "E_NUMERIC"}
MODELS = {"qLL": 0, "qLLG": 1}
SCHEMES = {"RK1": 1, "RK2": 2, "RK3": 3, "RK4": 4, "AB2": 12, "AB3": 13, "AB4": 14}
PRECISIONS = {"fp64": 0, "mixed": 1}
WARM = {"plain": 0, "analytic": 1, "learned": 2, "predict_identity": 3, "predict_cayley": 4}


class lrei_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("eig_tol", ctypes.c_double),
                ("eig_max_sweeps", ctypes.c_int), ("warm", ctypes.c_int),
                ("ab_bootstrap", ctypes.c_int), ("householder_mode", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("deterministic", ctypes.c_int),
                ("autotune_cache", ctypes.c_char_p), ("mixed_pivot_floor", ctypes.c_double),
                ("fail_after_steps", ctypes.c_int), ("site_order", ctypes.c_int)]


class lrei_stats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int64), ("eigensolves", ctypes.c_int64),
                ("warm_accepted", ctypes.c_int64), ("warm_rejected", ctypes.c_int64),
                ("warm_iterations", ctypes.c_int64), ("dropped_directions", ctypes.c_int32),
                ("precision_promoted", ctypes.c_int32), ("min_pivot_ratio", ctypes.c_double),
                ("ortho_error", ctypes.c_double), ("energy", ctypes.c_double),
                ("last_step_ms", ctypes.c_double), ("phase_ms", ctypes.c_double * 8),
                ("eig_phase_ms", ctypes.c_double * 6)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["phase_ms"] = list(self.phase_ms)
        d["eig_phase_ms"] = list(self.eig_phase_ms)
        return d


TUNE_MAX = 128  # LREI_TUNE_MAX


class lrei_tune_result(ctypes.Structure):
    _fields_ = [("epl", ctypes.c_int), ("grid", ctypes.c_int), ("win_bits", ctypes.c_int),
                ("n_sweeps", ctypes.c_int), ("ms", ctypes.c_double),
                ("from_cache", ctypes.c_int), ("n_tried", ctypes.c_int),
                ("tried_epl", ctypes.c_int * TUNE_MAX), ("tried_grid", ctypes.c_int * TUNE_MAX),
                ("tried_win", ctypes.c_int * TUNE_MAX), ("tried_ms", ctypes.c_double * TUNE_MAX),
                ("tile_bits", ctypes.c_int), ("tile_waves", ctypes.c_int), ("tried_tile", ctypes.c_int * TUNE_MAX),
                ("compact", ctypes.c_int), ("overlap_grid", ctypes.c_int)]


BATCH_TUNE_CLASSES = 32


class lrei_batch_tune_result(ctypes.Structure):
    _fields_ = [("n_classes", ctypes.c_int), ("rank", ctypes.c_int * BATCH_TUNE_CLASSES),
                ("epl", ctypes.c_int * BATCH_TUNE_CLASSES), ("wg_cap", ctypes.c_int * BATCH_TUNE_CLASSES),
                ("ms_default", ctypes.c_double), ("ms", ctypes.c_double), ("n_tried", ctypes.c_int),
                ("tried_rank", ctypes.c_int * TUNE_MAX), ("tried_epl", ctypes.c_int * TUNE_MAX),
                ("tried_cap", ctypes.c_int * TUNE_MAX), ("tried_ms", ctypes.c_double * TUNE_MAX)]


class lrei_traj_desc(ctypes.Structure):
    _fields_ = [("n_spins", ctypes.c_int), ("n_bonds", ctypes.c_int), ("bond_ij", ctypes.c_void_p),
                ("bond_J", ctypes.c_void_p), ("site_h", ctypes.c_void_p), ("r", ctypes.c_int),
                ("lambda_", ctypes.c_void_p), ("V", ctypes.c_void_p), ("model", ctypes.c_int),
                ("kappa", ctypes.c_double)]


class lrei_adapt_result(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("h_next", ctypes.c_double), ("err_last", ctypes.c_double),
                ("err_max", ctypes.c_double), ("accepted", ctypes.c_int), ("rejected", ctypes.c_int),
                ("attempts", ctypes.c_int), ("reached", ctypes.c_int)]


PAIRS = {"HE21": 21, "BS32": 32, "RK43": 43}


class LreiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "lrei_default_options": (None, [ctypes.POINTER(lrei_options)]),
    "lrei_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, ctypes.POINTER(lrei_options)]),
    "lrei_destroy": (None, [_P]),
    "lrei_last_error": (ctypes.c_char_p, [_P]),
    "lrei_set_hamiltonian": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P, _P, ctypes.c_double]),
    "lrei_set_rho": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int]),
    "lrei_step": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int]),
    "lrei_evolve_adaptive": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int, ctypes.POINTER(lrei_adapt_result)]),
    "lrei_get_rho": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "lrei_observables": (ctypes.c_int, [_P, _P, _P]),
    "lrei_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(lrei_stats)]),
    "lrei_apply_hamiltonian": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int]),
    "lrei_apply_hamiltonian_noalloc": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "lrei_get_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_size_t)]),
    "lrei_set_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "lrei_profile_kernels": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int, _P]),
    "lrei_synchronize": (ctypes.c_int, [_P]),
    "lrei_autotune": (ctypes.c_int, [_P, ctypes.POINTER(lrei_tune_result)]),
    "lrei_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P, ctypes.POINTER(lrei_options),
                                         ctypes.c_int, ctypes.POINTER(lrei_traj_desc), ctypes.c_double]),
    "lrei_batch_destroy": (None, [_P]),
    "lrei_batch_last_error": (ctypes.c_char_p, [_P]),
    "lrei_batch_step": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_int]),
    "lrei_batch_get_rho": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int]),
    "lrei_batch_energies": (ctypes.c_int, [_P, _P]),
    "lrei_batch_profile_kernels": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_int, _P]),
    "lrei_batch_synchronize": (ctypes.c_int, [_P]),
    "lrei_batch_autotune": (ctypes.c_int, [_P, ctypes.c_int, _P]),
    "lrei_net_param_count": (ctypes.c_longlong, [ctypes.c_int]),
    "lrei_net_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int, _P, ctypes.c_uint64]),
    "lrei_net_destroy": (None, [_P]),
    "lrei_net_last_error": (ctypes.c_char_p, [_P]),
    "lrei_net_rank": (ctypes.c_int, [_P]),
    "lrei_net_get_params": (ctypes.c_int, [_P, _P]),
    "lrei_net_set_params": (ctypes.c_int, [_P, _P]),
    "lrei_net_loss_grad": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P]),
    "lrei_net_rotations": (ctypes.c_int, [_P, _P, ctypes.c_int, _P]),
    "lrei_net_train": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                                      ctypes.c_uint64, _P]),
    "lrei_record": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "lrei_record_count": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)]),
    "lrei_attach_net": (ctypes.c_int, [_P, _P]),
    "lrei_pair_density": (ctypes.c_int, [_P, ctypes.c_int, _P, _P]),
    "lrei_set_mixing": (ctypes.c_int, [_P, ctypes.c_double]),
    "lrei_set_rho_factor": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_int]),
    "lrei_get_rank": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int)]),
    "lrei_pair_entanglement": (ctypes.c_int, [_P, _P, _P, _P]),
}


def load(path=LIB_PATH):
    """Loads liblrei.so and declares every entry point; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _ptr(a):
    """(pointer, is_device) for a numpy array or a torch tensor."""
    if a is None:
        return None, 0
    if isinstance(a, np.ndarray):
        return a.ctypes.data, 0
    if hasattr(a, "data_ptr"):
        return a.data_ptr(), int(a.is_cuda)
    raise TypeError(type(a))


class Context:
    """One LREI context (one trajectory) on a HIP device."""

    def __init__(self, device=0, stream=None, precision="fp64", eig_tol=1e-15, eig_max_sweeps=40,
                 warm="analytic", householder_mode=0, use_graph=True, autotune_cache=None,
                 mixed_pivot_floor=None, fail_after_steps=0, site_order=0):
        self.lib = load()
        opt = lrei_options()
        self.lib.lrei_default_options(ctypes.byref(opt))
        if mixed_pivot_floor is not None:
            opt.mixed_pivot_floor = float(mixed_pivot_floor)
        opt.fail_after_steps = int(fail_after_steps)
        opt.site_order = int(site_order)
        opt.precision = PRECISIONS[precision]
        opt.eig_tol = eig_tol
        opt.eig_max_sweeps = eig_max_sweeps
        opt.warm = WARM[warm]
        opt.householder_mode = householder_mode
        opt.use_graph = int(bool(use_graph))
        self._cache = None if autotune_cache is None else str(autotune_cache).encode()
        opt.autotune_cache = self._cache
        h = _P()
        st = self.lib.lrei_create(ctypes.byref(h), int(device), stream, ctypes.byref(opt))
        if st != LREI_OK:
            raise LreiError(st, "lrei_create failed")
        self.h = h
        self.precision = precision
        self.n = None
        self.r = None

    def _check(self, st):
        if st != LREI_OK:
            raise LreiError(st, self.lib.lrei_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.lrei_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_hamiltonian(self, n, bonds, J, h=None, hbar=1.0):
        bonds = np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1, 2))
        J = np.ascontiguousarray(np.asarray(J, dtype=np.float64).reshape(-1, 3, 3))
        hh = None if h is None else np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(n, 3))
        self._check(self.lib.lrei_set_hamiltonian(self.h, int(n), bonds.shape[0], bonds.ctypes.data,
                                                  J.ctypes.data, None if hh is None else hh.ctypes.data,
                                                  float(hbar)))
        self.n = int(n)
        self._keep = (bonds, J, hh)

    def set_rho(self, lam, V):
        lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
        if isinstance(V, np.ndarray):
            V = np.ascontiguousarray(V, dtype=np.complex128)
        p, dev = _ptr(V)
        self._check(self.lib.lrei_set_rho(self.h, lam.size, lam.ctypes.data, p, dev))
        self.r = lam.size

    def step(self, model, scheme, dt, kappa, n_steps=1):
        self._check(self.lib.lrei_step(self.h, MODELS[model], SCHEMES[scheme], float(dt), float(kappa),
                                       int(n_steps)))

    def evolve_adaptive(self, model, kappa, t_span, tol, h_init, h_min=None, h_max=None, max_attempts=100000,
                        pair="RK43"):
        """Advances by t_span with step-size control (lrei_evolve_adaptive).
        Returns a dict with t, h_next, err_last, err_max, accepted, rejected,
        attempts and status ('done', 'h_min' or 'max_attempts'); other
        failures raise LreiError."""
        h_min = float(h_init) * 1e-6 if h_min is None else float(h_min)
        h_max = float(t_span) if h_max is None else float(h_max)
        res = lrei_adapt_result()
        st = self.lib.lrei_evolve_adaptive(self.h, MODELS[model], PAIRS[pair], float(kappa), float(t_span),
                                           float(tol), float(h_init), h_min, h_max, int(max_attempts),
                                           ctypes.byref(res))
        out = {k: getattr(res, k) for k, _ in lrei_adapt_result._fields_}
        out["reached"] = bool(out["reached"])
        if st == LREI_OK:
            out["status"] = "done"
            return out
        msg = self.lib.lrei_last_error(self.h).decode() if st == LREI_E_NOTCONVERGED else ""
        if msg.startswith("an attempt at h <= h_min"):
            out["status"] = "h_min"
        elif msg.startswith("max_attempts reached"):
            out["status"] = "max_attempts"
        else:
            self._check(st)
        return out

    def get_rho(self, out=None):
        lam = np.zeros(self.r, dtype=np.float64)
        if out is None:
            out = np.zeros((2 ** self.n, self.r), dtype=np.complex128)
        p, dev = _ptr(out)
        self._check(self.lib.lrei_get_rho(self.h, lam.ctypes.data, p, dev))
        return lam, out

    def observables(self):
        e = ctypes.c_double()
        m = (ctypes.c_double * 3)()
        self._check(self.lib.lrei_observables(self.h, ctypes.byref(e), m))
        return e.value, np.array(list(m))

    def stats(self):
        s = lrei_stats()
        self._check(self.lib.lrei_get_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def apply_hamiltonian(self, X, out=None):
        if isinstance(X, np.ndarray):
            X = np.ascontiguousarray(X, dtype=np.complex128)
            if out is None:
                out = np.zeros_like(X)
        px, dev = _ptr(X)
        py, _ = _ptr(out)
        self._check(self.lib.lrei_apply_hamiltonian(self.h, X.shape[1], px, py, dev))
        return out

    def apply_hamiltonian_noalloc(self, X, Y):
        """Y = H X into the caller's device tensors (complex128, N x r,
        contiguous) without device allocation; enqueued on the context's
        stream (call synchronize() before reading Y)."""
        assert X.is_cuda and Y.is_cuda and X.is_contiguous() and Y.is_contiguous()
        assert X.shape == Y.shape and X.dim() == 2
        self._check(self.lib.lrei_apply_hamiltonian_noalloc(self.h, int(X.shape[1]), ctypes.c_void_p(X.data_ptr()),
                                                             ctypes.c_void_p(Y.data_ptr())))
        return Y

    def get_state(self):
        n = ctypes.c_size_t()
        self._check(self.lib.lrei_get_state(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self.lib.lrei_get_state(self.h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def set_state(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.lrei_set_state(self.h, buf, len(blob)))
        hdr = np.frombuffer(blob[:24], dtype=np.uint64)
        self.r = int(hdr[2])

    def profile_kernels(self, model, scheme, dt, kappa, iters=20):
        """Average per-launch ms of (H.V pass, reduction, projected step, combination)."""
        ms = (ctypes.c_double * 4)()
        self._check(self.lib.lrei_profile_kernels(self.h, MODELS[model], SCHEMES[scheme], float(dt),
                                                  float(kappa), int(iters), ms))
        return dict(hv_pass=ms[0], reduce=ms[1], projected_step=ms[2], combine=ms[3])

    def autotune(self):
        """Times the H.V launch variants and keeps the fastest; returns the choice and all timings."""
        t = lrei_tune_result()
        self._check(self.lib.lrei_autotune(self.h, ctypes.byref(t)))
        return {"epl": t.epl, "grid": t.grid, "win_bits": t.win_bits, "n_sweeps": t.n_sweeps, "ms": t.ms,
                "from_cache": bool(t.from_cache), "tile_bits": t.tile_bits, "tile_waves": t.tile_waves,
                "compact": bool(t.compact), "overlap_grid": t.overlap_grid,
                "tried": [(t.tried_epl[i], t.tried_grid[i], t.tried_win[i], t.tried_ms[i])
                          for i in range(t.n_tried)],
                "tried_tile": [t.tried_tile[i] for i in range(t.n_tried)]}

    def synchronize(self):
        self._check(self.lib.lrei_synchronize(self.h))

    def set_rho_factor(self, A):
        """rho = A A* / Tr(A A*) from a factor A (N x m, any columns); sets r = rank."""
        if isinstance(A, np.ndarray):
            A = np.ascontiguousarray(A, dtype=np.complex128)
        p, dev = _ptr(A)
        self._check(self.lib.lrei_set_rho_factor(self.h, A.shape[1], p, dev))
        r = ctypes.c_int()
        self._check(self.lib.lrei_get_rank(self.h, ctypes.byref(r)))
        self.r = r.value

    def set_mixing(self, p):
        """State p I / N + (1 - p) V Lambda V* from now on (see lrei_set_mixing)."""
        self._check(self.lib.lrei_set_mixing(self.h, float(p)))

    def pair_density(self, pairs):
        """Two-spin reduced density matrices, (n_pairs, 4, 4) complex."""
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        out = np.zeros((pr.shape[0], 4, 4), dtype=np.complex128)
        self._check(self.lib.lrei_pair_density(self.h, pr.shape[0], pr.ctypes.data, out.ctypes.data))
        return out

    def record(self, samples, capacity=None):
        """Records a training sample per RK stage into `samples` (a device
        float32 tensor of capacity x net_sample_floats(r)); None stops."""
        if samples is None:
            self._check(self.lib.lrei_record(self.h, None, 0))
            self._rec = None
            return
        cap = samples.shape[0] if capacity is None else int(capacity)
        p, dev = _ptr(samples)
        if not dev:
            raise LreiError(LREI_E_INVALID, "the sample buffer must be device memory")
        self._check(self.lib.lrei_record(self.h, p, cap))
        self._rec = samples

    def record_count(self):
        c = ctypes.c_int()
        self._check(self.lib.lrei_record_count(self.h, ctypes.byref(c)))
        return c.value

    def attach_net(self, net):
        """Network for warm="learned" (None detaches); it must outlive the attachment."""
        self._check(self.lib.lrei_attach_net(self.h, None if net is None else net.h))
        self._net = net


def pair_entanglement(R):
    """(concurrence, negativity, chsh) of a 4 x 4 two-spin density matrix."""
    lib = load()
    R = np.ascontiguousarray(np.asarray(R, dtype=np.complex128).reshape(4, 4))
    c, n, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = lib.lrei_pair_entanglement(R.ctypes.data, ctypes.byref(c), ctypes.byref(n), ctypes.byref(b))
    if st != LREI_OK:
        raise LreiError(st, "invalid two-spin density matrix")
    return c.value, n.value, b.value


def net_sample_floats(r):
    return 4 * r * r + 2


class Net:
    """The learned start rotation's network for rank r (lrei_net_* entry points)."""

    def __init__(self, r, device=0, params=None, seed=0):
        self.lib = load()
        self.r = int(r)
        h = _P()
        init = None
        if params is not None:
            init = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
            if init.size != self.param_count(self.r):
                raise LreiError(LREI_E_INVALID, "wrong parameter count")
        st = self.lib.lrei_net_create(ctypes.byref(h), int(device), self.r,
                                      None if init is None else init.ctypes.data, int(seed))
        if st != LREI_OK:
            raise LreiError(st, "lrei_net_create failed")
        self.h = h

    @staticmethod
    def param_count(r):
        return int(load().lrei_net_param_count(int(r)))

    def _check(self, st):
        if st != LREI_OK:
            raise LreiError(st, self.lib.lrei_net_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.lrei_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        out = np.zeros(self.param_count(self.r), dtype=np.float32)
        self._check(self.lib.lrei_net_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        if p.size != self.param_count(self.r):
            raise LreiError(LREI_E_INVALID, "wrong parameter count")
        self._check(self.lib.lrei_net_set_params(self.h, p.ctypes.data))

    def loss_grad(self, samples, n=None, grad=True):
        """Mean loss over the first n samples (device float32 tensor) and the gradient."""
        n = samples.shape[0] if n is None else int(n)
        loss = ctypes.c_double()
        g = np.zeros(self.param_count(self.r), dtype=np.float32) if grad else None
        p, dev = _ptr(samples)
        if not dev:
            raise LreiError(LREI_E_INVALID, "the samples must be device memory")
        self._check(self.lib.lrei_net_loss_grad(self.h, p, n, ctypes.byref(loss),
                                                None if g is None else g.ctypes.data))
        return loss.value, g

    def rotations(self, samples, n=None):
        n = samples.shape[0] if n is None else int(n)
        R = np.zeros((n, self.r, self.r), dtype=np.complex128)
        p, dev = _ptr(samples)
        if not dev:
            raise LreiError(LREI_E_INVALID, "the samples must be device memory")
        self._check(self.lib.lrei_net_rotations(self.h, p, n, R.ctypes.data))
        return R

    def train(self, samples, n=None, batch=256, epochs=10, lr=1e-3, seed=0):
        n = samples.shape[0] if n is None else int(n)
        losses = np.zeros(max(epochs, 1), dtype=np.float64)
        p, dev = _ptr(samples)
        if not dev:
            raise LreiError(LREI_E_INVALID, "the samples must be device memory")
        self._check(self.lib.lrei_net_train(self.h, p, n, int(batch), int(epochs), float(lr), int(seed),
                                            losses.ctypes.data))
        return losses[:epochs]


class Batch:
    """Many independent trajectories advanced together (lrei_batch_* entry points).

    trajs: list of dicts with keys n, bonds, J, h (or None), lam, V (host
    complex128), model ("qLL"/"qLLG") and kappa.
    """

    def __init__(self, trajs, device=0, stream=None, precision="fp64", use_graph=True, hbar=1.0,
                 householder_mode=0, warm="analytic"):
        self.lib = load()
        opt = lrei_options()
        self.lib.lrei_default_options(ctypes.byref(opt))
        opt.precision = PRECISIONS[precision]
        opt.use_graph = int(bool(use_graph))
        opt.householder_mode = householder_mode
        opt.warm = WARM[warm]
        descs = (lrei_traj_desc * len(trajs))()
        keep = []
        self.shapes = []
        for q, t in enumerate(trajs):
            n = int(t["n"])
            bonds = np.ascontiguousarray(np.asarray(t["bonds"], dtype=np.int32).reshape(-1, 2))
            J = np.ascontiguousarray(np.asarray(t["J"], dtype=np.float64).reshape(-1, 3, 3))
            hh = None if t.get("h") is None else np.ascontiguousarray(
                np.asarray(t["h"], dtype=np.float64).reshape(n, 3))
            lam = np.ascontiguousarray(np.asarray(t["lam"], dtype=np.float64))
            V = np.ascontiguousarray(np.asarray(t["V"]), dtype=np.complex128)
            keep.append((bonds, J, hh, lam, V))
            d = descs[q]
            d.n_spins = n
            d.n_bonds = bonds.shape[0]
            d.bond_ij = bonds.ctypes.data
            d.bond_J = J.ctypes.data
            d.site_h = None if hh is None else hh.ctypes.data
            d.r = lam.size
            d.lambda_ = lam.ctypes.data
            d.V = V.ctypes.data
            d.model = MODELS[t["model"]]
            d.kappa = float(t["kappa"])
            self.shapes.append((n, lam.size))
        h = _P()
        st = self.lib.lrei_batch_create(ctypes.byref(h), int(device), stream, ctypes.byref(opt), len(trajs),
                                        descs, float(hbar))
        if st != LREI_OK:
            raise LreiError(st, self.lib.lrei_batch_last_error(None).decode())
        self.h = h
        self.precision = precision

    def _check(self, st):
        if st != LREI_OK:
            raise LreiError(st, self.lib.lrei_batch_last_error(self.h).decode())

    def __len__(self):
        return len(self.shapes)

    def close(self):
        if getattr(self, "h", None):
            self.lib.lrei_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, scheme, dt, n_steps=1):
        self._check(self.lib.lrei_batch_step(self.h, SCHEMES[scheme], float(dt), int(n_steps)))

    def get_rho(self, traj, out=None):
        if not 0 <= traj < len(self.shapes):  # the library reports the bad index
            self._check(self.lib.lrei_batch_get_rho(self.h, int(traj), None, None, 0))
        n, r = self.shapes[traj]
        lam = np.zeros(r, dtype=np.float64)
        if out is None:
            out = np.zeros((2 ** n, r), dtype=np.complex128)
        p, dev = _ptr(out)
        self._check(self.lib.lrei_batch_get_rho(self.h, int(traj), lam.ctypes.data, p, dev))
        return lam, out

    def profile_kernels(self, scheme, dt, iters=20):
        """Average ms of (H.V pass, reduction, projected step, combination) for the whole batch."""
        ms = (ctypes.c_double * 4)()
        self._check(self.lib.lrei_batch_profile_kernels(self.h, SCHEMES[scheme], float(dt), int(iters), ms))
        return dict(hv_pass=ms[0], reduce=ms[1], projected_step=ms[2], combine=ms[3])

    def autotune(self, iters=10):
        """Chooses the batched H.V launch shape per rank class (lrei_batch_autotune);
        returns the choice per rank and every timing."""
        t = lrei_batch_tune_result()
        self._check(self.lib.lrei_batch_autotune(self.h, int(iters), ctypes.byref(t)))
        return {"ms_default": t.ms_default, "ms": t.ms,
                "choice": {t.rank[k]: {"epl": t.epl[k], "wg_cap": t.wg_cap[k]} for k in range(t.n_classes)},
                "tried": [(t.tried_rank[i], t.tried_epl[i], t.tried_cap[i], t.tried_ms[i])
                          for i in range(min(t.n_tried, TUNE_MAX))]}

    def energies(self):
        e = np.zeros(len(self.shapes), dtype=np.float64)
        self._check(self.lib.lrei_batch_energies(self.h, e.ctypes.data))
        return e

    def synchronize(self):
        self._check(self.lib.lrei_batch_synchronize(self.h))
