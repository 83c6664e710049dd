"""ctypes binding of libmcmg.so (argument marshalling only).

The names mirror the C ABI in include/mcmg.h.  Device arrays are passed as
torch tensors on the GPU (complex128 fields on the extended grid, float32
features); PyTorch only provides device memory and streams.  Every call
runs in the HIP library; when the library is missing the calls raise.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmcmg.so")

MCMG_OK = 0
MCMG_NOT_CONVERGED = 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "E_ARG", -2: "E_OOM", -3: "E_HIP",
          -4: "E_WEIGHTS", -5: "E_NONFINITE", -6: "E_BREAKDOWN", -7: "E_BUDGET"}
PRECISION = {"fp32": 0, "bf16": 1}


class McmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3)]


class Pml(ctypes.Structure):
    _fields_ = [("ncells", ctypes.c_int), ("sigma_max", ctypes.c_double), ("kind", ctypes.c_int)]


ABSORBER = {"pml": 0, "sponge": 1}
BORN_MCMG, BORN_CBS = 0, 1


class Weights(ctypes.Structure):
    _fields_ = [("blob", ctypes.c_void_p), ("bytes", ctypes.c_size_t)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("restart", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("ortho", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("relres_true", ctypes.c_double), ("relres_est", ctypes.c_double),
                ("status", ctypes.c_int), ("hist", ctypes.POINTER(ctypes.c_double)),
                ("hist_cap", ctypes.c_int), ("hist_len", ctypes.c_int)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_int),
                ("graphs", ctypes.c_int)]


class Completion(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("status", ctypes.c_int), ("nrhs", ctypes.c_int),
                ("iters_total", ctypes.c_int), ("iters_max", ctypes.c_int),
                ("relres_max", ctypes.c_double), ("queue_s", ctypes.c_double),
                ("latency_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("bytes_in_use", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t),
                ("media", ctypes.c_int), ("slots", ctypes.c_int), ("inflight", ctypes.c_int),
                ("queued", ctypes.c_int), ("completed", ctypes.c_int),
                ("inflight_peak", ctypes.c_int), ("ticks", ctypes.c_longlong), ("rebuilds", ctypes.c_longlong)]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


_lib = None

EXPORTS = {
    "mcmg_setup": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), Grid, ctypes.c_double,
                                  ctypes.c_double, Pml, Weights, ctypes.POINTER(Opts),
                                  ctypes.POINTER(ctypes.c_void_p)]),
    "mcmg_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mcmg_apply_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mcmg_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mcmg_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_double, ctypes.c_int, ctypes.POINTER(Info)]),
    "mcmg_stationary": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_double, ctypes.c_int, ctypes.POINTER(Info)]),
    "mcmg_train_step": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Adam),
                                       ctypes.POINTER(ctypes.c_double)]),
    "mcmg_train_loss_grad": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
    "mcmg_train_set_trainable": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                                ctypes.c_int]),
    "mcmg_train_commit": (ctypes.c_int, [ctypes.c_void_p]),
    "mcmg_weights_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "mcmg_get_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                        ctypes.c_size_t]),
    "mcmg_born_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]),
    "mcmg_born_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "mcmg_born_green": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mcmg_born_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mcmg_born_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                                       ctypes.POINTER(Info)]),
    "mcmg_solve_batch": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                        ctypes.c_double, ctypes.c_int, ctypes.POINTER(Info)]),
    "mcmg_grid_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "mcmg_device_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "mcmg_destroy": (None, [ctypes.c_void_p]),
    "mcmg_last_error": (ctypes.c_char_p, []),
    "mcmg_prof_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "mcmg_prof_report": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t]),
    "mcmg_prof_replay": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int)]),
    "mcmg_debug_set_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "mcmg_debug_get_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                               ctypes.c_void_p]),
    "mcmg_debug_level_shape": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_int),
                                              ctypes.POINTER(ctypes.c_int)]),
    "mcmg_server_create": (ctypes.c_int, [ctypes.POINTER(ServerOpts), ctypes.POINTER(ctypes.c_void_p)]),
    "mcmg_server_add_medium": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), Grid,
                                              ctypes.c_double, ctypes.c_double, Pml, Weights,
                                              ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_int)]),
    "mcmg_server_add_handle": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(ctypes.c_int)]),
    "mcmg_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_double,
                                          ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]),
    "mcmg_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Completion), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "mcmg_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "mcmg_server_destroy": (None, [ctypes.c_void_p]),
}


def lib():
    """Load libmcmg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2606_30495_amd.build first")
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(l, name)
            fn.restype = res
            fn.argtypes = args
        _lib = l
    return _lib


def _check(st):
    if st < 0:
        raise McmgError(st, lib().mcmg_last_error().decode())
    return st


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Handle:
    """One medium: setup once (Alg. 1), then apply / matvec / solve."""

    def __init__(self, c, omega, h, npml, blob, precision="fp32", restart=30, sigma_max=0.0,
                 stream=None, ortho=0, absorber="pml"):
        c = np.ascontiguousarray(c, dtype=np.float64)
        g = Grid(c.ndim, (ctypes.c_int * 3)(*(list(c.shape) + [1] * (3 - c.ndim))))
        self._blob = bytes(blob)
        w = Weights(ctypes.cast(ctypes.c_char_p(self._blob), ctypes.c_void_p), len(self._blob))
        opts = Opts(PRECISION[precision], int(restart), _stream_ptr(stream), int(ortho))
        out = ctypes.c_void_p()
        _check(lib().mcmg_setup(c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), g, float(omega),
                                float(h), Pml(int(npml), float(sigma_max), ABSORBER[absorber]), w,
                                ctypes.byref(opts), ctypes.byref(out)))
        self.ptr = out
        d = ctypes.c_int()
        ne = (ctypes.c_int * 3)()
        npm = ctypes.c_int()
        _check(lib().mcmg_grid_shape(self.ptr, ctypes.byref(d), ne, ctypes.byref(npm)))
        self.dim = d.value
        self.ext_shape = tuple(ne[: self.dim])
        self.npml = npm.value
        self.restart = restart

    def close(self):
        if getattr(self, "ptr", None):
            lib().mcmg_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self):
        return lib().mcmg_device_bytes(self.ptr)

    def _shape_check(self, *ts):
        import torch
        for t in ts:
            if t.dtype != torch.complex128 or tuple(t.shape) != self.ext_shape:
                raise ValueError(f"expected complex128 {self.ext_shape}, got {t.dtype} {tuple(t.shape)}")

    def apply(self, r, z):
        self._shape_check(r, z)
        _check(lib().mcmg_apply(self.ptr, _ptr(r), _ptr(z)))

    def apply_noalloc(self, r, z):
        """z = MG(r) with the level state in the library's static device
        array (mcmg_apply_noalloc): no allocation."""
        self._shape_check(r, z)
        _check(lib().mcmg_apply_noalloc(self.ptr, _ptr(r), _ptr(z)))

    def matvec(self, u, Au):
        self._shape_check(u, Au)
        _check(lib().mcmg_matvec(self.ptr, _ptr(u), _ptr(Au)))

    def _solve(self, fn, f, u, tol, maxit, hist_cap):
        self._shape_check(f, u)
        hist = (ctypes.c_double * max(1, hist_cap))()
        info = Info(0, 0, 0.0, 0.0, 0, hist, hist_cap, 0)
        st = _check(fn(self.ptr, _ptr(f), _ptr(u), float(tol), int(maxit), ctypes.byref(info)))
        return {"status": st, "iters": info.iters, "restarts": info.restarts,
                "relres_true": info.relres_true, "relres_est": info.relres_est,
                "hist": list(hist[: info.hist_len]), "converged": st == MCMG_OK}

    def solve(self, f, u, tol=1e-6, maxit=500, hist_cap=4096):
        return self._solve(lib().mcmg_solve, f, u, tol, maxit, hist_cap)

    def stationary(self, f, u, tol=1e-6, maxit=500, hist_cap=4096):
        return self._solve(lib().mcmg_stationary, f, u, tol, maxit, hist_cap)

    # ---- training (L_H, Adam, LLPF) ----
    def weights_size(self):
        nt, nf = ctypes.c_int(), ctypes.c_size_t()
        _check(lib().mcmg_weights_size(self.ptr, ctypes.byref(nt), ctypes.byref(nf)))
        return nt.value, nf.value

    def get_weights(self):
        """Current parameters as a float32 vector in canonical order."""
        _, nf = self.weights_size()
        out = np.empty(nf, dtype=np.float32)
        _check(lib().mcmg_get_weights(self.ptr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), nf))
        return out

    def export_blob(self):
        """The current parameters as a weight blob (same model as the handle's)."""
        from .weights import build_blob, parse_blob, split_flat
        head, tens = parse_blob(self._blob)
        return build_blob(head, split_flat(tens, self.get_weights()))

    def set_trainable(self, mask):
        m = (ctypes.c_int * len(mask))(*[1 if v else 0 for v in mask])
        _check(lib().mcmg_train_set_trainable(self.ptr, m, len(mask)))

    def commit(self):
        _check(lib().mcmg_train_commit(self.ptr))

    # ---- Born-series form (periodic operator, discrete Green operator) ----
    def born_setup(self, k0sq=0.0, eps=0.0):
        _check(lib().mcmg_born_setup(self.ptr, float(k0sq), float(eps)))

    def born_params(self):
        k0sq, eps = ctypes.c_double(), ctypes.c_double()
        _check(lib().mcmg_born_params(self.ptr, ctypes.byref(k0sq), ctypes.byref(eps)))
        return k0sq.value, eps.value

    def born_green(self, x, y):
        self._shape_check(x, y)
        _check(lib().mcmg_born_green(self.ptr, _ptr(x), _ptr(y)))

    def born_matvec(self, u, Au):
        self._shape_check(u, Au)
        _check(lib().mcmg_born_matvec(self.ptr, _ptr(u), _ptr(Au)))

    def born_solve(self, f, u, method="mcmg", tol=1e-6, maxit=500, hist_cap=4096):
        m = {"mcmg": BORN_MCMG, "cbs": BORN_CBS}[method]
        fn = lib().mcmg_born_solve
        return self._solve(lambda h, fp, up, t, mi, inf: fn(h, m, fp, up, t, mi, inf),
                           f, u, tol, maxit, hist_cap)

    def prof_enable(self, on=True):
        _check(lib().mcmg_prof_enable(self.ptr, 1 if on else 0))

    def prof_report(self):
        import json
        buf = ctypes.create_string_buffer(1 << 20)
        _check(lib().mcmg_prof_report(self.ptr, buf, len(buf)))
        return json.loads(buf.value.decode())

    def prof_replay(self, name, reps=1):
        avg = ctypes.c_double()
        n = ctypes.c_int()
        _check(lib().mcmg_prof_replay(self.ptr, name.encode(), int(reps), ctypes.byref(avg),
                                      ctypes.byref(n)))
        return avg.value, n.value

    def level_shape(self, level):
        n = (ctypes.c_int * 3)()
        c = ctypes.c_int()
        _check(lib().mcmg_debug_level_shape(self.ptr, int(level), n, ctypes.byref(c)))
        return tuple(n[: self.dim]), c.value

    def set_features(self, level, a, s):
        _check(lib().mcmg_debug_set_features(self.ptr, int(level), _ptr(a), _ptr(s)))

    def get_features(self, level, a, s):
        _check(lib().mcmg_debug_get_features(self.ptr, int(level), _ptr(a), _ptr(s)))


def solve_batch(handles, fs, us, tol=1e-6, maxit=500, hist_cap=0):
    nb = len(handles)
    H = (ctypes.c_void_p * nb)(*[h.ptr.value for h in handles])
    F = (ctypes.c_void_p * nb)(*[f.data_ptr() for f in fs])
    U = (ctypes.c_void_p * nb)(*[u.data_ptr() for u in us])
    for h, f, u in zip(handles, fs, us):
        h._shape_check(f, u)
    infos = (Info * nb)()
    hists = []
    for i in range(nb):
        hb = (ctypes.c_double * max(1, hist_cap))()
        hists.append(hb)
        infos[i].hist = hb
        infos[i].hist_cap = hist_cap
    st = _check(lib().mcmg_solve_batch(H, F, U, nb, float(tol), int(maxit), infos))
    out = []
    for i in range(nb):
        out.append({"status": infos[i].status, "iters": infos[i].iters,
                    "relres_true": infos[i].relres_true, "restarts": infos[i].restarts,
                    "hist": list(hists[i][: infos[i].hist_len]),
                    "converged": infos[i].status == MCMG_OK})
    return st, out


class Server:
    """Serving loop (continuous batching under an HBM budget); see the
    mcmg_server_* entry points.  Media are Handles (ownership moves to the
    server) or set up in place; requests carry device f / u tensors that
    must stay alive until their completion is polled."""

    def __init__(self, hbm_budget, max_inflight=0, graphs=True):
        out = ctypes.c_void_p()
        o = ServerOpts(int(hbm_budget), int(max_inflight), 1 if graphs else 0)
        _check(lib().mcmg_server_create(ctypes.byref(o), ctypes.byref(out)))
        self.ptr = out
        self._shapes = []
        self._held = {}

    def add_handle(self, handle):
        mid = ctypes.c_int()
        ptr, handle.ptr = handle.ptr, None        # the server owns it now
        _check(lib().mcmg_server_add_handle(self.ptr, ptr, ctypes.byref(mid)))
        self._shapes.append(handle.ext_shape)
        return mid.value

    def add_medium(self, c, omega, h, npml, blob, precision="bf16", restart=30, sigma_max=0.0,
                   ortho=0, absorber="pml"):
        c = np.ascontiguousarray(c, dtype=np.float64)
        g = Grid(c.ndim, (ctypes.c_int * 3)(*(list(c.shape) + [1] * (3 - c.ndim))))
        b = bytes(blob)
        w = Weights(ctypes.cast(ctypes.c_char_p(b), ctypes.c_void_p), len(b))
        opts = Opts(PRECISION[precision], int(restart), None, int(ortho))
        mid = ctypes.c_int()
        _check(lib().mcmg_server_add_medium(self.ptr, c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            g, float(omega), float(h),
                                            Pml(int(npml), float(sigma_max), ABSORBER[absorber]),
                                            w, ctypes.byref(opts), ctypes.byref(mid)))
        self._shapes.append(tuple(s + 2 * int(npml) for s in c.shape))
        return mid.value

    def submit(self, medium, fs, us, tol=1e-6, maxit=500):
        import torch
        shape = self._shapes[medium]
        for t in list(fs) + list(us):
            if t.dtype != torch.complex128 or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"expected contiguous complex128 {shape}")
        n = len(fs)
        F = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        U = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
        rid = ctypes.c_uint64()
        _check(lib().mcmg_server_submit(self.ptr, int(medium), F, U, n, float(tol), int(maxit),
                                        ctypes.byref(rid)))
        self._held[rid.value] = (list(fs), list(us))
        return rid.value

    def poll(self, max_n=64, wait_ms=0):
        buf = (Completion * max_n)()
        n = ctypes.c_int()
        _check(lib().mcmg_server_poll(self.ptr, buf, max_n, ctypes.byref(n), int(wait_ms)))
        out = []
        for i in range(n.value):
            c = buf[i]
            self._held.pop(c.req_id, None)
            out.append({"req_id": c.req_id, "status": c.status, "nrhs": c.nrhs,
                        "iters_total": c.iters_total, "iters_max": c.iters_max,
                        "relres_max": c.relres_max, "queue_s": c.queue_s,
                        "latency_s": c.latency_s})
        return out

    def stats(self):
        st = ServerStats()
        _check(lib().mcmg_server_get_stats(self.ptr, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "ptr", None):
            lib().mcmg_server_destroy(self.ptr)
            self.ptr = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _train_args(handles, residuals):
    if len(handles) != len(residuals) or not handles:
        raise ValueError("one residual per handle")
    for H, r in zip(handles, residuals):
        H._shape_check(r)
    hs = (ctypes.c_void_p * len(handles))(*[H.ptr.value for H in handles])
    rs = (ctypes.c_void_p * len(residuals))(*[_ptr(r) for r in residuals])
    return hs, rs


def train_step(handles, residuals, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on handles[0]'s parameters from L_H over the batch
    (handles[i], residuals[i]); returns L_H before the update."""
    hs, rs = _train_args(handles, residuals)
    loss = ctypes.c_double()
    opt = Adam(lr, beta1, beta2, eps)
    _check(lib().mcmg_train_step(hs, len(handles), rs, ctypes.byref(opt), ctypes.byref(loss)))
    return loss.value


def train_loss_grad(handles, residuals):
    """(L_H, gradient as a float32 vector in canonical order) without an update."""
    hs, rs = _train_args(handles, residuals)
    _, nf = handles[0].weights_size()
    g = np.empty(nf, dtype=np.float32)
    loss = ctypes.c_double()
    _check(lib().mcmg_train_loss_grad(hs, len(handles), rs, ctypes.byref(loss),
                                      g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), nf))
    return loss.value, g
