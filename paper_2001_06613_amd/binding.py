"""ctypes binding of libstml.so (C-ABI declared in include/stml.h).

Argument marshalling only: every step of the registration path runs in the
HIP library.  PyTorch supplies device memory (the workspace and the caller's
buffers) and the HIP stream.  If the library is missing or cannot load, every
call raises; there is no fallback.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstml.so")

STML_OK = 0
STML_EINVAL = -1
STML_ENOMEM = -2
STML_EDEVICE = -3
STML_ESTATE = -4
STML_EBREAKDOWN = -5
STML_WLINESEARCH = 2
MAX_FRAMES = 256

REG = {"diffusion": 0, "curvature": 1}
MODEL = {"field": 0, "affine": 1}


class stml_opts(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n_spatial", ctypes.c_int),
        ("n_temporal", ctypes.c_int),
        ("regulariser", ctypes.c_int),
        ("alpha", ctypes.c_double),
        ("lambda_", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("eps_stop", ctypes.c_double),
        ("gn_max", ctypes.c_int),
        ("cg_max", ctypes.c_int),
        ("cg_rtol", ctypes.c_double),
        ("ls_max", ctypes.c_int),
        ("c1", ctypes.c_double),
        ("tol_J", ctypes.c_double),
        ("tol_u", ctypes.c_double),
        ("predictor", ctypes.c_int),
        ("parity_mode", ctypes.c_int),
        ("stop_relative", ctypes.c_int),
        ("model", ctypes.c_int),
        ("lbfgs_mem", ctypes.c_int),
    ]


class stml_gir_log(ctypes.Structure):
    _fields_ = [
        ("level", ctypes.c_int),
        ("q", ctypes.c_int),
        ("n_frames", ctypes.c_int),
        ("gn_iterations", ctypes.c_int),
        ("status", ctypes.c_int),
        ("J0", ctypes.c_double),
        ("J", ctypes.c_double),
        ("D", ctypes.c_double),
        ("S", ctypes.c_double),
        ("P", ctypes.c_double),
        ("cg_iterations", ctypes.c_int * 64),
        ("step", ctypes.c_double * 64),
        ("J_iter", ctypes.c_double * 64),
        ("du_max", ctypes.c_double * 64),
        ("du_rms", ctypes.c_double * 64),
        ("predictor", ctypes.c_int),
        ("J_paper", ctypes.c_double),
        ("J_learned", ctypes.c_double),
    ]


class stml_tuning(ctypes.Structure):
    _fields_ = [("tile_blocks", ctypes.c_int), ("vox_blocks", ctypes.c_int),
                ("hv_blocks", ctypes.c_int)]


# every symbol include/stml.h declares, with (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_IP = ctypes.POINTER(ctypes.c_int)
_DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "stml_default_opts": (None, [ctypes.POINTER(stml_opts)]),
    "stml_workspace_bytes": (ctypes.c_size_t,
                             [ctypes.POINTER(stml_opts), _I, _IP]),
    "stml_create": (_I, [ctypes.POINTER(stml_opts), _I, _IP, _P, _P,
                         ctypes.c_size_t, ctypes.POINTER(_P)]),
    "stml_destroy": (None, [_P]),
    "stml_last_error": (ctypes.c_char_p, [_P]),
    "stml_set_sequence": (_I, [_P, _P]),
    "stml_get_level_frames": (_I, [_P, _I, _P]),
    "stml_level_extent": (_I, [_P, _I, _IP]),
    "stml_temporal_set": (_I, [_P, _I, _IP, _I]),
    "stml_predict": (_I, [_P, _I, _I]),
    "stml_register_level": (_I, [_P, _I, _I]),
    "stml_correct": (_I, [_P, _I, _I]),
    "stml_run": (_I, [_P]),
    "stml_set_targets": (_I, [_P, _DP]),
    "stml_get_stop_trace": (_I, [_P, _I, _DP, _I, _IP]),
    "stml_get_displacements": (_I, [_P, _I, _P]),
    "stml_set_displacements": (_I, [_P, _I, _P]),
    "stml_get_prediction": (_I, [_P, _I, _P]),
    "stml_set_prediction": (_I, [_P, _I, _P]),
    "stml_log_count": (_I, [_P]),
    "stml_get_log": (_I, [_P, _I, ctypes.POINTER(stml_gir_log)]),
    "stml_get_params": (_I, [_P, _I, _DP]),
    "stml_set_params": (_I, [_P, _I, _DP]),
    "stml_eval_params": (_I, [_P, _I, _IP, _I, _DP, _DP, _DP]),
    "stml_eval": (_I, [_P, _I, _IP, _I, _P, _DP, _P, _P]),
    "stml_hessvec": (_I, [_P, _I, _IP, _I, _P, _P, _P, _DP]),
    "stml_gn_direction": (_I, [_P, _I, _IP, _I, _P, _P, _IP]),
    "stml_force_cg_breakdown": (_I, [_P, _I]),
    "stml_net_param_count": (_I, [_I]),
    "stml_net_workspace_bytes": (ctypes.c_size_t, [_I, _I, _IP]),
    "stml_net_create": (_I, [_I, _I, _IP, _P, _P, ctypes.c_size_t,
                             ctypes.POINTER(_P)]),
    "stml_net_destroy": (None, [_P]),
    "stml_net_set_params": (_I, [_P, _P]),
    "stml_net_get_params": (_I, [_P, _P]),
    "stml_net_set_input": (_I, [_P, _P, _I, _P, _I, _IP]),
    "stml_net_assemble": (_I, [_P, _P, _P, _I, _IP, ctypes.c_double, _IP,
                               _I, _I]),
    "stml_net_forward": (_I, [_P, _P]),
    "stml_net_emit": (_I, [_P, ctypes.c_double, _P]),
    "stml_net_gradient": (_I, [_P, _P, _DP]),
    "stml_net_train_step": (_I, [_P, ctypes.c_double, _DP]),
    "stml_set_predictor_net": (_I, [_P, _P]),
    "stml_batch_workspace_bytes": (ctypes.c_size_t, [_I]),
    "stml_batch_create": (_I, [ctypes.POINTER(_P), _I, _P, _P,
                               ctypes.c_size_t, ctypes.POINTER(_P)]),
    "stml_batch_destroy": (None, [_P]),
    "stml_batch_last_error": (ctypes.c_char_p, [_P]),
    "stml_batch_set_graph": (_I, [_P, _I]),
    "stml_batch_predict": (_I, [_P, _I, _I]),
    "stml_batch_register_level": (_I, [_P, _I, _I]),
    "stml_batch_run": (_I, [_P]),
    "stml_set_tuning": (_I, [_P, ctypes.POINTER(stml_tuning)]),
    "stml_get_tuning": (_I, [_P, ctypes.POINTER(stml_tuning)]),
    "stml_eval_noalloc": (_I, [ctypes.POINTER(stml_opts), _I, _IP,
                               ctypes.c_double, _P, _IP, _I, _P, _DP, _P, _P,
                               _P]),
    "stml_noalloc_last_error": (ctypes.c_char_p, []),
    "stml_timing": (_I, [_P, _I]),
    "stml_timing_every": (_I, [_P, _I, _I]),
    "stml_timing_get": (_I, [_P, _I, _I, _DP,
                             ctypes.POINTER(ctypes.c_longlong), _DP, _DP]),
}

KERNELS = {"eval": 0, "hessvec": 1, "cg_update": 2, "cg_pupdate": 3,
           "trial": 4, "cg_init": 5, "accept": 6, "predict": 7,
           "restrict": 8}

_lib = None


class STMLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stml error {code}: {msg}")
        self.code = code


def load(path=LIB_PATH):
    """Load libstml.so and declare every exported entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise STMLError(STML_EDEVICE,
                        f"{path} is missing: build it with "
                        "`python -c 'import __graft_entry__ as g; g.build()'`")
    # torch first: the library then binds to the HIP runtime torch loaded
    # (one runtime per process, so torch's streams and memory are valid
    # handles for the library)
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def default_opts(**kw):
    lib = load()
    o = stml_opts()
    lib.stml_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "lam" or k == "lambda":
            k = "lambda_"
        if k == "reg":
            k, v = "regulariser", REG[v]
        if k == "model" and isinstance(v, str):
            v = MODEL[v]
        if k in ("parity_mode", "stop_relative"):
            v = int(bool(v))
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _int_array(vals):
    arr = (ctypes.c_int * len(vals))(*[int(v) for v in vals])
    return arr


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def eval_noalloc(frames, u, K, h=1.0, opts=None, grad=None, dW=None,
                 stream=None, **kw):
    """stml_eval_noalloc: objective, gradient and dW/du over the frames K
    of `frames` ([n][extent...] float32, on the device) at u
    ([n][dim][extent...]), with no context and no library allocation.
    grad and dW ([|K|][dim][extent...] float32) are allocated by torch here
    unless given.  Returns (dict J, D, S, P, grad, dW)."""
    import torch

    lib = load()
    o = opts if opts is not None else default_opts(**kw)
    n, ext = frames.shape[0], tuple(frames.shape[1:])
    shape = (len(K), len(ext)) + ext
    if grad is None:
        grad = torch.empty(shape, dtype=torch.float32, device=frames.device)
    if dW is None:
        dW = torch.empty(shape, dtype=torch.float32, device=frames.device)
    for t, want in ((frames, (n,) + ext), (u, (n, len(ext)) + ext),
                    (grad, shape), (dW, shape)):
        if tuple(t.shape) != want or t.dtype != torch.float32 or \
                not t.is_contiguous() or not t.is_cuda:
            raise STMLError(STML_EINVAL, f"need a contiguous float32 device "
                                         f"tensor of shape {want}")
    s = stream if stream is not None else torch.cuda.current_stream()
    out = (ctypes.c_double * 4)()
    rc = lib.stml_eval_noalloc(ctypes.byref(o), n, _int_array(ext), float(h),
                               _ptr(frames), _int_array(K), len(K), _ptr(u),
                               out, _ptr(grad), _ptr(dW),
                               ctypes.c_void_p(s.cuda_stream))
    if rc != STML_OK:
        raise STMLError(rc, lib.stml_noalloc_last_error().decode())
    return {"J": out[0], "D": out[1], "S": out[2], "P": out[3],
            "g": grad, "dW": dW}


class STML:
    """One registration context on the current torch device and stream.

    Mirrors the C-ABI one to one: set_sequence, predict, register_level,
    correct, run, get/set_displacements, eval, hessvec, gn_direction.
    """

    def __init__(self, n, extent, opts=None, stream=None,
                 workspace_fill=None, **kw):
        """workspace_fill: byte value written over the fresh workspace
        before the context is created (tests: state must not depend on
        what the memory held)."""
        import torch

        self.torch = torch
        self.lib = load()
        self.opts = opts if opts is not None else default_opts(**kw)
        self.n = int(n)
        self.extent = tuple(int(m) for m in extent)
        self.dim = len(self.extent)
        if self.dim != self.opts.dim:
            raise STMLError(STML_EINVAL, "extent does not match opts.dim")
        ext = _int_array(self.extent)
        nbytes = self.lib.stml_workspace_bytes(ctypes.byref(self.opts),
                                               self.n, ext)
        if nbytes == 0:
            raise STMLError(STML_EINVAL, "invalid options or shape")
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8,
                                     device=self.device)
        if workspace_fill is not None:
            self.workspace.fill_(int(workspace_fill))
        self.stream = stream if stream is not None else \
            torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        rc = self.lib.stml_create(ctypes.byref(self.opts), self.n, ext,
                                  ctypes.c_void_p(self.stream.cuda_stream),
                                  _ptr(self.workspace), nbytes,
                                  ctypes.byref(ctx))
        if rc != STML_OK:
            raise STMLError(rc, "stml_create failed")
        self.ctx = ctx
        self.levels = self.opts.n_spatial

    # -- helpers
    def _check(self, rc, allow_warn=True):
        if rc < 0 or (rc > 0 and not allow_warn):
            msg = self.lib.stml_last_error(self.ctx).decode()
            raise STMLError(rc, msg)
        return rc

    def _sync_in(self):
        # the library works on self.stream; order it after torch's work
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.stml_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_extent(self, level):
        out = (ctypes.c_int * self.dim)()
        self._check(self.lib.stml_level_extent(self.ctx, level, out))
        return tuple(out)

    def temporal_set(self, q):
        out = (ctypes.c_int * MAX_FRAMES)()
        cnt = self._check(self.lib.stml_temporal_set(self.ctx, q, out,
                                                     MAX_FRAMES))
        return list(out[:cnt])

    def _field(self, level, frames=None):
        ext = self.level_extent(level)
        nf = self.n if frames is None else frames
        return self.torch.empty((nf, self.dim) + ext, dtype=self.torch.float32,
                                device=self.device)

    def _dev(self, t, shape=None):
        t = self.torch.as_tensor(t).to(self.device,
                                        self.torch.float32).contiguous()
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise STMLError(STML_EINVAL, f"shape {tuple(t.shape)} != {shape}")
        return t

    # -- C-ABI entry points
    def set_sequence(self, frames):
        f = self._dev(frames, (self.n,) + self.extent)
        self._sync_in()
        return self._check(self.lib.stml_set_sequence(self.ctx, _ptr(f)))

    def get_level_frames(self, level):
        out = self.torch.empty((self.n,) + self.level_extent(level),
                               dtype=self.torch.float32, device=self.device)
        self._check(self.lib.stml_get_level_frames(self.ctx, level, _ptr(out)))
        return out

    def predict(self, level, q_next):
        return self._check(self.lib.stml_predict(self.ctx, level, q_next))

    def register_level(self, level, q):
        return self._check(self.lib.stml_register_level(self.ctx, level, q))

    def correct(self, level, q_next):
        return self._check(self.lib.stml_correct(self.ctx, level, q_next))

    def run(self):
        return self._check(self.lib.stml_run(self.ctx))

    def get_displacements(self, level=None):
        level = self.levels - 1 if level is None else level
        out = self._field(level)
        self._check(self.lib.stml_get_displacements(self.ctx, level,
                                                    _ptr(out)))
        return out

    def set_displacements(self, level, u):
        u = self._dev(u, (self.n, self.dim) + self.level_extent(level))
        self._sync_in()
        return self._check(self.lib.stml_set_displacements(self.ctx, level,
                                                           _ptr(u)))

    def get_prediction(self, level):
        out = self._field(level)
        self._check(self.lib.stml_get_prediction(self.ctx, level, _ptr(out)))
        return out

    def set_prediction(self, level, z):
        z = self._dev(z, (self.n, self.dim) + self.level_extent(level))
        self._sync_in()
        return self._check(self.lib.stml_set_prediction(self.ctx, level,
                                                        _ptr(z)))

    # -- affine model: parameters [n][p] (host float64 arrays)
    @property
    def n_params(self):
        return self.dim * self.dim + self.dim

    def get_params(self, level=None):
        level = self.levels - 1 if level is None else level
        out = np.zeros((self.n, self.n_params), np.float64)
        self._check(self.lib.stml_get_params(
            self.ctx, level, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def set_params(self, level, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        if th.shape != (self.n, self.n_params):
            raise STMLError(STML_EINVAL, f"need ({self.n}, {self.n_params})")
        return self._check(self.lib.stml_set_params(
            self.ctx, level, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def eval_params(self, level, frames, theta, grad=True):
        """(dict J, D, P) and the gradient [|K|][p] at theta [n][p]."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        if th.shape != (self.n, self.n_params):
            raise STMLError(STML_EINVAL, f"need ({self.n}, {self.n_params})")
        out = (ctypes.c_double * 3)()
        g = np.zeros((len(frames), self.n_params), np.float64) if grad \
            else None
        dp = ctypes.POINTER(ctypes.c_double)
        self._sync_in()
        self._check(self.lib.stml_eval_params(
            self.ctx, level, _int_array(frames), len(frames),
            th.ctypes.data_as(dp), out,
            g.ctypes.data_as(dp) if grad else None))
        return {"J": out[0], "D": out[1], "P": out[2]}, g

    def set_targets(self, targets):
        """Objective targets [levels][n_temporal] (NaN-free; -inf for
        none), or None to clear."""
        if targets is None:
            return self._check(self.lib.stml_set_targets(self.ctx, None))
        t = np.ascontiguousarray(targets, dtype=np.float64)
        if t.shape != (self.levels, self.opts.n_temporal):
            raise STMLError(STML_EINVAL, "need (levels, n_temporal) targets")
        return self._check(self.lib.stml_set_targets(
            self.ctx, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def stop_trace(self, level=None):
        """Eq. (3) record of the last run on `level`: (D_q list, stop q or
        -1)."""
        level = self.levels - 1 if level is None else level
        buf = (ctypes.c_double * 64)()
        q = ctypes.c_int(-1)
        cnt = self._check(self.lib.stml_get_stop_trace(self.ctx, level, buf,
                                                       64, ctypes.byref(q)))
        return list(buf[:min(cnt, 64)]), q.value

    def logs(self):
        out = []
        for i in range(self.lib.stml_log_count(self.ctx)):
            lg = stml_gir_log()
            self._check(self.lib.stml_get_log(self.ctx, i, ctypes.byref(lg)))
            it = lg.gn_iterations
            out.append({"level": lg.level, "q": lg.q, "nK": lg.n_frames,
                        "gn": it, "status": lg.status, "J0": lg.J0,
                        "J": lg.J, "D": lg.D, "S": lg.S, "P": lg.P,
                        "cg": list(lg.cg_iterations[:max(it, 0)]),
                        "steps": list(lg.step[:max(it, 0)]),
                        "J_iter": list(lg.J_iter[:max(it, 0)]),
                        "du_max": list(lg.du_max[:max(it, 0)]),
                        "du_rms": list(lg.du_rms[:max(it, 0)]),
                        "predictor": lg.predictor, "J_paper": lg.J_paper,
                        "J_learned": lg.J_learned})
        return out

    def set_predictor_net(self, net):
        self._net_ref = net
        return self._check(self.lib.stml_set_predictor_net(
            self.ctx, net.net if net is not None else None))

    def set_tuning(self, tile_blocks, vox_blocks, hv_blocks):
        t = stml_tuning(int(tile_blocks), int(vox_blocks), int(hv_blocks))
        return self._check(self.lib.stml_set_tuning(self.ctx, ctypes.byref(t)))

    def get_tuning(self):
        t = stml_tuning()
        self._check(self.lib.stml_get_tuning(self.ctx, ctypes.byref(t)))
        return {"tile_blocks": t.tile_blocks, "vox_blocks": t.vox_blocks,
                "hv_blocks": t.hv_blocks}

    def timing(self, kernels, every=1):
        """Start timing the named kernel classes (True: all), or stop (None,
        False or an empty list); every > 1 times only every every-th launch
        of each class."""
        if kernels is True:
            mask = (1 << len(KERNELS)) - 1
        elif not kernels:
            mask = 0
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << KERNELS[k]
        return self._check(self.lib.stml_timing_every(self.ctx, mask,
                                                      int(every)))

    def timing_get(self, kernel, level=-1):
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        vf = ctypes.c_double()
        nbytes = ctypes.c_double()
        self._check(self.lib.stml_timing_get(self.ctx, KERNELS[kernel], level,
                                             ctypes.byref(ms), ctypes.byref(n),
                                             ctypes.byref(vf),
                                             ctypes.byref(nbytes)))
        return {"ms": ms.value, "launches": n.value, "voxel_frames": vf.value,
                "bytes": nbytes.value}

    def eval(self, level, frames, u, want_grad=True):
        """Objective {J, D, S, P}, gradient and dW/du at u (all frames)."""
        u = self._dev(u, (self.n, self.dim) + self.level_extent(level))
        fr = _int_array(frames)
        out = (ctypes.c_double * 4)()
        g = self._field(level, len(frames)) if want_grad else None
        dW = self._field(level, len(frames)) if want_grad else None
        self._sync_in()
        self._check(self.lib.stml_eval(
            self.ctx, level, fr, len(frames), _ptr(u), out,
            _ptr(g) if g is not None else None,
            _ptr(dW) if dW is not None else None))
        return {"J": out[0], "D": out[1], "S": out[2], "P": out[3],
                "g": g, "dW": dW}

    def hessvec(self, level, frames, u, v):
        ext = self.level_extent(level)
        u = self._dev(u, (self.n, self.dim) + ext)
        v = self._dev(v, (len(frames), self.dim) + ext)
        hv = self._field(level, len(frames))
        vhv = ctypes.c_double()
        self._sync_in()
        self._check(self.lib.stml_hessvec(self.ctx, level,
                                          _int_array(frames), len(frames),
                                          _ptr(u), _ptr(v), _ptr(hv),
                                          ctypes.byref(vhv)))
        return hv, vhv.value

    def gn_direction(self, level, frames, u, allow_breakdown=False):
        """(delta, CG iterations); with allow_breakdown a CG breakdown
        returns (delta, iterations, STML_EBREAKDOWN) instead of raising."""
        u = self._dev(u, (self.n, self.dim) + self.level_extent(level))
        delta = self._field(level, len(frames))
        cg = ctypes.c_int()
        self._sync_in()
        rc = self.lib.stml_gn_direction(self.ctx, level, _int_array(frames),
                                        len(frames), _ptr(u), _ptr(delta),
                                        ctypes.byref(cg))
        if allow_breakdown and rc == STML_EBREAKDOWN:
            return delta, cg.value, rc
        self._check(rc)
        return (delta, cg.value, rc) if allow_breakdown else (delta, cg.value)

    def force_cg_breakdown(self, it):
        """Make CG step it break down as if p.Hp <= 0 (-1: off)."""
        self._check(self.lib.stml_force_cg_breakdown(self.ctx, it))


class Batch:
    """Several STML contexts registered together (stml_batch_* entry
    points): one launch per kernel per Gauss-Newton step over the tiles of
    every sequence, the iteration replayed from a captured HIP graph."""

    def __init__(self, stmls, stream=None, graph=True):
        import torch

        self.torch = torch
        self.lib = load()
        self.stmls = list(stmls)
        n = len(self.stmls)
        if n < 1:
            raise STMLError(STML_EINVAL, "empty batch")
        nbytes = self.lib.stml_batch_workspace_bytes(n)
        dev = self.stmls[0].device
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else \
            torch.cuda.current_stream(dev)
        arr = (_P * n)(*[st.ctx.value for st in self.stmls])
        b = ctypes.c_void_p()
        rc = self.lib.stml_batch_create(arr, n,
                                        ctypes.c_void_p(self.stream.cuda_stream),
                                        _ptr(self.workspace), nbytes,
                                        ctypes.byref(b))
        if rc != STML_OK:
            raise STMLError(rc, "stml_batch_create failed (contexts must "
                            "agree in dim 2, levels and solver options)")
        self.batch = b
        self.set_graph(graph)

    def _check(self, rc):
        if rc < 0:
            raise STMLError(rc, self.lib.stml_batch_last_error(
                self.batch).decode())
        return rc

    def close(self):
        if getattr(self, "batch", None):
            self.lib.stml_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, on):
        return self._check(self.lib.stml_batch_set_graph(self.batch,
                                                         int(bool(on))))

    def predict(self, level, q_next):
        return self._check(self.lib.stml_batch_predict(self.batch, level,
                                                       q_next))

    def register_level(self, level, q):
        return self._check(self.lib.stml_batch_register_level(self.batch,
                                                              level, q))

    def run(self):
        return self._check(self.lib.stml_batch_run(self.batch))


class Net:
    """The learned predictor network (stml_net_* entry points)."""

    OUT_LD = 32

    def __init__(self, max_batch, max_extent, dim=2, stream=None):
        import torch

        self.torch = torch
        self.lib = load()
        self.dim = dim
        ext = _int_array(max_extent)
        nbytes = self.lib.stml_net_workspace_bytes(dim, max_batch, ext)
        if nbytes == 0:
            raise STMLError(STML_EINVAL, "invalid network shape")
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8,
                                     device=self.device)
        self.stream = stream if stream is not None else \
            torch.cuda.current_stream(self.device)
        net = ctypes.c_void_p()
        rc = self.lib.stml_net_create(dim, max_batch, ext,
                                      ctypes.c_void_p(self.stream.cuda_stream),
                                      _ptr(self.workspace), nbytes,
                                      ctypes.byref(net))
        if rc != STML_OK:
            raise STMLError(rc, "stml_net_create failed")
        self.net = net
        self.nparam = self.lib.stml_net_param_count(dim)

    def _check(self, rc):
        if rc != STML_OK:
            raise STMLError(rc, "stml_net call failed")

    def close(self):
        if getattr(self, "net", None):
            self.lib.stml_net_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = self.torch.as_tensor(params, dtype=self.torch.float32).to(
            self.device).contiguous()
        self._check(self.lib.stml_net_set_params(self.net, _ptr(p)))

    def get_params(self):
        p = self.torch.empty(self.nparam, dtype=self.torch.float32,
                             device=self.device)
        self._check(self.lib.stml_net_get_params(self.net, _ptr(p)))
        return p

    def set_input(self, x, target=None):
        """x: [B][C][*extent] float32 (C <= 32, extent of dim axes);
        target [B][*extent][dim]."""
        x = self.torch.as_tensor(x, dtype=self.torch.float32).to(
            self.device).contiguous()
        if x.dim() != self.dim + 2:
            raise STMLError(STML_EINVAL, "x must be [B][C][*extent]")
        B, C, ext = x.shape[0], x.shape[1], tuple(x.shape[2:])
        t = None
        if target is not None:
            t = self.torch.as_tensor(target, dtype=self.torch.float32).to(
                self.device).contiguous()
            if tuple(t.shape) != (B,) + ext + (self.dim,):
                raise STMLError(STML_EINVAL, "target must be [B][*extent][dim]")
        self._input_refs = (x, t)
        self._check(self.lib.stml_net_set_input(
            self.net, _ptr(x), C, _ptr(t) if t is not None else None, B,
            _int_array(ext)))
        self.cur = (B,) + ext

    def assemble(self, frames, u, h, triples, with_target=False):
        """frames [n][*extent], u [n][dim][*extent] float32 device tensors;
        triples [(t, l, r), ...] with 0 <= l < t < r < n."""
        torch = self.torch
        n, ext = frames.shape[0], tuple(frames.shape[1:])
        if (len(ext) != self.dim or frames.dtype != torch.float32 or
                u.dtype != torch.float32 or
                tuple(u.shape) != (n, self.dim) + ext or not frames.is_cuda or
                not u.is_cuda or not frames.is_contiguous() or
                not u.is_contiguous()):
            raise STMLError(STML_EINVAL, "frames [n][*extent] and u "
                            "[n][dim][*extent] contiguous float32 device "
                            "tensors expected")
        flat = [int(v) for tr in triples for v in tr]
        self._check(self.lib.stml_net_assemble(
            self.net, _ptr(frames), _ptr(u), int(n), _int_array(ext),
            float(h), _int_array(flat), len(triples), int(bool(with_target))))
        self.cur = (len(triples),) + ext
        self.cur_n = int(n)

    def forward(self):
        out = self.torch.empty(self.cur + (self.OUT_LD,),
                               dtype=self.torch.float32, device=self.device)
        self._check(self.lib.stml_net_forward(self.net, _ptr(out)))
        return out[..., :self.dim]

    def emit(self, h, u):
        """u [n][dim][*extent] (n and extent as last assembled) receives the
        predictions of the assembled frames."""
        ext = tuple(self.cur[1:])
        if (u.dtype != self.torch.float32 or not u.is_cuda or
                not u.is_contiguous() or
                tuple(u.shape) != (getattr(self, "cur_n", -1), self.dim) + ext):
            raise STMLError(STML_EINVAL, "u must match the assembled frames")
        self._check(self.lib.stml_net_emit(self.net, float(h), _ptr(u)))

    def gradient(self):
        g = self.torch.empty(self.nparam, dtype=self.torch.float32,
                             device=self.device)
        loss = ctypes.c_double()
        self._check(self.lib.stml_net_gradient(self.net, _ptr(g),
                                               ctypes.byref(loss)))
        return loss.value, g

    def train_step(self, lr):
        loss = ctypes.c_double()
        self._check(self.lib.stml_net_train_step(self.net, float(lr),
                                                 ctypes.byref(loss)))
        return loss.value


def exported_symbols(path=LIB_PATH):
    """Names of the C-ABI functions that libstml.so exports (no GPU call)."""
    lib = ctypes.CDLL(path)
    return [n for n in SIGNATURES if hasattr(lib, n)]


def as_numpy(t):
    return t.detach().cpu().numpy().astype(np.float64)
