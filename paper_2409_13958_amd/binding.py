"""ctypes binding of the pmfem C ABI (include/pmfem.h); argument marshalling only.

Every computation happens in ``libpmfem.so``. Device buffers are torch
tensors on the context's GPU; their ``data_ptr()`` and the current HIP
stream are passed through. If the library has not been built the import of
``load_library`` raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import enum
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmfem.so")

TERM_EX = 1
TERM_MS = 2


class Status(enum.IntEnum):
    OK = 0
    EINVAL = -1
    EMESH = -2
    EPBC = -3
    EGRID = -4
    ENOMEM = -5
    EHIP = -6
    ESTATE = -7
    ECONV = -8


class PmfemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{Status(code).name}: {msg}")
        self.code = Status(code)


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_U32 = ctypes.c_uint32
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)
_U64 = ctypes.c_uint64

_SIGS = {
    "pmfem_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P]),
    "pmfem_set_mesh": (ctypes.c_int, [_P, _I64, _P, _I64, _P, _P]),
    "pmfem_set_materials": (ctypes.c_int, [_P, _I32, _P, _P]),
    "pmfem_set_periodicity": (ctypes.c_int, [_P, _U32, _P, _D]),
    "pmfem_set_aim": (ctypes.c_int, [_P, _P, _I32, _I32, _D, _I32]),
    "pmfem_set_variant": (ctypes.c_int, [_P, ctypes.c_char_p, _I32]),
    "pmfem_build": (ctypes.c_int, [_P]),
    "pmfem_query": (ctypes.c_int, [_P, ctypes.POINTER(_I64), _P, _P, _DP]),
    "pmfem_heff": (ctypes.c_int, [_P, _P, _P, _U32, _P]),
    "pmfem_heff_parts": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "pmfem_grid_convolve": (ctypes.c_int, [_P, _P, _P]),
    "pmfem_grid_convolve_noalloc": (ctypes.c_int, [_P, _P, _P]),
    "pmfem_llg_step": (ctypes.c_int, [_P, _P, _D, _D, _I32, _P]),
    "pmfem_llg_step_graph": (ctypes.c_int, [_P, _P, _D, _D, _I32, _P]),
    "pmfem_llg_implicit": (ctypes.c_int, [_P, _P, _D, _D, _I32, _U32, _P, _D, _I32, _P]),
    "pmfem_llg_implicit_adaptive": (ctypes.c_int, [_P, _P, _D, _P, _D, _U32, _P, _D, _D, _I32,
                                                   _I32, _P, _P, _I32]),
    "pmfem_llg_bdf2_adaptive": (ctypes.c_int, [_P, _P, _D, _P, _D, _U32, _P, _D, _D, _I32,
                                               _I32, _P, _P, _I32]),
    "pmfem_energy": (ctypes.c_int, [_P, _P, _DP, _DP]),
    "pmfem_profile_begin": (ctypes.c_int, [_P, _I32]),
    "pmfem_profile_end": (ctypes.c_int, [_P, ctypes.POINTER(_I32), _P, _P, _P]),
    "pmfem_export": (ctypes.c_int, [_P, ctypes.c_char_p, _P, ctypes.POINTER(_I64),
                                    ctypes.POINTER(_I32)]),
    "pmfem_pgf_eval": (ctypes.c_int, [_U32, _P, _D, _I64, _P, _P]),
    "pmfem_autotune": (ctypes.c_int, [_P, _I32, _P, _DP]),
    "pmfem_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _P, _P, _I32]),
    "pmfem_batch_query": (ctypes.c_int, [_P, ctypes.POINTER(_I64), _P, _DP]),
    "pmfem_batch_heff": (ctypes.c_int, [_P, _P, _P, _U32]),
    "pmfem_batch_llg_step": (ctypes.c_int, [_P, _P, _D, _D, _I32]),
    "pmfem_batch_llg_step_graph": (ctypes.c_int, [_P, _P, _D, _D, _I32]),
    "pmfem_surrogate_init": (ctypes.c_int, [_P, _I32, _U64, _I32]),
    "pmfem_surrogate_param_count": (ctypes.c_int, [_P, ctypes.POINTER(_I64)]),
    "pmfem_surrogate_set_params": (ctypes.c_int, [_P, _P, _I64, _P]),
    "pmfem_surrogate_get_params": (ctypes.c_int, [_P, _P, _I64, _P]),
    "pmfem_surrogate_apply": (ctypes.c_int, [_P, _P, _P]),
    "pmfem_surrogate_loss_grad": (ctypes.c_int, [_P, _P, _P, _DP, _P, _I64]),
    "pmfem_surrogate_profile": (ctypes.c_int, [_P, _P, _P, _I32, _P]),
    "pmfem_surrogate_texture": (ctypes.c_int, [_P, _I32, _U64, _P]),
    "pmfem_surrogate_train": (ctypes.c_int, [_P, _I32, _D, _U64, _U32, _P]),
    "pmfem_surrogate_enable": (ctypes.c_int, [_P, _I32]),
    "pmfem_llg_step_judged": (ctypes.c_int, [_P, _P, _D, _D, _I32, _P, _I32, _D, _P]),
    "pmfem_batch_last_error": (ctypes.c_char_p, [_P]),
    "pmfem_batch_destroy": (None, [_P]),
    "pmfem_last_error": (ctypes.c_char_p, [_P]),
    "pmfem_destroy": (None, [_P]),
}

EXPORTED = tuple(_SIGS)


def load_library(path=LIB_PATH):
    """Load libpmfem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2409_13958_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def pgf_eval(mask, L, r, eta=0.0):
    """Library's periodic Green's function at points r[n,3] (host, FP64)."""
    lib = load_library()
    r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1, 3)
    L = np.ascontiguousarray(L, dtype=np.float64)
    out = np.empty(r.shape[0])
    rc = lib.pmfem_pgf_eval(mask, _ptr(L), float(eta), r.shape[0], _ptr(r), _ptr(out))
    if rc:
        raise PmfemError(rc, "pmfem_pgf_eval")
    return out


def _dev_ptr(t, dtype, shape=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One pmfem context on a HIP device (device=-1: host-only setup)."""

    def __init__(self, device=0, stream=None):
        self.lib = load_library()
        self.device = device
        h = _P()
        if device >= 0 and stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        rc = self.lib.pmfem_create(ctypes.byref(h), device, _P(stream) if stream else None)
        if rc:
            raise PmfemError(rc, "pmfem_create")
        self.h = h
        self.n = None
        self._keep = []

    def _check(self, rc, what):
        if rc:
            msg = self.lib.pmfem_last_error(self.h)
            raise PmfemError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None):
            self.lib.pmfem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup -------------------------------------------------------------
    def set_mesh(self, xyz, tets, region):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        region = np.ascontiguousarray(region, dtype=np.int32)
        self._check(self.lib.pmfem_set_mesh(self.h, xyz.shape[0], _ptr(xyz), tets.shape[0],
                                            _ptr(tets), _ptr(region)), "set_mesh")

    def set_materials(self, Ms, Aex):
        Ms = np.ascontiguousarray(Ms, dtype=np.float64)
        Aex = np.ascontiguousarray(Aex, dtype=np.float64)
        self._check(self.lib.pmfem_set_materials(self.h, Ms.size, _ptr(Ms), _ptr(Aex)),
                    "set_materials")

    def set_periodicity(self, mask, L, tol=0.0):
        L = np.ascontiguousarray(L, dtype=np.float64)
        self._check(self.lib.pmfem_set_periodicity(self.h, int(mask), _ptr(L), float(tol)),
                    "set_periodicity")

    def set_variant(self, stage, variant):
        self._check(self.lib.pmfem_set_variant(self.h, stage.encode(), int(variant)),
                    "set_variant")

    def set_aim(self, grid, order_p=3, near_boxes=2, z0_radius=1.0, precision=0):
        g = np.ascontiguousarray(grid, dtype=np.int32)
        self._check(self.lib.pmfem_set_aim(self.h, _ptr(g), int(order_p), int(near_boxes),
                                           float(z0_radius), int(precision)), "set_aim")

    def build(self):
        self._check(self.lib.pmfem_build(self.h), "build")
        n = _I64()
        self._check(self.lib.pmfem_query(self.h, ctypes.byref(n), None, None, None), "query")
        self.n = int(n.value)

    @classmethod
    def from_problem(cls, prob, device=0, stream=None, order_p=None, near_boxes=None,
                     z0_radius=None, precision=0):
        ctx = cls(device, stream)
        ctx.set_mesh(prob.xyz, prob.tets, prob.region)
        ctx.set_materials(prob.Ms, prob.Aex)
        ctx.set_periodicity(prob.periodic, prob.L)
        ctx.set_aim(prob.grid, prob.order_p if order_p is None else order_p,
                    prob.near_boxes if near_boxes is None else near_boxes,
                    prob.z0_radius if z0_radius is None else z0_radius, precision)
        ctx.build()
        return ctx

    def query(self):
        n = _I64()
        bpe = _D()
        self._check(self.lib.pmfem_query(self.h, ctypes.byref(n), None, None, ctypes.byref(bpe)),
                    "query")
        nn = self.export("unk_of_node").size
        uon = np.empty(nn, dtype=np.int64)
        nou = np.empty(n.value, dtype=np.int64)
        self._check(self.lib.pmfem_query(self.h, ctypes.byref(n), _ptr(uon), _ptr(nou), None),
                    "query")
        return int(n.value), uon, nou, float(bpe.value)

    def export(self, name):
        cnt = _I64()
        eb = _I32()
        self._check(self.lib.pmfem_export(self.h, name.encode(), None, ctypes.byref(cnt),
                                          ctypes.byref(eb)), f"export {name}")
        dt = {4: np.float32, 8: np.float64}[eb.value]
        if name in ("loc_rowptr", "loc_col", "z0_rowptr", "z0_col", "p_rowptr", "p_col",
                    "box_start", "sc_plan", "sc_list", "sc_lstart", "sc_tab"):
            dt = np.int32
        if name in ("unk_of_node", "node_of_unk"):
            dt = np.int64
        out = np.empty(cnt.value, dtype=dt)
        self._check(self.lib.pmfem_export(self.h, name.encode(), _ptr(out), ctypes.byref(cnt),
                                          ctypes.byref(eb)), f"export {name}")
        return out

    # -- evaluation ----------------------------------------------------------
    def heff(self, m, h, terms=TERM_EX | TERM_MS, h_applied=None):
        import torch
        ha = None
        if h_applied is not None:
            ha = np.ascontiguousarray(h_applied, dtype=np.float64)
        self._check(self.lib.pmfem_heff(self.h, _dev_ptr(m, torch.float32, (self.n, 3), "m"),
                                        _dev_ptr(h, torch.float32, (self.n, 3), "h"), int(terms),
                                        _ptr(ha)), "heff")
        return h

    def heff_parts(self, m, h, q=None, u=None, hex=None):
        import torch

        def opt(t, shape, name):
            return None if t is None else _dev_ptr(t, torch.float32, shape, name)
        self._check(self.lib.pmfem_heff_parts(self.h, _dev_ptr(m, torch.float32, (self.n, 3), "m"),
                                              _dev_ptr(h, torch.float32, (self.n, 3), "h"),
                                              opt(q, (self.n,), "q"), opt(u, (self.n,), "u"),
                                              opt(hex, (self.n, 3), "hex")), "heff_parts")

    def grid_convolve(self, qg, ug):
        import torch
        info = self.export("grid_info")
        shape = (int(info[2]), int(info[1]), int(info[0]))
        self._check(self.lib.pmfem_grid_convolve(self.h, _dev_ptr(qg, torch.float32, shape, "qg"),
                                                 _dev_ptr(ug, torch.float32, shape, "ug")),
                    "grid_convolve")

    def grid_convolve_noalloc(self, qg, ug):
        import torch
        info = self.export("grid_info")
        shape = (int(info[2]), int(info[1]), int(info[0]))
        self._check(self.lib.pmfem_grid_convolve_noalloc(
            self.h, _dev_ptr(qg, torch.float32, shape, "qg"),
            _dev_ptr(ug, torch.float32, shape, "ug")), "grid_convolve_noalloc")

    def llg_step(self, m64, dt, alpha, n_steps=1, h_applied=None):
        import torch
        ha = None if h_applied is None else np.ascontiguousarray(h_applied, dtype=np.float64)
        self._check(self.lib.pmfem_llg_step(self.h, _dev_ptr(m64, torch.float64, (self.n, 3), "m"),
                                            float(dt), float(alpha), int(n_steps), _ptr(ha)),
                    "llg_step")

    def llg_step_graph(self, m64, dt, alpha, n_steps=1, h_applied=None):
        """RK4 steps as launches of a captured HIP graph of one step."""
        import torch
        ha = None if h_applied is None else np.ascontiguousarray(h_applied, dtype=np.float64)
        self._check(self.lib.pmfem_llg_step_graph(
            self.h, _dev_ptr(m64, torch.float64, (self.n, 3), "m"), float(dt), float(alpha),
            int(n_steps), _ptr(ha)), "llg_step_graph")

    def llg_implicit(self, m64, dt, alpha, n_steps=1, terms=TERM_EX | TERM_MS, h_applied=None,
                     tol=0.0, krylov_dim=0):
        """Implicit midpoint steps; returns (Newton iterations, Krylov iterations)."""
        import torch
        ha = None if h_applied is None else np.ascontiguousarray(h_applied, dtype=np.float64)
        its = np.zeros(2, dtype=np.int32)
        self._check(self.lib.pmfem_llg_implicit(
            self.h, _dev_ptr(m64, torch.float64, (self.n, 3), "m"), float(dt), float(alpha),
            int(n_steps), int(terms), _ptr(ha), float(tol), int(krylov_dim), _ptr(its)),
            "llg_implicit")
        return int(its[0]), int(its[1])

    def llg_implicit_adaptive(self, m64, t_end, dt0, alpha, lte_tol=1e-6, terms=TERM_EX | TERM_MS,
                              h_applied=None, newton_tol=0.0, krylov_dim=0, max_steps=0,
                              log_steps=0, scheme="midpoint"):
        """Adaptive implicit steps (scheme "midpoint" or "bdf2") from 0 to
        t_end; returns a dict with the accepted and rejected steps, Newton and
        Krylov iterations, the proposed next step, the step sizes of the first
        log_steps attempts ("attempts", negative where rejected) and those of
        the accepted ones ("dts")."""
        import torch
        fn = {"midpoint": self.lib.pmfem_llg_implicit_adaptive,
              "bdf2": self.lib.pmfem_llg_bdf2_adaptive}[scheme]
        ha = None if h_applied is None else np.ascontiguousarray(h_applied, dtype=np.float64)
        st = np.zeros(5, dtype=np.int32)
        dt = np.array([float(dt0)], dtype=np.float64)
        log = np.zeros(max(int(log_steps), 1), dtype=np.float64)
        self._check(fn(
            self.h, _dev_ptr(m64, torch.float64, (self.n, 3), "m"), float(t_end),
            _ptr(dt), float(alpha), int(terms), _ptr(ha), float(lte_tol),
            float(newton_tol), int(krylov_dim), int(max_steps), _ptr(st),
            _ptr(log) if log_steps else None, int(log_steps)), "llg_implicit_adaptive")
        att = log[:min(int(st[0] + st[1] + st[2]), int(log_steps))].copy()
        return dict(accepted=int(st[0]), rejected=int(st[1] + st[2]), rejected_error=int(st[1]),
                    rejected_newton=int(st[2]), newton=int(st[3]), krylov=int(st[4]),
                    dt_next=float(dt[0]), attempts=att, dts=att[att > 0])

    # -- learned surrogate of the grid convolution -------------------------
    def _grid_shape(self):
        info = self.export("grid_info")
        return (int(info[2]), int(info[1]), int(info[0]))

    def surrogate_init(self, depth=6, seed=0, bf16_activations=False):
        self._check(self.lib.pmfem_surrogate_init(self.h, int(depth), int(seed),
                                                  int(bool(bf16_activations))), "surrogate_init")
        self.surrogate_depth = int(depth)

    def surrogate_param_count(self):
        n = _I64(0)
        self._check(self.lib.pmfem_surrogate_param_count(self.h, ctypes.byref(n)),
                    "surrogate_param_count")
        return int(n.value)

    def surrogate_set_params(self, params, scales=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        sc = None if scales is None else np.ascontiguousarray(scales, dtype=np.float64)
        self._check(self.lib.pmfem_surrogate_set_params(self.h, _ptr(p), p.size, _ptr(sc)),
                    "surrogate_set_params")

    def surrogate_get_params(self):
        """(parameter vector, (s_in, s_out))"""
        p = np.empty(self.surrogate_param_count(), np.float32)
        sc = np.zeros(2, np.float64)
        self._check(self.lib.pmfem_surrogate_get_params(self.h, _ptr(p), p.size, _ptr(sc)),
                    "surrogate_get_params")
        return p, (float(sc[0]), float(sc[1]))

    def surrogate_apply(self, qg, ug):
        import torch
        shape = self._grid_shape()
        self._check(self.lib.pmfem_surrogate_apply(
            self.h, _dev_ptr(qg, torch.float32, shape, "qg"),
            _dev_ptr(ug, torch.float32, shape, "ug")), "surrogate_apply")

    def surrogate_profile(self, qg, ug, reps=10):
        """Mean milliseconds of each layer over reps applications."""
        import torch
        shape = self._grid_shape()
        ms = np.zeros(self.surrogate_depth, np.float64)
        self._check(self.lib.pmfem_surrogate_profile(
            self.h, _dev_ptr(qg, torch.float32, shape, "qg"),
            _dev_ptr(ug, torch.float32, shape, "ug"), int(reps), _ptr(ms)), "surrogate_profile")
        return ms

    def surrogate_loss_grad(self, qg, tg):
        """(loss, gradient vector) of one forward/backward pass."""
        import torch
        shape = self._grid_shape()
        g = np.empty(self.surrogate_param_count(), np.float32)
        loss = ctypes.c_double(0.0)
        self._check(self.lib.pmfem_surrogate_loss_grad(
            self.h, _dev_ptr(qg, torch.float32, shape, "qg"),
            _dev_ptr(tg, torch.float32, shape, "tg"), ctypes.byref(loss), _ptr(g), g.size),
            "surrogate_loss_grad")
        return float(loss.value), g

    def surrogate_texture(self, m64, kind, seed=0):
        import torch
        self._check(self.lib.pmfem_surrogate_texture(
            self.h, int(kind), int(seed), _dev_ptr(m64, torch.float64, (self.n, 3), "m")),
            "surrogate_texture")

    def surrogate_train(self, n_pairs, lr=1e-3, seed=0, kinds=0b111):
        """Trains on n_pairs AIM pairs; returns the loss of every pair."""
        log = np.zeros(max(1, int(n_pairs)), np.float64)
        self._check(self.lib.pmfem_surrogate_train(self.h, int(n_pairs), float(lr), int(seed),
                                                   int(kinds), _ptr(log)), "surrogate_train")
        return log[:int(n_pairs)]

    def surrogate_enable(self, on=True):
        self._check(self.lib.pmfem_surrogate_enable(self.h, int(bool(on))), "surrogate_enable")

    def llg_step_judged(self, m64, dt, alpha, n_steps, check_every=50, tol=1e-3,
                        h_applied=None):
        """RK4 steps with the surrogate, judged by the plain AIM; returns a dict
        (checks, max_error, last_error, fallback_step)."""
        import torch
        ha = None if h_applied is None else np.ascontiguousarray(h_applied, dtype=np.float64)
        rep = np.zeros(4, np.float64)
        self._check(self.lib.pmfem_llg_step_judged(
            self.h, _dev_ptr(m64, torch.float64, (self.n, 3), "m"), float(dt), float(alpha),
            int(n_steps), _ptr(ha), int(check_every), float(tol), _ptr(rep)), "llg_step_judged")
        return dict(checks=int(rep[0]), max_error=float(rep[1]), last_error=float(rep[2]),
                    fallback_step=int(rep[3]))

    def autotune(self, trials=20):
        """Pick the fastest kernel forms; returns ({stage: form}, ms per evaluation)."""
        ch = np.zeros(4, dtype=np.int32)
        ms = _D()
        self._check(self.lib.pmfem_autotune(self.h, int(trials), _ptr(ch), ctypes.byref(ms)),
                    "autotune")
        return dict(zip(("anterp", "interp", "fft", "spmv"), ch.tolist())), ms.value

    def energy(self, m64):
        import torch
        a, b = _D(), _D()
        self._check(self.lib.pmfem_energy(self.h, _dev_ptr(m64, torch.float64, (self.n, 3), "m"),
                                          ctypes.byref(a), ctypes.byref(b)), "energy")
        return a.value, b.value

    def profile_begin(self, max_calls):
        self._check(self.lib.pmfem_profile_begin(self.h, int(max_calls)), "profile_begin")

    def profile_end(self):
        nk = _I32()
        ms = np.zeros(16)
        cnt = np.zeros(16, dtype=np.int32)
        names = (ctypes.c_char * 32 * 16)()
        self._check(self.lib.pmfem_profile_end(self.h, ctypes.byref(nk), _ptr(ms), _ptr(cnt),
                                               ctypes.cast(names, _P)), "profile_end")
        return {names[k].value.decode(): (float(ms[k]), int(cnt[k])) for k in range(nk.value)}



class Batch:
    """Independent built contexts on one device, evaluated with one launch per
    stage for all of them. Vectors are packed in cell order (see offsets)."""

    def __init__(self, contexts, stream=None, spmv_lanes=0):
        self.lib = load_library()
        self.cells = list(contexts)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(self.cells[0].device).cuda_stream
        arr = (_P * len(self.cells))(*[c.h for c in self.cells])
        h = _P()
        rc = self.lib.pmfem_batch_create(ctypes.byref(h), len(self.cells), ctypes.cast(arr, _P),
                                         _P(stream) if stream else None, int(spmv_lanes))
        self.h = h if h.value else None
        if rc:
            msg = self.lib.pmfem_batch_last_error(h) if h.value else b""
            self.close()
            raise PmfemError(rc, f"pmfem_batch_create: {msg.decode() if msg else ''}")
        n = _I64()
        self.offsets = np.zeros(len(self.cells) + 1, dtype=np.int64)
        bpe = _D()
        self._check(self.lib.pmfem_batch_query(self.h, ctypes.byref(n), _ptr(self.offsets),
                                               ctypes.byref(bpe)), "batch_query")
        self.n = int(n.value)
        self.bytes_per_eval = float(bpe.value)

    def _check(self, rc, what):
        if rc:
            msg = self.lib.pmfem_batch_last_error(self.h)
            raise PmfemError(rc, f"{what}: {msg.decode() if msg else ''}")

    def heff(self, m, h, terms=TERM_EX | TERM_MS):
        import torch
        self._check(self.lib.pmfem_batch_heff(self.h, _dev_ptr(m, torch.float32, (self.n, 3), "m"),
                                              _dev_ptr(h, torch.float32, (self.n, 3), "h"),
                                              int(terms)), "batch_heff")

    def llg_step(self, m64, dt, alpha, n_steps=1):
        import torch
        self._check(self.lib.pmfem_batch_llg_step(
            self.h, _dev_ptr(m64, torch.float64, (self.n, 3), "m"), float(dt), float(alpha),
            int(n_steps)), "batch_llg_step")

    def llg_step_graph(self, m64, dt, alpha, n_steps=1):
        """RK4 steps of the batch as launches of a captured HIP graph of one step."""
        import torch
        self._check(self.lib.pmfem_batch_llg_step_graph(
            self.h, _dev_ptr(m64, torch.float64, (self.n, 3), "m"), float(dt), float(alpha),
            int(n_steps)), "batch_llg_step_graph")

    def close(self):
        if getattr(self, "h", None):
            self.lib.pmfem_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
