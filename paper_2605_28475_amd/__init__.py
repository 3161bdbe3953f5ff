"""wefq: Wigner-Eckart factorized Boltzmann collision operator on MI355X.

Thin Python binding over libwefq.so (C ABI in include/wefq.h).  PyTorch is used
only to hold device memory and to name the HIP stream; every step of the
computation runs in the library's HIP kernels.  There is no CPU fallback: the
calls raise if the HIP library is missing.
"""
import ctypes
import math

import numpy as np

from . import _lib
from ._lib import (BF16X3, FP32, FP64, FP64_NAIVE, HARD_SPHERE, MAXWELL, RK_CLASSIC4, RK_EULER, RK_HEUN,
                   RK_SSP3, VHS, WefqError)

MODELS = {"maxwell": MAXWELL, "mm": MAXWELL, "hard_sphere": HARD_SPHERE, "hs": HARD_SPHERE, "vhs": VHS}
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp64_naive": FP64_NAIVE,
              "bilinear": _lib.PREP_BILINEAR, "radial": _lib.PREP_RADIAL}
RK_SCHEMES = {"euler": RK_EULER, "heun": RK_HEUN, "ssp3": RK_SSP3, "rk4": RK_CLASSIC4}


def num_modes(K, L):
    return (K + 1) * (L + 1) ** 2


def _check_tensor(name, t, want, rows, N, device=None):
    """Refuse a tensor the library would read or write out of bounds: dtype, CUDA device,
    unit stride in the last dimension, at least `rows` rows of exactly N modes."""
    if t.dtype != want or t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError(f"{name} must be a CUDA {want} tensor on {device or 'the GPU'}")
    if t.dim() != 2 or t.shape[1] != N or t.shape[0] < rows:
        raise ValueError(f"{name} must have shape ({rows}, {N}); got {tuple(t.shape)}")
    if t.stride(-1) != 1 or (t.shape[0] > 1 and t.stride(0) < N):
        raise ValueError(f"{name} must have unit stride in the last dimension and rows at least N apart")


def _stream_ptr(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


class Core:
    """A built radial core (wefq_build_core) resident on one GPU.

    beta: Legendre coefficients of the angular factor of B(u, cos chi) = b0 u^gamma
    beta(cos chi), or None for the isotropic kernel.  rad_pad, ang_pad: extra points in the
    radial and angular Gauss rules beyond the exact counts (self-convergence studies)."""

    def __init__(self, model, K, L, gamma=None, b0=0.0, precisions=("fp64", "fp32", "bf16x3"),
                 device=0, stream=None, beta=None, rad_pad=0, ang_pad=0):
        m = MODELS[model] if isinstance(model, str) else int(model)
        if gamma is None:
            gamma = {MAXWELL: 0.0, HARD_SPHERE: 1.0}.get(m, 0.5)
        mask = 0
        for p in precisions:
            mask |= PRECISIONS[p] if isinstance(p, str) else int(p)
        coef = [] if beta is None else [float(b) for b in beta]
        arr = (ctypes.c_double * max(1, len(coef)))(*coef)
        desc = _lib.CoreDesc(m, float(gamma), float(b0), int(K), int(L), mask, int(device),
                             len(coef), ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)) if coef else None,
                             int(rad_pad), int(ang_pad))
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().wefq_build_core(ctypes.byref(desc), _stream_ptr(stream, device), ctypes.byref(h)))
        self._adopt(h, device)

    def _adopt(self, h, device):
        self._h = h
        self.device = device
        info = _lib.CoreInfo()
        _lib.check(_lib.lib().wefq_core_info_get(h, ctypes.byref(info)))
        self.info = {name: getattr(info, name) for name, _ in _lib.CoreInfo._fields_ if name != "beta"}
        self.N = int(info.N)
        self.K = int(info.NK) - 1
        self.L = int(round(math.sqrt(int(info.NQ)))) - 1
        self.model, self.gamma = int(info.model), float(info.gamma)
        nb = int(info.n_beta)
        self.beta = tuple(float(info.beta[j]) for j in range(nb)) if nb else None

    @classmethod
    def load(cls, path, precisions=("fp64", "fp32", "bf16x3"), device=0, stream=None):
        """A core rebuilt from a file written by save() (wefq_core_load), without the quadrature."""
        mask = 0
        for p in precisions:
            mask |= PRECISIONS[p] if isinstance(p, str) else int(p)
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().wefq_core_load(str(path).encode(), mask, int(device), _stream_ptr(stream, device),
                                             ctypes.byref(h)))
        core = cls.__new__(cls)
        core._adopt(h, device)
        return core

    def save(self, path):
        """Write the core (parameters and raw radial tensor) to a file (wefq_core_save)."""
        _lib.check(_lib.lib().wefq_core_save(self._h, str(path).encode()))

    @property
    def handle(self):
        return self._h

    def download_R(self):
        NK = self.K + 1
        out = np.empty((self.info["N_T"], NK, NK, NK), dtype=np.float64)
        _lib.check(_lib.lib().wefq_core_download_R(self._h, out.ctypes.data_as(ctypes.c_void_p), out.size))
        return out

    def _prec(self, f, precision):
        import torch
        if precision is None:
            return FP64 if f.dtype == torch.float64 else FP32
        return PRECISIONS[precision] if isinstance(precision, str) else int(precision)

    def apply_Q(self, f, out=None, precision=None, stream=None):
        """Q(f, f) for a [B, N] (or [N]) device tensor; returns a new tensor unless out is given."""
        import torch
        squeeze = f.dim() == 1
        f2 = f.unsqueeze(0) if squeeze else f
        prec = self._prec(f2, precision)
        want = torch.float64 if prec in (FP64, FP64_NAIVE) else torch.float32
        _check_tensor("f", f2, want, f2.shape[0], self.N)
        B = f2.shape[0]
        if out is None:
            out = torch.empty((B, self.N), dtype=want, device=f2.device)
        else:
            out = out.unsqueeze(0) if (squeeze and out.dim() == 1) else out
            _check_tensor("out", out, want, B, self.N, f2.device)
        _lib.check(_lib.lib().wefq_apply_Q(self._h, prec, ctypes.c_void_p(f2.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), B, f2.stride(0) if B > 1 else f2.shape[1],
                                           out.stride(0) if B > 1 else out.shape[1],
                                           _stream_ptr(stream, f2.device)))
        return out[0] if squeeze else out

    def mode_index(self, k, l, m):
        """Flat index n = (l^2 + l + m) NK + k of phi_klm in a coefficient vector (wefq_mode_index)."""
        n = ctypes.c_int64()
        _lib.check(_lib.lib().wefq_mode_index(self._h, int(k), int(l), int(m), ctypes.byref(n)))
        return n.value

    def radial_workspace_bytes(self, chunk):
        """Workspace bytes of apply_Q_radial for chunks of `chunk` cells (wefq_radial_workspace)."""
        n = ctypes.c_int64()
        _lib.check(_lib.lib().wefq_radial_workspace(self._h, int(chunk), ctypes.byref(n)))
        return n.value

    def apply_Q_radial(self, f, out=None, work=None, chunk=None, stream=None):
        """Q(f, f) in FP64 by the radial-first ordering (wefq_apply_Q_radial; core built with
        "radial").  work: a uint8 device tensor; by default one is allocated for chunks of
        `chunk` cells (default: the batch, capped so that the workspace stays under 1 GiB)."""
        import torch
        if f.dim() != 2:
            raise ValueError("f must be a [B, N] tensor")
        B = f.shape[0]
        _check_tensor("f", f, torch.float64, B, self.N)
        if out is None:
            out = torch.empty((B, self.N), dtype=torch.float64, device=f.device)
        else:
            _check_tensor("out", out, torch.float64, B, self.N, f.device)
        if work is not None and (work.device != f.device or not work.is_contiguous()):
            raise ValueError("work must be a contiguous tensor on the device of f")
        if work is None:
            per64 = self.radial_workspace_bytes(64)
            if chunk is None:
                chunk = max(64, min(((B + 63) // 64) * 64, (1 << 30) // per64 * 64))
            work = torch.empty(self.radial_workspace_bytes(chunk), dtype=torch.uint8, device=f.device)
        _lib.check(_lib.lib().wefq_apply_Q_radial(self._h, ctypes.c_void_p(f.data_ptr()),
                                                  ctypes.c_void_p(out.data_ptr()), B, f.stride(0), out.stride(0),
                                                  ctypes.c_void_p(work.data_ptr()), work.numel(),
                                                  _stream_ptr(stream, f.device)))
        return out

    def dense_bytes(self):
        """Bytes of the dense weak-form tensor C (wefq_dense_bytes; needs the FP64 tables)."""
        n = ctypes.c_int64()
        _lib.check(_lib.lib().wefq_dense_bytes(self._h, ctypes.byref(n)))
        return n.value

    def dense_assemble(self, C=None, stream=None):
        """Assemble the dense tensor C = g R (wefq_dense_assemble) into a uint8 device tensor of
        dense_bytes() bytes (allocated here when None) and return it."""
        import torch
        nb = self.dense_bytes()
        if C is None:
            C = torch.empty(nb, dtype=torch.uint8, device=torch.device("cuda", self.device))
        elif C.device.type != "cuda" or not C.is_contiguous() or C.numel() * C.element_size() < nb:
            raise ValueError(f"C must be a contiguous device tensor of at least {nb} bytes")
        _lib.check(_lib.lib().wefq_dense_assemble(self._h, ctypes.c_void_p(C.data_ptr()), C.numel() * C.element_size(),
                                                  _stream_ptr(stream, C.device)))
        return C

    def apply_Q_dense(self, C, f, out=None, stream=None):
        """Q(f, f) in FP64 by the dense Cartesian contraction with an assembled C (wefq_apply_Q_dense)."""
        import torch
        if f.dim() != 2:
            raise ValueError("f must be a [B, N] tensor")
        B = f.shape[0]
        _check_tensor("f", f, torch.float64, B, self.N)
        if C.device != f.device or not C.is_contiguous():
            raise ValueError("C must be a contiguous tensor on the device of f")
        if out is None:
            out = torch.empty((B, self.N), dtype=torch.float64, device=f.device)
        else:
            _check_tensor("out", out, torch.float64, B, self.N, f.device)
        _lib.check(_lib.lib().wefq_apply_Q_dense(self._h, ctypes.c_void_p(C.data_ptr()), C.numel() * C.element_size(),
                                                 ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()), B,
                                                 f.stride(0) if B > 1 else self.N,
                                                 out.stride(0) if B > 1 else self.N, _stream_ptr(stream, f.device)))
        return out

    def apply_J(self, c, d, out=None, precision=None, stream=None):
        """Jacobian-vector product J(c) d = Q(c, d) + Q(d, c) for [B, N] device tensors."""
        return self._two_input("wefq_apply_J", c, d, out, precision, stream)

    def apply_Qfg(self, f, g, out=None, precision=None, stream=None):
        """Bilinear form Q(f, g) for [B, N] device tensors (core built with "bilinear")."""
        return self._two_input("wefq_apply_Qfg", f, g, out, precision, stream)

    def _two_input(self, fn, c, d, out, precision, stream):
        import torch
        squeeze = c.dim() == 1
        c2 = c.unsqueeze(0) if squeeze else c
        d2 = d.unsqueeze(0) if d.dim() == 1 else d
        prec = self._prec(c2, precision)
        want = torch.float64 if prec == FP64 else torch.float32
        B = c2.shape[0]
        _check_tensor("c", c2, want, B, self.N)
        _check_tensor("d", d2, want, B, self.N, c2.device)
        if d2.shape != c2.shape:
            raise ValueError("c and d must have the same shape")
        if out is None:
            out = torch.empty((B, self.N), dtype=want, device=c2.device)
        else:
            out = out.unsqueeze(0) if (squeeze and out.dim() == 1) else out
            _check_tensor("out", out, want, B, self.N, c2.device)
        ld = lambda t: t.stride(0) if B > 1 else t.shape[1]
        _lib.check(getattr(_lib.lib(), fn)(self._h, prec, ctypes.c_void_p(c2.data_ptr()),
                                           ctypes.c_void_p(d2.data_ptr()), ctypes.c_void_p(out.data_ptr()), B,
                                           ld(c2), ld(d2), ld(out), _stream_ptr(stream, c2.device)))
        return out[0] if squeeze else out

    def check_conservation(self, Q, precision=None, stream=None):
        import torch
        Q2 = Q.unsqueeze(0) if Q.dim() == 1 else Q
        prec = self._prec(Q2, precision)
        _check_tensor("Q", Q2, torch.float64 if prec in (FP64, FP64_NAIVE) else torch.float32, Q2.shape[0], self.N)
        res = ctypes.c_double()
        _lib.check(_lib.lib().wefq_check_conservation(self._h, prec, ctypes.c_void_p(Q2.data_ptr()), Q2.shape[0],
                                                      Q2.stride(0) if Q2.shape[0] > 1 else Q2.shape[1],
                                                      ctypes.byref(res), _stream_ptr(stream, Q2.device)))
        return res.value

    def rk_workspace_bytes(self, B, scheme="rk4", precision="fp32"):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        n = ctypes.c_int64()
        _lib.check(_lib.lib().wefq_rk_workspace(self._h, prec, RK_SCHEMES.get(scheme, scheme), int(B), ctypes.byref(n)))
        return n.value

    def rk_integrate(self, c, dt, nsteps, scheme="rk4", precision=None, work=None, check=True, stream=None):
        """Advance the [B, N] device tensor c in place by nsteps explicit Runge-Kutta steps
        of dc/dt = Q(c) (wefq_rk_integrate).  work: optional uint8 device tensor of at least
        rk_workspace_bytes(B) bytes (allocated here when None).  Returns the FP64 maximum of
        |Q| over the invariant rows of every stage evaluation when check is true."""
        import torch
        c2 = c.unsqueeze(0) if c.dim() == 1 else c
        prec = self._prec(c2, precision)
        want = torch.float64 if prec in (FP64, FP64_NAIVE) else torch.float32
        B = c2.shape[0]
        _check_tensor("c", c2, want, B, self.N)
        sch = RK_SCHEMES.get(scheme, scheme)
        need = self.rk_workspace_bytes(B, sch, prec)
        if work is None:
            work = torch.empty(need, dtype=torch.uint8, device=c2.device)
        elif work.device != c2.device or not work.is_contiguous():
            raise ValueError("work must be a contiguous tensor on the device of c")
        res = ctypes.c_double()
        _lib.check(_lib.lib().wefq_rk_integrate(self._h, prec, int(sch), ctypes.c_void_p(c2.data_ptr()), B,
                                                c2.stride(0) if B > 1 else c2.shape[1], float(dt), int(nsteps),
                                                ctypes.c_void_p(work.data_ptr()), work.numel(),
                                                ctypes.byref(res) if check else None, _stream_ptr(stream, c2.device)))
        return res.value if check else None

    def tune_set(self, precision, slots, block):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _lib.check(_lib.lib().wefq_tune_set(self._h, prec, int(slots), int(block)))

    def tune_get(self, precision):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        s, b = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.lib().wefq_tune_get(self._h, prec, ctypes.byref(s), ctypes.byref(b)))
        return s.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.check(_lib.lib().wefq_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def host_coo(L):
    """Real-Gaunt COO table from the library's host code (no GPU needed)."""
    n = ctypes.c_int64()
    _lib.check(_lib.lib().wefq_host_coo(L, ctypes.byref(n), None, None, None, None, None))
    cnt = n.value
    arrs = {k: np.empty(cnt, dtype=np.int32) for k in ("q1", "q2", "q3", "c")}
    g = np.empty(cnt, dtype=np.float64)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _lib.check(_lib.lib().wefq_host_coo(L, ctypes.byref(n), ptr(arrs["q1"]), ptr(arrs["q2"]), ptr(arrs["q3"]),
                                        ptr(arrs["c"]), ptr(g)))
    arrs["g"] = g
    return arrs


def host_gauss(kind, n, alpha=0.0):
    x = np.empty(n); w = np.empty(n)
    _lib.check(_lib.lib().wefq_host_gauss(kind, n, alpha, x.ctypes.data_as(ctypes.c_void_p),
                                          w.ctypes.data_as(ctypes.c_void_p)))
    return x, w


PROBES = {"mfma_f32": _lib.PROBE_MFMA_F32, "mfma_f64": _lib.PROBE_MFMA_F64, "mfma_bf16": _lib.PROBE_MFMA_BF16,
          "valu_f32": _lib.PROBE_VALU_F32, "valu_f64": _lib.PROBE_VALU_F64}


def peak_probe(kind, device=0, stream=None):
    """Measured attainable rate (TFLOP/s) of one kind of arithmetic on the device."""
    out = ctypes.c_double()
    _lib.check(_lib.lib().wefq_peak_probe(device, PROBES[kind], ctypes.byref(out), _stream_ptr(stream, device)))
    return out.value


class Plan:
    """Uneven batch in one persistent, graph-captured launch (wefq_plan_*).

    segments: list of (core, f, Q) or (core, f, Q, slots) with f, Q CUDA tensors of
    shape [B_i, N_i].  The plan keeps references to the tensors and cores.
    """

    def __init__(self, segments, precision="fp32", block=512, stream=None):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        arr = (_lib.Segment * len(segments))()
        self._keep = []
        dev = None
        import torch
        want = torch.float64 if prec == FP64 else torch.float32
        for i, seg in enumerate(segments):
            core, f, Q = seg[:3]
            slots = seg[3] if len(seg) > 3 else 0
            B = f.shape[0]
            _check_tensor(f"segment {i} f", f, want, B, core.N, dev)
            _check_tensor(f"segment {i} Q", Q, want, B, core.N, f.device)
            arr[i] = _lib.Segment(core.handle, prec, int(slots), f.data_ptr(), Q.data_ptr(), B,
                                  f.stride(0) if B > 1 else f.shape[1], Q.stride(0) if B > 1 else Q.shape[1])
            self._keep.append((core, f, Q))
            dev = f.device
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().wefq_plan_create(len(segments), ctypes.cast(arr, ctypes.c_void_p), int(block),
                                               _stream_ptr(stream, dev), ctypes.byref(h)))
        self._h = h
        self.device = dev
        items, lds, grid = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _lib.check(_lib.lib().wefq_plan_info(h, ctypes.byref(items), ctypes.byref(lds), ctypes.byref(grid)))
        self.info = {"work_items": items.value, "lds_bytes": lds.value, "grid": grid.value, "block": block}

    def launch(self, stream=None, graph=True):
        fn = _lib.lib().wefq_plan_launch if graph else _lib.lib().wefq_plan_launch_direct
        _lib.check(fn(self._h, _stream_ptr(stream, self.device)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.check(_lib.lib().wefq_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Runner:
    """One persistent launch per call over any mix of segments (wefq_runner_*): the scheduling
    tick of the continuous-batching server.  Segments are (core, f, Q) with f, Q CUDA tensors of
    shape [B_i, N_i]; they must stay alive until the launch has completed (the caller records
    an event after launch())."""

    def __init__(self, device=0, precision="fp32", max_segments=4096, max_items=1 << 20, block=512):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.prec = prec
        self.device = device
        self.max_segments = int(max_segments)
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().wefq_runner_create(int(device), prec, self.max_segments, int(max_items), int(block),
                                                 ctypes.byref(h)))
        self._h = h
        self._arr = (_lib.Segment * self.max_segments)()

    def launch(self, segments, stream=None):
        import torch
        want = torch.float64 if self.prec == FP64 else torch.float32
        n = len(segments)
        if n > self.max_segments:
            raise ValueError(f"at most {self.max_segments} segments per launch")
        dev = None
        for i, (core, f, Q) in enumerate(segments):
            B = f.shape[0]
            _check_tensor(f"segment {i} f", f, want, B, core.N, dev)
            _check_tensor(f"segment {i} Q", Q, want, B, core.N, f.device)
            dev = f.device
            self._arr[i] = _lib.Segment(core.handle, self.prec, 0, f.data_ptr(), Q.data_ptr(), B,
                                        f.stride(0) if B > 1 else core.N, Q.stride(0) if B > 1 else core.N)
        _lib.check(_lib.lib().wefq_runner_launch(self._h, n, ctypes.cast(self._arr, ctypes.c_void_p),
                                                 _stream_ptr(stream, dev if dev is not None else self.device)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.check(_lib.lib().wefq_runner_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
