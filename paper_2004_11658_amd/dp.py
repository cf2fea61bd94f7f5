"""Thin Python binding of libdp.so (the C ABI in include/dp.h).

Argument marshalling only: torch supplies device memory and the current HIP stream;
every step of the computation runs in the library's HIP kernels.  Importing this
module raises if the library has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdp.so")

DP_OK = 0
DP_WARN_SEL_OVERFLOW = 1
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
STAGES = {"nlist": 0, "embed_fwd": 1, "fit": 2, "embed_bwd": 3, "reduce": 4, "md": 5, "fallback": 6}


class DPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libdp error %d: %s" % (code, msg))
        self.code = code


class _Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("deterministic", C.c_int32), ("skin", C.c_double)]


class _NptOptions(C.Structure):
    _fields_ = [("pressure_bar", C.c_double), ("tau_p_fs", C.c_double), ("temperature_K", C.c_double),
                ("tau_t_fs", C.c_double), ("min_scale", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdp.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2004_11658_amd.build)")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "dp_init": ([C.c_char_p, P, P], C.c_int),
        "dp_free": ([P], None),
        "dp_model_info": ([P, P, P, P, P, P, P], C.c_int),
        "dp_device_bytes": ([P, P], C.c_int),
        "dp_upload": ([P, P, SZ, P], C.c_int),
        "dp_student_bytes": ([P, P], C.c_int),
        "dp_workspace_size": ([P, I32, P, P, P], C.c_int),
        "dp_compute": ([P, I64, P, P, P, P, P, P, P, P, SZ, P], C.c_int),
        "dp_compute_batch": ([P, I32, P, P, P, P, P, P, P, P, P, SZ, P], C.c_int),
        "dp_compute_atomic": ([P, I64, P, P, P, P, P, P, P, P, P, SZ, P], C.c_int),
        "dp_compute_local_workspace_size": ([P, I64, I64, P, P], C.c_int),
        "dp_compute_local": ([P, I64, I64, P, P, P, P, P, P, P, P, P, SZ, P], C.c_int),
        "dp_nlist": ([P, I64, P, P, P, P, P, P, P, SZ, P], C.c_int),
        "dp_descriptor": ([P, I64, P, P, P, P, P, P, SZ, P], C.c_int),
        "dp_status": ([P, P, P, P, P], C.c_int),
        "dp_fallback_rows": ([P, P, P, P], C.c_int),
        "dp_md_run": ([P, I64, P, P, P, P, P, D, I32, I32, P, P, P, SZ, P], C.c_int),
        "dp_md_npt_workspace_size": ([P, I64, P, D, P], C.c_int),
        "dp_md_run_npt": ([P, I64, P, P, P, P, P, P, D, I32, I32, P, P, P, P, P, SZ, P], C.c_int),
        "dp_profile": ([P, I32], C.c_int),
        "dp_profile_stages": ([P, C.c_uint32], C.c_int),
        "dp_set_params": ([P, P, P], C.c_int),
        "dp_get_params": ([P, P, P], C.c_int),
        "dp_param_grad_workspace_size": ([P, I32, P, P, I64, P], C.c_int),
        "dp_param_grad": ([P, I32, P, P, P, P, P, P, P, I64, P, SZ, P], C.c_int),
        "dp_student_samples_workspace_size": ([P, I64, P, P], C.c_int),
        "dp_student_samples": ([P, I32, I32, I64, P, P, P, P, D, P, I64, P, P, SZ, P], C.c_int),
        "dp_embed_eval": ([P, I32, I32, I64, P, P, P], C.c_int),
        "dp_student_scratch_size": ([I32, I32, I64, P], C.c_int),
        "dp_student_loss_grad": ([I32, I32, I64, P, P, P, P, P, P, SZ, P], C.c_int),
        "dp_adam": ([I64, P, P, P, P, I32, D, D, D, D, P], C.c_int),
        "dp_student_lsq_scratch_size": ([I32, I32, I64, P], C.c_int),
        "dp_student_lsq": ([I32, I32, I64, P, P, P, D, P, SZ, P], C.c_int),
        "dp_set_student": ([P, I32, P, P, P, I32, P, SZ, P], C.c_int),
        "dp_profile_read": ([P, I32, P, P], C.c_int),
        "dp_strerror": ([C.c_int], C.c_char_p),
        "dp_last_error": ([P], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


_lib = _load()


def lib():
    return _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _box9(box) -> np.ndarray:
    b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(-1, 9))
    return b


class DPModel:
    """A DP-SE model on the current HIP device."""

    def __init__(self, model_path: str, precision: str = "fp64", skin: float = 0.0,
                 deterministic: bool = False):
        opt = _Options(PRECISIONS[precision], 1 if deterministic else 0, float(skin))
        h = C.c_void_p()
        rc = _lib.dp_init(model_path.encode(), C.byref(opt), C.byref(h))
        if rc != DP_OK:
            raise DPError(rc, _lib.dp_last_error(None).decode())
        self.h = h
        self.precision = precision
        nt, nm, M, m2 = (C.c_int32() for _ in range(4))
        rcut, npar = C.c_double(), C.c_int64()
        _lib.dp_model_info(h, C.byref(nt), C.byref(nm), C.byref(M), C.byref(m2), C.byref(rcut),
                           C.byref(npar))
        self.ntypes, self.nm, self.M, self.m2 = nt.value, nm.value, M.value, m2.value
        self.rc, self.nparams = rcut.value, npar.value
        self._ws = None
        self._pg_ws = None    # parameter-gradient workspace (reused between calls)
        self.device = torch.device("cuda", torch.cuda.current_device())
        # the weight region is caller memory: a torch buffer the library lays its layouts in
        nb = C.c_size_t()
        self._check(_lib.dp_device_bytes(h, C.byref(nb)))
        self._weights = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=self.device)
        self._check(_lib.dp_upload(h, _ptr(self._weights), self._weights.numel(), _stream()))
        self._student_mem = None

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:   # _lib is gone at interpreter exit
            _lib.dp_free(h)
            self.h = None

    # ------------------------------------------------------------------ helpers
    def _check(self, rc: int):
        if rc < 0:
            raise DPError(rc, _lib.dp_last_error(self.h).decode())
        return rc

    def workspace(self, offsets: np.ndarray, boxes: np.ndarray) -> torch.Tensor:
        nb = C.c_size_t()
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        boxes = _box9(boxes)
        self._check(_lib.dp_workspace_size(self.h, len(offsets) - 1, offsets.ctypes.data_as(C.c_void_p),
                                           boxes.ctypes.data_as(C.c_void_p), C.byref(nb)))
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = torch.empty(int(nb.value * 1.1) + 4096, dtype=torch.uint8, device=self.device)
        return self._ws

    def fallback_rows(self) -> int:
        """Neighbour rows the last force evaluation handed from the student nets to the
        full net (dp_fallback_rows)."""
        rows = C.c_int64()
        self._check(_lib.dp_fallback_rows(self.h, _ptr(self._ws), _stream(), C.byref(rows)))
        return int(rows.value)

    def status(self) -> int:
        flags, det = C.c_int32(), C.c_int64()
        rc = _lib.dp_status(self.h, _ptr(self._ws), _stream(), C.byref(flags), C.byref(det))
        self._check(rc)
        return rc

    @staticmethod
    def _dev(x, dtype):
        t = torch.as_tensor(x)
        if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
            t = t.to(device="cuda", dtype=dtype).contiguous()
        return t

    # ------------------------------------------------------------------ compute
    def compute(self, coords, types, box, atom_energy: bool = False, check: bool = True):
        """E [1], F [N][3], W [3][3] (and E_i [N]) of one frame; device tensors."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        b = _box9(box)
        ws = self.workspace(np.array([0, n]), b)
        E = torch.empty(1, dtype=torch.float64, device=x.device)
        F = torch.empty(n, 3, dtype=torch.float64, device=x.device)
        W = torch.empty(9, dtype=torch.float64, device=x.device)
        Ei = torch.empty(n, dtype=torch.float64, device=x.device) if atom_energy else None
        self._check(_lib.dp_compute(self.h, n, _ptr(x), _ptr(t), b.ctypes.data_as(C.c_void_p), _ptr(E),
                                    _ptr(F), _ptr(W), _ptr(Ei), _ptr(ws), ws.numel(), _stream()))
        if check:
            self.status()
        return (E, F, W.view(3, 3), Ei) if atom_energy else (E, F, W.view(3, 3))

    def compute_atomic(self, coords, types, box, check: bool = True):
        """E [1], F [N][3], W [3][3], E_i [N], W_i [N][3][3] of one periodic frame."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        b = _box9(box)
        ws = self.workspace(np.array([0, n]), b)
        E = torch.empty(1, dtype=torch.float64, device=x.device)
        F = torch.empty(n, 3, dtype=torch.float64, device=x.device)
        W = torch.empty(9, dtype=torch.float64, device=x.device)
        Ei = torch.empty(n, dtype=torch.float64, device=x.device)
        Wi = torch.empty(n, 9, dtype=torch.float64, device=x.device)
        self._check(_lib.dp_compute_atomic(self.h, n, _ptr(x), _ptr(t), b.ctypes.data_as(C.c_void_p), _ptr(E),
                                           _ptr(F), _ptr(W), _ptr(Ei), _ptr(Wi), _ptr(ws), ws.numel(), _stream()))
        if check:
            self.status()
        return E, F, W.view(3, 3), Ei, Wi.view(n, 3, 3)

    def compute_local(self, coords, types, nlocal: int, bounds=None, check: bool = True):
        """Engine-facing evaluation: atoms [0, nlocal) are local, the rest caller-supplied
        ghosts (no periodic box).  Returns E [1] (local atoms), F [nlocal + nghost][3]
        (forces on locals and ghosts), W [3][3], E_i [nlocal], W_i [nlocal][3][3]."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        if bounds is None:
            xc = x.detach().cpu().numpy()
            bounds = np.concatenate([xc.min(axis=0), xc.max(axis=0)])
        bd = np.ascontiguousarray(bounds, dtype=np.float64).reshape(6)
        nb = C.c_size_t()
        self._check(_lib.dp_compute_local_workspace_size(self.h, int(nlocal), int(n - nlocal),
                                                         bd.ctypes.data_as(C.c_void_p), C.byref(nb)))
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = torch.empty(int(nb.value * 1.1) + 4096, dtype=torch.uint8, device=self.device)
        ws = self._ws
        E = torch.empty(1, dtype=torch.float64, device=x.device)
        F = torch.empty(n, 3, dtype=torch.float64, device=x.device)
        W = torch.empty(9, dtype=torch.float64, device=x.device)
        Ei = torch.empty(nlocal, dtype=torch.float64, device=x.device)
        Wi = torch.empty(nlocal, 9, dtype=torch.float64, device=x.device)
        self._check(_lib.dp_compute_local(self.h, int(nlocal), int(n - nlocal), _ptr(x), _ptr(t),
                                          bd.ctypes.data_as(C.c_void_p), _ptr(E), _ptr(F), _ptr(W), _ptr(Ei),
                                          _ptr(Wi), _ptr(ws), ws.numel(), _stream()))
        if check:
            self.status()
        return E, F, W.view(3, 3), Ei, Wi.view(nlocal, 3, 3)

    def compute_batch(self, coords, types, offsets: Sequence[int], boxes, atom_energy: bool = False,
                      check: bool = True):
        """Energies [nf], forces [N][3], virials [nf][3][3] of a ragged batch."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        nf = len(off) - 1
        b = _box9(boxes)
        assert b.shape[0] == nf and off[-1] == x.shape[0]
        ws = self.workspace(off, b)
        E = torch.empty(nf, dtype=torch.float64, device=x.device)
        F = torch.empty(x.shape[0], 3, dtype=torch.float64, device=x.device)
        W = torch.empty(nf, 9, dtype=torch.float64, device=x.device)
        Ei = torch.empty(x.shape[0], dtype=torch.float64, device=x.device) if atom_energy else None
        self._check(_lib.dp_compute_batch(self.h, nf, off.ctypes.data_as(C.c_void_p), _ptr(x), _ptr(t),
                                          b.ctypes.data_as(C.c_void_p), _ptr(E), _ptr(F), _ptr(W),
                                          _ptr(Ei), _ptr(ws), ws.numel(), _stream()))
        if check:
            self.status()
        return (E, F, W.view(nf, 3, 3), Ei) if atom_energy else (E, F, W.view(nf, 3, 3))

    def nlist(self, coords, types, box, check: bool = True):
        """Formatted neighbour list (owner index, image code) and per-type counts."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        b = _box9(box)
        ws = self.workspace(np.array([0, n]), b)
        nl = torch.empty(n, self.nm, dtype=torch.int32, device=x.device)
        img = torch.empty(n, self.nm, dtype=torch.int32, device=x.device)
        nn = torch.empty(n, self.ntypes, dtype=torch.int32, device=x.device)
        self._check(_lib.dp_nlist(self.h, n, _ptr(x), _ptr(t), b.ctypes.data_as(C.c_void_p), _ptr(nl),
                                  _ptr(img), _ptr(nn), _ptr(ws), ws.numel(), _stream()))
        rc = self.status() if check else 0
        return nl, img, nn, rc

    def descriptor(self, coords, types, box, check: bool = True):
        """T = G^T R / N_m and dE/dT per atom, [N][M][4] doubles."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        b = _box9(box)
        ws = self.workspace(np.array([0, n]), b)
        T = torch.empty(n, self.M, 4, dtype=torch.float64, device=x.device)
        gT = torch.empty(n, self.M, 4, dtype=torch.float64, device=x.device)
        self._check(_lib.dp_descriptor(self.h, n, _ptr(x), _ptr(t), b.ctypes.data_as(C.c_void_p),
                                       _ptr(T), _ptr(gT), _ptr(ws), ws.numel(), _stream()))
        if check:
            self.status()
        return T, gT

    def md_run(self, x: torch.Tensor, v: torch.Tensor, types, masses, box, dt: float, nsteps: int,
               thermo_every: int = 0, forces: Optional[torch.Tensor] = None, check: bool = True):
        """Velocity Verlet in place on device tensors x, v; returns the thermo rows tensor."""
        assert x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()
        assert v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        b = _box9(box)
        ms = np.ascontiguousarray(masses, dtype=np.float64)
        ws = self.workspace(np.array([0, n]), b)
        nrow = 1 + (nsteps // thermo_every if thermo_every > 0 else 0)
        th = torch.zeros(nrow, 6, dtype=torch.float64, device=x.device)
        self._check(_lib.dp_md_run(self.h, n, _ptr(x), _ptr(v), _ptr(t), ms.ctypes.data_as(C.c_void_p),
                                   b.ctypes.data_as(C.c_void_p), float(dt), int(nsteps),
                                   int(thermo_every), _ptr(th), _ptr(forces), _ptr(ws), ws.numel(),
                                   _stream()))
        if check:
            self.status()
        return th

    def md_run_npt(self, x: torch.Tensor, v: torch.Tensor, types, masses, box, pressure_bar: float,
                   tau_p: float, temperature: float, tau_t: float, dt: float, nsteps: int,
                   thermo_every: int = 0, min_scale: float = 0.9, forces: Optional[torch.Tensor] = None,
                   check: bool = True):
        """Isobaric MD in place on device tensors x, v (dp_md_run_npt); returns the thermo
        rows [step, PE, KE, T, Etot, P(bar), V, H], the final box (3 x 3) and
        (p_eps, xi, p_xi), device tensors."""
        assert x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()
        assert v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        b = _box9(box)
        ms = np.ascontiguousarray(masses, dtype=np.float64)
        nb = C.c_size_t()
        self._check(_lib.dp_md_npt_workspace_size(self.h, n, b.ctypes.data_as(C.c_void_p), float(min_scale),
                                                  C.byref(nb)))
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = torch.empty(int(nb.value * 1.1) + 4096, dtype=torch.uint8, device=self.device)
        ws = self._ws
        opt = _NptOptions(float(pressure_bar), float(tau_p), float(temperature), float(tau_t), float(min_scale))
        nrow = 1 + (nsteps // thermo_every if thermo_every > 0 else 0)
        th = torch.zeros(nrow, 8, dtype=torch.float64, device=x.device)
        box_out = torch.zeros(9, dtype=torch.float64, device=x.device)
        state = torch.zeros(3, dtype=torch.float64, device=x.device)
        self._check(_lib.dp_md_run_npt(self.h, n, _ptr(x), _ptr(v), _ptr(t), ms.ctypes.data_as(C.c_void_p),
                                       b.ctypes.data_as(C.c_void_p), C.byref(opt), float(dt), int(nsteps),
                                       int(thermo_every), _ptr(th), _ptr(box_out), _ptr(state), _ptr(forces),
                                       _ptr(ws), ws.numel(), _stream()))
        if check:
            self.status()
        return th, box_out.view(3, 3), state

    def profile(self, enable: bool, stages=None):
        """Stage timing on (all stages, or only the named ones) or off."""
        if enable and stages is not None:
            mask = 0
            for s in stages:
                mask |= 1 << STAGES[s]
            self._check(_lib.dp_profile_stages(self.h, mask))
        else:
            self._check(_lib.dp_profile(self.h, 1 if enable else 0))

    def profile_read(self, stage: str):
        """(total milliseconds, launches) of one stage since profile(True)."""
        ms, cnt = C.c_double(), C.c_int64()
        self._check(_lib.dp_profile_read(self.h, STAGES[stage], C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    # ------------------------------------------------------------------ student
    def student_samples(self, alpha: int, beta: int, coords, types, box, uniforms: torch.Tensor,
                        keep: float, cap: int):
        """s of real (alpha, beta) neighbours kept where uniforms < keep (slot order)."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        n = x.shape[0]
        b = _box9(box)
        nb = C.c_size_t()
        self._check(_lib.dp_student_samples_workspace_size(self.h, n, b.ctypes.data_as(C.c_void_p), C.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
        out = torch.empty(max(cap, 1), dtype=torch.float64, device=x.device)
        cnt = C.c_int64()
        u = uniforms.to(device=x.device, dtype=torch.float32).contiguous()
        assert u.numel() == n * self.nm
        self._check(_lib.dp_student_samples(self.h, alpha, beta, n, _ptr(x), _ptr(t), b.ctypes.data_as(C.c_void_p),
                                            _ptr(u), float(keep), _ptr(out), cap, C.byref(cnt), _ptr(ws),
                                            ws.numel(), _stream()))
        return out[:min(cnt.value, cap)], cnt.value

    def embed_eval(self, alpha: int, beta: int, s: torch.Tensor) -> torch.Tensor:
        """The full embedding net G^{alpha,beta}(s) in FP64: [n][M]."""
        s = self._dev(s, torch.float64)
        G = torch.empty(s.numel(), self.M, dtype=torch.float64, device=s.device)
        self._check(_lib.dp_embed_eval(self.h, alpha, beta, s.numel(), _ptr(s), _ptr(G), _stream()))
        return G

    def set_student(self, hidden: int, theta_s: Optional[torch.Tensor], s_lo=None, s_hi=None, enable: bool = True):
        if not enable:
            self._check(_lib.dp_set_student(self.h, hidden, None, None, None, 0, None, 0, _stream()))
            self._ws = None
            return
        th = self._dev(theta_s, torch.float64)
        assert th.numel() == self.ntypes ** 2 * student_size(hidden, self.M)
        lo = np.ascontiguousarray(s_lo, dtype=np.float64)
        hi = np.ascontiguousarray(s_hi, dtype=np.float64)
        nb = C.c_size_t()
        self._check(_lib.dp_student_bytes(self.h, C.byref(nb)))
        if self._student_mem is None or self._student_mem.numel() < nb.value:
            self._student_mem = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self._check(_lib.dp_set_student(self.h, hidden, _ptr(th), lo.ctypes.data_as(C.c_void_p),
                                        hi.ctypes.data_as(C.c_void_p), 1, _ptr(self._student_mem),
                                        self._student_mem.numel(), _stream()))
        self._ws = None       # workspace layout changes with the student's fallback list

    # ------------------------------------------------------------------ parameters
    def get_params(self) -> torch.Tensor:
        th = torch.empty(self.nparams, dtype=torch.float64, device=self.device)
        self._check(_lib.dp_get_params(self.h, _ptr(th), _stream()))
        return th

    def set_params(self, theta: torch.Tensor):
        th = self._dev(theta.detach(), torch.float64)
        assert th.numel() == self.nparams
        self._check(_lib.dp_set_params(self.h, _ptr(th), _stream()))

    def param_grad(self, coords, types, offsets, boxes, gE, gF, max_atoms: int = 0) -> torch.Tensor:
        """sum_f gE_f dE_f/dtheta + sum_i gF_i . dF_i/dtheta for a ragged batch (FP64); the
        library splits the batch into chunks of whole frames of at most max_atoms atoms
        (0: its default)."""
        x = self._dev(coords, torch.float64)
        t = self._dev(types, torch.int32)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        b = _box9(boxes)
        nf = len(off) - 1
        gE = self._dev(gE, torch.float64).reshape(nf)
        gF = self._dev(gF, torch.float64).reshape(-1, 3)
        gt = torch.zeros(self.nparams, dtype=torch.float64, device=x.device)
        nb = C.c_size_t()
        self._check(_lib.dp_param_grad_workspace_size(self.h, nf, off.ctypes.data_as(C.c_void_p),
                                                      b.ctypes.data_as(C.c_void_p), int(max_atoms), C.byref(nb)))
        if self._pg_ws is None or self._pg_ws.numel() < nb.value:
            self._pg_ws = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
        ws = self._pg_ws
        self._check(_lib.dp_param_grad(self.h, nf, off.ctypes.data_as(C.c_void_p), _ptr(x), _ptr(t),
                                       b.ctypes.data_as(C.c_void_p), _ptr(gE), _ptr(gF), _ptr(gt), int(max_atoms),
                                       _ptr(ws), ws.numel(), _stream()))
        return gt


def student_size(hidden: int, M: int) -> int:
    return 2 * hidden + hidden * M + M


def student_loss_grad(hidden: int, M: int, s: torch.Tensor, G: torch.Tensor, theta_s: torch.Tensor,
                      scratch: Optional[torch.Tensor] = None):
    """Student MSE loss and gradient on the GPU (loss [1], grad [size] device tensors)."""
    n = s.numel()
    nb = C.c_size_t()
    _lib.dp_student_scratch_size(hidden, M, n, C.byref(nb))
    if scratch is None or scratch.numel() < nb.value:
        scratch = torch.empty(nb.value, dtype=torch.uint8, device=s.device)
    loss = torch.zeros(1, dtype=torch.float64, device=s.device)
    grad = torch.empty(student_size(hidden, M), dtype=torch.float64, device=s.device)
    rc = _lib.dp_student_loss_grad(hidden, M, n, _ptr(s), _ptr(G), _ptr(theta_s), _ptr(loss), _ptr(grad),
                                   _ptr(scratch), scratch.numel(), _stream())
    if rc != DP_OK:
        raise DPError(rc, "dp_student_loss_grad failed")
    return loss, grad, scratch


def student_lsq(hidden: int, M: int, s: torch.Tensor, G: torch.Tensor, theta_s: torch.Tensor,
                ridge: float = 1e-13):
    """Least-squares output layer (W2, b2 of theta_s) for the given hidden layer."""
    nb = C.c_size_t()
    _lib.dp_student_lsq_scratch_size(hidden, M, s.numel(), C.byref(nb))
    scratch = torch.empty(nb.value, dtype=torch.uint8, device=s.device)
    rc = _lib.dp_student_lsq(hidden, M, s.numel(), _ptr(s), _ptr(G), _ptr(theta_s), float(ridge),
                             _ptr(scratch), scratch.numel(), _stream())
    if rc != DP_OK:
        raise DPError(rc, "dp_student_lsq failed")


def adam_step(theta: torch.Tensor, m: torch.Tensor, v: torch.Tensor, g: torch.Tensor, step: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    rc = _lib.dp_adam(theta.numel(), _ptr(theta), _ptr(m), _ptr(v), _ptr(g), int(step), float(lr), b1, b2, eps,
                      _stream())
    if rc != DP_OK:
        raise DPError(rc, "dp_adam failed")


class DPEnergyForce(torch.autograd.Function):
    """(E [nframes], F [natoms][3]) = DP-SE(theta; batch), differentiable in theta.

    forward runs dp_compute_batch with theta installed; backward runs dp_param_grad,
    which returns sum_f gE_f dE_f/dtheta + sum_i gF_i . dF_i/dtheta exactly.
    Coordinates, types and boxes receive no gradient."""

    @staticmethod
    def forward(ctx, theta, model: DPModel, coords, types, offsets, boxes):
        model.set_params(theta)
        E, F, _ = model.compute_batch(coords, types, offsets, boxes)
        ctx.model = model
        ctx.batch = (coords, types, offsets, boxes)
        ctx.save_for_backward(theta)
        return E, F

    @staticmethod
    def backward(ctx, gE, gF):
        (theta,) = ctx.saved_tensors
        model = ctx.model
        coords, types, offsets, boxes = ctx.batch
        nf = len(offsets) - 1
        if gE is None:
            gE = torch.zeros(nf, dtype=torch.float64, device=theta.device)
        if gF is None:
            gF = torch.zeros(int(offsets[-1]), 3, dtype=torch.float64, device=theta.device)
        model.set_params(theta)
        g = model.param_grad(coords, types, offsets, boxes, gE.contiguous(), gF.contiguous())
        return g.to(theta.dtype), None, None, None, None, None
