"""ctypes wrapper of the plain FP64 CPU oracle (dp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "dp_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11", "-Wall",
               "-shared", "-fPIC", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.or_load.restype = P
        L.or_load.argtypes = [C.c_char_p]
        L.or_free.argtypes = [P]
        L.or_info.argtypes = [P] + [P] * 6
        L.or_get_params.argtypes = [P, P]
        L.or_set_params.argtypes = [P, P]
        L.or_smooth_vec.argtypes = [P, I64, P, P, P]
        L.or_env_row.argtypes = [P, P, P, P]
        L.or_nlist.argtypes = [P, I64, P, P, P, I64, P, P, P, P, P]
        L.or_eval.argtypes = [P, I64, P, P, P, P, P, P, P, P, P, P]
        L.or_eval_sampled.argtypes = [P, I64, P, P, P, I64, P, P, P]
        L.or_eval_atomic.argtypes = [P, I64, P, P, P, P, P, P, P, P]
        L.or_md.argtypes = [P, I64, P, P, P, P, P, D, C.c_int, C.c_int, P]
        L.or_md_npt.argtypes = [P, I64, P, P, P, P, P, D, D, D, D, D, C.c_int, C.c_int, P, P]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def set_threads(n: int):
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return lib().or_get_threads()


class Oracle:
    def __init__(self, model_path: str):
        self.h = lib().or_load(model_path.encode())
        if not self.h:
            raise ValueError("oracle: cannot read model file %s" % model_path)
        nt, nm, M, m2 = (C.c_int32() for _ in range(4))
        rc, npar = C.c_double(), C.c_int64()
        lib().or_info(self.h, C.byref(nt), C.byref(nm), C.byref(M), C.byref(m2),
                      C.byref(rc), C.byref(npar))
        self.ntypes, self.nm, self.M, self.m2 = nt.value, nm.value, M.value, m2.value
        self.rc, self.nparams = rc.value, npar.value

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_free(self.h)
            self.h = None

    # parameters ------------------------------------------------------------------
    def get_params(self):
        p = np.empty(self.nparams)
        lib().or_get_params(self.h, _p(p))
        return p

    def set_params(self, p):
        p = _f64(p)
        assert p.size == self.nparams
        lib().or_set_params(self.h, _p(p))

    # pieces ----------------------------------------------------------------------
    def smooth(self, r):
        r = _f64(np.atleast_1d(r))
        s, ds = np.empty_like(r), np.empty_like(r)
        lib().or_smooth_vec(self.h, r.size, _p(r), _p(s), _p(ds))
        return s, ds

    def env_row(self, d):
        d = _f64(d)
        R, dR = np.empty(4), np.empty((4, 3))
        lib().or_env_row(self.h, _p(d), _p(R), _p(dR))
        return R, dR

    def nlist(self, coords, types, box, centers=None):
        coords, types, box = _f64(coords), _i32(types), _f64(box)
        n = len(types)
        cent = None if centers is None else np.ascontiguousarray(centers, dtype=np.int64)
        nc = n if cent is None else len(cent)
        nl = np.empty((nc, self.nm), np.int32)
        img = np.empty((nc, self.nm), np.int32)
        nnei = np.empty((nc, self.ntypes), np.int32)
        ovf = C.c_int32(0)
        rc = lib().or_nlist(self.h, n, _p(coords), _p(types), _p(box), nc, _p(cent), _p(nl),
                            _p(img), _p(nnei), C.byref(ovf))
        if rc < 0:
            raise ValueError("oracle nlist error %d" % rc)
        return nl, img, nnei, bool(ovf.value)

    # evaluation ------------------------------------------------------------------
    def eval(self, coords, types, box, dumps: bool = False):
        coords, types, box = _f64(coords), _i32(types), _f64(box)
        n = len(types)
        E = np.zeros(1)
        F = np.empty((n, 3))
        W = np.empty(9)
        Ei = np.empty(n)
        T = np.empty((n, self.M, 4)) if dumps else None
        D = np.empty((n, self.M, self.m2)) if dumps else None
        gT = np.empty((n, self.M, 4)) if dumps else None
        rc = lib().or_eval(self.h, n, _p(coords), _p(types), _p(box), _p(E), _p(F), _p(W),
                           _p(Ei), _p(T), _p(D), _p(gT))
        if rc < 0:
            raise ValueError("oracle eval error %d" % rc)
        out = dict(E=float(E[0]), F=F, W=W.reshape(3, 3), Ei=Ei, overflow=bool(rc == 1))
        if dumps:
            out.update(T=T, D=D, gT=gT)
        return out

    def eval_atomic(self, coords, types, box):
        """E, F, W with the per-atom energies Ei [n] and per-centre virials Wi [n][3][3]
        (W_i = -sum_j d_ij (x) dE_i/dd_ij; sum_i W_i = W)."""
        coords, types, box = _f64(coords), _i32(types), _f64(box)
        n = len(types)
        E = np.zeros(1)
        F = np.zeros((n, 3))
        W = np.zeros(9)
        Ei = np.zeros(n)
        Wi = np.zeros((n, 9))
        rc = lib().or_eval_atomic(self.h, n, _p(coords), _p(types), _p(box), _p(E), _p(F), _p(W), _p(Ei), _p(Wi))
        if rc < 0:
            raise ValueError("oracle eval error %d" % rc)
        return dict(E=float(E[0]), F=F, W=W.reshape(3, 3), Ei=Ei, Wi=Wi.reshape(n, 3, 3), overflow=bool(rc == 1))

    def eval_sampled(self, coords, types, box, samples):
        coords, types, box = _f64(coords), _i32(types), _f64(box)
        s = np.ascontiguousarray(samples, dtype=np.int64)
        Ei = np.empty(len(s))
        F = np.empty((len(s), 3))
        rc = lib().or_eval_sampled(self.h, len(types), _p(coords), _p(types), _p(box), len(s),
                                   _p(s), _p(Ei), _p(F))
        if rc < 0:
            raise ValueError("oracle eval_sampled error %d" % rc)
        return Ei, F

    def md(self, x, v, types, masses, box, dt, nsteps, thermo_every):
        x, v = _f64(x).copy(), _f64(v).copy()
        types, box, masses = _i32(types), _f64(box), _f64(masses)
        nrow = 1 + (nsteps // thermo_every if thermo_every > 0 else 0)
        th = np.zeros((nrow, 6))
        rc = lib().or_md(self.h, len(types), _p(x), _p(v), _p(types), _p(masses), _p(box),
                         float(dt), int(nsteps), int(thermo_every), _p(th))
        if rc < 0:
            raise ValueError("oracle md error %d" % rc)
        return x, v, th

    def md_npt(self, x, v, types, masses, box, pext_bar, tau_p, temp, tau_t, dt, nsteps, thermo_every):
        """Isotropic isobaric MD (Martyna-Tobias-Klein barostat, optional Nose-Hoover
        thermostat: tau_t <= 0 gives the isoenthalpic form).  Returns x, v, box, thermo
        rows [step, PE, KE, T, Etot, P(bar), V, H] and (p_eps, xi, p_xi)."""
        x, v = _f64(x).copy(), _f64(v).copy()
        types, masses = _i32(types), _f64(masses)
        box = _f64(box).reshape(9).copy()
        nrow = 1 + (nsteps // thermo_every if thermo_every > 0 else 0)
        th = np.zeros((nrow, 8))
        st = np.zeros(3)
        rc = lib().or_md_npt(self.h, len(types), _p(x), _p(v), _p(types), _p(masses), _p(box),
                             float(pext_bar), float(tau_p), float(temp), float(tau_t), float(dt), int(nsteps),
                             int(thermo_every), _p(th), _p(st))
        if rc < 0:
            raise ValueError("oracle md_npt error %d" % rc)
        return x, v, box.reshape(3, 3), th, st
