"""FP64 CPU oracle of the discretised elastic 2->2 collision operator.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark load it; the product library never does.  It is a thin ctypes
wrapper over ``kxg_oracle.c`` (plain C loops, FP64), which shares no code with
the GPU library.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kxg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# another build of the same source to load instead (the sanitizer build of
# the CPU tests); it is used as it is, never rebuilt
LIB_OVERRIDE = os.environ.get("ORACLE_LIBRARY")

GL, EXACT = 0, 1          # angular quadrature: Gauss-Legendre in mu, closed form
LIN, LOG = 0, 1           # interpolation of f at the fourth momentum

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True, sanitize: bool = False, out: Optional[str] = None) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FMA contraction);
    with sanitize, into `out` with AddressSanitizer and
    UndefinedBehaviorSanitizer (the loading process preloads libasan)."""
    lib = out or LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        tmp = lib + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
        if sanitize:
            cmd[1:1] = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib)
    return lib


def lib():
    global _lib
    if _lib is None:
        if LIB_OVERRIDE:
            L = ctypes.CDLL(LIB_OVERRIDE)
        else:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            L = ctypes.CDLL(LIB)
        L.or_angular_gl.restype = ctypes.c_double
        L.or_angular_exact.restype = ctypes.c_double
        L.or_weight.restype = ctypes.c_double
        L.or_drift.restype = ctypes.c_double
        L.or_heun.restype = ctypes.c_int
        L.or_deposit.restype = ctypes.c_int
        L.or_condensate_a3nu.restype = ctypes.c_double
        L.or_gamma22.restype = ctypes.c_double
        L.or_freeze_in.restype = ctypes.c_int
        L.or_heun_comoving.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timing only)."""
    os.environ["OMP_NUM_THREADS"] = str(n)
    lib().or_set_threads(ctypes.c_int(int(n)))


def max_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(lib().or_max_threads())


class Grid:
    """Grid quantities p, dp, E, K, h of the oracle (App. B)."""

    def __init__(self, p, mass: float = 1.0, dp: Optional[np.ndarray] = None):
        self.p = _f64(p)
        self.n = len(self.p)
        self.mass = float(mass)
        self.dp_override = None if dp is None else _f64(dp)
        n = self.n
        self.dp, self.E, self.K, self.h = (np.empty(n) for _ in range(4))
        lib().or_grid(ctypes.c_int(n), _p(self.p), ctypes.c_double(self.mass),
                      _p(self.dp_override), _p(self.dp), _p(self.E), _p(self.K),
                      _p(self.h))


def gauss_legendre(n: int) -> Tuple[np.ndarray, np.ndarray]:
    x, w = np.empty(n), np.empty(n)
    lib().or_gauss_legendre(ctypes.c_int(n), _p(x), _p(w))
    return x, w


def angular_gl(pi, pn, pm, mass=1.0, nmu=18) -> float:
    x, w = gauss_legendre(nmu)
    K = lambda q: q * q / (np.sqrt(q * q + mass * mass) + mass)
    return lib().or_angular_gl(ctypes.c_double(pi), ctypes.c_double(pn),
                               ctypes.c_double(pm), ctypes.c_double(K(pi)),
                               ctypes.c_double(K(pn)), ctypes.c_double(K(pm)),
                               ctypes.c_int(nmu), _p(x), _p(w))


def angular_exact(p1, p2, p3, p4) -> float:
    return lib().or_angular_exact(*(ctypes.c_double(v) for v in (p1, p2, p3, p4)))


class Operator:
    """Precomputed A[i,n,m], R[i,j] of the oracle (linear interpolation)."""

    def __init__(self, p, mass=1.0, gdof=1.0, m2=1.0, quad=GL, nmu=18,
                 dp: Optional[np.ndarray] = None, keep_bracket: bool = False):
        self.grid = Grid(p, mass, dp)
        n = self.grid.n
        self.n, self.mass, self.gdof, self.m2 = n, float(mass), float(gdof), float(m2)
        self.quad, self.nmu = int(quad), int(nmu)
        self.A = np.empty((n, n, n))
        self.R = np.empty((n, n))
        self.jl = np.empty((n, n, n), dtype=np.int32) if keep_bracket else None
        self.wr = np.empty((n, n, n)) if keep_bracket else None
        lib().or_kernel_build(
            ctypes.c_int(n), _p(self.grid.p), _p(self.grid.dp_override),
            ctypes.c_double(self.mass), ctypes.c_double(self.gdof),
            ctypes.c_double(self.m2), ctypes.c_int(self.quad), ctypes.c_int(self.nmu),
            _p(self.A), _p(self.R),
            None if self.jl is None else self.jl.ctypes.data_as(_ip),
            _p(self.wr))

    # -- the operator --------------------------------------------------------
    def collision(self, f, project: bool = False):
        """Returns (C, gain, loss) for f of shape [N] or [B, N]."""
        f = _f64(f)
        one = f.ndim == 1
        fb = f.reshape(1, -1) if one else f
        nb = fb.shape[0]
        g, l, c = np.empty_like(fb), np.empty_like(fb), np.empty_like(fb)
        lib().or_collision_ar(ctypes.c_int(self.n), ctypes.c_int(nb), _p(self.A),
                              _p(self.R), _p(fb), _p(g), _p(l), _p(c))
        if project:
            c = np.stack([self.project(fb[b], c[b])[0] for b in range(nb)])
        if one:
            return c[0], g[0], l[0]
        return c, g, l

    def project(self, f, craw, eps_supp: float = 1e-12):
        f, craw = _f64(f), _f64(craw)
        out = np.empty(self.n)
        diag = np.empty(8)
        lib().or_project(ctypes.c_int(self.n), _p(self.grid.h), _p(self.grid.E),
                         _p(f), _p(craw), ctypes.c_double(eps_supp), _p(out), _p(diag))
        return out, diag

    def moments(self, f):
        out = np.empty(3)
        lib().or_moments(ctypes.c_int(self.n), _p(self.grid.h), _p(self.grid.E),
                         _p(_f64(f)), _p(out))
        return out

    def rk4(self, f0, lam: float, dt: float, nsteps: int, project: bool = True,
            traj: bool = False):
        f = _f64(f0).copy()
        tr = np.empty((nsteps, self.n)) if traj else None
        lib().or_rk4(ctypes.c_int(self.n), _p(self.A), _p(self.R), _p(self.grid.h),
                     _p(self.grid.E), _p(f), ctypes.c_double(lam), ctypes.c_double(dt),
                     ctypes.c_int(nsteps), ctypes.c_int(int(project)), _p(tr))
        return (f, tr) if traj else f

    def heun(self, x0, lam: float, Hi: float, u_end: float, dt0: float,
             expansion: bool = True, project: bool = True, rtol: float = 1e-6,
             atol: Optional[float] = None, safety: float = 0.9, fmin: float = 0.2,
             fmax: float = 5.0, max_steps: int = 10000, replay_dt=None, u0: float = 0.0):
        """Adaptive (or replayed) Heun in u.  Returns dict with the final state,
        accepted (u, dt), outflow, rejection count and the log of attempts
        (dt, error estimate, accepted) in the order they were made."""
        x = _f64(x0).copy()
        if atol is None:
            atol = 1e-12 * float(np.max(np.abs(x)))
        nrep = 0 if replay_dt is None else len(replay_dt)
        cap = max(nrep, max_steps)
        acc_u, acc_dt = np.empty(cap), np.empty(cap)
        rd = None if replay_dt is None else _f64(replay_dt)
        outflow = ctypes.c_double(0.0)
        nrej = ctypes.c_int(0)
        att_cap = 4 * cap + 64
        att_dt, att_err = np.empty(att_cap), np.empty(att_cap)
        att_ok = np.empty(att_cap, dtype=np.int32)
        natt = ctypes.c_int(0)
        nacc = lib().or_heun(
            ctypes.c_int(self.n), _p(self.A), _p(self.R), _p(self.grid.p),
            _p(self.grid.dp_override), ctypes.c_double(self.mass), _p(x),
            ctypes.c_int(int(expansion)), ctypes.c_int(int(project)),
            ctypes.c_double(lam), ctypes.c_double(Hi), ctypes.c_double(u0),
            ctypes.c_double(u_end), ctypes.c_double(dt0), ctypes.c_double(rtol),
            ctypes.c_double(atol), ctypes.c_double(safety), ctypes.c_double(fmin),
            ctypes.c_double(fmax), ctypes.c_int(max_steps), ctypes.c_int(nrep), _p(rd),
            _p(acc_u), _p(acc_dt), ctypes.byref(outflow), ctypes.byref(nrej),
            ctypes.c_int(att_cap), _p(att_dt), _p(att_err), att_ok.ctypes.data_as(_ip),
            ctypes.byref(natt))
        na = min(natt.value, att_cap)
        return {"x": x, "u": acc_u[:nacc], "dt": acc_dt[:nacc],
                "outflow": outflow.value, "rejected": nrej.value,
                "attempts": {"dt": att_dt[:na], "err": att_err[:na],
                             "accepted": att_ok[:na].astype(bool)}}

    # -- freeze-in sources and the two regimes of the evolution (Sec. 3, 4.2) --
    def deposit(self, p0: float):
        """(j, w_j, w_{j+1}): nodes and energy-linear weights sharing the
        condensate injection at momentum p0 (j = -1 outside the grid)."""
        return deposit(self.grid, p0)

    def sources(self, u: float, Hi: float, **kw):
        """Freeze-in source vector S_i(u) in the units of C (see sources())."""
        return sources(self.grid, u, Hi, **kw)

    def gamma22(self, f, lam: float = 1.0) -> float:
        """Effective self-scattering rate n<sigma v>: the per-particle loss
        rate lam (R f)_i averaged over the particles of f."""
        return float(lib().or_gamma22(ctypes.c_int(self.n), _p(self.R), _p(self.grid.h),
                                      _p(_f64(f)), ctypes.c_double(lam)))

    def freeze_in(self, x0, lam: float, Hi: float, u_end: float, du: float,
                  eps_switch: float = 1e-2, N0: float = 0.0, Gamma: float = 0.0,
                  p0: float = 1.0, kappa: float = 0.0, mh: float = 250.0, Ti: float = 1.0,
                  dt0: float = 1e-3, project: bool = True, rtol: float = 1e-6,
                  atol_rel: float = 1e-12, safety: float = 0.9, fmin: float = 0.2,
                  fmax: float = 5.0, max_steps: int = 100000, replay_dt=None, u0: float = 0.0):
        """Source-only RK4 on fixed du until Gamma_22/H > eps_switch, then
        adaptive (or replayed) Heun with the elastic operator (atol =
        atol_rel max|x| at the switch); state g = a^3 p^3 f.  Returns dict: x, n_src, u_switch, regime-2 accepted
        (u, dt), outflow, rejected."""
        x = _f64(x0).copy()
        nrep = 0 if replay_dt is None else len(replay_dt)
        cap = max(nrep, max_steps) + 1
        acc_u, acc_dt = np.empty(cap), np.empty(cap)
        rd = None if replay_dt is None else _f64(replay_dt)
        nsrc, usw = ctypes.c_int(0), ctypes.c_double(0.0)
        outflow, nrej = ctypes.c_double(0.0), ctypes.c_int(0)
        nacc = lib().or_freeze_in(
            ctypes.c_int(self.n), _p(self.A), _p(self.R), _p(self.grid.p),
            _p(self.grid.dp_override), ctypes.c_double(self.mass), _p(x),
            ctypes.c_int(int(project)), ctypes.c_double(lam), ctypes.c_double(Hi),
            ctypes.c_double(u0), ctypes.c_double(u_end), ctypes.c_double(du),
            ctypes.c_double(eps_switch), ctypes.c_double(N0), ctypes.c_double(Gamma),
            ctypes.c_double(p0), ctypes.c_double(kappa), ctypes.c_double(mh),
            ctypes.c_double(Ti), ctypes.c_double(dt0), ctypes.c_double(rtol),
            ctypes.c_double(atol_rel), ctypes.c_double(safety), ctypes.c_double(fmin),
            ctypes.c_double(fmax), ctypes.c_int(max_steps), ctypes.c_int(nrep), _p(rd),
            _p(acc_u), _p(acc_dt), ctypes.byref(nsrc), ctypes.byref(usw),
            ctypes.byref(outflow), ctypes.byref(nrej))
        return {"x": x, "n_src": nsrc.value, "u_switch": usw.value, "u": acc_u[:nacc],
                "dt": acc_dt[:nacc], "outflow": outflow.value, "rejected": nrej.value}

    def gamma0(self, f) -> float:
        """Largest loss rate max_i sum_j R_ij f_j (the initial scattering rate)."""
        return float(np.max(self.R @ _f64(f)))


class Comoving:
    """The operator on a fixed comoving grid q (Sec. 4.1: p = q / a) at u = ln a,
    exact (the tensors of the grid q / a rebuilt at every u; ntab = 0) or
    tabulated (the tensors at ntab nodes of u in [umin, umax], mixed linearly
    in u between the two that bracket it)."""

    def __init__(self, q, mass=1.0, gdof=1.0, m2=1.0, quad=GL, nmu=18, ntab: int = 0,
                 umin: float = 0.0, umax: float = 0.0):
        self.q = _f64(q)
        self.n = len(self.q)
        self.mass, self.gdof, self.m2 = float(mass), float(gdof), float(m2)
        self.quad, self.nmu = int(quad), int(nmu)
        self.ntab, self.umin = int(ntab), float(umin)
        self.du = (float(umax) - float(umin)) / (ntab - 1) if ntab > 1 else 1.0
        n = self.n
        if self.ntab > 0:
            assert self.ntab >= 2 and umax > umin
            self.tabA = np.empty((self.ntab, n, n, n))
            self.tabR = np.empty((self.ntab, n, n))
            for j in range(self.ntab):
                A, R = self.tensors(self.umin + j * self.du)
                self.tabA[j], self.tabR[j] = A, R
        else:
            self.tabA = self.tabR = None

    def tensors(self, u: float):
        """A, R of the physical grid q / e^u."""
        n = self.n
        A, R = np.empty((n, n, n)), np.empty((n, n))
        lib().or_comoving_tensors(ctypes.c_int(n), _p(self.q), ctypes.c_double(u),
                                  ctypes.c_double(self.mass), ctypes.c_double(self.gdof),
                                  ctypes.c_double(self.m2), ctypes.c_int(self.quad),
                                  ctypes.c_int(self.nmu), _p(A), _p(R))
        return A, R

    def grid(self, u: float) -> Grid:
        """Grid quantities of the physical grid q / e^u."""
        return Grid(self.q / np.exp(u), self.mass)

    def collision(self, f, u: float, project: bool = True):
        out = np.empty(self.n)
        lib().or_comoving_collision(
            ctypes.c_int(self.n), _p(self.q), ctypes.c_double(u), ctypes.c_double(self.mass),
            ctypes.c_double(self.gdof), ctypes.c_double(self.m2), ctypes.c_int(self.quad),
            ctypes.c_int(self.nmu), ctypes.c_int(self.ntab), ctypes.c_double(self.umin),
            ctypes.c_double(self.du), _p(self.tabA), _p(self.tabR), _p(_f64(f)),
            ctypes.c_int(int(project)), _p(out))
        return out

    def heun(self, x0, lam: float, Hi: float, u_end: float, dt0: float, u0: float = 0.0,
             project: bool = True, rtol: float = 1e-6, atol: Optional[float] = None,
             safety: float = 0.9, fmin: float = 0.2, fmax: float = 5.0,
             max_steps: int = 10000, replay_dt=None):
        """Adaptive (or replayed) Heun in u on the comoving grid (state f)."""
        x = _f64(x0).copy()
        if atol is None:
            atol = 1e-12 * float(np.max(np.abs(x)))
        nrep = 0 if replay_dt is None else len(replay_dt)
        cap = max(nrep, max_steps)
        acc_u, acc_dt = np.empty(cap), np.empty(cap)
        rd = None if replay_dt is None else _f64(replay_dt)
        nrej = ctypes.c_int(0)
        nacc = lib().or_heun_comoving(
            ctypes.c_int(self.n), _p(self.q), ctypes.c_double(self.mass),
            ctypes.c_double(self.gdof), ctypes.c_double(self.m2), ctypes.c_int(self.quad),
            ctypes.c_int(self.nmu), ctypes.c_int(self.ntab), ctypes.c_double(self.umin),
            ctypes.c_double(self.du), _p(self.tabA), _p(self.tabR), _p(x),
            ctypes.c_int(int(project)), ctypes.c_double(lam), ctypes.c_double(Hi),
            ctypes.c_double(u0), ctypes.c_double(u_end), ctypes.c_double(dt0),
            ctypes.c_double(rtol), ctypes.c_double(atol), ctypes.c_double(safety),
            ctypes.c_double(fmin), ctypes.c_double(fmax), ctypes.c_int(max_steps),
            ctypes.c_int(nrep), _p(rd), _p(acc_u), _p(acc_dt), ctypes.byref(nrej))
        return {"x": x, "u": acc_u[:nacc], "dt": acc_dt[:nacc], "rejected": nrej.value}


def direct(p, f, mass=1.0, gdof=1.0, m2=1.0, quad=GL, nmu=18, interp=LIN,
           dp: Optional[np.ndarray] = None, eta: int = 0):
    """Direct per-(i,n,m) evaluation of eq. app_dense_collision; eta = +1/-1
    adds the Bose-Einstein/Fermi-Dirac factors of eq. Lambda_quantum."""
    p, f = _f64(p), _f64(f)
    n = len(p)
    g, l, c = np.empty(n), np.empty(n), np.empty(n)
    lib().or_collision_direct_q(ctypes.c_int(n), _p(p), _p(None if dp is None else _f64(dp)),
                                ctypes.c_double(mass), ctypes.c_double(gdof),
                                ctypes.c_double(m2), ctypes.c_int(quad), ctypes.c_int(nmu),
                                ctypes.c_int(interp), ctypes.c_int(int(eta)), _p(f), _p(g),
                                _p(l), _p(c))
    return c, g, l


def deposit(grid: Grid, p0: float):
    """(j, w_j, w_{j+1}) of the condensate injection at momentum p0."""
    wl, wr = ctypes.c_double(0.0), ctypes.c_double(0.0)
    j = lib().or_deposit(ctypes.c_int(grid.n), _p(grid.p), ctypes.c_double(grid.mass),
                         ctypes.c_double(p0), ctypes.byref(wl), ctypes.byref(wr))
    return j, wl.value, wr.value


def sources(grid: Grid, u: float, Hi: float, N0: float = 0.0, Gamma: float = 0.0,
            p0: float = 1.0, kappa: float = 0.0, mh: float = 250.0, Ti: float = 1.0):
    """Freeze-in source vector S_i(u) on a grid, in the units of C: the
    condensate injection (a^3 nu_Phi = N0 at u = 0, decay rate Gamma, decay
    momentum p0) and the Higgs decay (amplitude kappa, mass mh, bath
    temperature Ti at u = 0)."""
    j, wl, wr = deposit(grid, p0) if N0 > 0.0 else (-1, 0.0, 0.0)
    S = np.empty(grid.n)
    lib().or_sources(ctypes.c_int(grid.n), _p(grid.p), _p(grid.h), _p(grid.E),
                     ctypes.c_double(grid.mass), ctypes.c_double(u), ctypes.c_double(Hi),
                     ctypes.c_double(N0), ctypes.c_double(Gamma), ctypes.c_int(j),
                     ctypes.c_double(wl), ctypes.c_double(wr), ctypes.c_double(kappa),
                     ctypes.c_double(mh), ctypes.c_double(Ti), _p(S))
    return S


def condensate_a3nu(N0: float, Gamma: float, Hi: float, u: float) -> float:
    """a^3 nu_Phi(u): the solution of the condensate's decay law in the
    radiation era (code units, nu = (2 pi^2 / g) n)."""
    return float(lib().or_condensate_a3nu(ctypes.c_double(N0), ctypes.c_double(Gamma),
                                          ctypes.c_double(Hi), ctypes.c_double(u)))


def drift(p, dp, g):
    out = np.empty(len(p))
    o = lib().or_drift(ctypes.c_int(len(p)), _p(_f64(p)), _p(_f64(dp)), _p(_f64(g)), _p(out))
    return out, o
