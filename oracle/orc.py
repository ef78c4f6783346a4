"""ctypes binding of the FP64 CPU oracle (orc.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product library never loads it.

Array conventions: positions in cell units, SoA ``pos[3, n]``; proper
velocities ``u[3, n]``; vector mesh fields ``F[3, nz, ny, nx]`` (x fastest),
scalar mesh fields ``[nz, ny, nx]``.  All float64, C-contiguous.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")
_LIB_OMP = os.path.join(_HERE, "liborc_omp.so")


def _compile(out: str, extra, force: bool) -> str:
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", *extra, "-o", tmp, _SRC, "-lm"],
                              stderr=subprocess.DEVNULL)
        os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile orc.c twice with gcc: liborc.so (plain -O2, scalar, single thread: the checker)
    and liborc_omp.so (the same source with -fopenmp: loops over particles use one current
    buffer per thread, loops over cells and lines are split among the threads).  Returns the
    path of the plain library."""
    _compile(_LIB_OMP, ["-fopenmp"], force)
    return _compile(_LIB, [], force)


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("d", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("c", ctypes.c_double),
        ("eps0", ctypes.c_double),
        ("shape_order", ctypes.c_int32),
        ("field_order", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("pusher", ctypes.c_int32),
        ("relax_tol", ctypes.c_double),
        ("relax_max_iter", ctypes.c_int32),
        ("rho_background", ctypes.c_double),
        ("rad_tau", ctypes.c_double),
        ("current_scheme", ctypes.c_int32),
        ("gauss_passes", ctypes.c_int32),
        ("time_order", ctypes.c_int32),
        ("gauss_every", ctypes.c_int32),
    ]


def make_params(n=(16, 16, 16), d=(1.0, 1.0, 1.0), dt=0.4, c=1.0, eps0=1.0, shape_order=2,
                field_order=2, alpha=0.55, pusher=0, relax_tol=1e-14, relax_max_iter=200,
                rho_background=0.0, rad_tau=0.0, current_scheme=0, gauss_passes=0, time_order=2,
                gauss_every=1) -> Params:
    p = Params()
    p.n[:] = [int(v) for v in n]
    p.d[:] = [float(v) for v in d]
    p.dt, p.c, p.eps0 = float(dt), float(c), float(eps0)
    p.shape_order, p.field_order = int(shape_order), int(field_order)
    p.alpha, p.pusher = float(alpha), int(pusher)
    p.relax_tol, p.relax_max_iter = float(relax_tol), int(relax_max_iter)
    p.rho_background = float(rho_background)
    p.rad_tau = float(rad_tau)
    p.current_scheme, p.gauss_passes = int(current_scheme), int(gauss_passes)
    p.time_order = int(time_order)
    p.gauss_every = int(gauss_every)
    return p


# Fourth-order composition (Forest & Ruth 1990; Candy & Rozmus 1991; Yoshida 1990): with
# theta = 1/(2 - 2^(1/3)) the position form D(th/2) K(th) D((1-th)/2) K(1-2th) D((1-th)/2)
# K(th) D(th/2) keeps every position at the middle of the momentum interval of its kick.
# Merging the trailing and leading half drifts of consecutive steps gives three leapfrog
# substeps per step, (kick, drift) = (th, (1-th)/2), (1-2th, (1-th)/2), (th, th) times dt,
# with the positions and fields of the state a drift of th dt/2 ahead of the momenta.
FR_THETA = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
FR_SUBSTEPS = ((FR_THETA, 0.5 * (1.0 - FR_THETA)), (1.0 - 2.0 * FR_THETA, 0.5 * (1.0 - FR_THETA)),
               (FR_THETA, FR_THETA))


def substep_params(P: Params, drift: float) -> Params:
    """A copy of P whose time step is the drift of a substep."""
    Q = Params()
    ctypes.pointer(Q)[0] = P
    Q.dt = drift
    return Q


_libs = {}
_use_omp = False
_D = ctypes.POINTER(ctypes.c_double)
_P = ctypes.POINTER(Params)


class openmp:
    """Context manager: inside it every oracle call goes to the OpenMP build (threads from
    OMP_NUM_THREADS), outside it to the plain scalar build."""

    def __enter__(self):
        global _use_omp
        self._prev, _use_omp = _use_omp, True
        return self

    def __exit__(self, *exc):
        global _use_omp
        _use_omp = self._prev
        return False


def num_threads() -> int:
    """Threads the active build uses (1 for the plain build)."""
    return int(lib().orc_num_threads())


def lib():
    key = "omp" if _use_omp else "plain"
    if key not in _libs:
        build()
        _libs[key] = ctypes.CDLL(_LIB_OMP if _use_omp else _LIB)
        L = _libs[key]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_W.restype = ctypes.c_double
        L.orc_W.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_gather.argtypes = [_P, _D, _D, _D, _D, _D]
        L.orc_push.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, _D, _D, _D]
        L.orc_push_rad.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.orc_rad_bracket.restype = ctypes.c_double
        L.orc_rad_bracket.argtypes = [ctypes.c_double, _D, _D]
        L.orc_deposit_direct.argtypes = [_P, ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.orc_gauss_kappa.restype = ctypes.c_double
        L.orc_gauss_kappa.argtypes = [_P]
        L.orc_gauss_filter.argtypes = [_P, _D, _D, ctypes.c_int]
        L.orc_step_species_kd.restype = ctypes.c_int
        L.orc_step_species_kd.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int64, _D, _D, _D, _D, _D]
        L.orc_step_species.restype = ctypes.c_int
        L.orc_step_species.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int64, _D, _D, _D, _D, _D]
        L.orc_deposit_current.argtypes = [_P, ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.orc_deposit_rho.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int64, _D, _D]
        L.orc_fd_coeffs.argtypes = [ctypes.c_int, _D]
        L.orc_deriv.argtypes = [_P, _D, _D, ctypes.c_int, ctypes.c_int]
        for name in ("orc_curl_up", "orc_curl_down", "orc_div_down", "orc_div_up", "orc_laplacian_B"):
            getattr(L, name).argtypes = [_P, _D, _D]
        L.orc_field_step.restype = ctypes.c_int
        L.orc_field_step.argtypes = [_P, _D, _D, _D, _D]
        L.orc_current_high_order.argtypes = [_P, _D]
        L.orc_species_moments.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int64, _D, _D, _D]
        L.orc_field_energy.argtypes = [_P, _D, _D, _D]
    return _libs[key]


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], (a.dtype, a.flags)
    return a.ctypes.data_as(_D)


def _vec(P: Params):
    nx, ny, nz = P.n[0], P.n[1], P.n[2]
    return (3, nz, ny, nx)


def _scal(P: Params):
    return (P.n[2], P.n[1], P.n[0])


# -- single-particle pieces ------------------------------------------------------------------
def W(order: int, delta: float) -> float:
    return lib().orc_W(int(order), float(delta))


def gather(P: Params, E: np.ndarray, B: np.ndarray, X) -> tuple[np.ndarray, np.ndarray]:
    X = np.ascontiguousarray(X, dtype=np.float64)
    Ep = np.zeros(3)
    Bp = np.zeros(3)
    lib().orc_gather(ctypes.byref(P), _ptr(E), _ptr(B), _ptr(X), _ptr(Ep), _ptr(Bp))
    return Ep, Bp


def push(pusher: int, q: float, m: float, dt: float, c: float, E, B, u) -> np.ndarray:
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    uu = np.array(u, dtype=np.float64)
    lib().orc_push(int(pusher), q, m, dt, c, _ptr(E), _ptr(B), _ptr(uu))
    return uu


def push_rad(pusher: int, q: float, m: float, dt: float, c: float, rad_tau: float, E, B, u) -> np.ndarray:
    """Electromagnetic push followed by one step of radiative cooling."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    uu = np.array(u, dtype=np.float64)
    lib().orc_push_rad(int(pusher), q, m, dt, c, rad_tau, _ptr(E), _ptr(B), _ptr(uu))
    return uu


def rad_bracket(c: float, u, udot) -> float:
    """|du/dt|^2 + |du/dt x u|^2 / c^2 (radiated power over mu0 q^2 / (6 pi c))."""
    return lib().orc_rad_bracket(c, _ptr(np.array(u, dtype=np.float64)), _ptr(np.array(udot, dtype=np.float64)))


def deposit_direct(P: Params, q: float, w: float, X, v, J: np.ndarray | None = None) -> np.ndarray:
    """Direct current (eq. "jj2") of one particle at X with three-velocity v."""
    if J is None:
        J = np.zeros(_vec(P))
    lib().orc_deposit_direct(ctypes.byref(P), q, w, _ptr(np.array(X, dtype=np.float64)),
                             _ptr(np.array(v, dtype=np.float64)), _ptr(J))
    return J


def gauss_kappa(P: Params) -> float:
    return lib().orc_gauss_kappa(ctypes.byref(P))


def gauss_filter(P: Params, E: np.ndarray, rho: np.ndarray, passes: int) -> np.ndarray:
    """Gauss-law filter passes on E in place (rho: charge density at E's time)."""
    lib().orc_gauss_filter(ctypes.byref(P), _ptr(E), _ptr(rho), int(passes))
    return E


def deposit_current(P: Params, q: float, w: float, X0, X1, J: np.ndarray | None = None) -> np.ndarray:
    if J is None:
        J = np.zeros(_vec(P))
    X0 = np.ascontiguousarray(X0, dtype=np.float64)
    X1 = np.ascontiguousarray(X1, dtype=np.float64)
    lib().orc_deposit_current(ctypes.byref(P), q, w, _ptr(X0), _ptr(X1), _ptr(J))
    return J


# -- whole-array steps -----------------------------------------------------------------------
def step_species_kd(P: Params, kick, q, m, w, pos: np.ndarray, u: np.ndarray, E, B, J) -> int:
    """Steps 1-3 with the momentum update over ``kick`` and the drift over P.dt."""
    n = pos.shape[1]
    return lib().orc_step_species_kd(ctypes.byref(P), kick, q, m, w, n, _ptr(pos), _ptr(u), _ptr(E), _ptr(B),
                                     _ptr(J))


def step_species(P: Params, q, m, w, pos: np.ndarray, u: np.ndarray, E, B, J) -> int:
    """Steps 1-3 for one species, in place on pos/u, accumulating into J."""
    n = pos.shape[1]
    return lib().orc_step_species(ctypes.byref(P), q, m, w, n, _ptr(pos), _ptr(u), _ptr(E), _ptr(B), _ptr(J))


def deposit_rho(P: Params, q, w, pos: np.ndarray, rho: np.ndarray | None = None) -> np.ndarray:
    if rho is None:
        rho = np.zeros(_scal(P))
    lib().orc_deposit_rho(ctypes.byref(P), q, w, pos.shape[1], _ptr(pos), _ptr(rho))
    return rho


def fd_coeffs(order: int) -> np.ndarray:
    a = np.zeros(3)
    lib().orc_fd_coeffs(int(order), _ptr(a))
    return a


def deriv(P: Params, f: np.ndarray, dim: int, up: bool) -> np.ndarray:
    out = np.zeros_like(f)
    lib().orc_deriv(ctypes.byref(P), _ptr(f), _ptr(out), int(dim), int(bool(up)))
    return out


def curl_up(P: Params, F):
    out = np.zeros(_vec(P))
    lib().orc_curl_up(ctypes.byref(P), _ptr(F), _ptr(out))
    return out


def curl_down(P: Params, F):
    out = np.zeros(_vec(P))
    lib().orc_curl_down(ctypes.byref(P), _ptr(F), _ptr(out))
    return out


def div_down(P: Params, F):
    out = np.zeros(_scal(P))
    lib().orc_div_down(ctypes.byref(P), _ptr(F), _ptr(out))
    return out


def div_up(P: Params, F):
    out = np.zeros(_scal(P))
    lib().orc_div_up(ctypes.byref(P), _ptr(F), _ptr(out))
    return out


def laplacian_B(P: Params, B):
    out = np.zeros(_vec(P))
    lib().orc_laplacian_B(ctypes.byref(P), _ptr(B), _ptr(out))
    return out


def field_step(P: Params, E: np.ndarray, B: np.ndarray, J: np.ndarray) -> tuple[int, float]:
    res = np.zeros(1)
    it = lib().orc_field_step(ctypes.byref(P), _ptr(E), _ptr(B), _ptr(J), _ptr(res))
    return it, float(res[0])


def current_high_order(P: Params, J: np.ndarray) -> np.ndarray:
    lib().orc_current_high_order(ctypes.byref(P), _ptr(J))
    return J


def species_moments(P: Params, m, w, u: np.ndarray):
    kin = np.zeros(1)
    mom = np.zeros(3)
    lib().orc_species_moments(ctypes.byref(P), m, w, u.shape[1], _ptr(u), _ptr(kin), _ptr(mom))
    return float(kin[0]), mom


def field_energy(P: Params, E, B):
    out = np.zeros(3)
    lib().orc_field_energy(ctypes.byref(P), _ptr(E), _ptr(B), _ptr(out))
    return out  # (U_E, U_B, U_Ex)


# -- one full time step (paper Sec. III order) -------------------------------------------------
class Run:
    """Oracle state for a whole run: species + mesh, stepped in the paper's order:
    particles (gather, push, move, charge-conserving J), high-order current, fields."""

    def __init__(self, P: Params, species, E=None, B=None):
        self.P = P
        self.species = [dict(q=float(s["q"]), m=float(s["m"]), w=float(s["w"]),
                             pos=np.ascontiguousarray(s["pos"], dtype=np.float64).copy(),
                             u=np.ascontiguousarray(s["u"], dtype=np.float64).copy()) for s in species]
        self.E = np.zeros(_vec(P)) if E is None else np.ascontiguousarray(E, dtype=np.float64).copy()
        self.B = np.zeros(_vec(P)) if B is None else np.ascontiguousarray(B, dtype=np.float64).copy()
        self.J = np.zeros(_vec(P))
        self.flags = 0
        self.relax = (0, 0.0)
        self.nstep = 0  # completed steps

    def particles_step(self, P=None, kick=None):
        P = self.P if P is None else P
        kick = P.dt if kick is None else kick
        self.J[:] = 0.0
        for s in self.species:
            self.flags |= step_species_kd(P, kick, s["q"], s["m"], s["w"], s["pos"], s["u"], self.E, self.B, self.J)
        if P.current_scheme == 0:  # the line solve belongs to the charge-conserving current
            current_high_order(P, self.J)

    def fields_step(self, P=None):
        P = self.P if P is None else P
        self.relax = field_step(P, self.E, self.B, self.J)
        # Gauss-law filter with the charge density of x^{n+1}, after every step or (in single
        # precision, the paper's cadence) after every k-th
        every = max(1, P.gauss_every)
        if P.gauss_passes > 0 and (self.nstep + (1 if P.time_order != 4 else 0)) % every == 0:
            r = np.zeros(_scal(P))
            for s in self.species:
                deposit_rho(P, s["q"], s["w"], s["pos"], r)
            gauss_filter(P, self.E, r, P.gauss_passes)

    def step(self):
        if self.P.time_order == 4:  # three leapfrog substeps (FR_SUBSTEPS)
            for kick, drift in FR_SUBSTEPS:
                Q = substep_params(self.P, drift * self.P.dt)
                self.particles_step(Q, kick * self.P.dt)
                self.fields_step(Q)
            return
        self.particles_step()
        self.fields_step()
        self.nstep += 1

    def rho(self):
        r = np.zeros(_scal(self.P))
        for s in self.species:
            deposit_rho(self.P, s["q"], s["w"], s["pos"], r)
        return r + self.P.rho_background
