"""ctypes wrapper of the FP64 CPU oracle (``lbm_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the package smoke check and the CPU-baseline
leg of ``bench.py``. The HIP product path never imports this module, and this module imports
nothing from the product package.

The oracle follows Yao, Liu, Zhong & Wen, arXiv 2203.04508: equilibrium eq. 14, exact-difference
forcing eq. 13, collision eq. 4 with a single relaxation time, streaming eq. 5, wall density
eq. 15 (first solid layer), curved boundary eqs. 16-17 and the mass modification eq. 18.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

ONE = 65536  # one lattice spacing in the fixed-point geometry units


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call([
            "g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-shared", "-fPIC", "-o", tmp, SRC,
        ])
        os.replace(tmp, LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("tau", C.c_double), ("G", C.c_double),
        ("eos_a", C.c_double), ("eos_b", C.c_double), ("eos_R", C.c_double), ("eos_T", C.c_double),
    ]


def make_params(dim, nx, ny, nz=1, tau=1.0, G=-1.0, a=1.0, b=4.0, R=1.0, T=0.066) -> Params:
    return Params(dim, nx, ny, nz if dim == 3 else 1, tau, G, a, b, R, T)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.POINTER(Params)
        vp = C.c_void_p
        L.or_num_threads.restype = C.c_int
        L.or_lattice.argtypes = [C.c_int, vp, vp, vp, vp]
        L.or_lattice.restype = C.c_int
        L.or_equilibrium.argtypes = [C.c_int, C.c_double, vp, vp]
        L.or_edm_terms.argtypes = [C.c_int, C.c_double, vp, vp, vp]
        L.or_p_eos.argtypes = [P, C.c_double]
        L.or_p_eos.restype = C.c_double
        L.or_psi.argtypes = [P, C.c_double]
        L.or_psi.restype = C.c_double
        L.or_curved_bc.argtypes = [C.c_double, C.c_int] + [C.c_double] * 4
        L.or_curved_bc.restype = C.c_double
        L.or_classify.argtypes = [P, vp, C.c_int64, vp]
        L.or_classify.restype = C.c_int
        L.or_count_links.argtypes = [P, vp]
        L.or_count_links.restype = C.c_int64
        L.or_fill_links.argtypes = [P, vp, C.c_int64, vp, vp, vp, vp, vp, C.c_int64]
        L.or_fill_links.restype = C.c_int
        L.or_wall_nodes.argtypes = [P, vp, vp, C.c_int64]
        L.or_wall_nodes.restype = C.c_int64
        L.or_sim_create.argtypes = [P, vp, vp, vp, vp, C.c_int64]
        L.or_sim_create.restype = vp
        L.or_sim_destroy.argtypes = [vp]
        L.or_sim_set_chempot.argtypes = [vp] + [C.c_double] * 7
        L.or_sim_set_chempot.restype = C.c_int
        L.or_sim_set_mu_wall.argtypes = [vp, vp]
        L.or_sim_set_mu_wall.restype = C.c_int
        L.or_sim_cp_fields.argtypes = [vp, vp, vp]
        L.or_sim_cp_fields.restype = C.c_int
        L.or_pr_p.argtypes = [C.c_double] * 6
        L.or_pr_p.restype = C.c_double
        L.or_pr_mu.argtypes = [C.c_double] * 6
        L.or_pr_mu.restype = C.c_double
        L.or_pr_critical.argtypes = [C.c_double] * 3 + [vp, vp]
        L.or_pr_critical.restype = None
        L.or_sim_set_gravity.argtypes = [vp, C.c_double, C.c_double, C.c_double]
        L.or_sim_set_gravity.restype = C.c_int
        L.or_sim_set_mrt.argtypes = [vp, C.c_double, C.c_double, C.c_double]
        L.or_sim_set_mrt.restype = C.c_int
        L.or_sim_set_bc_mode.argtypes = [vp, C.c_int]
        L.or_sim_set_bc_mode.restype = C.c_int
        L.or_sim_n_wall.argtypes = [vp]
        L.or_sim_n_wall.restype = C.c_int64
        L.or_sim_set_phi.argtypes = [vp, vp]
        L.or_sim_set_phi.restype = C.c_int
        L.or_sim_set_f.argtypes = [vp, vp]
        L.or_sim_set_f.restype = C.c_int
        L.or_sim_init_eq.argtypes = [vp, vp, vp]
        L.or_sim_init_eq.restype = C.c_int
        L.or_sim_step.argtypes = [vp, C.c_int64, vp]
        L.or_sim_step.restype = C.c_int
        L.or_sim_get_f.argtypes = [vp, vp]
        L.or_sim_moments.argtypes = [vp, vp, vp, vp]
        L.or_sim_mass.argtypes = [vp]
        L.or_sim_mass.restype = C.c_double
        L.or_sim_dm_last.argtypes = [vp]
        L.or_sim_dm_last.restype = C.c_double
        L.or_sim_wall_rho.argtypes = [vp, vp, vp]
        L.or_sim_wall_rho.restype = C.c_int64
        L.or_sim_loss.argtypes = [vp, C.c_int, vp, vp]
        L.or_sim_loss.restype = C.c_int
        L.or_dual_kd.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = None
        L.or_dsim_create.argtypes = [P, vp, vp, vp, vp, C.c_int64]
        L.or_dsim_create.restype = vp
        L.or_dsim_destroy.argtypes = [vp]
        L.or_dsim_set_phi.argtypes = [vp, vp, vp]
        L.or_dsim_set_phi.restype = C.c_int
        L.or_dsim_set_chempot.argtypes = [vp] + [C.c_double] * 7
        L.or_dsim_set_chempot.restype = C.c_int
        L.or_dsim_set_mu_wall.argtypes = [vp, vp, vp]
        L.or_dsim_set_mu_wall.restype = C.c_int
        L.or_dsim_set_mrt.argtypes = [vp, C.c_double, C.c_double, C.c_double]
        L.or_dsim_set_mrt.restype = C.c_int
        L.or_dsim_set_gravity.argtypes = [vp, C.c_double, C.c_double, C.c_double]
        L.or_dsim_set_gravity.restype = C.c_int
        L.or_dsim_set_bc_mode.argtypes = [vp, C.c_int]
        L.or_dsim_set_bc_mode.restype = C.c_int
        L.or_dsim_init_eq.argtypes = [vp, vp]
        L.or_dsim_init_eq.restype = C.c_int
        L.or_dsim_step.argtypes = [vp, C.c_int64]
        L.or_dsim_step.restype = C.c_int
        L.or_dsim_loss.argtypes = [vp, C.c_int, vp, vp]
        L.or_dsim_loss.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (timing only; results do not depend on it)."""
    lib().or_set_threads(int(n))


# ---------------------------------------------------------------------------- pointwise pieces
def lattice(dim: int):
    e = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    wf = np.zeros(19)
    opp = np.zeros(19, np.int32)
    Q = lib().or_lattice(dim, _p(e), _p(w), _p(wf), _p(opp))
    return e[:Q].copy(), w[:Q].copy(), wf[:Q].copy(), opp[:Q].copy()


def equilibrium(dim, rho, u):
    Q = 9 if dim == 2 else 19
    out = np.zeros(Q)
    uu = np.zeros(3)
    uu[: len(u)] = u
    lib().or_equilibrium(dim, float(rho), _p(uu), _p(out))
    return out


def edm_terms(dim, rho, u, F):
    Q = 9 if dim == 2 else 19
    out = np.zeros(Q)
    uu = np.zeros(3)
    FF = np.zeros(3)
    uu[: len(u)] = u
    FF[: len(F)] = F
    lib().or_edm_terms(dim, float(rho), _p(uu), _p(FF), _p(out))
    return out


def p_eos(params: Params, rho: float) -> float:
    return lib().or_p_eos(C.byref(params), float(rho))


def psi(params: Params, rho: float) -> float:
    return lib().or_psi(C.byref(params), float(rho))


PR_PAPER = dict(a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344)


def pr_p(rho, T, a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344) -> float:
    """eq. 10 with alpha(T) of Sec. 2.2"""
    return lib().or_pr_p(a, b, R, T, omega, rho)


def pr_mu(rho, T, a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344) -> float:
    """eq. 11 without the gradient term (nan outside 0 < rho < 1/b)"""
    return lib().or_pr_mu(a, b, R, T, omega, rho)


def pr_critical(a=2.0 / 49.0, b=2.0 / 21.0, R=1.0):
    Tc, rc = C.c_double(), C.c_double()
    lib().or_pr_critical(a, b, R, C.byref(Tc), C.byref(rc))
    return Tc.value, rc.value


def curved_bc(q, x2_fluid, ft_i_x1, ft_i_x2, ft_ibar_x1, F_i) -> float:
    return lib().or_curved_bc(float(q), int(bool(x2_fluid)), float(ft_i_x1), float(ft_i_x2),
                              float(ft_ibar_x1), float(F_i))


# ---------------------------------------------------------------------------- geometry
def classify(params: Params, shapes: np.ndarray) -> np.ndarray:
    shapes = np.ascontiguousarray(shapes, np.int64).reshape(-1, 8)
    N = params.nx * params.ny * (params.nz if params.dim == 3 else 1)
    solid = np.zeros(N, np.uint8)
    rc = lib().or_classify(C.byref(params), _p(shapes), len(shapes), _p(solid))
    if rc != 0:
        raise ValueError(f"or_classify failed ({rc})")
    return solid


def links(params: Params, shapes: np.ndarray, solid: np.ndarray):
    """Canonical link list: (node int64, dir int32, cls int32, q_fixed uint32)."""
    shapes = np.ascontiguousarray(shapes, np.int64).reshape(-1, 8)
    n = lib().or_count_links(C.byref(params), _p(solid))
    node = np.zeros(n, np.int64)
    d = np.zeros(n, np.int32)
    cls = np.zeros(n, np.int32)
    q = np.zeros(n, np.uint32)
    rc = lib().or_fill_links(C.byref(params), _p(shapes), len(shapes), _p(solid), _p(node), _p(d), _p(cls), _p(q), n)
    if rc != 0:
        raise ValueError(f"or_fill_links failed ({rc})")
    return node, d, cls, q


def wall_nodes(params: Params, solid: np.ndarray) -> np.ndarray:
    n = lib().or_wall_nodes(C.byref(params), _p(solid), None, 0)
    out = np.zeros(n, np.int64)
    lib().or_wall_nodes(C.byref(params), _p(solid), _p(out), n)
    return out


# ---------------------------------------------------------------------------- simulation
# boundary schemes (Secs. 1, 3 and 4): the present one and the three the paper compares it with
BC_PRESENT, BC_IBC, BC_MIBC, BC_HBBC = 0, 1, 2, 3


class OracleError(RuntimeError):
    pass


class Sim:
    """FP64 reference simulation. State = post-collision populations f~(t) plus the moments
    (rho, u, F) of time t, which eqs. 16-17 need for the forcing term of the next step."""

    def __init__(self, params: Params, solid, lk_node, lk_dir, lk_q):
        self.params = params
        self.dim = params.dim
        self.Q = 9 if self.dim == 2 else 19
        self.N = params.nx * params.ny * (params.nz if self.dim == 3 else 1)
        self._keep = [np.ascontiguousarray(solid, np.uint8), np.ascontiguousarray(lk_node, np.int64),
                      np.ascontiguousarray(lk_dir, np.int32), np.ascontiguousarray(lk_q, np.uint32)]
        s, n, d, q = self._keep
        self.h = lib().or_sim_create(C.byref(params), _p(s), _p(n), _p(d), _p(q), len(n))
        if not self.h:
            raise OracleError("or_sim_create rejected the parameters or the link list")
        self.n_wall = lib().or_sim_n_wall(self.h)

    def close(self):
        if self.h:
            lib().or_sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _check(rc, what):
        if rc == -4:
            raise OracleError(f"{what}: psi domain error (rho <= 0 or negative square-root argument)")
        if rc == -5:
            raise OracleError(f"{what}: non-finite population")
        if rc != 0:
            raise OracleError(f"{what}: error {rc}")

    def set_chempot(self, T, k=1.0, kappa=0.0, a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344):
        """The chemical-potential model (2-D, eqs. 9-12) with the Peng-Robinson EOS for the collisions
        that follow; defaults are the paper's a, b, R and the acentric factor of water."""
        self._check(lib().or_sim_set_chempot(self.h, a, b, R, T, omega, k, kappa), "set_chempot")

    def set_mu_wall(self, mu_s):
        """Assigned chemical potential per first-layer wall node (the wettability, Sec. 2.3)."""
        mu_s = np.ascontiguousarray(np.broadcast_to(np.asarray(mu_s, np.float64), (self.n_wall,)))
        self._check(lib().or_sim_set_mu_wall(self.h, _p(mu_s)), "set_mu_wall")

    def cp_fields(self):
        """(rho, mu) on fluid nodes and the two solid layers as the last collision used them."""
        rho, mu = np.zeros(self.N), np.zeros(self.N)
        self._check(lib().or_sim_cp_fields(self.h, _p(rho), _p(mu)), "cp_fields")
        return rho, mu

    def set_gravity(self, g):
        """Uniform body acceleration (2 or 3 components) added to the force of later collisions."""
        g = list(g) + [0.0] * (3 - len(g))
        self._check(lib().or_sim_set_gravity(self.h, *map(float, g)), "set_gravity")

    def set_mrt(self, se=1.64, seps=1.54, sq=1.7):
        """Multiple-relaxation-time collision (D2Q9, eqs. 1-4) for the collisions that follow, with
        S = diag(1, se, seps, 1, sq, 1, sq, 1/tau, 1/tau); the defaults are the rates of eq. 3."""
        self._check(lib().or_sim_set_mrt(self.h, se, seps, sq), "set_mrt")

    def set_bc_mode(self, mode: int):
        """0 present scheme (eqs. 16-18), 1 IBC (eqs. 16-17 without the forcing term, no eq. 18),
        2 MIBC (IBC with eq. 18), 3 halfway bounce-back."""
        self._check(lib().or_sim_set_bc_mode(self.h, int(mode)), "set_bc_mode")

    def set_phi(self, phi):
        phi = np.ascontiguousarray(np.broadcast_to(np.asarray(phi, np.float64), (self.n_wall,)))
        self._check(lib().or_sim_set_phi(self.h, _p(phi)), "set_phi")

    def init_eq(self, rho0, u0=None):
        rho0 = np.ascontiguousarray(rho0, np.float64).reshape(-1)
        up = None
        if u0 is not None:
            u0 = np.ascontiguousarray(u0, np.float64).reshape(-1)
            up = _p(u0)
        self._check(lib().or_sim_init_eq(self.h, _p(rho0), up), "init_eq")

    def set_f(self, fpre):
        fpre = np.ascontiguousarray(fpre, np.float64).reshape(-1)
        assert fpre.size == self.Q * self.N
        self._check(lib().or_sim_set_f(self.h, _p(fpre)), "set_f")

    def step(self, n=1, record_dm=False):
        hist = np.zeros(max(n, 1)) if record_dm else None
        self._check(lib().or_sim_step(self.h, n, _p(hist) if record_dm else None), "step")
        return hist

    def get_f(self):
        f = np.zeros(self.Q * self.N)
        lib().or_sim_get_f(self.h, _p(f))
        return f.reshape(self.Q, self.N)

    def moments(self):
        rho = np.zeros(self.N)
        v = np.zeros(self.dim * self.N)
        F = np.zeros(self.dim * self.N)
        lib().or_sim_moments(self.h, _p(rho), _p(v), _p(F))
        return rho, v.reshape(self.dim, self.N), F.reshape(self.dim, self.N)

    def mass(self) -> float:
        return lib().or_sim_mass(self.h)

    def dm_last(self) -> float:
        return lib().or_sim_dm_last(self.h)

    def wall_rho(self):
        """(wall node indices, eq. 15 density of each wall node before the wettability factor)."""
        nodes = np.zeros(self.n_wall, np.int64)
        r = np.zeros(self.n_wall)
        lib().or_sim_wall_rho(self.h, _p(nodes), _p(r))
        return nodes, r


def sim_from_shapes(params: Params, shapes):
    solid = classify(params, shapes)
    node, d, cls, q = links(params, shapes, solid)
    return Sim(params, solid, node, d, q), (solid, node, d, cls, q)


# ---------------------------------------------------------------------------- losses and derivatives
LOSS_COM_X, LOSS_WETTED_LENGTH, LOSS_TOTAL_MASS = 0, 1, 2


def sim_loss(sim: Sim, kind: int, prm=(0.0, 1.0)) -> float:
    """Loss of the stored state f~(T) (kinds: 0 centre of mass in x, 1 smooth wetted length,
    2 total mass)."""
    prm = np.ascontiguousarray(prm, np.float64)
    out = np.zeros(1)
    Sim._check(lib().or_sim_loss(sim.h, kind, _p(prm), _p(out)), "loss")
    return float(out[0])


def dual_kd() -> int:
    return lib().or_dual_kd()


class DualSim:
    """The same simulation in forward-mode dual numbers: the wettability factors carry up to
    KD tangent directions, and loss() returns the loss with its directional derivatives."""

    def __init__(self, params: Params, solid, lk_node, lk_dir, lk_q):
        self.params = params
        self.N = params.nx * params.ny * (params.nz if params.dim == 3 else 1)
        self._keep = [np.ascontiguousarray(solid, np.uint8), np.ascontiguousarray(lk_node, np.int64),
                      np.ascontiguousarray(lk_dir, np.int32), np.ascontiguousarray(lk_q, np.uint32)]
        s, n, d, q = self._keep
        self.h = lib().or_dsim_create(C.byref(params), _p(s), _p(n), _p(d), _p(q), len(n))
        if not self.h:
            raise OracleError("or_dsim_create rejected the parameters or the link list")
        self.kd = dual_kd()

    def close(self):
        if self.h:
            lib().or_dsim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_phi(self, phi, directions=None):
        """phi: (n_wall,); directions: up to KD tangent vectors, shape (m, n_wall)."""
        phi = np.ascontiguousarray(phi, np.float64)
        d = None
        if directions is not None:
            directions = np.atleast_2d(np.asarray(directions, np.float64))
            assert directions.shape[0] <= self.kd and directions.shape[1] == len(phi)
            d = np.zeros((self.kd, len(phi)))
            d[: directions.shape[0]] = directions
        Sim._check(lib().or_dsim_set_phi(self.h, _p(phi), _p(d) if d is not None else None), "set_phi")

    def set_mrt(self, se=1.64, seps=1.54, sq=1.7):
        Sim._check(lib().or_dsim_set_mrt(self.h, se, seps, sq), "set_mrt")

    def set_chempot(self, T, k=1.0, kappa=0.0, a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344):
        Sim._check(lib().or_dsim_set_chempot(self.h, a, b, R, T, omega, k, kappa), "set_chempot")

    def set_mu_wall(self, mu_s, directions=None):
        """mu_s: (n_wall,) assigned wall chemical potentials; directions: up to KD tangent vectors,
        shape (m, n_wall)."""
        mu_s = np.ascontiguousarray(mu_s, np.float64)
        nw = len(mu_s)
        d = None
        if directions is not None:
            d = np.zeros((dual_kd(), nw))
            dd = np.asarray(directions, np.float64).reshape(-1, nw)
            d[: len(dd)] = dd
            d = np.ascontiguousarray(d)
        Sim._check(lib().or_dsim_set_mu_wall(self.h, _p(mu_s), _p(d) if d is not None else None), "set_mu_wall")

    def set_gravity(self, g):
        g = list(g) + [0.0] * (3 - len(g))
        Sim._check(lib().or_dsim_set_gravity(self.h, *map(float, g)), "set_gravity")

    def set_bc_mode(self, mode: int):
        Sim._check(lib().or_dsim_set_bc_mode(self.h, int(mode)), "set_bc_mode")

    def init_eq(self, rho0):
        rho0 = np.ascontiguousarray(rho0, np.float64).reshape(-1)
        Sim._check(lib().or_dsim_init_eq(self.h, _p(rho0)), "init_eq")

    def step(self, n=1):
        Sim._check(lib().or_dsim_step(self.h, n), "step")

    def loss(self, kind: int, prm=(0.0, 1.0)):
        """(value, array of KD directional derivatives)."""
        prm = np.ascontiguousarray(prm, np.float64)
        out = np.zeros(1 + self.kd)
        Sim._check(lib().or_dsim_loss(self.h, kind, _p(prm), _p(out)), "loss")
        return float(out[0]), out[1:].copy()
