"""Python binding of libmcb (``include/mcb.h``): one function per C entry point, same names,
argument marshalling only.  Every step of the simulation runs in the HIP kernels of the library;
torch provides the device arenas and the stream.

:class:`Lattice` strings the calls together (create -> bind -> geometry -> links -> state ->
step -> observe) and owns the torch tensors that back the device arenas.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcb.so")

MCB_OK, MCB_EINVAL, MCB_ESIZE, MCB_EHIP, MCB_EDOMAIN, MCB_ENAN, MCB_ESTATE, MCB_ENOTSUP = 0, -1, -2, -3, -4, -5, -6, -7
MCB_F64, MCB_F32S, MCB_F16S = 0, 1, 2
MCB_BC_PRESENT, MCB_BC_IBC, MCB_BC_MIBC, MCB_BC_HBBC = 0, 1, 2, 3
MCB_COLL_BGK, MCB_COLL_MRT = 0, 1
MCB_MODEL_PSEUDO, MCB_MODEL_CHEMPOT = 0, 1
PR_PAPER = dict(a=2.0 / 49.0, b=2.0 / 21.0, R=1.0, omega=0.344)  # Sec. 2.2: a, b, R, water's omega
MRT_RATES_PAPER = (1.64, 1.54, 1.7)  # s_e, s_epsilon, s_q of eq. 3
BC_MODES = {"present": MCB_BC_PRESENT, "ibc": MCB_BC_IBC, "mibc": MCB_BC_MIBC, "hbbc": MCB_BC_HBBC}
MCB_COUNT, MCB_FILL = 0, 1
PRECISIONS = {"f64": MCB_F64, "f32s": MCB_F32S, "f16s": MCB_F16S}
STATUS_NAMES = {0: "MCB_OK", -1: "MCB_EINVAL", -2: "MCB_ESIZE", -3: "MCB_EHIP", -4: "MCB_EDOMAIN",
                -5: "MCB_ENAN", -6: "MCB_ESTATE", -7: "MCB_ENOTSUP"}


class mcb_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("tau", C.c_double), ("G", C.c_double),
                ("eos_a", C.c_double), ("eos_b", C.c_double), ("eos_R", C.c_double), ("eos_T", C.c_double),
                ("precision", C.c_int32), ("bc_mode", C.c_int32), ("rho_ref", C.c_double),
                ("collision", C.c_int32), ("track_dm", C.c_int32),
                ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double), ("gravity", C.c_double * 3),
                ("model", C.c_int32), ("reserved2", C.c_int32), ("pr_omega", C.c_double),
                ("cp_k", C.c_double), ("cp_kappa", C.c_double)]


class mcb_shape(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("kind", "cx", "cy", "cz", "radius", "lo", "hi", "group")]


class mcb_link(C.Structure):
    _fields_ = [("node", C.c_int64), ("dir", C.c_int32), ("cls", C.c_int32), ("q_fixed", C.c_uint32), ("pad", C.c_uint32)]


LINK_DTYPE = np.dtype([("node", np.int64), ("dir", np.int32), ("cls", np.int32), ("q_fixed", np.uint32), ("pad", np.uint32)])


class mcb_sizes(C.Structure):
    _fields_ = [("lattice_bytes", C.c_int64), ("links_bytes", C.c_int64)]


class mcb_buffers(C.Structure):
    _fields_ = [("lattice", C.c_void_p), ("lattice_bytes", C.c_int64), ("links", C.c_void_p), ("links_bytes", C.c_int64)]


class mcb_mass_report(C.Structure):
    _fields_ = [("M", C.c_double), ("J", C.c_double * 3), ("dM_last", C.c_double),
                ("n_nan", C.c_int64), ("n_domain", C.c_int64), ("t", C.c_int64), ("dM_cum", C.c_double)]


EXPORTS = [
    "mcb_create", "mcb_destroy", "mcb_last_error", "mcb_required_sizes", "mcb_bind_buffers",
    "mcb_set_geometry", "mcb_build_links", "mcb_get_links", "mcb_get_wall_nodes", "mcb_set_links",
    "mcb_set_wettability", "mcb_init_equilibrium", "mcb_set_f", "mcb_get_f", "mcb_step",
    "mcb_moments", "mcb_max_speed", "mcb_mass", "mcb_mass_static", "mcb_sync", "mcb_timing", "mcb_timing_report",
    "mcb_adj_required_bytes", "mcb_adj_bind", "mcb_adj_forward", "mcb_adj_generation", "mcb_adj_backward",
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libmcb.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libmcb.so not found at {path}: build it with paper_2203_04508_amd/build.py")
    L = C.CDLL(path)
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    P = C.POINTER
    sig = {
        "mcb_create": ([P(mcb_params), P(vp)], i32),
        "mcb_destroy": ([vp], None),
        "mcb_last_error": ([vp], C.c_char_p),
        "mcb_required_sizes": ([P(mcb_params), i64, i64, i64, i64, P(mcb_sizes)], i32),
        "mcb_bind_buffers": ([vp, P(mcb_buffers), vp], i32),
        "mcb_set_geometry": ([vp, vp, i64], i32),
        "mcb_build_links": ([vp, i32, P(i64), P(i64), P(i64)], i32),
        "mcb_get_links": ([vp, vp, i64], i32),
        "mcb_get_wall_nodes": ([vp, vp, i64], i32),
        "mcb_set_links": ([vp, vp, i64], i32),
        "mcb_set_wettability": ([vp, vp, i64], i32),
        "mcb_init_equilibrium": ([vp, vp, vp], i32),
        "mcb_set_f": ([vp, vp], i32),
        "mcb_get_f": ([vp, vp], i32),
        "mcb_step": ([vp, i64], i32),
        "mcb_moments": ([vp, vp, vp], i32),
        "mcb_max_speed": ([vp, vp, vp], i32),
        "mcb_mass": ([vp, P(mcb_mass_report)], i32),
        "mcb_mass_static": ([vp, P(mcb_mass_report)], i32),
        "mcb_sync": ([vp], i32),
        "mcb_timing": ([vp, i32], i32),
        "mcb_timing_report": ([vp, P(C.c_double), P(i64)], i32),
        "mcb_adj_required_bytes": ([vp, i64, i64, P(i64)], i32),
        "mcb_adj_bind": ([vp, vp, i64], i32),
        "mcb_adj_forward": ([vp, vp, i64, i64, i32, vp, P(C.c_double)], i32),
        "mcb_adj_generation": ([vp, P(i64)], i32),
        "mcb_adj_backward": ([vp, i64, C.c_double, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


class MCBError(RuntimeError):
    def __init__(self, code, where, msg):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(ctx, code, where):
    if code != MCB_OK:
        msg = load().mcb_last_error(ctx) if ctx else b""
        raise MCBError(code, where, (msg or b"").decode())


# ---------------------------------------------------------------- one wrapper per entry point
def mcb_create(params: mcb_params):
    h = C.c_void_p()
    code = load().mcb_create(C.byref(params), C.byref(h))
    if code != MCB_OK:
        raise MCBError(code, "mcb_create", "unsupported combination" if code == -7 else "invalid parameters")
    return h


def mcb_destroy(ctx):
    load().mcb_destroy(ctx)


def mcb_last_error(ctx) -> str:
    return (load().mcb_last_error(ctx) or b"").decode()


def mcb_required_sizes(params: mcb_params, n_shapes=0, n_links=0, n_bnodes=0, n_wall=0) -> mcb_sizes:
    out = mcb_sizes()
    code = load().mcb_required_sizes(C.byref(params), n_shapes, n_links, n_bnodes, n_wall, C.byref(out))
    if code != MCB_OK:
        raise MCBError(code, "mcb_required_sizes", "invalid arguments")
    return out


def mcb_bind_buffers(ctx, lattice_ptr, lattice_bytes, links_ptr, links_bytes, stream_handle):
    b = mcb_buffers(lattice_ptr, lattice_bytes, links_ptr, links_bytes)
    _check(ctx, load().mcb_bind_buffers(ctx, C.byref(b), C.c_void_p(stream_handle)), "mcb_bind_buffers")


def mcb_set_geometry(ctx, shapes: np.ndarray):
    shapes = np.ascontiguousarray(shapes, np.int64).reshape(-1, 8)
    _check(ctx, load().mcb_set_geometry(ctx, _ptr(shapes), len(shapes)), "mcb_set_geometry")


def mcb_build_links(ctx, phase):
    nl, nb, nw = C.c_int64(), C.c_int64(), C.c_int64()
    _check(ctx, load().mcb_build_links(ctx, phase, C.byref(nl), C.byref(nb), C.byref(nw)), "mcb_build_links")
    return nl.value, nb.value, nw.value


def mcb_get_links(ctx, n_links) -> np.ndarray:
    out = np.zeros(n_links, LINK_DTYPE)
    _check(ctx, load().mcb_get_links(ctx, _ptr(out), n_links), "mcb_get_links")
    return out


def mcb_get_wall_nodes(ctx, n_wall) -> np.ndarray:
    out = np.zeros(n_wall, np.int64)
    _check(ctx, load().mcb_get_wall_nodes(ctx, _ptr(out), n_wall), "mcb_get_wall_nodes")
    return out


def mcb_set_links(ctx, links: np.ndarray):
    links = np.ascontiguousarray(links, LINK_DTYPE)
    _check(ctx, load().mcb_set_links(ctx, _ptr(links), len(links)), "mcb_set_links")


def mcb_set_wettability(ctx, phi: np.ndarray):
    phi = np.ascontiguousarray(phi, np.float64)
    _check(ctx, load().mcb_set_wettability(ctx, _ptr(phi), len(phi)), "mcb_set_wettability")


def mcb_init_equilibrium(ctx, rho: np.ndarray, u: np.ndarray | None = None):
    rho = np.ascontiguousarray(rho, np.float64)
    u = None if u is None else np.ascontiguousarray(u, np.float64)
    _check(ctx, load().mcb_init_equilibrium(ctx, _ptr(rho), _ptr(u)), "mcb_init_equilibrium")


def mcb_set_f(ctx, f: np.ndarray):
    f = np.ascontiguousarray(f, np.float64)
    _check(ctx, load().mcb_set_f(ctx, _ptr(f)), "mcb_set_f")


def mcb_get_f(ctx, Q, N) -> np.ndarray:
    f = np.zeros((Q, N))
    _check(ctx, load().mcb_get_f(ctx, _ptr(f)), "mcb_get_f")
    return f


def mcb_step(ctx, n):
    _check(ctx, load().mcb_step(ctx, int(n)), "mcb_step")


def mcb_moments(ctx, dim, N):
    rho = np.zeros(N)
    v = np.zeros((dim, N))
    _check(ctx, load().mcb_moments(ctx, _ptr(rho), _ptr(v)), "mcb_moments")
    return rho, v


def mcb_max_speed(ctx):
    """(largest |v| over the fluid nodes, smallest node index attaining it)."""
    v = C.c_double()
    n = C.c_int64()
    _check(ctx, load().mcb_max_speed(ctx, C.byref(v), C.byref(n)), "mcb_max_speed")
    return v.value, n.value


def mcb_mass(ctx) -> mcb_mass_report:
    r = mcb_mass_report()
    _check(ctx, load().mcb_mass(ctx, C.byref(r)), "mcb_mass")
    return r


def mcb_mass_static(ctx) -> mcb_mass_report:
    r = mcb_mass_report()
    _check(ctx, load().mcb_mass_static(ctx, C.byref(r)), "mcb_mass_static")
    return r


def mcb_sync(ctx):
    _check(ctx, load().mcb_sync(ctx), "mcb_sync")


def mcb_timing(ctx, enable: bool):
    _check(ctx, load().mcb_timing(ctx, 1 if enable else 0), "mcb_timing")


def mcb_timing_report(ctx):
    """(total ms of the fused step kernel, number of timed launches)"""
    ms = C.c_double()
    n = C.c_int64()
    _check(ctx, load().mcb_timing_report(ctx, C.byref(ms), C.byref(n)), "mcb_timing_report")
    return ms.value, n.value


MCB_LOSS_COM_X, MCB_LOSS_WETTED_LENGTH, MCB_LOSS_TOTAL_MASS = 0, 1, 2
LOSS_COM_X, LOSS_WETTED_LENGTH, LOSS_TOTAL_MASS = MCB_LOSS_COM_X, MCB_LOSS_WETTED_LENGTH, MCB_LOSS_TOTAL_MASS

# Per-boundary-node storage of the step kernel (compute-type values), for traffic accounting: the
# boundary record (forcing terms, populations, eq. 18 correction) and the link-coefficient slots.
REC2, REC3 = 16, 28
Q2_LINKS, Q3_LINKS = 8, 20


def mcb_adj_required_bytes(ctx, nsteps, k) -> int:
    b = C.c_int64()
    _check(ctx, load().mcb_adj_required_bytes(ctx, int(nsteps), int(k), C.byref(b)), "mcb_adj_required_bytes")
    return b.value


def mcb_adj_bind(ctx, dev_ptr, nbytes):
    _check(ctx, load().mcb_adj_bind(ctx, C.c_void_p(dev_ptr), int(nbytes)), "mcb_adj_bind")


def mcb_adj_forward(ctx, rho0, nsteps, k, kind, prm) -> float:
    rho0 = np.ascontiguousarray(rho0, np.float64).reshape(-1)
    prm = np.ascontiguousarray(np.resize(np.asarray(prm, np.float64), 2))
    v = C.c_double()
    _check(ctx, load().mcb_adj_forward(ctx, _ptr(rho0), int(nsteps), int(k), int(kind), _ptr(prm), C.byref(v)),
           "mcb_adj_forward")
    return v.value


def mcb_adj_generation(ctx) -> int:
    g = C.c_int64()
    _check(ctx, load().mcb_adj_generation(ctx, C.byref(g)), "mcb_adj_generation")
    return g.value


def mcb_adj_backward(ctx, generation, dloss, n_wall) -> np.ndarray:
    d = np.zeros(max(n_wall, 1))
    _check(ctx, load().mcb_adj_backward(ctx, int(generation), float(dloss), _ptr(d)), "mcb_adj_backward")
    return d[:n_wall]


# ---------------------------------------------------------------- convenience object
class Lattice:
    """A context plus the torch tensors backing its device arenas."""

    def __init__(self, dim, dims, tau, T, precision="f64", rho_ref=0.0, G=-1.0, a=None, b=None, R=1.0,
                 device="cuda:0", stream=None, bc_mode="present", collision="bgk", mrt_rates=MRT_RATES_PAPER,
                 gravity=(0.0, 0.0, 0.0), model="pseudo", cp_k=1.0, cp_kappa=0.0, pr_omega=PR_PAPER["omega"],
                 track_dm=False):
        """model "pseudo": pseudopotential with the Carnahan-Starling EOS (a, b default 1, 4);
        model "chempot": the chemical-potential model with the Peng-Robinson EOS (a, b default to the
        paper's 2/49, 2/21), mesh scaling cp_k and gradient coefficient cp_kappa.  track_dm: sum each
        step's eq. 18 total into the mass report's dM_cum."""
        import torch

        self.torch = torch
        self.device = torch.device(device)
        nz = dims[2] if dim == 3 else 1
        cp = model == "chempot"
        if a is None:
            a = PR_PAPER["a"] if cp else 1.0
        if b is None:
            b = PR_PAPER["b"] if cp else 4.0
        self.params = mcb_params(dim, dims[0], dims[1], nz, tau, G, a, b, R, T,
                                 PRECISIONS[precision] if isinstance(precision, str) else precision,
                                 BC_MODES[bc_mode] if isinstance(bc_mode, str) else bc_mode, rho_ref,
                                 {"bgk": MCB_COLL_BGK, "mrt": MCB_COLL_MRT}[collision], 1 if track_dm else 0, *mrt_rates,
                                 (C.c_double * 3)(*(list(gravity) + [0.0] * (3 - len(gravity)))),
                                 MCB_MODEL_CHEMPOT if cp else MCB_MODEL_PSEUDO, 0, pr_omega, cp_k, cp_kappa)
        self.dim = dim
        self.Q = 9 if dim == 2 else 19
        self.N = int(dims[0]) * int(dims[1]) * int(nz)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = mcb_create(self.params)
        self.lat = None
        self.lnk = None
        self.n_links = self.n_bnodes = self.n_wall = 0

    def close(self):
        if getattr(self, "ctx", None):
            mcb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind(self):
        lp = self.lat.data_ptr()
        kp = self.lnk.data_ptr() if self.lnk is not None and self.lnk.numel() else None
        mcb_bind_buffers(self.ctx, lp, self.lat.numel(), kp, 0 if kp is None else self.lnk.numel(),
                         self.stream.cuda_stream)

    def set_geometry(self, shapes):
        torch = self.torch
        shapes = np.ascontiguousarray(shapes, np.int64).reshape(-1, 8)
        sz = mcb_required_sizes(self.params, len(shapes))
        if self.lat is None or self.lat.numel() < sz.lattice_bytes:
            self.lat = torch.empty(sz.lattice_bytes, dtype=torch.uint8, device=self.device)
        self._bind()
        mcb_set_geometry(self.ctx, shapes)
        self.n_links, self.n_bnodes, self.n_wall = mcb_build_links(self.ctx, MCB_COUNT)
        sz = mcb_required_sizes(self.params, len(shapes), self.n_links, self.n_bnodes, self.n_wall)
        if sz.links_bytes > 0:
            self.lnk = torch.empty(sz.links_bytes, dtype=torch.uint8, device=self.device)
        self._bind()
        mcb_build_links(self.ctx, MCB_FILL)
        return self.n_links, self.n_bnodes, self.n_wall

    def links(self):
        return mcb_get_links(self.ctx, self.n_links)

    def wall_nodes(self):
        return mcb_get_wall_nodes(self.ctx, self.n_wall)

    def set_links(self, links):
        mcb_set_links(self.ctx, links)

    def set_wettability(self, phi):
        phi = np.ascontiguousarray(np.broadcast_to(np.asarray(phi, np.float64), (self.n_wall,)))
        mcb_set_wettability(self.ctx, phi)

    def init_equilibrium(self, rho, u=None):
        mcb_init_equilibrium(self.ctx, np.asarray(rho, np.float64).reshape(-1),
                             None if u is None else np.asarray(u, np.float64).reshape(-1))

    def set_f(self, f):
        mcb_set_f(self.ctx, np.asarray(f, np.float64).reshape(self.Q, self.N))

    def get_f(self):
        return mcb_get_f(self.ctx, self.Q, self.N)

    def step(self, n=1):
        mcb_step(self.ctx, n)

    def moments(self):
        return mcb_moments(self.ctx, self.dim, self.N)

    def mass(self):
        return mcb_mass(self.ctx)

    def mass_static(self):
        return mcb_mass_static(self.ctx)

    def max_speed(self):
        return mcb_max_speed(self.ctx)

    def sync(self):
        mcb_sync(self.ctx)

    def timing(self, enable=True):
        mcb_timing(self.ctx, enable)

    def timing_report(self):
        return mcb_timing_report(self.ctx)

    # ---- reverse mode
    def adj_forward(self, rho0, nsteps, k, kind=MCB_LOSS_COM_X, prm=(0.0, 1.0)) -> float:
        """Equilibrium start from rho0, nsteps steps with a checkpoint every k; returns the loss."""
        need = mcb_adj_required_bytes(self.ctx, nsteps, k)
        if getattr(self, "adj", None) is None or self.adj.numel() < need:
            self.adj = None
            self.adj = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        mcb_adj_bind(self.ctx, self.adj.data_ptr(), self.adj.numel())
        val = mcb_adj_forward(self.ctx, rho0, nsteps, k, kind, prm)
        self.adj_gen = mcb_adj_generation(self.ctx)
        return val

    def adj_backward(self, dloss=1.0, generation=None) -> np.ndarray:
        """dloss * d loss / d phi per wall node, for the forward pass of the given generation (default:
        the last adj_forward); MCBError (MCB_ESTATE) once that pass is superseded or its state changed."""
        gen = self.adj_gen if generation is None else generation
        return mcb_adj_backward(self.ctx, gen, dloss, self.n_wall)


def _wettability_loss_class():
    import torch

    class WettabilityLoss(torch.autograd.Function):
        """loss(phi) of the state after nsteps steps from the equilibrium start rho0, with the
        hand-written reverse mode of the step as its backward.

        forward(phi, lattice, rho0, nsteps, k, kind, prm): phi is a float64 tensor with one
        entry per wall node (any device); returns a 0-d float64 tensor on phi's device."""

        @staticmethod
        def forward(ctx, phi, lattice, rho0, nsteps, k, kind=MCB_LOSS_COM_X, prm=(0.0, 1.0)):
            lattice.set_wettability(phi.detach().to("cpu", torch.float64).numpy())
            val = lattice.adj_forward(rho0, nsteps, k, kind, prm)
            ctx.lattice = lattice
            ctx.generation = lattice.adj_gen  # backward refuses once another forward pass has run
            ctx.phi_device = phi.device
            return torch.tensor(val, dtype=torch.float64, device=phi.device)

        @staticmethod
        def backward(ctx, g):
            d = ctx.lattice.adj_backward(float(g), generation=ctx.generation)
            return torch.from_numpy(d).to(ctx.phi_device), None, None, None, None, None, None

    return WettabilityLoss


def __getattr__(name):
    if name == "WettabilityLoss":
        cls = _wettability_loss_class()
        globals()["WettabilityLoss"] = cls
        return cls
    raise AttributeError(name)
