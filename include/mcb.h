/*
 * mcb.h -- C ABI of libmcb: one pseudopotential multiphase lattice Boltzmann time step with the
 * multiphase curved wetting boundary of Yao, Liu, Zhong & Wen, "Multiphase curved boundary
 * condition in lattice Boltzmann method" (arXiv 2203.04508), on AMD Instinct MI355X (gfx950).
 *
 * The step (Sec. 2-3 of the paper):
 *   streaming, eq. 5, pull form; incoming populations across fluid-solid links from the curved
 *   boundary condition, eq. 16 (0 <= q < 1/2) and eq. 17 (1/2 <= q <= 1), each carrying the
 *   nonideal forcing term F_i(x1, t) of eq. 13; the interpolation-error mass modification of
 *   eq. 18 added to the rest population of every boundary-fluid node; then density, velocity,
 *   the EOS-based pseudopotential psi(rho) with first-layer wall densities from eq. 15 times a
 *   wettability factor phi, the nearest-neighbour interaction force, and single-relaxation-time
 *   collision (eq. 4 with S = I/tau) with exact-difference forcing (eqs. 13-14).
 *
 * Conventions
 *   - Every function returns an mcb_status: 0 on success, a negative MCB_E* code otherwise.
 *     Nothing throws across the ABI. mcb_last_error() returns a description of the last error of
 *     a context (a pointer owned by the context, valid until its next call).
 *   - Host arrays passed in are owned by the caller and copied before the call returns.
 *   - Device memory is owned by the caller: mcb_required_sizes() gives the byte sizes of two
 *     arenas (lattice, links) that the caller allocates (e.g. as torch tensors) and binds with
 *     mcb_bind_buffers(). The library allocates no device memory. Arenas must stay alive and
 *     bound while the context uses them; mcb_bind_buffers() may be called again (e.g. once the
 *     link counts are known).
 *   - Work is queued on the HIP stream given to mcb_bind_buffers(). mcb_step() and the geometry
 *     FILL phase are asynchronous; faults detected on the device (non-finite populations, psi
 *     domain errors) are reported by the next synchronising call: mcb_mass, mcb_moments,
 *     mcb_get_f, mcb_sync.
 *   - A context is used by one host thread at a time.
 *   - Node linear index: x + nx * (y + ny * z). Population arrays on the host are SoA, [Q][N].
 *   - D2Q9 velocity order is the column order of the moment matrix M (eq. 2):
 *     (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
 *     D3Q19: rest, (+-1,0,0), (0,+-1,0), (0,0,+-1), then (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0)
 *     (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).
 */
#ifndef MCB_H
#define MCB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mcb_status;

enum {
    MCB_OK = 0,
    MCB_EINVAL = -1,   /* bad argument */
    MCB_ESIZE = -2,    /* a buffer or capacity is too small */
    MCB_EHIP = -3,     /* a HIP runtime call failed */
    MCB_EDOMAIN = -4,  /* psi undefined: rho <= 0 or negative square-root argument */
    MCB_ENAN = -5,     /* non-finite population */
    MCB_ESTATE = -6,   /* call out of order */
    MCB_ENOTSUP = -7   /* unsupported combination */
};

/* storage of the populations */
enum {
    MCB_F64 = 0,   /* FP64 storage and arithmetic */
    MCB_F32S = 1,  /* shifted FP32 storage g_i = f_i - w_i rho_ref, FP32 arithmetic */
    MCB_F16S = 2   /* shifted FP16 storage, FP32 arithmetic */
};

/* boundary scheme on fluid-solid links: the paper's (Sec. 3) and the three it is compared with
 * (Secs. 1 and 4).  All four coincide at q = 1/2. */
enum {
    MCB_BC_PRESENT = 0, /* eqs. 16-18: interpolation with the forcing term, plus mass modification */
    MCB_BC_IBC = 1,     /* eqs. 16-17 without the forcing term, no eq. 18 */
    MCB_BC_MIBC = 2,    /* eqs. 16-17 without the forcing term, with eq. 18 */
    MCB_BC_HBBC = 3     /* halfway bounce-back on every link (q ignored; eq. 18 terms are zero) */
};

/* collision operator */
enum {
    MCB_COLL_BGK = 0,  /* eq. 4 with S = I/tau (single relaxation time) */
    MCB_COLL_MRT = 1   /* eqs. 1-4: moment matrix of eq. 2, S = diag(1, s_e, s_eps, 1, s_q, 1, s_q,
                          1/tau, 1/tau) of eq. 3; D2Q9 only (MCB_ENOTSUP from mcb_create for dim 3) */
};

/* multiphase model */
enum {
    MCB_MODEL_PSEUDO = 0,  /* pseudopotential, psi from the Carnahan-Starling EOS; wettability phi scales
                              the first-layer wall density of eq. 15 */
    MCB_MODEL_CHEMPOT = 1  /* the paper's chemical-potential model (Secs. 2.2-2.3), D2Q9 only: Peng-Robinson
                              EOS (eq. 10; eos_a, eos_b, eos_R, eos_T are its a, b, R, T; G is ignored),
                              mu = k^2 mu_PR(rho) - kappa lap(rho) (eqs. 11-12), F = -rho grad mu +
                              grad(rho)/3 (eq. 9) by fourth-order central differences, densities on two solid
                              layers by eq. 15; the wettability values are the assigned chemical potential of
                              each wall node (both layers take it) */
};

/* build_links phases */
enum { MCB_COUNT = 0, MCB_FILL = 1 };

/* shape kinds (units: 2^-16 lattice spacings) */
enum { MCB_SHAPE_BALL = 1, MCB_SHAPE_BAND_Y = 2 };

/* link classes */
enum { MCB_CLS_EQ16 = 0, MCB_CLS_HBB = 1, MCB_CLS_EQ17 = 2 };

typedef struct mcb_ctx mcb_ctx;

typedef struct {
    int32_t dim;            /* 2 (D2Q9) or 3 (D3Q19) */
    int32_t nx, ny, nz;     /* periodic box, each in [3, 32768]; nz = 1 for dim 2; N < 2^31 */
    double tau;             /* relaxation time, > 1/2 */
    double G;               /* interaction strength of the pseudopotential force, < 0 */
    double eos_a, eos_b, eos_R, eos_T;  /* Carnahan-Starling EOS parameters and temperature */
    int32_t precision;      /* MCB_F64, MCB_F32S, MCB_F16S */
    int32_t bc_mode;        /* MCB_BC_PRESENT, MCB_BC_IBC, MCB_BC_MIBC, MCB_BC_HBBC */
    double rho_ref;         /* shift of the stored populations (ignored for MCB_F64) */
    int32_t collision;      /* MCB_COLL_BGK (0, the default of a zeroed struct) or MCB_COLL_MRT */
    int32_t track_dm;       /* nonzero: every mcb_step also adds the step's eq. 18 total (Delta M of
                               Sec. 3.2) to an FP64 sum on the device, reported as dM_cum (two small
                               extra launches per step); 0: dM_cum is reported as NaN */
    double s_e, s_eps, s_q; /* MRT rates of the energy, energy-square and heat-flux moments, each in
                               (0, 2) for MCB_COLL_MRT (the paper's: 1.64, 1.54, 1.7); ignored for BGK */
    double gravity[3];      /* uniform body acceleration g (lattice units): the force of eq. 13 and of
                               eqs. 16-17 becomes F_nonideal + rho g (Sec. 4.5 runs with gravity);
                               finite; gravity[2] = 0 for dim 2; zero = no body force */
    int32_t model;          /* MCB_MODEL_PSEUDO (0) or MCB_MODEL_CHEMPOT (dim 2 only, else MCB_ENOTSUP) */
    int32_t reserved2;      /* 0 */
    double pr_omega;        /* MCB_MODEL_CHEMPOT: acentric factor of alpha(T) (water: 0.344) */
    double cp_k, cp_kappa;  /* MCB_MODEL_CHEMPOT: mesh scaling k > 0 and gradient coefficient kappa >= 0 (eq. 12) */
} mcb_params;

/* A solid shape. kind MCB_SHAPE_BALL: centre (cx, cy, cz) and radius; a node is solid when it
 * lies strictly inside. kind MCB_SHAPE_BAND_Y: the periodic band lo <= y < hi (x, z free).
 * group is carried for the caller (e.g. a wettability table) and not used by the library. */
typedef struct {
    int64_t kind, cx, cy, cz, radius, lo, hi, group;
} mcb_shape;

/* One fluid-solid link (x1 fluid, x1 + e_dir solid). q = q_fixed / 2^16 is the first point of
 * the segment x1 -> x1 + e_dir inside or on a shape (Sec. 3.1, Figs. 1-2); cls is
 * MCB_CLS_EQ16 (q < 1/2, x2 = x1 - e_dir fluid), MCB_CLS_HBB (q < 1/2, x2 solid: halfway
 * bounce-back) or MCB_CLS_EQ17 (q >= 1/2). Canonical order: node ascending, then dir. */
typedef struct {
    int64_t node;
    int32_t dir, cls;
    uint32_t q_fixed, pad;
} mcb_link;

typedef struct {
    int64_t lattice_bytes;  /* populations (two lattices), node tags, scratch */
    int64_t links_bytes;    /* boundary-node, link and wall-node tables */
} mcb_sizes;

typedef struct {
    void* lattice;          /* device pointer, >= lattice_bytes, 256-byte aligned */
    int64_t lattice_bytes;
    void* links;            /* device pointer, >= links_bytes, 256-byte aligned; may be NULL
                               before the link counts are known */
    int64_t links_bytes;
} mcb_buffers;

typedef struct {
    double M;        /* total mass: sum over fluid nodes of the populations (FP64 reduction) */
    double J[3];     /* total post-collision momentum */
    double dM_last;  /* sum of the eq. 18 corrections of the last step (the paper's Delta M) */
    int64_t n_nan;   /* fluid nodes with a non-finite population */
    int64_t n_domain;/* psi domain errors since the state was set */
    int64_t t;       /* steps taken since the state was set */
    double dM_cum;   /* sum of dM_last over the mcb_step steps since the state was set (Sec. 3.2),
                        summed in FP64 in a fixed order; NaN unless params.track_dm */
} mcb_mass_report;

/* ---- context ---------------------------------------------------------------------------- */
/* Validates params (MCB_EINVAL otherwise; MCB_ENOTSUP for MCB_COLL_MRT or MCB_MODEL_CHEMPOT in 3-D) and creates a
 * context; no device work. */
mcb_status mcb_create(const mcb_params* params, mcb_ctx** out);
void mcb_destroy(mcb_ctx* ctx);
const char* mcb_last_error(const mcb_ctx* ctx);

/* Arena sizes for the given shape count and link/boundary-node/wall-node counts (pass zeros
 * before the counts are known: links_bytes is then 0). */
mcb_status mcb_required_sizes(const mcb_params* params, int64_t n_shapes, int64_t n_links,
                              int64_t n_bnodes, int64_t n_wall, mcb_sizes* out);

/* Binds caller-owned device arenas and the HIP stream (hipStream_t; NULL = default stream).
 * The lattice arena must be sized for the shape count later passed to mcb_set_geometry. */
mcb_status mcb_bind_buffers(mcb_ctx* ctx, const mcb_buffers* bufs, void* hip_stream);

/* ---- geometry (the exact integer pass) -------------------------------------------------- */
/* Copies the shape list to the device. Balls need 2 radius < box length on every axis. */
mcb_status mcb_set_geometry(mcb_ctx* ctx, const mcb_shape* shapes, int64_t n);

/* MCB_COUNT: classifies nodes on the device and returns the number of links, boundary-fluid
 * nodes and wall nodes (synchronises). MCB_FILL (after binding a links arena of the size
 * mcb_required_sizes gives for those counts): fills the link table with q and class, the
 * boundary-node and wall-node tables, and sets every wall node's phi to 1. */
mcb_status mcb_build_links(mcb_ctx* ctx, int32_t phase, int64_t* n_links, int64_t* n_bnodes,
                           int64_t* n_wall);

/* Copies the canonical link list to the host (cap entries available). */
mcb_status mcb_get_links(mcb_ctx* ctx, mcb_link* host, int64_t cap);

/* Wall nodes (solid nodes with a fluid neighbour), ascending linear index. */
mcb_status mcb_get_wall_nodes(mcb_ctx* ctx, int64_t* host, int64_t cap);

/* Test override of q: the (node, dir) sequence must equal the built list; q_fixed in [0, 2^16]
 * is taken from each entry and the class recomputed. */
mcb_status mcb_set_links(mcb_ctx* ctx, const mcb_link* links, int64_t n);

/* ---- wettability -------------------------------------------------------------------------- */
/* phi per wall node (ascending linear index), > 0: the virtual wall density is phi times the
 * eq. 15 first-layer average of the fluid neighbours. */
mcb_status mcb_set_wettability(mcb_ctx* ctx, const double* phi, int64_t n_wall);

/* ---- state -------------------------------------------------------------------------------- */
/* f(x, 0) = f^eq(rho, u) (eq. 14) on fluid nodes, then the first collision. rho: N doubles;
 * u: dim x N doubles or NULL (rest). Values on solid nodes are ignored. Synchronises. */
mcb_status mcb_init_equilibrium(mcb_ctx* ctx, const double* rho, const double* u);

/* Pre-collision populations f(x, t) (Q x N doubles, solid entries ignored) followed by one
 * collision: the state becomes the post-collision populations of time t. Synchronises. */
mcb_status mcb_set_f(mcb_ctx* ctx, const double* f);

/* Post-collision populations f~(x, t) of the current state (Q x N doubles; solid entries 0). */
mcb_status mcb_get_f(mcb_ctx* ctx, double* f);

/* ---- time stepping -------------------------------------------------------------------------- */
/* n steps, asynchronous on the bound stream. */
mcb_status mcb_step(mcb_ctx* ctx, int64_t n);

/* ---- observables ---------------------------------------------------------------------------- */
/* rho (N doubles) and the physical velocity v = u + F / (2 rho) (dim x N doubles; Sec. 2.2,
 * after eq. 14) of the current state. Either pointer may be NULL. Solid entries 0. */
mcb_status mcb_moments(mcb_ctx* ctx, double* rho, double* v);

/* Largest physical speed |v| over the fluid nodes of the current state (the spurious-current measure
 * of Sec. 4.4) in *vmax, and in *node the smallest linear index of a fluid node attaining it (-1 and
 * 0 without fluid nodes).  FP64, computed on the device, deterministic; non-finite speeds are
 * skipped (mcb_mass counts them).  Either pointer may be NULL.  Synchronises. */
mcb_status mcb_max_speed(mcb_ctx* ctx, double* vmax, int64_t* node);

/* FP64 mass / momentum / Delta M report (deterministic two-pass reduction). */
mcb_status mcb_mass(mcb_ctx* ctx, mcb_mass_report* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the report of mcb_mass, computed by the same kernels in
 * the same order (bit-identical results), with the reduction's partial sums and result slots kept
 * in a static device array of the library instead of the context's lattice arena.  Allocates
 * nothing.  The array holds 65,600 bytes (1024 x 8 partial sums and 8 result slots, a fixed grid
 * whatever the lattice size; MCB_ESIZE if the reduction ever needed more) on each device the
 * library runs on, until the process ends.  Every call on one device shares that device's array:
 * calls that overlap on one device (several host threads, or several streams) race and must be
 * serialised by the caller; each call writes every entry it reads, so nothing needs clearing.  The
 * current device must be the one the context's buffers were bound on (MCB_ESTATE otherwise).
 * Synchronises. */
mcb_status mcb_mass_static(mcb_ctx* ctx, mcb_mass_report* out);

/* Waits for the stream and reports device-detected faults. */
mcb_status mcb_sync(mcb_ctx* ctx);

/* ---- measurement ------------------------------------------------------------------------ */
/* enable != 0 starts timing of mcb_step with HIP events recorded on the bound stream around every
 * launch of the fused step kernel (totals reset); 0 stops it. */
mcb_status mcb_timing(mcb_ctx* ctx, int32_t enable);

/* Total milliseconds of the fused step kernel and the number of timed launches since timing was
 * enabled (synchronises). */
mcb_status mcb_timing_report(mcb_ctx* ctx, double* ms, int64_t* launches);

/* ---- differentiation: reverse mode with checkpoints ---------------------------------------- */
/* Gradient of a loss of the state after nsteps steps from the equilibrium start rho0 (the same
 * start as mcb_init_equilibrium with u = 0) with respect to the wettability factor phi of every
 * wall node, by the hand-written discrete adjoint of the step.  The forward pass stores the state
 * every k steps; the reverse pass recomputes each k-step segment from its checkpoint with the
 * fused step kernel and applies the transposed step backwards through it, then the transposed
 * first collision.  The adjoint arithmetic is FP64 in every storage precision (for the shifted
 * storages it is the adjoint of the FP64 step linearised at the stored states).
 *
 * Losses of the stored state f~(T), rho(x) = sum_i f~_i(x, T) on fluid nodes:
 *   MCB_LOSS_COM_X           sum_x X (rho - prm[0]) / sum_x (rho - prm[0]), X the node's x index
 *                            (prm[0] = rho_v: the centre of mass of the liquid)
 *   MCB_LOSS_WETTED_LENGTH   sum over links (x1, j) of |e_j| (1 + tanh((rho(x1) - prm[0]) / prm[1])) / 2
 *   MCB_LOSS_TOTAL_MASS      sum_x rho (its gradient is zero: eq. 18 conserves mass for any phi)
 */
enum { MCB_LOSS_COM_X = 0, MCB_LOSS_WETTED_LENGTH = 1, MCB_LOSS_TOTAL_MASS = 2 };

/* Device bytes of the reverse-mode arena for nsteps >= 0 steps with a checkpoint every k >= 1
 * steps (after mcb_build_links(FILL)).  Reverse mode covers both models (2-D for the chemical-potential
 * one), every boundary scheme, both collisions and the body force. */
mcb_status mcb_adj_required_bytes(mcb_ctx* ctx, int64_t nsteps, int64_t k, int64_t* bytes);

/* Binds the caller-owned reverse-mode arena (device memory, at least the required bytes, 256-byte
 * aligned); it must stay alive while mcb_adj_forward / mcb_adj_backward use it. */
mcb_status mcb_adj_bind(mcb_ctx* ctx, void* device_buffer, int64_t bytes);

/* Equilibrium start from rho0 (N doubles), nsteps steps with checkpoints, and the loss of the final
 * state in *value.  The context's state is then that final state (t = nsteps).  Each successful call
 * starts a new generation of the reverse mode (mcb_adj_generation).  Synchronises. */
mcb_status mcb_adj_forward(mcb_ctx* ctx, const double* rho0, int64_t nsteps, int64_t k, int32_t loss_kind,
                           const double* loss_prm, double* value);

/* The generation of the last mcb_adj_forward, while its gradient can still be taken; 0 once the
 * state, the wettability, the links or the geometry have changed since (mcb_step, mcb_set_f,
 * mcb_init_equilibrium, mcb_set_wettability, mcb_set_links, mcb_set_geometry, mcb_build_links,
 * mcb_adj_bind). */
mcb_status mcb_adj_generation(const mcb_ctx* ctx, int64_t* generation);

/* dphi[w] = dloss * d loss / d phi[w] (n_wall doubles, wall nodes in ascending linear index; phi is the
 * wettability value of mcb_set_wettability: the factor, or the assigned chemical potential) for
 * the forward pass of the given generation, which must be the last one, with nothing changed
 * since (MCB_ESTATE otherwise: a caller holding the losses of two forward passes on one context
 * cannot take the gradient of the first).  The context's state is left as it was.  Synchronises. */
mcb_status mcb_adj_backward(mcb_ctx* ctx, int64_t generation, double dloss, double* dphi);

#ifdef __cplusplus
}
#endif

#endif /* MCB_H */
