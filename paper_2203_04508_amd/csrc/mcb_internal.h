// Internal declarations of libmcb: context, arena layout, device lattice tables, launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/mcb.h"

namespace mcb {

constexpr int64_t ONE = 65536;            // one lattice spacing in fixed point
constexpr uint32_t NOHIT = 0xFFFFFFFFu;
constexpr uint32_t QMASK = 0x1FFFFu;      // q_fixed in bits 0..16 of a packed link word
constexpr int CLS_SHIFT = 30;             // link class in bits 30..31

constexpr int STRIP_HALO = 4;            // 2-D step: halo lanes per strip (two columns on each side)
constexpr int Q2_LINKS = 8;               // link-coefficient slots per boundary node: one per direction,
constexpr int Q3_LINKS = 20;              // 3-D: and two unused ones, so every node's slots start on 16 bytes
// Boundary record of a boundary-fluid node, written by its collision and read by the pull of the
// next step: the terms of its exact-difference forcing (rho, du = F / rho, s = 2u + du and
// duu = 1.5 du.s, from which F_j of eq. 13 follows per direction), its post-collision populations
// 1 .. Q-1 as stored, one slot (the sum of the node's own populations on its links, which the
// density of the next step adds: the 3-D density pass and the chemical-potential march; the 2-D
// step of the pseudopotential model keeps population 0 as stored there, which nothing reads), and
// the eq. 18 correction that the pull of that step applied.  The pull loads only the leading RF + Q - 1 values (a loaded value
// that is never used frees its register while the load is in flight, and the next write to it
// must wait for the load).
constexpr int REC2 = 16;                  // 6 + 8 + 1 + 1
constexpr int REC3 = 28;                  // 8 + 18 + 1 + 1
constexpr int RF2 = 6, RF3 = 8;           // offset of population 1
constexpr double NO_LINK = 2.0;           // coefficient of a direction without a link (|a| <= 1 on links)
constexpr int SCAN_BLOCK = 256;           // geometry scan granularity
constexpr int MON_BLOCKS = 1024;          // monitor partial sums
constexpr int MON_FIELDS = 8;             // M, Jx, Jy, Jz, dM, n_nan, then the max-speed pair
constexpr int MON_SPEED = 6;              // result slots of the largest speed and its node
constexpr int DM_BLOCKS = 256;            // workgroups of the per-step Delta M sum (track_dm)
constexpr int MAX_BANDS = 8;

// sticky device fault flags
enum { FLAG_DOMAIN = 0, FLAG_NOHIT = 1, FLAG_COUNT = 16 };

// ---------------------------------------------------------------- device lattice tables
// D2Q9 in the column order of the moment matrix (eq. 2); D3Q19 rest / axes / edges.
static __constant__ int c_ex[2][19] = {
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0}};
static __constant__ int c_ey[2][19] = {
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1}};
static __constant__ int c_ez[2][19] = {
    {0, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1}};
static __constant__ int c_opp[2][19] = {
    {0, 3, 4, 1, 2, 7, 8, 5, 6},
    {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17}};

struct GridDev {
    int dim, nx, ny, nz, Q;
    int64_t N;
};

// Byte offsets of the sub-buffers carved out of the two caller-owned arenas.
struct Layout {
    // lattice arena
    int64_t fa, fb, tag, nmask, rho3, dm, cp_rho, cp_mu, cp_layer, cp_l2, cp_l2n, solid, scratch, blocksums, flags, partials, result, shapes, lattice_bytes;
    // links arena
    int64_t bn_node, bn_mask, bn_link0, lk_qc, lk_a, rec[2], wl_node, wl_phi, wl_fac, links_bytes;
    int64_t rec_slots;   // link-coefficient slots: Q2_LINKS / Q3_LINKS per boundary node
    int64_t rec_stride;  // compute-type values per boundary record (REC2 / REC3)
};

Layout make_layout(const mcb_params& p, int64_t n_shapes, int64_t n_links, int64_t n_bnodes, int64_t n_wall);

// Reverse-mode arena (caller-owned): byte offsets of checkpoints, the recomputed segment, the
// adjoint states and the work arrays of the transposed step.
struct AdjPlan {
    int64_t nsteps, k, nck, state_b, rec_b, nslots;
    int64_t rho0, ck, ck_rec, seg, seg_rec, lam[2], lamR[2];
    int64_t p, pbar, rho, psi, dpsi, rave, den, rbar, qbar, Fbar, Fv, dphi, part, sums, bytes;
};

// device pointers of the work arrays
struct AdjWork {
    const double* rho0;
    double *p, *pbar, *rho, *psi, *dpsi, *rave, *den, *rbar, *qbar, *Fbar, *Fv, *dphi, *part, *sums;
};
int64_t storage_bytes(int precision);
// bytes of one population state (Q planes; FP16 storage keeps plane 0 in FP32) and the byte offset
// of plane i in it
int64_t state_bytes(int precision, int Q, int64_t N);
int64_t plane_bytes_off(int precision, int i, int64_t N);
int64_t compute_bytes(int precision);

// Peng-Robinson critical temperature (alpha = 1): x = b rho_c is the real root of
// x^3 + x^2 + x - 1/3 = 0 (d2p/drho2 = 0 on the curve dp/drho = 0), then
// R T_c b / a = (1 - x)^2 (2x + 2x^2) / (1 + 2x - x^2)^2
inline double pr_tc(double a, double b, double R) {
    const double r2 = std::sqrt(2.0);
    const double x = (std::cbrt(8.0 + 6.0 * r2) + std::cbrt(8.0 - 6.0 * r2) - 1.0) / 3.0;
    const double q = 1.0 + 2.0 * x - x * x;
    return a / (b * R) * (1.0 - x) * (1.0 - x) * 2.0 * x * (1.0 + x) / (q * q);
}

// a alpha(T) of the Peng-Robinson EOS (Sec. 2.2) with acentric factor omega
inline double pr_aalpha(double a, double b, double R, double T, double omega) {
    const double m = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    const double s = 1.0 + m * (1.0 - std::sqrt(T / pr_tc(a, b, R)));
    return a * s * s;
}

}  // namespace mcb

struct mcb_ctx {
    mcb_params p{};
    mcb::GridDev g{};
    hipStream_t stream = nullptr;
    int device = -1;      // the device current when the buffers were bound
    double* scratch = nullptr;  // that device's static scratch (mcb_mass_static), found at bind time
    hipError_t scratch_err = hipSuccess;
    int n_cu = 0;         // compute units of the device (sizes the step grids to whole rounds)
    char* lat = nullptr;
    int64_t lat_bytes = 0;
    char* lk = nullptr;
    int64_t lk_bytes = 0;
    int64_t n_shapes = 0, n_links = -1, n_bnodes = -1, n_wall = -1;
    int64_t n_l2 = 0;  // chemical-potential model: nodes of the second solid layer
    int64_t cap_shapes = 0;
    int occ[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // resident workgroups per CU of the step kernel variants and of
                                            // the largest-speed pass (0: not yet queried)
    int stage = 0;        // 0 created, 1 bound, 2 geometry set, 3 counted, 4 links filled, 5 state set
    bool swapped = false; // current post-collision state lives in fb instead of fa
    int64_t t = 0;
    double dm_host = 0.0;  // track_dm: host copy of the running Delta M sum, read by the mass reports
    int n_bands = 0;
    mcb_shape bands[mcb::MAX_BANDS]{};
    mcb::Layout L{};
    std::string err;
    // per-kernel event timing of mcb_step: a ring of event triples drained lazily
    bool timing = false;
    static constexpr int RING = 64;
    hipEvent_t ev[RING][2]{};
    bool ev_pending[RING]{};
    int ev_next = 0;
    bool ev_made = false;
    double ms_tot = 0.0;
    int64_t launches = 0;
    // reverse mode
    char* adj = nullptr;
    int64_t adj_bytes = 0;
    mcb::AdjPlan ap{};
    bool adj_ready = false;   // a forward pass with checkpoints has run and the state is its end
    int64_t adj_gen = 0;      // generation of the last forward pass (bumped by every mcb_adj_forward)
    int64_t adj_t_end = -1;
    int32_t adj_kind = 0;
    double adj_prm[2]{};
};

namespace mcb {

// ---------------------------------------------------------------- launchers (asynchronous)
// geometry.hip
hipError_t geom_classify(mcb_ctx* c);
hipError_t geom_count(mcb_ctx* c);                // block sums + scan, totals at the end
hipError_t geom_fill(mcb_ctx* c);                 // tags, boundary-node / wall tables, q, class
hipError_t geom_reclass(mcb_ctx* c);              // class from the current q (after an override)
hipError_t wall_factors(mcb_ctx* c);              // phi / (eq. 15 weight of the fluid neighbours) per wall node
hipError_t cp_wall_mu(mcb_ctx* c);                // chemical-potential model: mu of the solid layers from the assigned values

// step2d.hip / step3d.hip: one time step from the state (fcur, rcur) to (fnext, rnext), where r are
// the boundary records of the state (pull = false: collision of fcur in place of the pull)
hipError_t step_fused(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull);
hipError_t init_feq(mcb_ctx* c, const double* rho, const double* u, void* fout);

// adjoint.hip: one transposed step (pull = 0: the first collision from f^eq(rho0, 0)), and the
// loss of a state with (lam != nullptr) its gradient lam = dloss * d loss / d g
hipError_t adj_step(mcb_ctx* c, const AdjWork& w, const void* gt, const void* rec, int pull, const double* lam1,
                    const double* lamR1, double* lam0, double* lamR0);
hipError_t adj_loss(mcb_ctx* c, const AdjWork& w, const void* g, int kind, const double* prm, double dloss, double* lam);

// monitor.hip
// partials (MON_BLOCKS x MON_FIELDS doubles) and result (MON_FIELDS doubles): null = the context's
// lattice arena
hipError_t monitor(mcb_ctx* c, const void* fcur, const void* rcur, double* partials = nullptr, double* result = nullptr);
hipError_t moments_out(mcb_ctx* c, const void* fcur, double* rho, double* v);
hipError_t max_speed(mcb_ctx* c, const void* fcur);  // result slots MON_SPEED, MON_SPEED + 1
// track_dm: adds the eq. 18 total held in the records rcur (the step that wrote them) to the FP64
// sum at L.dm[DM_BLOCKS] (per-workgroup partials first, then one workgroup in a fixed order)
hipError_t dm_accumulate(mcb_ctx* c, const void* rcur);
// chemical-potential model: the density and chemical-potential fields of the collision that made
// the current state, from the populations fpre it collided (pulled with the records rpre when pull)
hipError_t cp_fields(mcb_ctx* c, const void* fpre, const void* rpre, bool pull);
hipError_t convert_plane_in(mcb_ctx* c, const double* src, void* dst_plane, int dir);
hipError_t convert_plane_out(mcb_ctx* c, const void* src_plane, double* dst, int dir);

}  // namespace mcb
