// Host side of the C ABI declared in include/mcb.h: argument checks, arena layout, call order,
// stream handling and error reporting.  Device work lives in geometry.hip, step2d.hip,
// step3d.hip and monitor.hip.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mcb_internal.h"

namespace mcb {

int64_t storage_bytes(int precision) { return precision == MCB_F64 ? 8 : (precision == MCB_F32S ? 4 : 2); }
int64_t state_bytes(int precision, int Q, int64_t N) {
    return (precision == MCB_F16S ? Q + 1 : Q) * N * storage_bytes(precision);
}
int64_t plane_bytes_off(int precision, int i, int64_t N) {
    const int64_t s = storage_bytes(precision);
    return (precision == MCB_F16S && i > 0 ? i + 1 : i) * N * s;
}
int64_t compute_bytes(int precision) { return precision == MCB_F64 ? 8 : 4; }

static int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

Layout make_layout(const mcb_params& p, int64_t n_shapes, int64_t n_links, int64_t n_bnodes, int64_t n_wall) {
    Layout L{};
    const int Q = p.dim == 2 ? 9 : 19;
    const int64_t N = int64_t(p.nx) * p.ny * (p.dim == 3 ? p.nz : 1);
    const int64_t s = storage_bytes(p.precision), cb = compute_bytes(p.precision);
    const int64_t nblk = (N + SCAN_BLOCK - 1) / SCAN_BLOCK;
    int64_t o = 0;
    auto take = [&](int64_t bytes) { const int64_t at = o; o = align256(o + bytes); return at; };
    L.fa = take(state_bytes(p.precision, Q, N));
    L.fb = take(state_bytes(p.precision, Q, N));
    L.tag = take(4 * N);
    L.nmask = take(p.dim == 3 ? 4 * N : 0);  // 3-D: link bits of each boundary node (bit j-1: x + e_j solid)
    L.rho3 = take(p.dim == 3 ? cb * N : 0);  // 3-D: density pass output of the step (compute type)
    L.dm = take(8 * (DM_BLOCKS + 1));         // track_dm: per-workgroup partials, then the running sum
    const bool cp = p.model == MCB_MODEL_CHEMPOT;
    L.cp_rho = take(cp ? cb * N : 0);        // chemical-potential model: density and chemical potential
    L.cp_mu = take(cp ? cb * N : 0);         // fields of the step (compute type), solid layer of each node
    L.cp_layer = take(cp ? N : 0);
    L.cp_l2 = take(cp ? 4 * N : 0);          // indices of the second-layer nodes, and their count
    L.cp_l2n = take(cp ? 8 : 0);
    L.solid = take(N);
    L.scratch = take(8 * N * (2 + p.dim));
    L.blocksums = take(8 * (3 * nblk + 3));
    L.flags = take(4 * FLAG_COUNT);
    L.partials = take(8 * MON_BLOCKS * MON_FIELDS);
    L.result = take(8 * MON_FIELDS);
    L.shapes = take(int64_t(sizeof(mcb_shape)) * (n_shapes > 0 ? n_shapes : 1));  // last: only it depends on n_shapes
    L.lattice_bytes = o;
    o = 0;
    const int64_t nb = n_bnodes > 0 ? n_bnodes : 0, nl = n_links > 0 ? n_links : 0, nw = n_wall > 0 ? n_wall : 0;
    L.bn_node = take(4 * nb);
    L.bn_mask = take(4 * nb);
    L.bn_link0 = take(4 * nb);
    L.lk_qc = take(4 * nl);
    // per boundary node: the signed interpolation coefficient a of each direction's link (fixed
    // slots), and the boundary records of the two lattice buffers (records of fa, records of fb)
    L.rec_slots = (p.dim == 2 ? Q2_LINKS : Q3_LINKS) * nb;
    L.rec_stride = p.dim == 2 ? REC2 : REC3;
    L.lk_a = take(cb * L.rec_slots);
    L.rec[0] = take(cb * L.rec_stride * nb);
    L.rec[1] = take(cb * L.rec_stride * nb);
    L.wl_node = take(4 * nw);
    L.wl_phi = take(8 * nw);
    L.wl_fac = take(8 * nw);  // compute type
    L.links_bytes = (nb + nl + nw) > 0 ? o : 0;
    return L;
}

AdjPlan adj_plan(const mcb_ctx* c, int64_t nsteps, int64_t k) {
    AdjPlan a{};
    const int64_t N = c->g.N, Q = c->g.Q;
    const int64_t cb = compute_bytes(c->p.precision);
    a.nsteps = nsteps;
    a.k = k;
    a.nck = nsteps == 0 ? 1 : (nsteps + k - 1) / k;
    a.state_b = align256(state_bytes(c->p.precision, int(Q), N));
    a.nslots = c->L.rec_slots;
    a.rec_b = align256(cb * c->L.rec_stride * (c->n_bnodes > 0 ? c->n_bnodes : 0));
    int64_t o = 0;
    auto take = [&](int64_t bytes) { const int64_t at = o; o = align256(o + bytes); return at; };
    a.rho0 = take(8 * N);
    a.ck = take(a.nck * a.state_b);
    a.ck_rec = take(a.nck * a.rec_b);
    a.seg = take((k - 1) * a.state_b);
    a.seg_rec = take((k - 1) * a.rec_b);
    for (int b = 0; b < 2; ++b) {
        a.lam[b] = take(8 * Q * N);
        a.lamR[b] = take(8 * (a.nslots > 0 ? a.nslots : 1));
    }
    a.p = take(8 * Q * N);
    a.pbar = take(8 * Q * N);
    a.rho = take(8 * N);
    a.psi = take(8 * N);
    a.dpsi = take(8 * N);
    a.rave = take(8 * N);
    a.den = take(8 * N);
    a.rbar = take(8 * N);
    a.qbar = take(8 * N);
    a.Fbar = take(8 * 3 * N);
    a.Fv = take(8 * 3 * N);
    a.dphi = take(8 * (c->n_wall > 0 ? c->n_wall : 1));
    a.part = take(8 * 2 * MON_BLOCKS);
    a.sums = take(8 * 2);
    a.bytes = o;
    return a;
}

}  // namespace mcb

using namespace mcb;

namespace {

// Device scratch of mcb_mass_static, for callers that cannot allocate: the monitor's per-workgroup
// FP64 partial sums followed by its result slots (65,600 bytes on each device the library runs on,
// held until the process ends).  Host code never passes the array's name to a kernel: each device's
// copy lives at its own address, which mcb_bind_buffers looks up once per device with that device
// current (hipGetSymbolAddress) and keeps in scratch_addr.
constexpr int64_t SCRATCH_DOUBLES = int64_t(MON_BLOCKS) * MON_FIELDS + MON_FIELDS;
__device__ __align__(256) double scratch[SCRATCH_DOUBLES];
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_addr[MAX_DEVICES] = {};

// the address of the current device's scratch (dev = the current device), looked up on first use
hipError_t scratch_of(int dev, double** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_addr[dev] = static_cast<double*>(p);
    }
    *out = scratch_addr[dev];
    return hipSuccess;
}

mcb_status fail(mcb_ctx* c, mcb_status code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return fail(c, MCB_EHIP, "%s: %s", #call, hipGetErrorString(e_));   \
    } while (0)

bool params_ok(const mcb_params* p, const char** why) {
    if (!p) { *why = "null params"; return false; }
    if (p->dim != 2 && p->dim != 3) { *why = "dim must be 2 or 3"; return false; }
    const int nz = p->dim == 3 ? p->nz : 1;
    if (p->nx < 3 || p->ny < 3 || p->nx > 32768 || p->ny > 32768 || (p->dim == 3 && (nz < 3 || nz > 32768))) {
        *why = "box sizes must lie in [3, 32768]";
        return false;
    }
    if (p->dim == 2 && p->nz != 1) { *why = "nz must be 1 in 2-D"; return false; }
    if (int64_t(p->nx) * p->ny * nz >= (int64_t(1) << 31)) { *why = "N must be < 2^31"; return false; }
    const int64_t sbytes = p->precision == MCB_F64 ? 8 : (p->precision == MCB_F32S ? 4 : 2);
    if (int64_t(p->nx) * p->ny * nz * (p->dim == 2 ? 9 : 19) * sbytes > int64_t(0xFFFFFE00u)) {
        *why = "one population lattice must stay below 4 GiB (32-bit buffer offsets)";
        return false;
    }
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) { *why = "tau must exceed 1/2"; return false; }
    if (p->model != MCB_MODEL_PSEUDO && p->model != MCB_MODEL_CHEMPOT) { *why = "unknown model"; return false; }
    if (p->model == MCB_MODEL_PSEUDO && (!(p->G < 0.0) || !std::isfinite(p->G))) { *why = "G must be negative"; return false; }
    if (p->model == MCB_MODEL_CHEMPOT &&
        (!(p->cp_k > 0.0) || !std::isfinite(p->cp_k) || !(p->cp_kappa >= 0.0) || !std::isfinite(p->cp_kappa) ||
         !std::isfinite(p->pr_omega) || !(p->eos_a > 0.0))) {
        *why = "bad chemical-potential parameters";
        return false;
    }
    if (!std::isfinite(p->eos_a) || !std::isfinite(p->eos_b) || !std::isfinite(p->eos_R) || !std::isfinite(p->eos_T) ||
        p->eos_b <= 0 || p->eos_R <= 0 || p->eos_T <= 0) {
        *why = "bad EOS parameters";
        return false;
    }
    if (p->precision < MCB_F64 || p->precision > MCB_F16S) { *why = "unknown precision"; return false; }
    if (p->bc_mode < MCB_BC_PRESENT || p->bc_mode > MCB_BC_HBBC) { *why = "unknown bc_mode"; return false; }
    if (p->precision != MCB_F64 && !(std::isfinite(p->rho_ref) && p->rho_ref >= 0.0)) { *why = "bad rho_ref"; return false; }
    if (p->collision != MCB_COLL_BGK && p->collision != MCB_COLL_MRT) { *why = "unknown collision"; return false; }
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(p->gravity[k])) { *why = "gravity must be finite"; return false; }
    if (p->dim == 2 && p->gravity[2] != 0.0) { *why = "gravity[2] must be 0 in 2-D"; return false; }
    if (p->collision == MCB_COLL_MRT)
        for (double r : {p->s_e, p->s_eps, p->s_q})
            if (!(r > 0.0 && r < 2.0)) { *why = "MRT rates must lie in (0, 2)"; return false; }
    return true;
}

void* fcur(mcb_ctx* c) { return c->lat + (c->swapped ? c->L.fb : c->L.fa); }
void* fnext(mcb_ctx* c) { return c->lat + (c->swapped ? c->L.fa : c->L.fb); }
// boundary records of the current and the next state (each lattice buffer has its own)
void* rcur(mcb_ctx* c) { return c->lk + c->L.rec[c->swapped ? 1 : 0]; }
void* rnext(mcb_ctx* c) { return c->lk + c->L.rec[c->swapped ? 0 : 1]; }

mcb_status check_flags(mcb_ctx* c, int64_t* n_domain_out) {
    int32_t flags[FLAG_COUNT];
    HIPCHK(hipMemcpyAsync(flags, c->lat + c->L.flags, sizeof flags, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (n_domain_out) *n_domain_out = flags[FLAG_DOMAIN] ? 1 : 0;
    if (flags[FLAG_NOHIT]) return fail(c, MCB_EINVAL, "a link's solid neighbour lies in no shape");
    if (flags[FLAG_DOMAIN]) {
        // a non-finite population fails the domain test too: tell the two apart by counting the
        // fluid nodes of the current state that hold one
        if (c->stage >= 5) {
            HIPCHK(monitor(c, fcur(c), rcur(c)));
            double r[MON_FIELDS];
            HIPCHK(hipMemcpyAsync(r, c->lat + c->L.result, sizeof r, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            if (r[5] > 0.0) return fail(c, MCB_ENAN, "%lld fluid nodes hold non-finite populations", (long long)r[5]);
        }
        return fail(c, MCB_EDOMAIN, "psi domain error: rho <= 0 or negative square-root argument");
    }
    return MCB_OK;
}

mcb_status clear_flags(mcb_ctx* c) {
    HIPCHK(hipMemsetAsync(c->lat + c->L.flags, 0, 4 * FLAG_COUNT, c->stream));
    return MCB_OK;
}

// host copy of the link tables, expanded to the canonical list
mcb_status expand_links(mcb_ctx* c, std::vector<mcb_link>& out) {
    const int64_t nb = c->n_bnodes, nl = c->n_links;
    std::vector<int32_t> node(nb), link0(nb);
    std::vector<uint32_t> mask(nb), qc(nl);
    if (nb > 0) {
        HIPCHK(hipMemcpyAsync(node.data(), c->lk + c->L.bn_node, 4 * nb, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(mask.data(), c->lk + c->L.bn_mask, 4 * nb, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(link0.data(), c->lk + c->L.bn_link0, 4 * nb, hipMemcpyDeviceToHost, c->stream));
    }
    if (nl > 0) HIPCHK(hipMemcpyAsync(qc.data(), c->lk + c->L.lk_qc, 4 * nl, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    out.assign(nl, mcb_link{});
    for (int64_t b = 0; b < nb; ++b) {
        int64_t l = link0[b];
        for (int j = 1; j < c->g.Q; ++j) {
            if (!((mask[b] >> j) & 1u)) continue;
            if (l >= nl) return fail(c, MCB_EINVAL, "corrupt link table");
            out[l].node = node[b];
            out[l].dir = j;
            out[l].cls = int32_t(qc[l] >> CLS_SHIFT);
            out[l].q_fixed = qc[l] & QMASK;
            out[l].pad = 0;
            ++l;
        }
    }
    return MCB_OK;
}

}  // namespace

extern "C" {

mcb_status mcb_create(const mcb_params* params, mcb_ctx** out) {
    if (!out) return MCB_EINVAL;
    *out = nullptr;
    const char* why = nullptr;
    if (!params_ok(params, &why)) return MCB_EINVAL;
    // the 3-D density pass takes the boundary nodes' density from the eq. 18 balance
    // the paper gives the moment basis of D2Q9 only; the chemical-potential path is two-dimensional
    if (params->dim == 3 && (params->collision == MCB_COLL_MRT || params->model == MCB_MODEL_CHEMPOT)) return MCB_ENOTSUP;
    auto* c = new (std::nothrow) mcb_ctx();
    if (!c) return MCB_EINVAL;
    c->p = *params;
    if (c->p.dim == 2) c->p.nz = 1;
    c->g.dim = c->p.dim;
    c->g.nx = c->p.nx;
    c->g.ny = c->p.ny;
    c->g.nz = c->p.nz;
    c->g.Q = c->p.dim == 2 ? 9 : 19;
    c->g.N = int64_t(c->p.nx) * c->p.ny * c->p.nz;
    c->L = make_layout(c->p, 0, 0, 0, 0);
    *out = c;
    return MCB_OK;
}

void mcb_destroy(mcb_ctx* c) {
    if (!c) return;
    if (c->ev_made)
        for (int r = 0; r < mcb_ctx::RING; ++r)
            for (int k = 0; k < 2; ++k) (void)hipEventDestroy(c->ev[r][k]);
    delete c;
}

const char* mcb_last_error(const mcb_ctx* c) { return c ? c->err.c_str() : "null context"; }

mcb_status mcb_required_sizes(const mcb_params* params, int64_t n_shapes, int64_t n_links, int64_t n_bnodes, int64_t n_wall,
                              mcb_sizes* out) {
    const char* why = nullptr;
    if (!out || !params_ok(params, &why)) return MCB_EINVAL;
    if (n_shapes < 0 || n_links < 0 || n_bnodes < 0 || n_wall < 0) return MCB_EINVAL;
    mcb_params p = *params;
    if (p.dim == 2) p.nz = 1;
    const Layout L = make_layout(p, n_shapes, n_links, n_bnodes, n_wall);
    out->lattice_bytes = L.lattice_bytes;
    out->links_bytes = L.links_bytes;
    return MCB_OK;
}

mcb_status mcb_bind_buffers(mcb_ctx* c, const mcb_buffers* b, void* stream) {
    if (!c) return MCB_EINVAL;
    if (!b || !b->lattice) return fail(c, MCB_EINVAL, "lattice arena missing");
    if ((reinterpret_cast<uintptr_t>(b->lattice) & 255) || (b->links && (reinterpret_cast<uintptr_t>(b->links) & 255)))
        return fail(c, MCB_EINVAL, "arenas must be 256-byte aligned");
    const Layout L0 = make_layout(c->p, 0, 0, 0, 0);
    if (b->lattice_bytes < L0.lattice_bytes)
        return fail(c, MCB_ESIZE, "lattice arena %lld < %lld bytes", (long long)b->lattice_bytes, (long long)L0.lattice_bytes);
    if (c->lat && c->lat != b->lattice && c->stage >= 2)
        return fail(c, MCB_ESTATE, "the lattice arena cannot move once geometry is set");
    c->lat = static_cast<char*>(b->lattice);
    c->lat_bytes = b->lattice_bytes;
    if (b->links) {
        if (c->lk && c->lk != b->links && c->stage >= 4)
            return fail(c, MCB_ESTATE, "the links arena cannot move once links are built");
        c->lk = static_cast<char*>(b->links);
        c->lk_bytes = b->links_bytes;
    }
    c->stream = static_cast<hipStream_t>(stream);
    {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
        c->device = dev;
        // the static scratch of mcb_mass_static; a failed lookup only disables that entry point
        c->scratch = nullptr;
        c->scratch_err = scratch_of(dev, &c->scratch);
    }
    if (c->stage < 1) c->stage = 1;
    // lattice offsets do not depend on the counts; refresh the link offsets if counts are known
    c->L = make_layout(c->p, c->n_shapes, c->n_links > 0 ? c->n_links : 0, c->n_bnodes > 0 ? c->n_bnodes : 0,
                       c->n_wall > 0 ? c->n_wall : 0);
    return MCB_OK;
}

mcb_status mcb_set_geometry(mcb_ctx* c, const mcb_shape* shapes, int64_t n) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 1) return fail(c, MCB_ESTATE, "bind buffers first");
    if (n < 0 || (n > 0 && !shapes)) return fail(c, MCB_EINVAL, "bad shape list");
    const int64_t len[3] = {int64_t(c->p.nx) * ONE, int64_t(c->p.ny) * ONE, int64_t(c->p.nz) * ONE};
    int nb = 0;
    for (int64_t s = 0; s < n; ++s) {
        const mcb_shape& h = shapes[s];
        if (h.kind == MCB_SHAPE_BALL) {
            if (h.radius <= 0) return fail(c, MCB_EINVAL, "shape %lld: radius must be positive", (long long)s);
            for (int k = 0; k < c->p.dim; ++k)
                if (2 * h.radius >= len[k]) return fail(c, MCB_EINVAL, "shape %lld: diameter exceeds the box", (long long)s);
            const int64_t cc[3] = {h.cx, h.cy, h.cz};
            for (int k = 0; k < 3; ++k)
                if (cc[k] < -(int64_t(1) << 40) || cc[k] > (int64_t(1) << 40))
                    return fail(c, MCB_EINVAL, "shape %lld: centre out of range", (long long)s);
        } else if (h.kind == MCB_SHAPE_BAND_Y) {
            if (h.hi <= h.lo || h.hi - h.lo >= len[1]) return fail(c, MCB_EINVAL, "shape %lld: bad band", (long long)s);
            if (nb >= MAX_BANDS) return fail(c, MCB_ENOTSUP, "at most %d bands", MAX_BANDS);
            c->bands[nb++] = h;
        } else {
            return fail(c, MCB_EINVAL, "shape %lld: unknown kind", (long long)s);
        }
    }
    const Layout L = make_layout(c->p, n, 0, 0, 0);
    if (c->lat_bytes < L.lattice_bytes)
        return fail(c, MCB_ESIZE, "lattice arena too small for %lld shapes", (long long)n);
    c->n_bands = nb;
    c->n_shapes = n;
    c->L = L;
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(c->lat + c->L.shapes, shapes, sizeof(mcb_shape) * n, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    c->n_links = c->n_bnodes = c->n_wall = -1;
    c->stage = 2;
    c->adj_ready = false;
    return MCB_OK;
}

mcb_status mcb_build_links(mcb_ctx* c, int32_t phase, int64_t* n_links, int64_t* n_bnodes, int64_t* n_wall) {
    if (!c) return MCB_EINVAL;
    c->adj_ready = false;
    if (phase == MCB_COUNT) {
        if (c->stage < 2) return fail(c, MCB_ESTATE, "set geometry first");
        mcb_status st = clear_flags(c);
        if (st) return st;
        HIPCHK(geom_classify(c));
        HIPCHK(geom_count(c));
        const int64_t nblk = (c->g.N + SCAN_BLOCK - 1) / SCAN_BLOCK;
        int64_t tot[3];
        HIPCHK(hipMemcpyAsync(tot, c->lat + c->L.blocksums + 8 * 3 * nblk, sizeof tot, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (tot[0] >= (int64_t(1) << 31)) return fail(c, MCB_ENOTSUP, "too many links");
        if (c->g.dim == 2 && tot[1] >= (int64_t(1) << 23)) return fail(c, MCB_ENOTSUP, "2-D tags hold at most 2^23 boundary nodes");
        if (tot[1] * (c->g.dim == 2 ? REC2 : REC3) * compute_bytes(c->p.precision) > int64_t(0xFFFFFE00u))
            return fail(c, MCB_ENOTSUP, "boundary records exceed 4 GiB");
        c->n_links = tot[0];
        c->n_bnodes = tot[1];
        c->n_wall = tot[2];
        c->stage = 3;
    } else if (phase == MCB_FILL) {
        if (c->stage < 3) return fail(c, MCB_ESTATE, "run the COUNT phase first");
        const Layout L = make_layout(c->p, c->n_shapes, c->n_links, c->n_bnodes, c->n_wall);
        if (L.links_bytes > 0 && (!c->lk || c->lk_bytes < L.links_bytes))
            return fail(c, MCB_ESIZE, "links arena too small: need %lld bytes", (long long)L.links_bytes);
        c->L = L;
        mcb_status st = clear_flags(c);
        if (st) return st;
        HIPCHK(geom_fill(c));
        st = check_flags(c, nullptr);
        if (st) return st;
        c->stage = 4;
        c->swapped = false;
    } else {
        return fail(c, MCB_EINVAL, "unknown phase");
    }
    if (n_links) *n_links = c->n_links;
    if (n_bnodes) *n_bnodes = c->n_bnodes;
    if (n_wall) *n_wall = c->n_wall;
    return MCB_OK;
}

mcb_status mcb_get_links(mcb_ctx* c, mcb_link* host, int64_t cap) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 4) return fail(c, MCB_ESTATE, "links not built");
    if (cap < c->n_links || (c->n_links > 0 && !host)) return fail(c, MCB_ESIZE, "capacity %lld < %lld links", (long long)cap, (long long)c->n_links);
    std::vector<mcb_link> v;
    mcb_status st = expand_links(c, v);
    if (st) return st;
    if (!v.empty()) std::memcpy(host, v.data(), v.size() * sizeof(mcb_link));
    return MCB_OK;
}

mcb_status mcb_get_wall_nodes(mcb_ctx* c, int64_t* host, int64_t cap) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 4) return fail(c, MCB_ESTATE, "links not built");
    if (cap < c->n_wall || (c->n_wall > 0 && !host)) return fail(c, MCB_ESIZE, "capacity too small");
    std::vector<int32_t> w(c->n_wall);
    if (c->n_wall > 0) {
        HIPCHK(hipMemcpyAsync(w.data(), c->lk + c->L.wl_node, 4 * c->n_wall, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    for (int64_t i = 0; i < c->n_wall; ++i) host[i] = w[i];
    return MCB_OK;
}

mcb_status mcb_set_links(mcb_ctx* c, const mcb_link* links, int64_t n) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 4) return fail(c, MCB_ESTATE, "links not built");
    if (n != c->n_links || (n > 0 && !links)) return fail(c, MCB_EINVAL, "link count differs from the built list");
    std::vector<mcb_link> cur;
    mcb_status st = expand_links(c, cur);
    if (st) return st;
    std::vector<uint32_t> qc(n);
    for (int64_t l = 0; l < n; ++l) {
        if (links[l].node != cur[l].node || links[l].dir != cur[l].dir)
            return fail(c, MCB_EINVAL, "link %lld: (node, dir) differs from the built list", (long long)l);
        if (links[l].q_fixed > uint32_t(ONE)) return fail(c, MCB_EINVAL, "link %lld: q_fixed > 2^16", (long long)l);
        qc[l] = links[l].q_fixed;
    }
    c->adj_ready = false;
    if (n > 0) HIPCHK(hipMemcpyAsync(c->lk + c->L.lk_qc, qc.data(), 4 * n, hipMemcpyHostToDevice, c->stream));
    st = clear_flags(c);
    if (st) return st;
    HIPCHK(geom_reclass(c));
    return check_flags(c, nullptr);
}

mcb_status mcb_set_wettability(mcb_ctx* c, const double* phi, int64_t n_wall) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 4) return fail(c, MCB_ESTATE, "links not built");
    if (n_wall != c->n_wall || (n_wall > 0 && !phi)) return fail(c, MCB_EINVAL, "phi needs %lld entries", (long long)c->n_wall);
    const bool cp = c->p.model == MCB_MODEL_CHEMPOT;  // values are assigned chemical potentials
    for (int64_t w = 0; w < n_wall; ++w)
        if (!std::isfinite(phi[w]) || (!cp && !(phi[w] > 0.0)))
            return fail(c, MCB_EINVAL, "phi[%lld] must be %s", (long long)w, cp ? "finite" : "positive");
    c->adj_ready = false;  // a gradient of the old wettability can no longer be taken
    if (n_wall > 0) {
        HIPCHK(hipMemcpyAsync(c->lk + c->L.wl_phi, phi, 8 * n_wall, hipMemcpyHostToDevice, c->stream));
        HIPCHK(wall_factors(c));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return MCB_OK;
}

static mcb_status collide_from(mcb_ctx* c, void* fpre) {
    c->adj_ready = false;  // a new state: the last forward pass no longer ends here
    // the running Delta M sum starts again with the state
    HIPCHK(hipMemsetAsync(c->lat + c->L.dm + 8 * DM_BLOCKS, 0, 8, c->stream));
    // fpre holds pre-collision populations in storage format; the collision writes the other lattice
    const bool to_fb = fpre != c->lat + c->L.fb;
    void* dst = to_fb ? c->lat + c->L.fb : c->lat + c->L.fa;
    HIPCHK(step_fused(c, fpre, nullptr, dst, c->lk + c->L.rec[to_fb ? 1 : 0], false));
    c->swapped = dst == c->lat + c->L.fb;
    c->t = 0;
    c->stage = 5;
    return check_flags(c, nullptr);
}

mcb_status mcb_init_equilibrium(mcb_ctx* c, const double* rho, const double* u) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 4) return fail(c, MCB_ESTATE, "links not built");
    if (!rho) return fail(c, MCB_EINVAL, "rho missing");
    double* srho = reinterpret_cast<double*>(c->lat + c->L.scratch);
    double* su = srho + 2 * c->g.N;
    mcb_status st = clear_flags(c);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(srho, rho, 8 * c->g.N, hipMemcpyHostToDevice, c->stream));
    if (u) HIPCHK(hipMemcpyAsync(su, u, 8 * c->g.N * c->g.dim, hipMemcpyHostToDevice, c->stream));
    void* tmp = c->lat + c->L.fb;
    HIPCHK(init_feq(c, srho, u ? su : nullptr, tmp));
    HIPCHK(hipStreamSynchronize(c->stream));
    return collide_from(c, tmp);
}

mcb_status mcb_set_f(mcb_ctx* c, const double* f) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 4) return fail(c, MCB_ESTATE, "links not built");
    if (!f) return fail(c, MCB_EINVAL, "f missing");
    double* stage_buf = reinterpret_cast<double*>(c->lat + c->L.scratch);
    mcb_status st = clear_flags(c);
    if (st) return st;
    char* tmp = c->lat + c->L.fb;
    for (int i = 0; i < c->g.Q; ++i) {
        HIPCHK(hipMemcpyAsync(stage_buf, f + i * c->g.N, 8 * c->g.N, hipMemcpyHostToDevice, c->stream));
        HIPCHK(convert_plane_in(c, stage_buf, tmp + plane_bytes_off(c->p.precision, i, c->g.N), i));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return collide_from(c, tmp);
}

mcb_status mcb_get_f(mcb_ctx* c, double* f) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 5) return fail(c, MCB_ESTATE, "no state");
    if (!f) return fail(c, MCB_EINVAL, "f missing");
    double* stage_buf = reinterpret_cast<double*>(c->lat + c->L.scratch);
    const char* cur = static_cast<const char*>(fcur(c));
    for (int i = 0; i < c->g.Q; ++i) {
        HIPCHK(convert_plane_out(c, cur + plane_bytes_off(c->p.precision, i, c->g.N), stage_buf, i));
        HIPCHK(hipMemcpyAsync(f + i * c->g.N, stage_buf, 8 * c->g.N, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return check_flags(c, nullptr);
}

static mcb_status drain_slot(mcb_ctx* c, int r) {
    if (!c->ev_pending[r]) return MCB_OK;
    HIPCHK(hipEventSynchronize(c->ev[r][1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[r][0], c->ev[r][1]));
    c->ms_tot += ms;
    c->launches += 1;
    c->ev_pending[r] = false;
    return MCB_OK;
}

mcb_status mcb_step(mcb_ctx* c, int64_t n) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 5) return fail(c, MCB_ESTATE, "no state");
    if (n < 0) return fail(c, MCB_EINVAL, "negative step count");
    if (n > 0) c->adj_ready = false;
    for (int64_t k = 0; k < n; ++k) {
        if (c->timing) {
            const int r = c->ev_next;
            c->ev_next = (r + 1) % mcb_ctx::RING;
            mcb_status st = drain_slot(c, r);
            if (st) return st;
            HIPCHK(hipEventRecord(c->ev[r][0], c->stream));
            HIPCHK(step_fused(c, fcur(c), rcur(c), fnext(c), rnext(c), true));
            HIPCHK(hipEventRecord(c->ev[r][1], c->stream));
            c->ev_pending[r] = true;
        } else {
            HIPCHK(step_fused(c, fcur(c), rcur(c), fnext(c), rnext(c), true));
        }
        c->swapped = !c->swapped;
        ++c->t;
        if (c->p.track_dm) HIPCHK(dm_accumulate(c, rcur(c)));
    }
    return MCB_OK;
}

static AdjWork adj_work(mcb_ctx* c) {
    const AdjPlan& a = c->ap;
    auto d = [&](int64_t off) { return reinterpret_cast<double*>(c->adj + off); };
    AdjWork w;
    w.rho0 = d(a.rho0);
    w.p = d(a.p);
    w.pbar = d(a.pbar);
    w.rho = d(a.rho);
    w.psi = d(a.psi);
    w.dpsi = d(a.dpsi);
    w.rave = d(a.rave);
    w.den = d(a.den);
    w.rbar = d(a.rbar);
    w.qbar = d(a.qbar);
    w.Fbar = d(a.Fbar);
    w.Fv = d(a.Fv);
    w.dphi = d(a.dphi);
    w.part = d(a.part);
    w.sums = d(a.sums);
    return w;
}

mcb_status mcb_adj_required_bytes(mcb_ctx* c, int64_t nsteps, int64_t k, int64_t* bytes) {
    if (!c || !bytes) return MCB_EINVAL;
    if (c->stage < 4) return fail(c, MCB_ESTATE, "links not built");
    if (nsteps < 0 || k < 1) return fail(c, MCB_EINVAL, "need nsteps >= 0 and k >= 1");
    *bytes = adj_plan(c, nsteps, k).bytes;
    return MCB_OK;
}

mcb_status mcb_adj_bind(mcb_ctx* c, void* buf, int64_t bytes) {
    if (!c) return MCB_EINVAL;
    if (!buf || bytes <= 0 || (reinterpret_cast<uintptr_t>(buf) & 255)) return fail(c, MCB_EINVAL, "bad reverse-mode arena");
    c->adj = static_cast<char*>(buf);
    c->adj_bytes = bytes;
    c->adj_ready = false;
    return MCB_OK;
}

mcb_status mcb_adj_forward(mcb_ctx* c, const double* rho0, int64_t nsteps, int64_t k, int32_t kind, const double* prm,
                           double* value) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 4) return fail(c, MCB_ESTATE, "links not built");
    if (!rho0 || !prm || !value) return fail(c, MCB_EINVAL, "missing argument");
    if (nsteps < 0 || k < 1) return fail(c, MCB_EINVAL, "need nsteps >= 0 and k >= 1");
    if (kind < MCB_LOSS_COM_X || kind > MCB_LOSS_TOTAL_MASS) return fail(c, MCB_EINVAL, "unknown loss");
    if (kind == MCB_LOSS_WETTED_LENGTH && !(prm[1] > 0.0)) return fail(c, MCB_EINVAL, "wetted length needs delta > 0");
    const AdjPlan a = adj_plan(c, nsteps, k);
    if (!c->adj || c->adj_bytes < a.bytes) return fail(c, MCB_ESIZE, "reverse-mode arena needs %lld bytes", (long long)a.bytes);
    c->adj_ready = false;
    c->ap = a;
    mcb_status st = mcb_init_equilibrium(c, rho0, nullptr);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(c->adj + a.rho0, rho0, 8 * c->g.N, hipMemcpyHostToDevice, c->stream));
    const int64_t rec_used = compute_bytes(c->p.precision) * c->L.rec_stride * (c->n_bnodes > 0 ? c->n_bnodes : 0);
    for (int64_t t = 0;; ++t) {
        if (t % k == 0 && t / k < a.nck) {
            HIPCHK(hipMemcpyAsync(c->adj + a.ck + (t / k) * a.state_b, fcur(c), state_bytes(c->p.precision, c->g.Q, c->g.N),
                                  hipMemcpyDeviceToDevice, c->stream));
            if (rec_used > 0)
                HIPCHK(hipMemcpyAsync(c->adj + a.ck_rec + (t / k) * a.rec_b, rcur(c), rec_used, hipMemcpyDeviceToDevice, c->stream));
        }
        if (t == nsteps) break;
        HIPCHK(step_fused(c, fcur(c), rcur(c), fnext(c), rnext(c), true));
        c->swapped = !c->swapped;
        ++c->t;
    }
    const AdjWork w = adj_work(c);
    HIPCHK(adj_loss(c, w, fcur(c), kind, prm, 0.0, nullptr));
    double sums[2];
    HIPCHK(hipMemcpyAsync(sums, w.sums, sizeof sums, hipMemcpyDeviceToHost, c->stream));
    st = check_flags(c, nullptr);
    if (st) return st;
    *value = kind == MCB_LOSS_COM_X ? sums[0] / sums[1] : sums[0];
    c->adj_kind = kind;
    c->adj_prm[0] = prm[0];
    c->adj_prm[1] = prm[1];
    c->adj_t_end = c->t;
    c->adj_ready = true;
    ++c->adj_gen;
    return MCB_OK;
}

mcb_status mcb_adj_generation(const mcb_ctx* c, int64_t* generation) {
    if (!c || !generation) return MCB_EINVAL;
    *generation = c->adj_ready ? c->adj_gen : 0;
    return MCB_OK;
}

mcb_status mcb_adj_backward(mcb_ctx* c, int64_t generation, double dloss, double* dphi) {
    if (!c) return MCB_EINVAL;
    if (!c->adj_ready || c->t != c->adj_t_end) return fail(c, MCB_ESTATE, "no matching mcb_adj_forward");
    if (generation != c->adj_gen)
        return fail(c, MCB_ESTATE, "forward pass %lld was superseded by pass %lld", (long long)generation,
                    (long long)c->adj_gen);
    if (c->n_wall > 0 && !dphi) return fail(c, MCB_EINVAL, "dphi missing");
    const AdjPlan& a = c->ap;
    const AdjWork w = adj_work(c);
    auto lam = [&](int b) { return reinterpret_cast<double*>(c->adj + a.lam[b]); };
    auto lamR = [&](int b) { return reinterpret_cast<double*>(c->adj + a.lamR[b]); };
    mcb_status st = clear_flags(c);
    if (st) return st;
    HIPCHK(hipMemsetAsync(w.dphi, 0, 8 * (c->n_wall > 0 ? c->n_wall : 1), c->stream));
    int cur = 0;
    HIPCHK(hipMemsetAsync(lamR(cur), 0, 8 * (a.nslots > 0 ? a.nslots : 1), c->stream));
    HIPCHK(adj_loss(c, w, fcur(c), c->adj_kind, c->adj_prm, dloss, lam(cur)));
    for (int64_t sg = a.nck - 1; sg >= 0; --sg) {
        const int64_t t0 = sg * a.k, t1 = std::min(a.nsteps, t0 + a.k);
        if (t0 >= t1) continue;
        char* ck = c->adj + a.ck + sg * a.state_b;
        char* ckr = c->adj + a.ck_rec + sg * a.rec_b;
        // recompute the states t0+1 .. t1-1 of the segment, each with its boundary records
        const char* prev = ck;
        const char* prev_rec = ckr;
        for (int64_t t = t0 + 1; t < t1; ++t) {
            char* dst = c->adj + a.seg + (t - t0 - 1) * a.state_b;
            char* dst_rec = c->adj + a.seg_rec + (t - t0 - 1) * a.rec_b;
            HIPCHK(step_fused(c, prev, prev_rec, dst, dst_rec, true));
            prev = dst;
            prev_rec = dst_rec;
        }
        for (int64_t t = t1 - 1; t >= t0; --t) {
            const void* gt = t == t0 ? static_cast<const void*>(ck) : c->adj + a.seg + (t - t0 - 1) * a.state_b;
            const void* rt = t == t0 ? static_cast<const void*>(ckr) : c->adj + a.seg_rec + (t - t0 - 1) * a.rec_b;
            HIPCHK(adj_step(c, w, gt, rt, 1, lam(cur), lamR(cur), lam(1 - cur), lamR(1 - cur)));
            cur = 1 - cur;
        }
    }
    // the first collision, from f^eq(rho0, 0)
    HIPCHK(adj_step(c, w, nullptr, nullptr, 0, lam(cur), lamR(cur), nullptr, nullptr));
    if (c->n_wall > 0) HIPCHK(hipMemcpyAsync(dphi, w.dphi, 8 * c->n_wall, hipMemcpyDeviceToHost, c->stream));
    return check_flags(c, nullptr);
}

mcb_status mcb_timing(mcb_ctx* c, int32_t enable) {
    if (!c) return MCB_EINVAL;
    if (enable) {
        if (!c->ev_made) {
            for (int r = 0; r < mcb_ctx::RING; ++r)
                for (int k = 0; k < 2; ++k) HIPCHK(hipEventCreate(&c->ev[r][k]));
            c->ev_made = true;
        }
        for (int r = 0; r < mcb_ctx::RING; ++r) c->ev_pending[r] = false;
        c->ev_next = 0;
        c->ms_tot = 0.0;
        c->launches = 0;
    }
    c->timing = enable != 0;
    return MCB_OK;
}

mcb_status mcb_timing_report(mcb_ctx* c, double* ms, int64_t* launches) {
    if (!c) return MCB_EINVAL;
    if (c->ev_made)
        for (int r = 0; r < mcb_ctx::RING; ++r) {
            mcb_status st = drain_slot(c, r);
            if (st) return st;
        }
    if (ms) *ms = c->ms_tot;
    if (launches) *launches = c->launches;
    return MCB_OK;
}

// chemical-potential model: the velocity output takes the force from the density and chemical-
// potential fields of the collision that made the current state; the step keeps them on chip, so
// they are formed here again from the populations that collision took (the other buffer of the
// pair, and its records), which no step has overwritten since
static hipError_t cp_fields_for_output(mcb_ctx* c) {
    if (c->p.model != MCB_MODEL_CHEMPOT) return hipSuccess;
    return cp_fields(c, fnext(c), rnext(c), c->t > 0);
}

mcb_status mcb_moments(mcb_ctx* c, double* rho, double* v) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 5) return fail(c, MCB_ESTATE, "no state");
    HIPCHK(cp_fields_for_output(c));
    HIPCHK(moments_out(c, fcur(c), rho, v));
    return check_flags(c, nullptr);
}

mcb_status mcb_max_speed(mcb_ctx* c, double* vmax, int64_t* node) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 5) return fail(c, MCB_ESTATE, "no state");
    HIPCHK(cp_fields_for_output(c));
    HIPCHK(max_speed(c, fcur(c)));
    double r[2];
    HIPCHK(hipMemcpyAsync(r, reinterpret_cast<double*>(c->lat + c->L.result) + MON_SPEED, sizeof r, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (vmax) *vmax = r[1] < 0.0 ? 0.0 : r[0];
    if (node) *node = int64_t(r[1]);
    return check_flags(c, nullptr);
}

// the running Delta M sum of track_dm (NaN when not tracked), as last copied to the host
static double dm_total(const mcb_ctx* c) { return c->p.track_dm ? c->dm_host : std::nan(""); }

mcb_status mcb_mass(mcb_ctx* c, mcb_mass_report* out) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 5) return fail(c, MCB_ESTATE, "no state");
    if (!out) return fail(c, MCB_EINVAL, "report missing");
    HIPCHK(monitor(c, fcur(c), rcur(c)));
    double r[MON_FIELDS];
    HIPCHK(hipMemcpyAsync(r, c->lat + c->L.result, sizeof r, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&c->dm_host, c->lat + c->L.dm + 8 * DM_BLOCKS, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memset(out, 0, sizeof *out);
    out->M = r[0];
    out->J[0] = r[1];
    out->J[1] = r[2];
    out->J[2] = r[3];
    out->dM_last = c->t > 0 ? r[4] : 0.0;
    out->n_nan = int64_t(r[5]);
    out->t = c->t;
    out->dM_cum = dm_total(c);
    int64_t nd = 0;
    mcb_status st = check_flags(c, &nd);
    out->n_domain = nd;
    if (st) return st;
    if (out->n_nan > 0) return fail(c, MCB_ENAN, "%lld fluid nodes hold non-finite populations", (long long)out->n_nan);
    return MCB_OK;
}

mcb_status mcb_mass_static(mcb_ctx* c, mcb_mass_report* out) {
    if (!c) return MCB_EINVAL;
    if (c->stage < 5) return fail(c, MCB_ESTATE, "no state");
    if (!out) return fail(c, MCB_EINVAL, "report missing");
    if (!c->scratch)
        return c->device < 0 ? fail(c, MCB_ESTATE, "no device scratch: bind buffers first")
                             : fail(c, MCB_EHIP, "device scratch not found: %s", hipGetErrorString(c->scratch_err));
    const int64_t need = int64_t(MON_BLOCKS) * MON_FIELDS + MON_FIELDS;  // the monitor's fixed grid
    if (need > SCRATCH_DOUBLES)
        return fail(c, MCB_ESIZE, "the reduction needs %lld doubles of scratch, the static array holds %lld", (long long)need,
                    (long long)SCRATCH_DOUBLES);
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != c->device) return fail(c, MCB_ESTATE, "device %d is current, the context's buffers are on device %d", cur, c->device);
    // every entry of the partials and the result is written before it is read: nothing to clear
    double* part = c->scratch;
    double* res = c->scratch + int64_t(MON_BLOCKS) * MON_FIELDS;
    HIPCHK(monitor(c, fcur(c), rcur(c), part, res));
    double r[MON_FIELDS];
    HIPCHK(hipMemcpyAsync(r, res, sizeof r, hipMemcpyDeviceToHost, c->stream));
    int32_t flags[FLAG_COUNT];
    HIPCHK(hipMemcpyAsync(flags, c->lat + c->L.flags, sizeof flags, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&c->dm_host, c->lat + c->L.dm + 8 * DM_BLOCKS, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::memset(out, 0, sizeof *out);
    out->M = r[0];
    out->J[0] = r[1];
    out->J[1] = r[2];
    out->J[2] = r[3];
    out->dM_last = c->t > 0 ? r[4] : 0.0;
    out->n_nan = int64_t(r[5]);
    out->n_domain = flags[FLAG_DOMAIN] ? 1 : 0;
    out->t = c->t;
    out->dM_cum = dm_total(c);
    if (out->n_nan > 0) return fail(c, MCB_ENAN, "%lld fluid nodes hold non-finite populations", (long long)out->n_nan);
    if (flags[FLAG_DOMAIN]) return fail(c, MCB_EDOMAIN, "psi domain error: rho <= 0 or negative square-root argument");
    return MCB_OK;
}

mcb_status mcb_sync(mcb_ctx* c) {
    if (!c) return MCB_EINVAL;
    if (!c->stream && !c->lat) return MCB_OK;
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->stage < 1) return MCB_OK;
    return check_flags(c, nullptr);
}

}  // extern "C"

namespace mcb {
hipError_t step2d(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull);
hipError_t step3d(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull);

hipError_t step_fused(mcb_ctx* c, const void* fcur, const void* rcur, void* fnext, void* rnext, bool pull) {
    return c->g.dim == 2 ? step2d(c, fcur, rcur, fnext, rnext, pull) : step3d(c, fcur, rcur, fnext, rnext, pull);
}
}  // namespace mcb
