// Host side of the C ABI declared in include/eelbm.h: parameter validation,
// layout of the caller-owned device state, launch sequencing on the caller's
// stream, read-out, diagnostics and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "eelbm.h"
#include "eelbm_internal.hpp"

using namespace eelbm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return EELBM_E_HIP;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    size_t pop[2], cf[2], lag, side[2], noise, stage, macro, partials, dout, spart, dscr, total;
};

struct Geometry {
    int D, Q;
    long long n;
    int flow_axis;
    long long face_n;
    size_t tsize, csize;
    dim3 grid, block;
    int nblocks;
    int ntx, nty, xcd_remap;
    bool channel;
    int bc_mode;  // kBc* configuration the step kernels are compiled for
};

int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return v && *v ? std::atoi(v) : dflt;
}

// LDS of a tile's staged record window (FP32 compute): 32 bytes for each
// node of the tile and its one-node halo, in three planes in D3Q19; the
// window must fit the 64 KiB a workgroup can address.
constexpr size_t kMaxWindowBytes = 65536;
// FP64 arithmetic and records (FP64 storage, or FP32 populations with FP64 arithmetic)
bool f64_compute(const eelbm_params& p) { return p.storage == EELBM_FP64 || p.storage == EELBM_FP32_F64; }
// bytes per stored population value: a direction's four sets take 4x this
// (mixed storage: 12 bytes, FP32 f_g and three FP16 values)
size_t pop_value_bytes(const eelbm_params& p) {
    switch (p.storage) {
        case EELBM_FP64: return 8;
        case EELBM_FP32:
        case EELBM_FP32_F64: return 4;
        case EELBM_MIXED: return 3;
        default: return 2;
    }
}
size_t window_bytes(const eelbm_params& p, int bx, int by) {
    if (f64_compute(p)) return 0;
    return (size_t)(bx + 2) * (by + 2) * (p.lattice == EELBM_D3Q19 ? 3 : 1) * 32;
}
bool tile_ok(const eelbm_params& p, int bx, int by) {
    return bx >= 64 && by >= 1 && bx % 64 == 0 && bx * by <= 256 && window_bytes(p, bx, by) <= kMaxWindowBytes;
}

// Launch shape: tiles of bx * by nodes (a whole number of 64-wide wavefronts,
// at most 256 threads), one workgroup per tile, tiles of all planes in one
// grid dimension.  bx = 0 picks the default: rows of up to 256 nodes in
// D2Q9, 64 x 4 tiles in D3Q19 (whose record window of a 256-node row would
// not fit the workgroup's LDS).  EELBM_TILE_X / EELBM_TILE_Y /
// EELBM_XCD_REMAP override the default.
void set_tiles(const eelbm_params& p, Geometry* g, int bx, int by, int xcd) {
    if (bx <= 0) {
        bx = env_int("EELBM_TILE_X", 0);
        by = env_int("EELBM_TILE_Y", 0);
    }
    if (!tile_ok(p, bx, by)) {
        if (p.lattice == EELBM_D3Q19) {
            bx = 64;
            by = 4;
        } else {
            bx = ((p.nx + 63) / 64) * 64;
            if (bx > 256) bx = 256;
            by = 1;
        }
    }
    if (xcd < 0) xcd = env_int("EELBM_XCD_REMAP", 1);
    g->block = dim3(bx, by, 1);
    g->ntx = (p.nx + bx - 1) / bx;
    g->nty = (p.ny + by - 1) / by;
    g->xcd_remap = xcd ? 1 : 0;
    g->nblocks = g->ntx * g->nty * p.nz;
    g->grid = dim3(g->nblocks, 1, 1);
}

bool periodic(const eelbm_params& p, int face) { return p.bc[face] == EELBM_BC_PERIODIC; }

int validate(const eelbm_params* pp, Geometry* g) {
    if (!pp) return fail(EELBM_E_PARAM, "params is NULL");
    const eelbm_params& p = *pp;
    if (p.abi_version != EELBM_ABI_VERSION) return fail(EELBM_E_PARAM, "abi_version mismatch");
    if (p.lattice != EELBM_D2Q9 && p.lattice != EELBM_D3Q19) return fail(EELBM_E_PARAM, "lattice must be D2Q9 or D3Q19");
    if (p.storage < EELBM_FP64 || p.storage > EELBM_MIXED) return fail(EELBM_E_PARAM, "unknown storage");
    const int D = p.lattice == EELBM_D2Q9 ? 2 : 3;
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return fail(EELBM_E_PARAM, "grid sizes must be >= 1");
    if (D == 2 && p.nz != 1) return fail(EELBM_E_PARAM, "D2Q9 needs nz = 1");
    if (p.ny > 65535 || p.nz > 65535) return fail(EELBM_E_PARAM, "ny and nz must be <= 65535");
    const long long n = (long long)p.nx * p.ny * p.nz;
    // every per-node array (the widest: 8-wide FP64 records) stays below 4 GiB,
    // so kernels address it with 32-bit byte offsets
    if ((unsigned long long)n * 8 * (f64_compute(p) ? 8 : 4) >= (1ull << 32))
        return fail(EELBM_E_PARAM, "too many nodes for one lattice");
    // ... and so does one z-plane of a population copy (buffer descriptors)
    {
        const unsigned long long tsz = pop_value_bytes(p);
        const unsigned long long plane = (unsigned long long)p.ny * ((p.nx + 63) / 64) * 64 * 4 * (D == 2 ? 9 : 19);
        if (plane * tsz >= (1ull << 32)) return fail(EELBM_E_PARAM, "lattice plane too large");
    }
    int flow_axis = -1;
    const int nn[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; ++a) {
        const int lo = p.bc[2 * a], hi = p.bc[2 * a + 1];
        for (int v : {lo, hi})
            if (v < EELBM_BC_PERIODIC || v > EELBM_BC_OUTLET) return fail(EELBM_E_PARAM, "unknown boundary type");
        if (a >= D) {
            if (lo != EELBM_BC_PERIODIC || hi != EELBM_BC_PERIODIC)
                return fail(EELBM_E_PARAM, "faces beyond the lattice dimension must be periodic");
            continue;
        }
        if ((lo == EELBM_BC_PERIODIC) != (hi == EELBM_BC_PERIODIC))
            return fail(EELBM_E_PARAM, "periodic faces come in pairs");
        const bool open = lo == EELBM_BC_INLET || lo == EELBM_BC_OUTLET || hi == EELBM_BC_INLET || hi == EELBM_BC_OUTLET;
        if (open) {
            if (flow_axis >= 0) return fail(EELBM_E_PARAM, "inlet/outlet faces on more than one axis");
            flow_axis = a;
            if (nn[a] < 4) return fail(EELBM_E_PARAM, "an axis with inlet/outlet faces needs >= 4 nodes");
        } else if (lo == EELBM_BC_WALL && nn[a] < 2) {
            return fail(EELBM_E_PARAM, "a walled axis needs >= 2 nodes");
        }
    }
    if (p.up_axis < 0 || p.up_axis >= D) return fail(EELBM_E_PARAM, "up_axis out of range");
    if (!(p.rho_g > 0 && p.rho_l > 0)) return fail(EELBM_E_PARAM, "densities must be > 0");
    for (double om : {p.omega_g, p.omega_l, p.omega_ag, p.omega_al})
        if (!(om > 0 && om < 2)) return fail(EELBM_E_PARAM, "relaxation rates must lie in (0, 2)");
    if (p.drag_model != EELBM_DRAG_CONST && p.drag_model != EELBM_DRAG_CGW) return fail(EELBM_E_PARAM, "unknown drag model");
    if (p.rho_ref_mode < EELBM_RHOREF_LIQUID || p.rho_ref_mode > EELBM_RHOREF_EXPLICIT)
        return fail(EELBM_E_PARAM, "unknown rho_ref_mode");
    if (p.n_gamma < 1) return fail(EELBM_E_PARAM, "n_gamma must be >= 1");
    if (!(p.alpha_min > 0)) return fail(EELBM_E_PARAM, "alpha_min must be > 0");
    if (p.flags & ~(EELBM_FLAG_NO_RENORM | EELBM_FLAG_NO_SIGMA_GRAD)) return fail(EELBM_E_PARAM, "unknown flags");
    if (!std::isfinite(p.g_hat) || !std::isfinite(p.gamma) || !std::isfinite(p.K_I) || !std::isfinite(p.kappa_I) ||
        !std::isfinite(p.K_W))
        return fail(EELBM_E_PARAM, "non-finite parameter");
    if (g) {
        g->D = D;
        g->Q = D == 2 ? 9 : 19;
        g->n = n;
        g->flow_axis = flow_axis;
        g->face_n = flow_axis < 0 ? 0 : n / nn[flow_axis];
        g->tsize = pop_value_bytes(p);
        g->csize = f64_compute(p) ? 8 : 4;
        set_tiles(p, g, 0, 0, -1);
        g->channel = false;
        for (int f = 0; f < 2 * D; ++f) g->channel = g->channel || p.bc[f] != EELBM_BC_PERIODIC;
        bool column = p.bc[2 * (D - 1)] == EELBM_BC_INLET && p.bc[2 * (D - 1) + 1] == EELBM_BC_OUTLET;
        for (int f = 0; f < 2 * (D - 1); ++f) column = column && p.bc[f] == EELBM_BC_WALL;
        g->bc_mode = !g->channel ? kBcPeriodic : (column ? kBcColumn : kBcGeneric);
    }
    return EELBM_OK;
}

// upper bound of the workgroup count over every allowed tile shape
// (bx * by >= 64): ceil(nx/bx) ceil(ny/by) <= nx ny / 64 + nx + ny + 1
size_t max_blocks(const eelbm_params& p) {
    return ((size_t)p.nx * p.ny / 64 + p.nx + p.ny + 2) * (size_t)p.nz;
}

// population copy: per z-plane, rows of 64-node x-blocks, each block holding
// its 4Q populations contiguously (the layout the step kernel reads)
int x_blocks(const eelbm_params& p) { return (p.nx + 63) / 64; }
size_t pop_plane_elems(const eelbm_params& p, const Geometry& g) {
    return (size_t)p.ny * x_blocks(p) * 4 * g.Q * 64;
}
size_t pop_bytes(const eelbm_params& p, const Geometry& g) { return (size_t)p.nz * pop_plane_elems(p, g) * g.tsize; }

// MI355X's last-level (Infinity) cache: populations written in one step are
// found there in the next when one set of them is smaller
constexpr size_t kLastLevelCacheBytes = 256ull << 20;

// imposed-velocity region of one ping-pong copy: [n] records of 2 + 2D
// values (8 in D3Q19, 6 in D2Q9), then [n] alpha_l values (used only without
// renormalisation)
size_t cf_records_bytes(const Geometry& g) { return align256((g.D == 3 ? 8 : 6) * (size_t)g.n * g.csize); }
size_t cf_region_bytes(const Geometry& g) { return cf_records_bytes(g) + (size_t)g.n * g.csize; }
// lag region: [n] 2-wide records (S''_g, S''_l), then [n] Lambda'
size_t lag_records_bytes(const Geometry& g) { return align256(2 * (size_t)g.n * g.csize); }
size_t lag_region_bytes(const eelbm_params& p, const Geometry& g) {
    if (p.n_gamma <= 1) return 0;
    return lag_records_bytes(g) + (size_t)g.n * g.csize;
}

Layout layout(const eelbm_params& p, const Geometry& g) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t n = (size_t)g.n;
    const int NV = 2 * g.D + 2;
    for (int k = 0; k < 2; ++k) L.pop[k] = take(pop_bytes(p, g));
    for (int k = 0; k < 2; ++k) L.cf[k] = take(cf_region_bytes(g));
    L.lag = take(lag_region_bytes(p, g));
    for (int k = 0; k < 2; ++k) L.side[k] = take((size_t)2 * 2 * NV * (size_t)g.face_n * g.csize);
    L.noise = take((size_t)g.face_n * 8);
    L.stage = take((size_t)(2 + 2 * g.D) * n * 8);
    L.macro = take((size_t)(3 + 2 * g.D) * n * 8);
    L.partials = take(max_blocks(p) * kNDiag * 8);
    L.dout = take((kNDiag + 1) * 8);
    L.spart = take(1024 * 8);
    L.dscr = take((size_t)kDiagGroups * kNDiag * 8);
    L.total = off;
    return L;
}


}  // namespace

struct eelbm_handle {
    eelbm_params p;
    Geometry g;
    Layout L;
    char* mem;
    size_t bytes;
    hipStream_t stream;
    int device;
    int64_t t;
    int cur;
    bool initialized;
    double rho_ref, b_g, b_l;
    double alpha_ref;  // mean initial gas fraction: reference of the f_alpha deviations
    int64_t diag_blocks;  // workgroups that wrote the current diagnostic partial sums
    KParams kp;
    uint64_t gen;  // bumped when the step parameters or tiles change (init, load, launch shape)
};

namespace {

KBuffers buffers(eelbm_handle* h, int in, int out) {
    KBuffers b{};
    char* m = h->mem;
    b.pop_in = m + h->L.pop[in];
    b.pop_out = m + h->L.pop[out];
    b.cf_in = m + h->L.cf[in];
    b.cf_out = m + h->L.cf[out];
    b.al_in = m + h->L.cf[in] + cf_records_bytes(h->g);
    b.al_out = m + h->L.cf[out] + cf_records_bytes(h->g);
    b.lag = m + h->L.lag;
    b.lag_lam = m + h->L.lag + lag_records_bytes(h->g);
    b.side_in = m + h->L.side[in];
    b.side_out = m + h->L.side[out];
    b.noise = reinterpret_cast<const double*>(m + h->L.noise);
    b.stage = reinterpret_cast<const double*>(m + h->L.stage);
    b.macro = reinterpret_cast<double*>(m + h->L.macro);
    b.partials = reinterpret_cast<double*>(m + h->L.partials);
    return b;
}

void fill_kparams(eelbm_handle* h) {
    const eelbm_params& p = h->p;
    KParams& k = h->kp;
    k = KParams{};
    k.nx = p.nx;
    k.ny = p.ny;
    k.nz = p.nz;
    k.n = h->g.n;
    k.ntx = h->g.ntx;
    k.nxb = x_blocks(p);
    k.plane = (long long)pop_plane_elems(p, h->g);
    k.nty = h->g.nty;
    k.xcd_remap = h->g.xcd_remap;
    for (int a = 0; a < 3; ++a) {
        k.per[a] = periodic(p, 2 * a);
        k.wall_lo[a] = p.bc[2 * a] == EELBM_BC_WALL;
        k.wall_hi[a] = p.bc[2 * a + 1] == EELBM_BC_WALL;
    }
    k.flow_axis = h->g.flow_axis;
    k.face_lo = h->g.flow_axis >= 0 ? p.bc[2 * h->g.flow_axis] : EELBM_BC_PERIODIC;
    k.face_hi = h->g.flow_axis >= 0 ? p.bc[2 * h->g.flow_axis + 1] : EELBM_BC_PERIODIC;
    k.face_n = h->g.face_n;
    k.up = p.up_axis;
    k.cgw = p.drag_model == EELBM_DRAG_CGW;
    k.use_lag = p.n_gamma > 1;
    k.renorm = !(p.flags & EELBM_FLAG_NO_RENORM);
    k.sigma_grad = !(p.flags & EELBM_FLAG_NO_SIGMA_GRAD);
    k.nt_store = pop_bytes(p, h->g) > kLastLevelCacheBytes;
    k.R = p.rho_l / p.rho_g;
    k.invR = p.rho_g / p.rho_l;
    k.rho_g = p.rho_g;
    k.rho_l = p.rho_l;
    k.omega_g = p.omega_g;
    k.omega_l = p.omega_l;
    k.psi_g = p.psi_g;
    k.psi_l = p.psi_l;
    k.omega_ag = p.omega_ag;
    k.omega_al = p.omega_al;
    k.K_I = p.K_I;
    k.kappa_I = p.kappa_I;
    k.K_W = p.K_W;
    k.b_g = h->b_g;
    k.b_l = h->b_l;
    k.gamma = p.gamma;
    k.alpha_min = p.alpha_min;
    k.n_gamma = p.n_gamma;
    k.a_in_max = p.alpha_in_max;
    k.a_in_min = p.alpha_in_min;
    k.ug_in_max = p.ug_in_max;
    k.ug_in_min = p.ug_in_min;
    k.ul_in_max = p.ul_in_max;
    k.ul_in_min = p.ul_in_min;
    k.n_ramp = p.n_ramp;
    k.alpha_ref = h->alpha_ref;
    // FP16 scales of the stored residuals (FP16 and mixed storage): 2^20
    // for f_g, f_ag, f_al, 2^20 * 2^round(log2 min(R, 64)) for the moving
    // populations of f_l (its rest population is stored unscaled)
    const double R = p.rho_l / p.rho_g;
    int e = (int)std::lround(std::log2(std::min(std::max(R, 1.0), 64.0)));
    k.h16_up[0] = std::ldexp(1.0f, 20);
    k.h16_up[1] = std::ldexp(1.0f, 20 + e);
    k.h16_down[0] = std::ldexp(1.0f, -20);
    k.h16_down[1] = std::ldexp(1.0f, -(20 + e));
}

int launch(eelbm_handle* h, bool init, int64_t t, bool last, const int32_t* gate = nullptr) {
    KCtl c{};
    c.t = t;
    c.gate = gate;
    // lagged S'' and Lambda' (Eqs. (133), (137)) refresh at t mod n_gamma == 0
    // and at the first step of a run or rebuild: fields bring no lagged values
    c.refresh = init || (t % h->p.n_gamma) == 0;
    c.write_macro = last;
    c.write_diag = last;
    // the state at time t is always copy t mod 2
    const int in = init ? 1 - (int)(t & 1) : h->cur;
    const int out = init ? (int)(t & 1) : 1 - h->cur;
    KBuffers b = buffers(h, in, out);
    hipError_t e = launch_step(h->p.lattice, h->p.storage, h->g.bc_mode, init, h->kp, b, c, h->g.grid, h->g.block,
                               h->stream);
    if (e != hipSuccess) return hip_fail(e, "k_step launch");
    if (last) h->diag_blocks = h->g.nblocks;
    h->cur = out;
    h->t = t;
    return EELBM_OK;
}

int copy_in(eelbm_handle* h, void* dst, const void* src, size_t bytes, int on_device) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (init fields)");
    return EELBM_OK;
}

}  // namespace

namespace eelbm {
// the thread-local message of eelbm_last_error, for entry points defined in
// the kernel files
int set_error(int code, const char* msg) { return fail(code, msg); }
}  // namespace eelbm

extern "C" {

int32_t eelbm_abi_version(void) { return EELBM_ABI_VERSION; }
size_t eelbm_params_size(void) { return sizeof(eelbm_params); }
const char* eelbm_last_error(void) { return g_err.c_str(); }

int eelbm_state_bytes(const eelbm_params* p, size_t* bytes) {
    Geometry g;
    int rc = validate(p, &g);
    if (rc) return rc;
    if (!bytes) return fail(EELBM_E_PARAM, "bytes is NULL");
    *bytes = layout(*p, g).total;
    return EELBM_OK;
}

int eelbm_create(const eelbm_params* p, void* device_mem, size_t bytes, void* hip_stream, eelbm_handle** out) {
    if (!out) return fail(EELBM_E_PARAM, "out is NULL");
    *out = nullptr;
    Geometry g;
    int rc = validate(p, &g);
    if (rc) return rc;
    Layout L = layout(*p, g);
    if (!device_mem) return fail(EELBM_E_PARAM, "device_mem is NULL");
    if (bytes < L.total) return fail(EELBM_E_SIZE, "device buffer smaller than eelbm_state_bytes");
    if (reinterpret_cast<uintptr_t>(device_mem) & 255) return fail(EELBM_E_PARAM, "device buffer not 256-byte aligned");
    eelbm_handle* h = new (std::nothrow) eelbm_handle();
    if (!h) return fail(EELBM_E_PARAM, "out of host memory");
    h->p = *p;
    h->g = g;
    h->L = L;
    h->mem = static_cast<char*>(device_mem);
    h->bytes = bytes;
    h->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipGetDevice");
    }
    h->t = 0;
    h->cur = 0;
    h->initialized = false;
    h->rho_ref = p->rho_l;
    *out = h;
    return EELBM_OK;
}

}  // extern "C"

namespace {
// initial state (keep = false) or rebuilt state at time t (keep = true:
// inlet noise, buoyancy reference and lag fields are those of the run)
int init_impl(eelbm_handle* h, int64_t t, const double* alpha_g, const double* u_g, const double* u_l,
              const double* dp_k, const double* inlet_noise, int on_device, bool keep,
              const int32_t* gate = nullptr) {
    if (!h) return fail(EELBM_E_PARAM, "handle is NULL");
    if (!alpha_g) return fail(EELBM_E_PARAM, "alpha_g is NULL");
    if (keep && !h->initialized) return fail(EELBM_E_STATE, "eelbm_init_fields not called");
    if (t < 0) return fail(EELBM_E_PARAM, "t < 0");
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const size_t n = (size_t)h->g.n;
    const int D = h->g.D;
    double* stage = reinterpret_cast<double*>(h->mem + h->L.stage);
    int rc = copy_in(h, stage, alpha_g, n * 8, on_device);
    if (rc) return rc;
    const double* parts[3] = {u_g, u_l, dp_k};
    const size_t offs[3] = {n, (size_t)(1 + D) * n, (size_t)(1 + 2 * D) * n};
    const size_t cnt[3] = {(size_t)D * n, (size_t)D * n, n};
    for (int k = 0; k < 3; ++k) {
        if (parts[k]) {
            rc = copy_in(h, stage + offs[k], parts[k], cnt[k] * 8, on_device);
        } else {
            e = hipMemsetAsync(stage + offs[k], 0, cnt[k] * 8, h->stream);
            rc = e == hipSuccess ? EELBM_OK : hip_fail(e, "hipMemsetAsync");
        }
        if (rc) return rc;
    }
    if (h->g.face_n > 0 && !keep) {
        double* noise = reinterpret_cast<double*>(h->mem + h->L.noise);
        if (inlet_noise) {
            rc = copy_in(h, noise, inlet_noise, (size_t)h->g.face_n * 8, on_device);
        } else {
            std::vector<double> ones((size_t)h->g.face_n, 1.0);
            e = hipMemcpyAsync(noise, ones.data(), ones.size() * 8, hipMemcpyHostToDevice, h->stream);
            rc = e == hipSuccess ? EELBM_OK : hip_fail(e, "hipMemcpyAsync (noise)");
            if (!rc) {
                e = hipStreamSynchronize(h->stream);
                if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
            }
        }
        if (rc) return rc;
    }
    // mean initial gas fraction: reference of the f_alpha deviations and,
    // for EELBM_RHOREF_MIXTURE_MEAN, of the buoyancy reference density (a
    // rebuild keeps both: no read-back, no synchronisation)
    const eelbm_params& p = h->p;
    double am = h->alpha_ref;
    if (!keep) {
        double* sp = reinterpret_cast<double*>(h->mem + h->L.spart);
        double* so = reinterpret_cast<double*>(h->mem + h->L.dout) + kNDiag;
        e = launch_sum(stage, (long long)n, sp, 1024, so, h->stream);
        if (e != hipSuccess) return hip_fail(e, "alpha sum launch");
        double sum = 0;
        e = hipMemcpyAsync(&sum, so, 8, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "alpha sum read-back");
        am = sum / (double)n;
    }
    if (!std::isfinite(am)) return fail(EELBM_E_NONFINITE, "non-finite initial gas fraction");
    if (!keep) h->alpha_ref = f64_compute(p) ? am : (double)(float)am;
    if (keep) {
        // buoyancy reference of the run
    } else if (p.rho_ref_mode == EELBM_RHOREF_LIQUID) {
        h->rho_ref = p.rho_l;
    } else if (p.rho_ref_mode == EELBM_RHOREF_EXPLICIT) {
        h->rho_ref = p.rho_ref;
    } else {
        h->rho_ref = am * p.rho_g + (1.0 - am) * p.rho_l;
    }
    h->b_g = (h->rho_ref / p.rho_g - 1.0) * p.g_hat;
    h->b_l = (h->rho_ref / p.rho_l - 1.0) * p.g_hat;
    fill_kparams(h);
    if (!keep) ++h->gen;
    rc = launch(h, true, t, true, gate);
    if (rc) return rc;
    if (!on_device) {
        // host inputs were copied from pageable memory; finish before returning
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    }
    h->initialized = true;
    return EELBM_OK;
}
}  // namespace

extern "C" {

int eelbm_init_fields(eelbm_handle* h, const double* alpha_g, const double* u_g, const double* u_l,
                      const double* dp_k, const double* inlet_noise, int on_device) {
    return init_impl(h, 0, alpha_g, u_g, u_l, dp_k, inlet_noise, on_device, false);
}

int eelbm_reinit_fields(eelbm_handle* h, int64_t t, const double* alpha_g, const double* u_g, const double* u_l,
                        const double* dp_k, int on_device) {
    return init_impl(h, t, alpha_g, u_g, u_l, dp_k, nullptr, on_device, true);
}

int eelbm_reinit_fields_gated(eelbm_handle* h, int64_t t, const double* alpha_g, const double* u_g, const double* u_l,
                              const double* dp_k, const int32_t* gate) {
    if (!gate) return fail(EELBM_E_PARAM, "gate is NULL");
    if (!u_g || !u_l || !dp_k) return fail(EELBM_E_PARAM, "a gated rebuild needs every field");
    return init_impl(h, t, alpha_g, u_g, u_l, dp_k, nullptr, 1, true, gate);
}

int eelbm_advance(eelbm_handle* h, int64_t nsteps) {
    if (!h) return fail(EELBM_E_PARAM, "handle is NULL");
    if (!h->initialized) return fail(EELBM_E_STATE, "eelbm_init_fields not called");
    if (nsteps < 0) return fail(EELBM_E_PARAM, "nsteps < 0");
    for (int64_t k = 1; k <= nsteps; ++k) {
        int rc = launch(h, false, h->t + 1, k == nsteps);
        if (rc) return rc;
    }
    return EELBM_OK;
}

int64_t eelbm_time(const eelbm_handle* h) { return h ? h->t : -1; }

int eelbm_set_launch(eelbm_handle* h, int32_t tile_x, int32_t tile_y, int32_t xcd_remap) {
    if (!h) return fail(EELBM_E_PARAM, "handle is NULL");
    if (tile_x < 64 || tile_y < 1 || tile_x % 64 != 0 || tile_x * tile_y > 256)
        return fail(EELBM_E_PARAM, "tile_x must be a multiple of 64 (one x-block per wavefront), at most 256 nodes");
    if (!tile_ok(h->p, tile_x, tile_y))
        return fail(EELBM_E_PARAM, "the tile's record window exceeds 64 KiB of LDS (D3Q19: at most 64x4 or 128x2)");
    if (h->g.D == 2 && tile_y > h->p.ny) return fail(EELBM_E_PARAM, "tile_y exceeds ny");
    set_tiles(h->p, &h->g, tile_x, tile_y, xcd_remap ? 1 : 0);
    fill_kparams(h);
    ++h->gen;
    return EELBM_OK;
}

int eelbm_get_launch(const eelbm_handle* h, int32_t* tile_x, int32_t* tile_y, int32_t* xcd_remap) {
    if (!h) return fail(EELBM_E_PARAM, "handle is NULL");
    if (tile_x) *tile_x = (int32_t)h->g.block.x;
    if (tile_y) *tile_y = (int32_t)h->g.block.y;
    if (xcd_remap) *xcd_remap = h->g.xcd_remap;
    return EELBM_OK;
}

int eelbm_read(eelbm_handle* h, int32_t field, void* dst, int32_t dst_dtype, int on_device) {
    if (!h) return fail(EELBM_E_PARAM, "handle is NULL");
    if (!h->initialized) return fail(EELBM_E_STATE, "eelbm_init_fields not called");
    if (!dst) return fail(EELBM_E_PARAM, "dst is NULL");
    if (dst_dtype != EELBM_DTYPE_F64 && dst_dtype != EELBM_DTYPE_F32) return fail(EELBM_E_PARAM, "unknown dtype");
    const size_t n = (size_t)h->g.n;
    const int D = h->g.D;
    size_t off, cnt;
    double add = 0.0;
    switch (field) {
        case EELBM_FIELD_ALPHA_G: off = 0; cnt = n; break;
        case EELBM_FIELD_ALPHA_L: off = n; cnt = n; break;
        case EELBM_FIELD_U_G: off = 2 * n; cnt = D * n; break;
        case EELBM_FIELD_U_L: off = (2 + D) * n; cnt = D * n; break;
        case EELBM_FIELD_P_K: off = (2 + 2 * D) * n; cnt = n; add = 1.0 / 3.0; break;
        case EELBM_FIELD_DP_K: off = (2 + 2 * D) * n; cnt = n; break;
        default: return fail(EELBM_E_PARAM, "unknown field");
    }
    const double* src = reinterpret_cast<const double*>(h->mem + h->L.macro) + off;
    hipError_t e;
    if (on_device) {
        e = launch_convert(src, dst, dst_dtype, (long long)cnt, add, 1.0, h->stream);
        if (e != hipSuccess) return hip_fail(e, "convert launch");
        return EELBM_OK;
    }
    if (dst_dtype == EELBM_DTYPE_F64 && add == 0.0) {
        e = hipMemcpyAsync(dst, src, cnt * 8, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_fail(e, "read-back");
        return EELBM_OK;
    }
    std::vector<double> tmp(cnt);
    e = hipMemcpyAsync(tmp.data(), src, cnt * 8, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "read-back");
    if (dst_dtype == EELBM_DTYPE_F64) {
        double* d = static_cast<double*>(dst);
        for (size_t i = 0; i < cnt; ++i) d[i] = tmp[i] + add;
    } else {
        float* d = static_cast<float*>(dst);
        for (size_t i = 0; i < cnt; ++i) d[i] = (float)(tmp[i] + add);
    }
    return EELBM_OK;
}

int eelbm_diag(eelbm_handle* h, eelbm_diagnostics* out) {
    if (!h || !out) return fail(EELBM_E_PARAM, "NULL argument");
    if (!h->initialized) return fail(EELBM_E_STATE, "eelbm_init_fields not called");
    double* parts = reinterpret_cast<double*>(h->mem + h->L.partials);
    double* d = reinterpret_cast<double*>(h->mem + h->L.dout);
    double* scr = reinterpret_cast<double*>(h->mem + h->L.dscr);
    hipError_t e = launch_diag_finalize(parts, (int)h->diag_blocks, scr, d, h->stream);
    if (e != hipSuccess) return hip_fail(e, "diag launch");
    double v[kNDiag];
    e = hipMemcpyAsync(v, d, sizeof(v), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "diag read-back");
    const double n = (double)h->g.n;
    std::memset(out, 0, sizeof(*out));
    out->t = h->t;
    out->a_g = v[0];
    out->a_l = v[1];
    out->alpha_g = v[2];
    out->alpha_l = v[3];
    out->deps_g = v[4];
    out->deps_l = v[5];
    for (int a = 0; a < 3; ++a) {
        out->u_g[a] = v[6 + a];
        out->u_l[a] = v[9 + a];
        out->momentum[a] = v[12 + a];
    }
    out->renorm_defect = v[15];
    out->nonfinite = (int64_t)v[16];
    (void)n;
    if (out->nonfinite > 0) return fail(EELBM_E_NONFINITE, "non-finite populations in the state");
    return EELBM_OK;
}

namespace {
struct SaveHeader {
    uint64_t magic;
    int32_t abi, lattice, storage, nx, ny, nz;
    int64_t t;
    double rho_ref, b_g, b_l, alpha_ref;
    int64_t diag_blocks;
    uint64_t pop_bytes, cf_bytes, lag_bytes, side_bytes, macro_bytes, part_bytes, noise_bytes;
    eelbm_params params;  // the run's parameters (reserved field cleared): a load must match them
};
constexpr uint64_t kMagic = 0x45454c424d434b32ull;  // "EELBMCK2"

eelbm_params canonical(const eelbm_params& p) {
    eelbm_params c;
    std::memset(&c, 0, sizeof(c));
    c = p;
    c.reserved_i = 0;
    return c;
}

void save_sizes(const eelbm_handle* h, SaveHeader* s) {
    const size_t n = (size_t)h->g.n;
    s->pop_bytes = pop_bytes(h->p, h->g);
    s->cf_bytes = cf_region_bytes(h->g);
    s->lag_bytes = lag_region_bytes(h->p, h->g);
    s->side_bytes = (size_t)2 * 2 * (2 * h->g.D + 2) * (size_t)h->g.face_n * h->g.csize;
    s->macro_bytes = (size_t)(3 + 2 * h->g.D) * n * 8;
    s->part_bytes = (size_t)h->diag_blocks * kNDiag * 8;
    s->noise_bytes = (size_t)h->g.face_n * 8;
}
}  // namespace

int eelbm_save(eelbm_handle* h, void* host_buf, size_t* bytes) {
    if (!h || !bytes) return fail(EELBM_E_PARAM, "NULL argument");
    if (!h->initialized) return fail(EELBM_E_STATE, "eelbm_init_fields not called");
    SaveHeader s{};
    save_sizes(h, &s);
    const size_t need = sizeof(s) + s.pop_bytes + s.cf_bytes + s.lag_bytes + s.side_bytes + s.macro_bytes + s.part_bytes +
                        s.noise_bytes;
    if (!host_buf) {
        *bytes = need;
        return EELBM_OK;
    }
    if (*bytes < need) return fail(EELBM_E_SIZE, "checkpoint buffer too small");
    s.magic = kMagic;
    s.abi = EELBM_ABI_VERSION;
    s.lattice = h->p.lattice;
    s.storage = h->p.storage;
    s.nx = h->p.nx;
    s.ny = h->p.ny;
    s.nz = h->p.nz;
    s.t = h->t;
    s.rho_ref = h->rho_ref;
    s.b_g = h->b_g;
    s.b_l = h->b_l;
    s.alpha_ref = h->alpha_ref;
    s.diag_blocks = h->diag_blocks;
    s.params = canonical(h->p);
    char* o = static_cast<char*>(host_buf);
    std::memcpy(o, &s, sizeof(s));
    o += sizeof(s);
    const char* m = h->mem;
    const std::pair<size_t, size_t> parts[7] = {{h->L.pop[h->cur], s.pop_bytes}, {h->L.cf[h->cur], s.cf_bytes},
                                               {h->L.lag, s.lag_bytes},         {h->L.side[h->cur], s.side_bytes},
                                               {h->L.macro, s.macro_bytes},     {h->L.partials, s.part_bytes},
                                               {h->L.noise, s.noise_bytes}};
    for (const auto& pr : parts) {
        if (pr.second == 0) continue;
        hipError_t e = hipMemcpyAsync(o, m + pr.first, pr.second, hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) return hip_fail(e, "save copy");
        o += pr.second;
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    *bytes = need;
    return EELBM_OK;
}

int eelbm_load(eelbm_handle* h, const void* host_buf, size_t bytes) {
    if (!h || !host_buf) return fail(EELBM_E_PARAM, "NULL argument");
    SaveHeader s{}, want{};
    if (bytes < sizeof(s)) return fail(EELBM_E_SIZE, "checkpoint too small");
    std::memcpy(&s, host_buf, sizeof(s));
    if (s.diag_blocks < 0 || (size_t)s.diag_blocks > max_blocks(h->p))
        return fail(EELBM_E_PARAM, "checkpoint does not match this lattice");
    const int64_t keep_blocks = h->diag_blocks;
    h->diag_blocks = s.diag_blocks;
    save_sizes(h, &want);
    h->diag_blocks = keep_blocks;
    if (s.magic != kMagic || s.abi != EELBM_ABI_VERSION || s.lattice != h->p.lattice || s.storage != h->p.storage ||
        s.nx != h->p.nx || s.ny != h->p.ny || s.nz != h->p.nz || s.pop_bytes != want.pop_bytes ||
        s.cf_bytes != want.cf_bytes || s.lag_bytes != want.lag_bytes || s.side_bytes != want.side_bytes ||
        s.macro_bytes != want.macro_bytes || s.part_bytes != want.part_bytes || s.noise_bytes != want.noise_bytes)
        return fail(EELBM_E_PARAM, "checkpoint does not match this lattice");
    const eelbm_params mine = canonical(h->p);
    if (std::memcmp(&mine, &s.params, sizeof(mine)) != 0)
        return fail(EELBM_E_PARAM, "checkpoint was saved with other physical or boundary parameters");
    const size_t need = sizeof(s) + s.pop_bytes + s.cf_bytes + s.lag_bytes + s.side_bytes + s.macro_bytes +
                        s.part_bytes + s.noise_bytes;
    if (bytes < need) return fail(EELBM_E_SIZE, "checkpoint truncated");
    // the copy holding the state at time t is always copy t mod 2
    h->cur = (int)(s.t & 1);
    const char* o = static_cast<const char*>(host_buf) + sizeof(s);
    const std::pair<size_t, size_t> parts[7] = {{h->L.pop[h->cur], s.pop_bytes}, {h->L.cf[h->cur], s.cf_bytes},
                                               {h->L.lag, s.lag_bytes},    {h->L.side[h->cur], s.side_bytes},
                                               {h->L.macro, s.macro_bytes}, {h->L.partials, s.part_bytes},
                                               {h->L.noise, s.noise_bytes}};
    for (const auto& pr : parts) {
        if (pr.second == 0) continue;
        hipError_t e = hipMemcpyAsync(h->mem + pr.first, o, pr.second, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) return hip_fail(e, "load copy");
        o += pr.second;
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    h->t = s.t;
    h->diag_blocks = s.diag_blocks;
    h->alpha_ref = s.alpha_ref;
    h->rho_ref = s.rho_ref;
    h->b_g = s.b_g;
    h->b_l = s.b_l;
    fill_kparams(h);
    ++h->gen;
    h->initialized = true;
    return EELBM_OK;
}

void eelbm_destroy(eelbm_handle* h) { delete h; }

int eelbm_map_physical(double g, double kappa_I, double g_hat, double kappa_hat, double* c_over_tau, double* c_tau,
                       double* c) {
    if (!(g > 0 && kappa_I > 0 && g_hat > 0 && kappa_hat > 0)) return fail(EELBM_E_PARAM, "inputs must be > 0");
    const double a = g / g_hat, b = kappa_hat / kappa_I;
    if (c_over_tau) *c_over_tau = a;
    if (c_tau) *c_tau = b;
    if (c) *c = std::sqrt(a * b);
    return EELBM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

struct eelbm_batch {
    std::vector<eelbm_handle*> m;
    std::vector<uint64_t> gen;  // members' generations when the batch copied their parameters
    int lattice, storage;
    int bc_mode;  // kBc* configuration of the step kernel; members agree on it or it is kBcGeneric
    char* mem;
    size_t bytes;
    hipStream_t user;     // caller's stream: advance is ordered after its work and before later work
    hipStream_t own;      // the batch's own stream (captures cannot use the legacy default stream)
    hipEvent_t ev_in, ev_out;
    size_t off_lat, off_work, off_clock;
    long long nwork;
    dim3 block;
    int graph_steps;
    hipGraphExec_t exec;
    int exec_steps;
    long long t_clock;  // time the device clock holds (members may be rebuilt at another time between advances)
    bool nt_store;      // the members' populations together exceed the last-level cache
    const int32_t* active;  // device flags per member (NULL: all advance)
    size_t off_moff, off_aoff, off_awork, off_count;
};

namespace {

long long tiles_for(const eelbm_params& p, int bx, int by) {
    return (long long)((p.nx + bx - 1) / bx) * ((p.ny + by - 1) / by) * p.nz;
}

int check_members(eelbm_handle* const* m, int32_t n, int32_t tx, int32_t ty) {
    if (!m || n < 1) return fail(EELBM_E_PARAM, "a batch needs at least one lattice");
    if (tx < 64 || ty < 1 || tx % 64 != 0 || tx * ty > 256)
        return fail(EELBM_E_PARAM, "tile_x must be a multiple of 64, tile_x * tile_y at most 256");
    for (int32_t i = 0; i < n; ++i) {
        const eelbm_handle* h = m[i];
        if (!h) return fail(EELBM_E_PARAM, "batch member is NULL");
        if (!h->initialized) return fail(EELBM_E_STATE, "batch member not initialised");
        if (h->p.lattice != m[0]->p.lattice || h->p.storage != m[0]->p.storage || h->g.channel != m[0]->g.channel)
            return fail(EELBM_E_PARAM, "batch members must share lattice, storage and boundary kind");
        if (h->p.storage == EELBM_FP32_F64 || h->p.storage == EELBM_MIXED)
            return fail(EELBM_E_PARAM, "EELBM_FP32_F64 and EELBM_MIXED lattices are not batched");
        if (h->device != m[0]->device) return fail(EELBM_E_PARAM, "batch members must live on one device");
        if (h->t != m[0]->t) return fail(EELBM_E_STATE, "batch members must be at the same time step");
        if (h->cur != (int)(h->t & 1)) return fail(EELBM_E_STATE, "internal: copy parity differs from time parity");
        for (int32_t j = 0; j < i; ++j)
            if (m[j] == h) return fail(EELBM_E_PARAM, "a lattice appears twice in the batch");
    }
    if (!tile_ok(m[0]->p, tx, ty))
        return fail(EELBM_E_PARAM, "the tile's record window exceeds 64 KiB of LDS (D3Q19: at most 64x4 or 128x2)");
    return EELBM_OK;
}

// device layout of a batch: member table | work list | clock | member
// offsets in the work list (n + 1) | active members' offsets (n) | work list
// of the active members | its length
struct BatchSizes {
    size_t lat, work, clock, moff, aoff, awork, count, total;
    long long nwork;
};
BatchSizes batch_sizes(eelbm_handle* const* m, int32_t n, int32_t tx, int32_t ty) {
    BatchSizes z{};
    for (int32_t i = 0; i < n; ++i) z.nwork += tiles_for(m[i]->p, tx, ty);
    z.lat = 0;
    z.work = align256((size_t)n * sizeof(BatchLattice));
    z.clock = z.work + align256((size_t)z.nwork * sizeof(uint2));
    z.moff = z.clock + 256;
    z.aoff = z.moff + align256((size_t)(n + 1) * sizeof(int));
    z.awork = z.aoff + align256((size_t)n * sizeof(int));
    z.count = z.awork + align256((size_t)z.nwork * sizeof(uint2));
    z.total = z.count + 256;
    return z;
}

int batch_step_launches(eelbm_batch* b, int64_t nsteps, hipStream_t s) {
    const BatchLattice* lat = reinterpret_cast<const BatchLattice*>(b->mem + b->off_lat);
    // with active flags: the compacted work list and its length on the device
    const uint2* work = reinterpret_cast<const uint2*>(b->mem + (b->active ? b->off_awork : b->off_work));
    const int* count = b->active ? reinterpret_cast<const int*>(b->mem + b->off_count) : nullptr;
    long long* clock = reinterpret_cast<long long*>(b->mem + b->off_clock);
    for (int64_t k = 0; k < nsteps; ++k) {
        hipError_t e = launch_batch_step(b->lattice, b->storage, b->bc_mode, b->nt_store, lat, work, b->nwork, clock, (int)k,
                                         k == nsteps - 1, count, b->block, s);
        if (e != hipSuccess) return hip_fail(e, "batch step launch");
    }
    hipError_t e = launch_clock_add(clock, nsteps, s);
    if (e != hipSuccess) return hip_fail(e, "batch clock launch");
    return EELBM_OK;
}

// tile_x = tile_y = 0: the autotuned tile of the largest member (by node count)
constexpr int kBatchTuneSteps = 20;
int resolve_batch_tile(eelbm_handle* const* members, int32_t n, int32_t* tile_x, int32_t* tile_y) {
    if (*tile_x != 0 || *tile_y != 0) return EELBM_OK;
    if (!members || n < 1) return fail(EELBM_E_PARAM, "a batch needs at least one lattice");
    eelbm_handle* big = nullptr;
    for (int32_t i = 0; i < n; ++i) {
        if (!members[i]) return fail(EELBM_E_PARAM, "batch member is NULL");
        if (!big || members[i]->g.n > big->g.n) big = members[i];
    }
    return eelbm_autotune(big, kBatchTuneSteps, 0, tile_x, tile_y, nullptr);
}

}  // namespace

extern "C" {

int eelbm_batch_bytes(eelbm_handle* const* members, int32_t n, int32_t tile_x, int32_t tile_y, size_t* bytes) {
    if (!bytes) return fail(EELBM_E_PARAM, "bytes is NULL");
    int rc = resolve_batch_tile(members, n, &tile_x, &tile_y);
    if (rc) return rc;
    rc = check_members(members, n, tile_x, tile_y);
    if (rc) return rc;
    *bytes = batch_sizes(members, n, tile_x, tile_y).total;
    return EELBM_OK;
}

int eelbm_batch_create(eelbm_handle* const* members, int32_t n, int32_t tile_x, int32_t tile_y, void* device_mem,
                       size_t bytes, void* hip_stream, eelbm_batch** out) {
    if (!out) return fail(EELBM_E_PARAM, "out is NULL");
    *out = nullptr;
    int rc = resolve_batch_tile(members, n, &tile_x, &tile_y);
    if (rc) return rc;
    rc = check_members(members, n, tile_x, tile_y);
    if (rc) return rc;
    const BatchSizes z = batch_sizes(members, n, tile_x, tile_y);
    if (!device_mem) return fail(EELBM_E_PARAM, "device_mem is NULL");
    if (reinterpret_cast<uintptr_t>(device_mem) & 255) return fail(EELBM_E_PARAM, "device buffer not 256-byte aligned");
    if (bytes < z.total) return fail(EELBM_E_SIZE, "device buffer smaller than eelbm_batch_bytes");
    if (z.nwork >= (1ll << 31)) return fail(EELBM_E_PARAM, "too many tiles in one batch");
    // every member takes the batch's tile shape (its own launches use it too)
    std::vector<BatchLattice> lat((size_t)n);
    size_t batch_pop = 0;
    std::vector<uint2> work;
    work.reserve((size_t)z.nwork);
    for (int32_t i = 0; i < n; ++i) {
        eelbm_handle* h = members[i];
        set_tiles(h->p, &h->g, tile_x, tile_y, h->g.xcd_remap);
        fill_kparams(h);
        lat[i].p = h->kp;
        batch_pop += pop_bytes(h->p, h->g);
        lat[i].buf[0] = buffers(h, 0, 1);
        lat[i].buf[1] = buffers(h, 1, 0);
        for (int t = 0; t < h->g.nblocks; ++t) work.push_back(make_uint2((unsigned)i, (unsigned)t));
    }
    // one step of the batch writes the populations of every member
    for (auto& l : lat) l.p.nt_store = batch_pop > kLastLevelCacheBytes;
    eelbm_batch* b = new (std::nothrow) eelbm_batch();
    if (!b) return fail(EELBM_E_PARAM, "out of host memory");
    b->nt_store = batch_pop > kLastLevelCacheBytes;
    b->m.assign(members, members + n);
    for (int32_t i = 0; i < n; ++i) b->gen.push_back(members[i]->gen);
    b->lattice = members[0]->p.lattice;
    b->storage = members[0]->p.storage;
    b->bc_mode = members[0]->g.bc_mode;
    for (int32_t i = 1; i < n; ++i)
        if (members[i]->g.bc_mode != b->bc_mode) b->bc_mode = kBcGeneric;
    b->mem = static_cast<char*>(device_mem);
    b->bytes = bytes;
    b->user = static_cast<hipStream_t>(hip_stream);
    b->off_lat = z.lat;
    b->off_work = z.work;
    b->off_clock = z.clock;
    b->off_moff = z.moff;
    b->off_aoff = z.aoff;
    b->off_awork = z.awork;
    b->off_count = z.count;
    b->nwork = z.nwork;
    b->block = dim3(tile_x, tile_y, 1);
    b->graph_steps = 0;
    b->exec = nullptr;
    b->exec_steps = 0;
    const long long t0 = members[0]->t;
    hipError_t e = hipStreamCreate(&b->own);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
    // the caller's memory may still be in use by work queued on the caller's
    // stream (an allocator that reuses a block as soon as that stream moves
    // on): the uploads below wait for it
    if (e == hipSuccess) e = hipEventRecord(b->ev_in, b->user);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->own, b->ev_in, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->mem + b->off_lat, lat.data(), lat.size() * sizeof(BatchLattice), hipMemcpyHostToDevice,
                           b->own);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->mem + b->off_work, work.data(), work.size() * sizeof(uint2), hipMemcpyHostToDevice,
                           b->own);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->mem + b->off_clock, &t0, sizeof(t0), hipMemcpyHostToDevice, b->own);
    std::vector<int> moff((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) moff[(size_t)i + 1] = moff[(size_t)i] + (int)members[i]->g.nblocks;
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->mem + b->off_moff, moff.data(), moff.size() * sizeof(int), hipMemcpyHostToDevice,
                           b->own);
    b->t_clock = t0;
    if (e == hipSuccess) e = hipStreamSynchronize(b->own);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch setup");
    }
    *out = b;
    return EELBM_OK;
}

int eelbm_batch_set_graph(eelbm_batch* b, int32_t steps_per_graph) {
    if (!b) return fail(EELBM_E_PARAM, "batch is NULL");
    if (steps_per_graph < 0 || steps_per_graph > 100000) return fail(EELBM_E_PARAM, "steps_per_graph out of range");
    b->graph_steps = steps_per_graph;
    return EELBM_OK;
}

int eelbm_batch_advance(eelbm_batch* b, int64_t nsteps) {
    if (!b) return fail(EELBM_E_PARAM, "batch is NULL");
    if (nsteps < 0) return fail(EELBM_E_PARAM, "nsteps < 0");
    if (nsteps == 0) return EELBM_OK;
    const long long t0 = b->m[0]->t;
    for (size_t i = 0; i < b->m.size(); ++i) {
        if (b->m[i]->t != t0) return fail(EELBM_E_STATE, "a batch member was advanced on its own");
        if (b->m[i]->gen != b->gen[i])
            return fail(EELBM_E_STATE,
                        "a batch member was initialised, loaded or given another launch shape after the batch was "
                        "created: create the batch again");
    }
    // order after the caller's stream
    hipError_t e = hipEventRecord(b->ev_in, b->user);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->own, b->ev_in, 0);
    if (e != hipSuccess) return hip_fail(e, "batch stream ordering");
    if (t0 != b->t_clock) {
        // the members were rebuilt at another time (eelbm_reinit_fields):
        // move the device clock there before any step
        long long* clock = reinterpret_cast<long long*>(b->mem + b->off_clock);
        e = launch_clock_add(clock, t0 - b->t_clock, b->own);
        if (e != hipSuccess) return hip_fail(e, "batch clock launch");
        b->t_clock = t0;
    }
    if (b->active) {
        // the work list of the members whose flags are set now
        e = launch_batch_compact(b->active, reinterpret_cast<const int*>(b->mem + b->off_moff), (int)b->m.size(),
                                 reinterpret_cast<int*>(b->mem + b->off_aoff),
                                 reinterpret_cast<int*>(b->mem + b->off_count),
                                 reinterpret_cast<const uint2*>(b->mem + b->off_work), b->nwork,
                                 reinterpret_cast<uint2*>(b->mem + b->off_awork), b->own);
        if (e != hipSuccess) return hip_fail(e, "batch work-list compaction");
    }
    int64_t left = nsteps;
    const int K = b->graph_steps;
    if (K > 0 && left >= K) {
        if (!b->exec || b->exec_steps != K) {
            if (b->exec) {
                (void)hipGraphExecDestroy(b->exec);
                b->exec = nullptr;
            }
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
            int rc = batch_step_launches(b, K, b->own);
            e = hipStreamEndCapture(b->own, &g);
            if (rc) return rc;
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                b->exec = nullptr;
                return hip_fail(e, "hipGraphInstantiate");
            }
            b->exec_steps = K;
        }
        for (; left >= K; left -= K) {
            e = hipGraphLaunch(b->exec, b->own);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        }
    }
    if (left > 0) {
        int rc = batch_step_launches(b, left, b->own);
        if (rc) return rc;
    }
    e = hipEventRecord(b->ev_out, b->own);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->user, b->ev_out, 0);
    if (e != hipSuccess) return hip_fail(e, "batch stream ordering");
    for (auto* h : b->m) {
        h->t += nsteps;
        h->cur = (int)(h->t & 1);
        h->diag_blocks = h->g.nblocks;
    }
    b->t_clock += nsteps;
    return EELBM_OK;
}

int eelbm_batch_set_active(eelbm_batch* b, const int32_t* active) {
    if (!b) return fail(EELBM_E_PARAM, "batch is NULL");
    if ((active == nullptr) != (b->active == nullptr) && b->exec) {
        // the captured launches read the full or the compacted work list
        (void)hipStreamSynchronize(b->own);
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    b->active = active;
    return EELBM_OK;
}

int eelbm_batch_rebuild_gated(eelbm_batch* b, int64_t t, const double* fields, const int32_t* gate) {
    if (!b) return fail(EELBM_E_PARAM, "batch is NULL");
    if (!fields || !gate) return fail(EELBM_E_PARAM, "fields or gate is NULL");
    size_t off = 0;
    for (size_t i = 0; i < b->m.size(); ++i) {
        eelbm_handle* h = b->m[i];
        const size_t n = (size_t)h->g.n;
        const int D = h->g.D;
        const double* f = fields + off;
        int rc = init_impl(h, t, f, f + n, f + (1 + D) * n, f + (1 + 2 * D) * n, nullptr, 1, true, gate + i);
        if (rc) return rc;
        off += (size_t)(2 + 2 * D) * n;
    }
    return EELBM_OK;
}

int eelbm_batch_read_fields(eelbm_batch* b, float* out) {
    if (!b) return fail(EELBM_E_PARAM, "batch is NULL");
    if (!out) return fail(EELBM_E_PARAM, "out is NULL");
    size_t off = 0;
    for (size_t i = 0; i < b->m.size(); ++i) {
        eelbm_handle* h = b->m[i];
        const size_t n = (size_t)h->g.n;
        const int D = h->g.D;
        const double* mac = reinterpret_cast<const double*>(h->mem + h->L.macro);
        // macro: alpha_g, alpha_l, u_g(D), u_l(D), dp_k -> alpha_g, u_g(D), u_l(D), dp_k
        hipError_t e = launch_convert(mac, out + off, EELBM_DTYPE_F32, (long long)n, 0.0, 1.0, h->stream);
        if (e == hipSuccess)
            e = launch_convert(mac + 2 * n, out + off + n, EELBM_DTYPE_F32, (long long)(2 * D * n), 0.0, 1.0,
                               h->stream);
        if (e == hipSuccess)
            e = launch_convert(mac + (2 + 2 * D) * n, out + off + (1 + 2 * D) * n, EELBM_DTYPE_F32, (long long)n, 0.0,
                               1.0, h->stream);
        if (e != hipSuccess) return hip_fail(e, "convert launch");
        off += (size_t)(2 + 2 * D) * n;
    }
    return EELBM_OK;
}

void eelbm_batch_destroy(eelbm_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    (void)hipStreamSynchronize(b->own);
    (void)hipEventDestroy(b->ev_in);
    (void)hipEventDestroy(b->ev_out);
    (void)hipStreamDestroy(b->own);
    delete b;
}

// ---------------------------------------------------------------- autotuner

int eelbm_autotune(eelbm_handle* h, int32_t steps, int32_t force, int32_t* tile_x, int32_t* tile_y,
                   int32_t* xcd_remap) {
    if (!h) return fail(EELBM_E_PARAM, "handle is NULL");
    if (!h->initialized) return fail(EELBM_E_STATE, "eelbm_init_fields not called");
    if (steps < 1) return fail(EELBM_E_PARAM, "steps < 1");
    // key: lattice, storage, boundary kind, size class (floor log2 of the node count)
    int cls = 0;
    for (long long v = h->g.n; v > 1; v >>= 1) ++cls;
    const long long key = (((long long)h->p.lattice * 8 + h->p.storage) * 3 + h->g.bc_mode) * 64 + cls;
    static std::mutex mu;
    static std::map<long long, std::array<int, 3>> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end() && !force) {
            set_tiles(h->p, &h->g, it->second[0], it->second[1], it->second[2]);
            fill_kparams(h);
            ++h->gen;
            if (tile_x) *tile_x = it->second[0];
            if (tile_y) *tile_y = it->second[1];
            if (xcd_remap) *xcd_remap = it->second[2];
            return EELBM_OK;
        }
    }
    // trials run on the handle's own state, which is saved to host memory
    // first and restored after every trial (bit for bit)
    size_t need = 0;
    int rc = eelbm_save(h, nullptr, &need);
    if (rc) return rc;
    std::vector<char> snap(need);
    rc = eelbm_save(h, snap.data(), &need);
    if (rc) return rc;
    const int bx_max = std::min(256, ((h->p.nx + 63) / 64) * 64);
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    float best = 1e30f;
    std::array<int, 3> pick = {(int)h->g.block.x, (int)h->g.block.y, h->g.xcd_remap};
    for (int bx = 64; bx <= bx_max; bx += 64) {
        for (int by = 1; bx * by <= 256; by *= 2) {
            if (by > h->p.ny) break;
            if (!tile_ok(h->p, bx, by)) continue;
            for (int xcd = 0; xcd < 2; ++xcd) {
                set_tiles(h->p, &h->g, bx, by, xcd);
                fill_kparams(h);
                rc = eelbm_advance(h, 2);
                if (!rc) e = hipEventRecord(e0, h->stream);
                if (!rc && e == hipSuccess) rc = eelbm_advance(h, steps);
                if (!rc && e == hipSuccess) e = hipEventRecord(e1, h->stream);
                if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (!rc && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                const int rc2 = eelbm_load(h, snap.data(), snap.size());
                if (rc || rc2 || e != hipSuccess) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    if (e != hipSuccess) return hip_fail(e, "autotune timing");
                    return rc ? rc : rc2;
                }
                if (ms < best) {
                    best = ms;
                    pick = {bx, by, xcd};
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_tiles(h->p, &h->g, pick[0], pick[1], pick[2]);
    fill_kparams(h);
    ++h->gen;
    {
        std::lock_guard<std::mutex> lk(mu);
        cache[key] = pick;
    }
    if (tile_x) *tile_x = pick[0];
    if (tile_y) *tile_y = pick[1];
    if (xcd_remap) *xcd_remap = pick[2];
    return EELBM_OK;
}

}  // extern "C"
