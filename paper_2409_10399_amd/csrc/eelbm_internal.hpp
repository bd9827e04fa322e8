// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace eelbm {

constexpr int kNDiag = 18;  // per-node diagnostic sums (see k_step)
// diagnostics finalize: at most kDiagGroups workgroups of the first pass, each
// over at least kDiagRowsPerGroup block partials (scratch: kDiagGroups rows)
constexpr int kDiagGroups = 256;
constexpr int kDiagRowsPerGroup = 1024;

// Scalars of the scheme, in lattice units, fixed for a run.
struct KParams {
    int nx, ny, nz;
    long long n;        // nodes
    int ntx, nty;       // tiles per plane along x and y (tile = blockDim.x * blockDim.y nodes)
    int nxb;            // 64-node x-blocks per row of the population layout
    long long plane;    // population elements of one z-plane (ny * nxb * 4Q * 64)
    int xcd_remap;      // map contiguous tile runs to one XCD
    int per[3];         // axis periodic?
    int wall_lo[3], wall_hi[3];
    int flow_axis;      // axis carrying the inlet/outlet faces, -1 if none
    int face_lo, face_hi;  // EELBM_BC_* of the two flow-axis faces
    long long face_n;   // nodes of one flow-axis face
    int up;             // buoyancy axis
    int cgw;            // Clift-Grace-Weber drag?
    int use_lag;        // n_gamma > 1: lag fields are stored
    int renorm;         // Spalding renormalisation on?
    int sigma_grad;     // sigma . grad(alpha) / alpha term on?
    int nt_store;       // the launches store populations with the nontemporal hint (one set larger than the last-level cache)
    double R, invR, rho_g, rho_l;
    double omega_g, omega_l, psi_g, psi_l, omega_ag, omega_al;
    double K_I, kappa_I, K_W;
    double b_g, b_l;    // buoyancy accelerations along up
    double gamma, alpha_min;
    double alpha_ref;   // reference of the f_alpha deviations (mean initial alpha_g)
    long long n_gamma;  // lag refresh period
    double a_in_max, a_in_min, ug_in_max, ug_in_min, ul_in_max, ul_in_min, n_ramp;  // inlet ramp, Eq. (153)
    float h16_up[2], h16_down[2];  // FP16 storage scales: [0] f_g, f_ag, f_al; [1] moving f_l
};

// Device pointers of one launch (ping-pong halves already selected).
struct KBuffers {
    const void* pop_in;   // [4][Q][n] storage type: deviations of f_g, f_l, f_ag, f_al
    void* pop_out;
    const void* cf_in;    // [n] records of 8 compute-type values: alpha_g, u_g(D), u_l(D),
    void* cf_out;         //     Lambda' (D2Q9), eps_g - 1
    const void* al_in;    // [n] alpha_l (read and written only without renormalisation)
    void* al_out;
    void* lag;            // [n] records of 2: S''_g, S''_l
    void* lag_lam;        // [n] Lambda' (D3Q19 only)
    const void* side_in;  // [2 faces][2 layers][NV][face_n] compute type
    void* side_out;
    const double* noise;  // [face_n] inlet gas-fraction factor
    const double* stage;  // init inputs [2 + 2D][n]: alpha_g, u_g(D), u_l(D), dp_k
    double* macro;        // outputs [3 + 2D][n]: alpha_g, alpha_l, u_g(D), u_l(D), dp_k
    double* partials;     // [blocks][kNDiag]
};

// Per-launch control.
struct KCtl {
    long long t;          // time of the collision performed by this launch
    int refresh;          // lag refresh: t mod n_gamma == 0 (Eqs. (133), (137))
    int write_macro;
    int write_diag;
    const int* gate;      // initialisation launches: skipped when *gate == 0 (device flag; NULL: run)
};

// One lattice of a batch: its parameters and its buffers for both parities
// (buf[0]: read copy 0 / write copy 1, the step from even to odd time).
struct BatchLattice {
    KParams p;
    KBuffers buf[2];
};

// boundary configuration a step is compiled for: every axis periodic; any
// mix of periodic, wall and inlet/outlet faces read from KParams; the
// standard column (inlet at the low and outlet at the high face of the last
// axis, walls on every face of the other axes)
constexpr int kBcPeriodic = 0;
constexpr int kBcGeneric = 1;
constexpr int kBcColumn = 2;

// storage: 0 FP64, 1 FP32, 2 FP16, 3 BF16; lattice: 2 D2Q9, 3 D3Q19; bc: kBc*
hipError_t launch_step(int lattice, int storage, int bc, bool init, const KParams& p,
                       const KBuffers& b, const KCtl& c, dim3 grid, dim3 block, hipStream_t s);
// one step of every lattice of a batch: grid = work items (lattice, tile)
hipError_t launch_batch_step(int lattice, int storage, int bc, bool nts, const BatchLattice* lat, const uint2* work,
                             long long nwork, const long long* clock, int k, int write_last, const int* count,
                             dim3 block, hipStream_t s);
hipError_t launch_batch_compact(const int* active, const int* moff, int n, int* aoff, int* count, const uint2* work,
                                long long nwork, uint2* awork, hipStream_t s);
hipError_t launch_clock_add(long long* clock, long long add, hipStream_t s);
hipError_t launch_sum(const double* x, long long n, double* partials, int nblocks, double* out,
                      hipStream_t s);
hipError_t launch_diag_finalize(const double* partials, int nblocks, double* scratch, double* out,
                                hipStream_t s);
// sets the message returned by eelbm_last_error and returns code
int set_error(int code, const char* msg);

hipError_t launch_convert(const double* src, void* dst, int dst_dtype, long long n, double add,
                          double scale, hipStream_t s);

}  // namespace eelbm
