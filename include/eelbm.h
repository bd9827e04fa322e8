/*
 * eelbm.h -- C ABI of the MI355X (gfx950) implementation of the six coupled
 * lattice Boltzmann schemes of Piredda & Asinari, "Lattice Boltzmann framework
 * for multiphase flows by Eulerian-Eulerian Navier-Stokes equations"
 * (arXiv:2409.10399).
 *
 * One time step updates, on one D2Q9 or D3Q19 lattice, the two artificially
 * compressible momentum schemes f_g, f_l (Sec. 2.1.1, Eqs. (34)-(42)), the two
 * volume-fraction schemes f_ag, f_al (Sec. 2.2, Eqs. (71)-(94)) and the two
 * continuity-source schemes f_bg, f_bl (Sec. 2.3, Eqs. (95)-(107)), with the
 * large-density-ratio stabilisers of Sec. 3.2 (Eqs. (128)-(133)), the
 * Clift-Grace-Weber drag of Sec. 3.3 (Eqs. (135)-(137)) and the boundary rules
 * of Sec. 3.5 (Tables 1-2, Eqs. (159)-(164)).
 *
 * The calls follow the paper's statement of the problem (Sec. 1: unknowns
 * alpha_g, p, u_g, u_l; Sec. 2.1: phase densities and the density ratio R):
 * create a lattice from the phase densities, relaxation rates, drag and
 * boundary parameters; set the initial fields; advance N steps; read the
 * volume fractions, phase velocities and kinematic pressure.
 *
 * Conventions
 *  - All quantities are in lattice units (the paper's hat quantities).
 *  - Fields are structure-of-arrays in C order with x fastest: a scalar field
 *    is [nz][ny][nx] (nz = 1 in 2D), a vector field is [D][nz][ny][nx] with
 *    component order (x, y, z).
 *  - Device memory for the state is owned by the caller (eelbm_state_bytes,
 *    then eelbm_create binds it); the handle never frees it.  Host arrays
 *    passed in are copied before the call returns and stay caller-owned.
 *  - Work is enqueued on the caller's HIP stream given at create time.
 *    eelbm_advance is asynchronous; eelbm_read to host, eelbm_diag and
 *    eelbm_save synchronise that stream.
 *  - Every call returns 0 on success or a negative EELBM_E_* code; no C++
 *    exception crosses the ABI.  eelbm_last_error() gives a thread-local
 *    message for the last failure.
 *  - Calls on one handle must not overlap (one host thread at a time).
 */
#ifndef EELBM_H
#define EELBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EELBM_ABI_VERSION 1

/* return codes */
#define EELBM_OK 0
#define EELBM_E_PARAM (-1)     /* invalid parameter value or combination */
#define EELBM_E_SIZE (-2)      /* buffer too small / size mismatch */
#define EELBM_E_HIP (-3)       /* a HIP runtime call or kernel launch failed */
#define EELBM_E_NONFINITE (-4) /* diagnostics found NaN or Inf in the state */
#define EELBM_E_STATE (-5)     /* call out of order (e.g. advance before init) */

/* lattice */
#define EELBM_D2Q9 2
#define EELBM_D3Q19 3

/* population storage: populations are stored as deviations from the rest
 * equilibrium w_q (w_q * 0 for f_ag); collision arithmetic is FP64 for FP64
 * storage and FP32 otherwise */
#define EELBM_FP64 0
#define EELBM_FP32 1
#define EELBM_FP16 2
#define EELBM_BF16 3
/* FP32 populations with the FP64 step's arithmetic and FP64 records: the
 * rounding of FP32 storage alone (single lattices; batches refuse it) */
#define EELBM_FP32_F64 4
/* Mixed storage: f_g in FP32, f_l, f_alpha_g, f_alpha_l in FP16 (scaled
 * residuals as in FP16 storage), 12 bytes per direction instead of 16; FP32
 * arithmetic (single lattices; batches refuse it) */
#define EELBM_MIXED 5

/* boundary type of one face (Sec. 3.5) */
#define EELBM_BC_PERIODIC 0
#define EELBM_BC_WALL 1   /* no-slip wall: bounce-back, zero flux, EQ(S)(1,0) for f_b */
#define EELBM_BC_INLET 2  /* Table 1 */
#define EELBM_BC_OUTLET 3 /* Table 2 */

/* drag model: constant K_I, or Clift-Grace-Weber K_I = kappa_I Lambda (Eq. (135)) */
#define EELBM_DRAG_CONST 0
#define EELBM_DRAG_CGW 1

/* buoyancy reference density (b_phi = (rho_ref/rho_phi - 1) g_hat along up) */
#define EELBM_RHOREF_LIQUID 0       /* rho_ref = rho_l: the kinematic pressure of Eqs. (108)-(110) */
#define EELBM_RHOREF_MIXTURE_MEAN 1 /* mean mixture density of the initial state (periodic boxes) */
#define EELBM_RHOREF_EXPLICIT 2     /* rho_ref given in the params */

/* flags */
#define EELBM_FLAG_NO_RENORM 1u     /* skip the Spalding renormalisation of Eq. (93) */
#define EELBM_FLAG_NO_SIGMA_GRAD 2u /* drop the sigma . grad(alpha) / alpha term of G (Eq. (92)) */

typedef struct eelbm_params {
    int32_t abi_version;   /* must be EELBM_ABI_VERSION */
    int32_t lattice;       /* EELBM_D2Q9 or EELBM_D3Q19 */
    int32_t storage;       /* EELBM_FP64 / FP32 / FP16 / BF16 / FP32_F64 / MIXED */
    int32_t nx, ny, nz;    /* nz = 1 for D2Q9 */
    int32_t bc[6];         /* faces x-, x+, y-, y+, z-, z+; periodic faces come in pairs */
    int32_t up_axis;       /* 0, 1, 2: direction of +buoyancy (and of the inlet flow) */
    int32_t drag_model;    /* EELBM_DRAG_* */
    int32_t rho_ref_mode;  /* EELBM_RHOREF_* */
    int32_t n_gamma;       /* lag period of Eqs. (133), (137); >= 1 */
    uint32_t flags;        /* EELBM_FLAG_* */
    int32_t reserved_i;
    double rho_g, rho_l;   /* phase densities; R = rho_l / rho_g */
    double omega_g, omega_l;   /* BGK relaxation of f_g, f_l: nu = c_s^2 (1/omega - 1/2), Eq. (65) */
    double psi_g, psi_l;       /* forcing-operator parameter, Eq. (66) */
    double omega_ag, omega_al; /* relaxation of f_ag, f_al: chi = c_s^2 (1/omega - 1/2), Eq. (88) */
    double K_I;            /* constant drag coefficient (EELBM_DRAG_CONST), Eq. (6) */
    double kappa_I;        /* Clift-Grace-Weber factor kappa_I (EELBM_DRAG_CGW) */
    double K_W;            /* liquid wall-friction coefficient, Eq. (119) (0: off) */
    double g_hat;          /* gravity magnitude */
    double rho_ref;        /* used with EELBM_RHOREF_EXPLICIT */
    double gamma;          /* dashpot constant, Eqs. (128), (131) */
    double alpha_min;      /* floor of alpha in 1/alpha factors (> 0) */
    /* inlet ramp y(t) = (max - min) tanh(t / n_ramp) + min, Eq. (153); n_ramp <= 0: max */
    double alpha_in_max, alpha_in_min;
    double ug_in_max, ug_in_min;
    double ul_in_max, ul_in_min;
    double n_ramp;
} eelbm_params;

typedef struct eelbm_handle eelbm_handle;

/* field ids for eelbm_read */
#define EELBM_FIELD_ALPHA_G 0 /* renormalised gas volume fraction (Eq. (93)), scalar */
#define EELBM_FIELD_ALPHA_L 1 /* 1 - alpha_g, scalar */
#define EELBM_FIELD_U_G 2     /* gas velocity, Eq. (41), vector */
#define EELBM_FIELD_U_L 3     /* liquid velocity, vector */
#define EELBM_FIELD_P_K 4     /* kinematic pressure p_k = c_s^2 eps_g (Eq. (111)), scalar */
#define EELBM_FIELD_DP_K 5    /* p_k - c_s^2, scalar */

/* dtype of eelbm_read destinations */
#define EELBM_DTYPE_F64 0
#define EELBM_DTYPE_F32 1

/* domain sums at the current time, accumulated in FP64 on the GPU */
typedef struct eelbm_diagnostics {
    int64_t t;               /* time step of the sums */
    int64_t nonfinite;       /* count of NaN/Inf populations read this step */
    double a_g, a_l;         /* sum of raw zeroth moments of f_ag, f_al (Eq. (73)) */
    double alpha_g, alpha_l; /* sum of renormalised volume fractions */
    double deps_g, deps_l;   /* sum of (eps - 1) of f_g, f_l (Eq. (40)) */
    double u_g[3], u_l[3];   /* sums of phase velocities */
    double momentum[3];      /* sum of rho_g alpha_g u_g + rho_l alpha_l u_l */
    double renorm_defect;    /* sum of (alpha_g - a_g) */
} eelbm_diagnostics;

/* Version of this ABI (EELBM_ABI_VERSION) and sizeof(eelbm_params), so that
 * a binding can check its mirror of the struct. */
int32_t eelbm_abi_version(void);
size_t eelbm_params_size(void);

/* Device bytes the state needs for *p (two population copies, imposed-velocity
 * fields, lag fields, boundary side buffers, output fields, staging and
 * diagnostics).  Returns EELBM_E_PARAM for invalid parameters. */
int eelbm_state_bytes(const eelbm_params* p, size_t* bytes);

/* Bind caller-owned device memory (at least eelbm_state_bytes bytes, 256-byte
 * aligned) and a caller-owned hipStream_t (NULL: the null stream).  *p is
 * copied.  The device current at the call is the one the handle uses. */
int eelbm_create(const eelbm_params* p, void* device_mem, size_t bytes, void* hip_stream,
                 eelbm_handle** out);

/* Initial macroscopic fields at t = 0.  f_g, f_l, f_ag, f_al start at the
 * local equilibria of these fields (eps_g = 1 + dp_k / c_s^2, eps_l = 1);
 * f_bg, f_bl start as if streamed from the equilibria f^eq(1, c_phi) of the
 * initial imposed velocities of Eq. (97).  alpha_g and dp_k (= p_k - c_s^2) are scalar fields, u_g and
 * u_l vector fields, all FP64.  inlet_noise is the factor multiplying the
 * inlet gas fraction per inlet-face node ([face rows][face cols], face axis
 * removed), or NULL for 1.  on_device = 1: all pointers are device pointers.
 * u_g, u_l, dp_k may be NULL (zero). */
int eelbm_init_fields(eelbm_handle* h, const double* alpha_g, const double* u_g, const double* u_l,
                      const double* dp_k, const double* inlet_noise, int on_device);

/* Rebuild the state at time t from macroscopic fields (the layout of
 * eelbm_init_fields): populations at the local equilibria of the fields as at
 * initialisation, the inlet ramp continuing from t, the inlet noise, the
 * buoyancy reference and the reference gas fraction of the f_alpha
 * deviations kept (nothing is read back: with on_device = 1 the call does not
 * wait for the device).  The lagged S''_g, S''_l and Lambda' of Sec. 3.2 and
 * Eq. (137) are taken afresh from the rebuilt state at t, as at t = 0: the
 * fields carry no lagged values, and the lag of the previous run belongs to
 * another state.  For restarting the
 * scheme from fields predicted elsewhere (the surrogate's re-anchoring); a
 * batch holding the lattice follows the new time at its next advance.
 * EELBM_E_STATE before eelbm_init_fields. */
int eelbm_reinit_fields(eelbm_handle* h, int64_t t, const double* alpha_g, const double* u_g, const double* u_l,
                        const double* dp_k, int on_device);

/* eelbm_reinit_fields from device fields (all four given), carried out only
 * if the device flag *gate (an int32 in device memory) is nonzero when the
 * rebuild runs on the device; with *gate == 0 the state is left as it was.
 * The host side (time, copy parity) is set to t either way, so a caller
 * gates only lattices already at t or lattices whose state it will not use
 * before another rebuild.  For rollouts that decide on the device which
 * lattices to rebuild, without waiting for the device. */
int eelbm_reinit_fields_gated(eelbm_handle* h, int64_t t, const double* alpha_g, const double* u_g,
                              const double* u_l, const double* dp_k, const int32_t* gate);

/* Advance nsteps time steps (asynchronous on the bound stream).  The last
 * step also writes the output fields and the diagnostic partial sums. */
int eelbm_advance(eelbm_handle* h, int64_t nsteps);

/* Copy a field at the current time into dst (dtype EELBM_DTYPE_*; host or
 * device pointer).  Vector fields take D * nodes elements. */
int eelbm_read(eelbm_handle* h, int32_t field, void* dst, int32_t dst_dtype, int on_device);

/* Domain sums at the current time (synchronises the stream).  Returns
 * EELBM_E_NONFINITE (and fills *out) if a non-finite population was seen. */
int eelbm_diag(eelbm_handle* h, eelbm_diagnostics* out);

/* Current time step (number of steps since eelbm_init_fields). */
int64_t eelbm_time(const eelbm_handle* h);

/* Launch shape of the step kernel (for tuning; results do not depend on it):
 * one workgroup per tile of tile_x * tile_y nodes of an (x, y) plane, tile_x
 * a multiple of 64 (a wavefront is one 64-node x-block of the population
 * layout) and tile_x * tile_y at most 256; xcd_remap = 1 hands each of the 8
 * XCDs one contiguous run of tiles.  EELBM_E_PARAM otherwise.  The diagnostics of the last
 * step refer to the shape they were produced with, so call this before
 * eelbm_advance. */
int eelbm_set_launch(eelbm_handle* h, int32_t tile_x, int32_t tile_y, int32_t xcd_remap);
int eelbm_get_launch(const eelbm_handle* h, int32_t* tile_x, int32_t* tile_y, int32_t* xcd_remap);

/* Checkpoint: bytes needed for a save (eelbm_save with host_buf = NULL sets
 * *bytes), save to a caller host buffer, load into a handle created with the
 * same parameters.  A loaded run continues bit-for-bit like the saved one.
 * The checkpoint carries the saving handle's eelbm_params; eelbm_load returns
 * EELBM_E_PARAM (state unchanged) when any of them differs from the loading
 * handle's (geometry, storage, densities, relaxation rates, drag, gravity,
 * stabilisers, boundary types or inlet ramp). */
int eelbm_save(eelbm_handle* h, void* host_buf, size_t* bytes);
int eelbm_load(eelbm_handle* h, const void* host_buf, size_t bytes);

/* Release the handle (not the caller's device memory or stream). */
void eelbm_destroy(eelbm_handle* h);

/* Thread-local message of the last failing call on this thread. */
const char* eelbm_last_error(void);

/* Similarity mapping of Sec. 3.3: from the physical gravity g, drag factor
 * kappa_I = 3 C_d / (4 d) and their lattice counterparts g_hat, kappa_hat,
 * c/tau = g / g_hat (Eq. (138)), c tau = kappa_hat / kappa_I (Eq. (139)),
 * c = sqrt((c/tau)(c tau)) (Eq. (140)); velocities convert as u_hat = u / c. */
int eelbm_map_physical(double g, double kappa_I, double g_hat, double kappa_hat, double* c_over_tau,
                       double* c_tau, double* c);

/* ----------------------------------------------------------------- batches
 * Many independent lattices (each with its own sizes and parameters, e.g. a
 * sweep of density ratio, bubble diameter and inlet gas fraction) advanced
 * together: one launch per time step covers every tile of every member (a
 * work list of (member, tile) pairs), and eelbm_batch_set_graph captures runs
 * of steps into a HIP graph that is replayed.  Members are handles created and
 * initialised as usual (same lattice, storage type, boundary kind and device;
 * all at the same time step); the batch does not own them.  Results equal
 * those of advancing every member on its own, bit for bit. */
typedef struct eelbm_batch eelbm_batch;

/* Device bytes of the batch's work area (member table, work list, clock) for
 * the tile shape tile_x * tile_y (tile_x a multiple of 64, at most 256 nodes).
 * tile_x = tile_y = 0 takes the tile eelbm_autotune picks for the largest
 * member (timed on that member alone, its state restored bit for bit; the
 * choice is cached per lattice, storage, boundary kind and size class, so
 * eelbm_batch_bytes and eelbm_batch_create given 0, 0 agree). */
int eelbm_batch_bytes(eelbm_handle* const* members, int32_t n, int32_t tile_x, int32_t tile_y, size_t* bytes);

/* Bind caller-owned device memory (eelbm_batch_bytes, 256-byte aligned) and
 * the caller's stream (NULL: the null stream).  Every member takes the tile
 * shape (its own eelbm_advance uses it too).  The batch runs on a stream of
 * its own, ordered after the caller's stream at each eelbm_batch_advance and
 * before the caller's later work.  Errors: EELBM_E_PARAM (mixed members, bad
 * shape, too many tiles), EELBM_E_STATE (member not initialised, times differ). */
int eelbm_batch_create(eelbm_handle* const* members, int32_t n, int32_t tile_x, int32_t tile_y, void* device_mem,
                       size_t bytes, void* hip_stream, eelbm_batch** out);

/* steps_per_graph = 0: one launch per step; > 0: runs of that many steps are
 * captured once into a HIP graph and replayed (the remainder of an advance is
 * launched directly).  Every step reads its time from a device clock, so a
 * replay is valid at any time. */
int eelbm_batch_set_graph(eelbm_batch* b, int32_t steps_per_graph);

/* Device flags, one int32 per member in member order (device memory the
 * caller keeps alive), read on the device at the start of every
 * eelbm_batch_advance: a member whose flag is 0 is not advanced by it.  Its
 * populations are left untouched while its time moves with the batch, so
 * its state is not valid until it is rebuilt (eelbm_reinit_fields,
 * eelbm_reinit_fields_gated): reads and diagnostics of it return stale
 * values.  The tiles of the active members are gathered into a work list of
 * their own on the device (so they spread over the whole GPU whichever
 * members are left out); flags may change on the device between advances,
 * also under graph replay.  NULL: every member advances.  For advancing only
 * the members a device-side test selected, without waiting for the device. */
int eelbm_batch_set_active(eelbm_batch* b, const int32_t* active);

/* eelbm_reinit_fields_gated for every member at time t, member i gated by
 * gate[i] (device int32 flags).  fields: device FP64, the members one after
 * the other, each [2 + 2D][n]: alpha_g, u_g (D planes), u_l (D planes), dp_k.
 * Asynchronous (no wait for the device). */
int eelbm_batch_rebuild_gated(eelbm_batch* b, int64_t t, const double* fields, const int32_t* gate);

/* The output fields of every member (as eelbm_read after the last advance),
 * FP32, into device memory laid out like the fields of
 * eelbm_batch_rebuild_gated.  Asynchronous. */
int eelbm_batch_read_fields(eelbm_batch* b, float* out);

/* Advance every member by nsteps (asynchronous).  The last step of the
 * advance (and of every replayed graph) writes the output fields and
 * diagnostics of every member, so eelbm_read / eelbm_diag on a member work as
 * after eelbm_advance.  EELBM_E_STATE if a member was advanced on its own,
 * or was initialised (eelbm_init_fields), loaded, autotuned or given another
 * launch shape after the batch copied its parameters (eelbm_reinit_fields
 * keeps them and is followed). */
int eelbm_batch_advance(eelbm_batch* b, int64_t nsteps);

/* Release the batch (not the members or the caller's memory). */
void eelbm_batch_destroy(eelbm_batch* b);

/* ---------------------------------------------------------------- autotuner
 * Choose the launch shape (tile_x, tile_y, xcd_remap) of a handle by timing
 * every allowed shape for `steps` steps on the handle's own state, which is
 * saved to host memory first and restored after every trial, so the state is
 * unchanged.  The choice is cached per (lattice, storage, boundary kind, size
 * class = floor(log2 nodes)) for the process; a later call for the same class
 * applies the cached shape without timing unless force != 0.  The chosen shape
 * is applied to the handle and returned through the non-NULL pointers. */
int eelbm_autotune(eelbm_handle* h, int32_t steps, int32_t force, int32_t* tile_x, int32_t* tile_y,
                   int32_t* xcd_remap);

/* --------------------------------------------------- learned surrogate
 * Kernels of a convolutional neural operator (U-Net of 3x3 convolutions)
 * that maps the macroscopic fields of a lattice to their change over a
 * fixed number of steps; a caller (the Python surrogate module) chains them
 * into forward and backward passes.  Not part of the paper: the surrogate is
 * judged against the step above.
 *
 * All pointers are device pointers, tensors NHWC FP32 (B images, H x W
 * pixels, C channels, C a multiple of 16), launches are asynchronous on
 * `stream` (a hipStream_t, NULL: the null stream).  Returns EELBM_OK,
 * EELBM_E_PARAM for NULL pointers or unsupported shapes (the message is not
 * set), EELBM_E_HIP if the launch failed.
 *
 * Convolution weights: FP32 master W[tap][ci][co] (tap = 3 (dy + 1) + dx + 1),
 * and two BF16 copies made by eelbm_cno_pack_weights: Wf[co][tap][ci] for the
 * forward pass and Wd[ci][8 - tap][co] (taps reversed) for the input
 * gradient, which is then a forward convolution of dout with Wd.  The
 * products run on the matrix cores in BF16 with FP32 accumulation. */

/* out = act(conv3x3(in; Wf) + bias), zero padding; act = leaky-ReLU with
 * `slope` if act != 0; bias may be NULL.  The weight copy (9 * Cin * Cout)
 * and the input and output tensors must each hold fewer than 2^31 values
 * (EELBM_E_PARAM otherwise). */
int eelbm_cno_conv_fwd(const float* in, int32_t B, int32_t H, int32_t W, int32_t Cin, const uint16_t* wf,
                       const float* bias, int32_t Cout, float* out, int32_t act, float slope, void* stream);
/* The same convolution of the channel concatenation [src0 | src1] (C0 + C1
 * input channels; src1 may be NULL with C1 = 0), src0 read with nearest 2x
 * upsampling from a (B, H/2, W/2, C0) image when up0 != 0: the decoder's
 * upsampling and skip concatenation fused into the convolution's input (no
 * intermediate tensors).  H and W must be even when up0 != 0. */
int eelbm_cno_conv_fwd_cat(const float* src0, int32_t C0, int32_t up0, const float* src1, int32_t C1, int32_t B,
                           int32_t H, int32_t W, const uint16_t* wf, const float* bias, int32_t Cout, float* out,
                           int32_t act, float slope, void* stream);
/* eelbm_cno_conv_fwd_cat with the activations of either side stored as BF16
 * (uint16 bit patterns, round to nearest even) when in_bf16 / out_bf16 != 0,
 * else FP32: src0 and src1 share the input type.  A BF16 output is the value
 * the FP32 output would give rounded to BF16, i.e. exactly what the next
 * convolution would have used; BF16 activations halve the traffic of
 * inference passes. */
int eelbm_cno_conv_fwd_cat_dt(const void* src0, int32_t C0, int32_t up0, const void* src1, int32_t C1, int32_t B,
                              int32_t H, int32_t W, const uint16_t* wf, const float* bias, int32_t Cout, void* out,
                              int32_t act, float slope, int32_t in_bf16, int32_t out_bf16, void* stream);
/* Tile of the forward and input-gradient convolutions, process-wide: mt
 * M-tiles of 16 pixels per wavefront (1, 2 or 4) x nt N-tiles of 16 output
 * channels per workgroup (1..4); (0, 0) restores the automatic choice (two
 * M-tiles once W >= 64, else one; two N-tiles if they divide Cout / 16, else
 * three, else one).  For tests and tuning.  A set tile applies to every later call; a
 * call whose Cout / 16 nt does not divide then returns EELBM_E_PARAM.
 * EELBM_E_PARAM for other values. */
int eelbm_cno_conv_set_tile(int32_t mt, int32_t nt);
/* din = gradient of the convolution wrt its input, given dout (the gradient
 * wrt the pre-activation output); the size limits of eelbm_cno_conv_fwd apply
 * with the roles of Cin and Cout exchanged. */
int eelbm_cno_conv_bwd_data(const float* dout, int32_t B, int32_t H, int32_t W, int32_t Cout, const uint16_t* wd,
                            int32_t Cin, float* din, void* stream);
/* dw[tap][ci][co] += sum over pixels of in(shifted) * dout; dbias[co] += sum
 * of dout (dbias may be NULL).  Accumulates: zero them first (eelbm_cno_fill).
 * Deterministic: per-chunk partial sums are added in chunk order (no
 * atomics), in a partial-sum workspace the library allocates per device on
 * first use and keeps (grown when a larger layer needs it; calls that
 * overlap on one device from different streams race on it).
 * Cout <= 256; B * H * W below 2^31 - 4096 pixels (EELBM_E_PARAM otherwise). */
int eelbm_cno_conv_bwd_weight(const float* in, const float* dout, int32_t B, int32_t H, int32_t W, int32_t Cin,
                              int32_t Cout, float* dw, float* dbias, void* stream);
/* Gas-volume defect of a surrogate jump f0 -> f1 of N channels, the test
 * that decides whether a predicted jump is kept or redone on the LBM.
 * f0, f1: (N, 6, ny, nx) FP32 field planes per channel (alpha_g, u_g,x,
 * u_g,y, u_l,x, u_l,y, dp_k), rows 0 = inlet .. ny - 1 = outlet; chi: N
 * FP32 diffusivities c_s^2 (1/omega_alpha - 1/2) of the volume-fraction
 * schemes (Sec. 2.2); defect: N FP64
 * results.  Net inflow per step = flux through the inlet row - flux through
 * the outlet row, each sum over x of alpha_g u_g,y - chi d(alpha_g)/dy (one-
 * sided difference between the end row and its neighbour); defect =
 * |V(f1) - V(f0) - jump (in(f0) + in(f1)) / 2| / |V(f0)|, V = sum of alpha_g.
 * FP64 sums in a fixed order.  ny >= 3 and f0, f1 16-byte aligned;
 * EELBM_E_PARAM otherwise. */
int eelbm_cno_volume_defect(const float* f0, const float* f1, int32_t N, int32_t ny, int32_t nx, int32_t jump,
                            const float* chi, double* defect, void* stream);
/* The re-anchoring decision of a surrogate rollout jump for N lattices, on
 * the device (one thread block, no host wait): mask[i] = 1 if defect[i]
 * exceeds defect_max or is not finite, or if force != 0; rebuild[i] =
 * mask[i] && !valid[i] (the lattice's LBM state is not at the current time
 * and must be rebuilt from the fields before it is advanced); then valid[i]
 * = mask[i] and *count += the number of masked lattices.  All arrays are
 * device memory: defect N doubles, valid, mask, rebuild N int32, count one
 * int64. */
int eelbm_cno_reanchor_policy(const double* defect, int32_t N, double defect_max, int32_t force, int32_t* valid,
                              int32_t* mask, int32_t* rebuild, int64_t* count, void* stream);
/* out[i] = mask[i / per] ? a[i] : b[i] for i < N * per (device arrays; out
 * may alias a or b): the fields of the re-anchored lattices taken from the
 * LBM, the others from the surrogate. */
int eelbm_cno_select(const int32_t* mask, int32_t N, int64_t per, const float* a, const float* b, float* out,
                     void* stream);
/* dx = dy where y > 0, slope * dy elsewhere (y: the leaky-ReLU output). */
int eelbm_cno_act_bwd(const float* y, const float* dy, int64_t n, float slope, float* dx, void* stream);
/* 2x2 average pooling (H, W even): forward (B, H, W, C) -> (B, H/2, W/2, C);
 * backward (backward = 1): the gradient of (B, H/2, W/2, C) spread back to
 * (B, H, W, C) (in = that gradient, H, W the full sizes). */
int eelbm_cno_pool(const float* in, int32_t B, int32_t H, int32_t W, int32_t C, float* out, int32_t backward,
                   void* stream);
/* 2x2 average pooling forward of BF16 activations (uint16 bit patterns):
 * the four values summed in FP32 in row order, times 1/4, rounded to BF16. */
int eelbm_cno_pool_bf16(const uint16_t* in, int32_t B, int32_t H, int32_t W, int32_t C, uint16_t* out,
                        void* stream);
/* nearest 2x upsampling: forward (B, H, W, C) -> (B, 2H, 2W, C); backward:
 * the gradient of (B, 2H, 2W, C) summed back to (B, H, W, C). */
int eelbm_cno_up(const float* in, int32_t B, int32_t H, int32_t W, int32_t C, float* out, int32_t backward,
                 void* stream);
/* out = [a | b] over channels, P pixels; split_add: da = d[:, :Ca],
 * db += d[:, Ca:]. */
int eelbm_cno_concat(const float* a, int32_t Ca, const float* b, int32_t Cb, int64_t P, float* out, void* stream);
int eelbm_cno_split_add(const float* d, int32_t Ca, int32_t Cb, int64_t P, float* da, float* db, void* stream);
/* mean squared error over the first Cused of C channels: partial[nblocks]
 * FP64 sums (their total is the loss), dpred = its gradient (may be NULL). */
int eelbm_cno_mse(const float* pred, const float* target, int64_t P, int32_t C, int32_t Cused, double* partial,
                  int32_t nblocks, float* dpred, void* stream);
/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving or training loops, harnesses that forbid allocation): the loss of
 * eelbm_cno_mse without a caller workspace.  *loss (device pointer) receives
 * the total of the nblocks partial sums, added in block order (bit-identical
 * to summing eelbm_cno_mse's partial[] in index order); dpred as in
 * eelbm_cno_mse (may be NULL).  The partial sums live in a fixed device array
 * of EELBM_CNO_MSE_MAX_BLOCKS doubles inside the library (one per GPU, kept
 * until the process ends); the call allocates nothing.  nblocks above
 * EELBM_CNO_MSE_MAX_BLOCKS: EELBM_E_SIZE with a message.  Calls on one GPU
 * share that array: calls that overlap in time on one GPU (different streams
 * without ordering) race and give undefined losses. */
#define EELBM_CNO_MSE_MAX_BLOCKS 1024
int eelbm_cno_mse_noalloc(const float* pred, const float* target, int64_t P, int32_t C, int32_t Cused,
                          int32_t nblocks, double* loss, float* dpred, void* stream);
/* Adam step `step` (>= 1) with decoupled weight decay on n FP32 values. */
int eelbm_cno_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                   int64_t step, float weight_decay, void* stream);
/* BF16 operand copies Wf and Wd of the FP32 master W (9 Cin Cout values). */
int eelbm_cno_pack_weights(const float* w, int32_t Cin, int32_t Cout, uint16_t* wf, uint16_t* wd, void* stream);
/* Network input: out[b][p][c] = (soa[b][c][p] - mean[c]) * inv_scale[c] for
 * c < nf (stacked field planes, P pixels per image; clamped to [-clip, clip]
 * if clip > 0), cond[b][c - nf] for nf <= c < nf + nc, 0 up to C. */
int eelbm_cno_pack(const float* soa, int64_t P, int32_t nf, const float* mean, const float* inv_scale,
                   const float* cond, int32_t nc, int32_t B, int32_t C, float clip, float* out, void* stream);
/* Fields after a jump: soa_out[b][f][p] = soa_in[b][f][p] + net[b][p][f] * dscale[f], f < nf. */
int eelbm_cno_unpack(const float* soa_in, const float* net, int64_t P, int32_t nf, int32_t C, const float* dscale,
                     int32_t B, float* soa_out, void* stream);
/* y += a x over n values. */
int eelbm_cno_axpy(const float* x, int64_t n, float a, float* y, void* stream);
/* p[0..n) = value (a kernel, usable inside captured graphs). */
int eelbm_cno_fill(float* p, int64_t n, float value, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* EELBM_H */
