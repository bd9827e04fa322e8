// HIP kernels of the six coupled LBM schemes for gfx950.
//
// One launch of k_step performs one full time step for every node: a pull
// gather of the post-collision populations of the previous step (streaming,
// left-hand sides of Eqs. (34), (35), (71), (95)), the boundary rules of
// Sec. 3.5 at the domain faces, the moments of all six sets, the Spalding
// renormalisation (Eq. (93)), the continuity sources from the source schemes
// (Eq. (107)) with the dashpots and lagged updates of Sec. 3.2, the volume-
// fraction gradients (Eqs. (91), (94)), the stresses (Eq. (70)), the drag
// (Eqs. (6), (135)-(137)), the forces (Eqs. (24), (26)) and the collisions
// (Eqs. (34)-(42), (71)-(72)), and writes the node's own post-collision
// populations (coalesced stores into the node's 64-node x-block, see
// pop_in_plane).
//
// State kept between launches, per node:
//  * f_g, f_l, f_ag, f_al, post-collision, in the storage type, as residuals
//    against the equilibrium part of their sender's record (see Rec8);
//  * one 8-wide record (alpha_g - alpha_r, u_g, u_l, eps_g - 1, and Lambda'
//    in D2Q9), the reference of those residuals; the post-collision f_b of
//    the lattice kinetic scheme is the pure function f^eq(1, c_phi) of
//    alpha_g and u_g - u_l (Eqs. (95), (97) with beta = 1), so f_b is rebuilt
//    at the gather from the upstream node's record instead of being stored;
//  * the lag fields S''_g, S''_l (and Lambda' in 3D) when n_gamma > 1;
//  * for the two node layers next to an inlet/outlet face, the macroscopic
//    values the boundary extrapolations of Eqs. (160)-(161) need at the next
//    step (u_g, u_l, alpha_g, alpha_l).
//
// Every node computes its pulls per lane (periodic wrap and the boundary
// rules included).  In FP32 compute the upstream records of a tile are staged
// in LDS first (one coalesced load per record of the tile and its halo).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "eelbm.h"
#include "eelbm_internal.hpp"
#include "lattice.hpp"

namespace eelbm {

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to nearest-even into one dword of two 16-bit
// numbers (lo in bits 0-15): one packed conversion instruction on gfx950
// instead of two conversions, a shift and an or.
__device__ __forceinline__ unsigned pack_f16x2(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, f16x2));
}
__device__ __forceinline__ unsigned pack_bf16x2(float lo, float hi) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}
typedef double f64x2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- storage
// Compute type of a storage type: FP64 storage computes in FP64, every other
// storage in FP32.  Populations are read exactly once per step: they are
// loaded nontemporally so that they do not displace the imposed-velocity
// records (read by nine nodes) and the freshly written populations, which the
// next step reads back, from L2 and the Infinity Cache.  Stores stay ordinary
// (measured: nontemporal stores, or nontemporal loads of the lag fields, are
// slower on gfx950; ordinary population loads cost 15 %).
template <class T>
struct Compute {
    using C = float;
};
template <>
struct Compute<double> {
    using C = double;
};
// FP32 populations with FP64 arithmetic and records (EELBM_FP32_F64): the
// storage of FP32 at the arithmetic precision of the FP64 step
struct F32D {
    float v;
};
template <>
struct Compute<F32D> {
    using C = double;
};

// Per-node record of 2 + 2D compute-type values written by every step (8 in
// D3Q19: two 16-byte vectors in FP32; 6 in D2Q9: 24 bytes in FP32, 48 in
// FP64): alpha_g - a_r (renormalised alpha_g as a deviation from the
// reference gas fraction a_r, so that carrying it from step to step rounds at
// the scale of the deviation), u_g, u_l and the gas density deviation
// eps_g - 1 of the node's collision.  It serves two purposes:
//  * the post-collision f_b of the lattice kinetic scheme is the pure
//    function f^eq(1, c_phi) of alpha_g and u_g - u_l (Eqs. (95), (97) with
//    beta = 1), so f_b is rebuilt at the gather from the upstream record
//    instead of being stored;
//  * populations are stored relative to the equilibrium part E_q(r) of their
//    sender's record r:
//        f_g:  w_q (de + 3 v_q.u_g)            f_l:  w_q 3 v_q.u_l
//        f_ag: w_q (da + 3 a v_q.u_g)          f_al: w_q (-da + 3 (1 - a) v_q.u_l)
//    (deviations; da = alpha_g - a_r from the record, a = a_r + da), so what is
//    stored is the non-equilibrium and second-order part only: in FP32 the
//    rounding no longer scales with the velocity, and 16-bit types keep
//    their precision for the small fields (the pressure deviation, the
//    liquid at large density ratios).  The receiver adds E of the sender's
//    record back; any rounding of the record is the same on both sides.
template <int D>
constexpr int kDe = 1 + 2 * D;  // slot of eps_g - 1
// bytes of one record in the record array (the stride between nodes)
template <int D, class C>
constexpr unsigned kRecBytes = (unsigned)((D == 3 ? 8 : 6) * sizeof(C));
template <class C>
struct alignas(8 * sizeof(C)) Rec8 {
    C v[8];
};
template <class C>
struct alignas(2 * sizeof(C)) Rec2 {
    C v[2];
};

__device__ __forceinline__ Rec8<float> ld_rec8(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float) {
    struct Two {
        u32x4 a, b;
    } t;
    t.a = __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0);
    t.b = __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)(so + 16), 0);
    return __builtin_bit_cast(Rec8<float>, t);
}
__device__ __forceinline__ Rec8<double> ld_rec8(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, double) {
    struct Four {
        u32x4 a, b, c, d;
    } t;
    t.a = __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0);
    t.b = __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)(so + 16), 0);
    t.c = __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)(so + 32), 0);
    t.d = __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)(so + 48), 0);
    return __builtin_bit_cast(Rec8<double>, t);
}
// one node's record: all 8 slots in D3Q19, slots 0-5 in D2Q9 (one 16-byte
// and one 8-byte load in FP32; the 24-byte stride leaves every second record
// 8-byte aligned, which buffer loads of several dwords accept)
template <int D>
__device__ __forceinline__ Rec8<float> ld_rec_up(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float c) {
    if constexpr (D == 3) {
        return ld_rec8(r, vo, so, c);
    } else {
        const f32x4 a = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0));
        const f32x2 bq = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)(so + 16), 0));
        Rec8<float> o;
        o.v[0] = a.x;
        o.v[1] = a.y;
        o.v[2] = a.z;
        o.v[3] = a.w;
        o.v[4] = bq.x;
        o.v[5] = bq.y;
        o.v[6] = 0.0f;
        o.v[7] = 0.0f;
        return o;
    }
}
template <int D>
__device__ __forceinline__ Rec8<double> ld_rec_up(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, double c) {
    if constexpr (D == 3) {
        return ld_rec8(r, vo, so, c);
    } else {
        Rec8<double> o;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const f64x2 v =
                __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)(so + 16 * k), 0));
            o.v[2 * k] = v.x;
            o.v[2 * k + 1] = v.y;
        }
        o.v[6] = 0.0;
        o.v[7] = 0.0;
        return o;
    }
}
// stores the slots ld_rec_up reads (kRecBytes<D, C> bytes at vo)
template <int D>
__device__ __forceinline__ void st_rec(__amdgpu_buffer_rsrc_t r, unsigned vo, const Rec8<float>& v) {
    struct Two {
        u32x4 a, b;
    };
    const Two t = __builtin_bit_cast(Two, v);
    __builtin_amdgcn_raw_buffer_store_b128(t.a, r, (int)vo, 0, 0);
    if constexpr (D == 3) {
        __builtin_amdgcn_raw_buffer_store_b128(t.b, r, (int)vo, 16, 0);
    } else {
        const u32x2 lo = {t.b.x, t.b.y};
        __builtin_amdgcn_raw_buffer_store_b64(lo, r, (int)vo, 16, 0);
    }
}
template <int D>
__device__ __forceinline__ void st_rec(__amdgpu_buffer_rsrc_t r, unsigned vo, const Rec8<double>& v) {
    struct Four {
        u32x4 a, b, c, d;
    };
    const Four t = __builtin_bit_cast(Four, v);
    __builtin_amdgcn_raw_buffer_store_b128(t.a, r, (int)vo, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b128(t.b, r, (int)vo, 16, 0);
    __builtin_amdgcn_raw_buffer_store_b128(t.c, r, (int)vo, 32, 0);
    if constexpr (D == 3) __builtin_amdgcn_raw_buffer_store_b128(t.d, r, (int)vo, 48, 0);
}

// Upstream records staged in LDS (FP32 compute): one 32-byte slot per node
// of the tile and its one-node halo; D2Q9 uses slots 0-5 of it.
extern __shared__ Rec8<float> lds_win[];

template <int D>
__device__ __forceinline__ void lds_put(Rec8<float>* d, const Rec8<float>& r) {
    if constexpr (D == 3) {
        *d = r;
    } else {
        *reinterpret_cast<f32x4*>(d->v) = f32x4{r.v[0], r.v[1], r.v[2], r.v[3]};
        *reinterpret_cast<f32x2*>(d->v + 4) = f32x2{r.v[4], r.v[5]};
    }
}
template <int D>
__device__ __forceinline__ Rec8<float> lds_get(const Rec8<float>* d) {
    if constexpr (D == 3) {
        return *d;
    } else {
        const f32x4 a = *reinterpret_cast<const f32x4*>(d->v);
        const f32x2 c = *reinterpret_cast<const f32x2*>(d->v + 4);
        Rec8<float> o;
        o.v[0] = a.x;
        o.v[1] = a.y;
        o.v[2] = a.z;
        o.v[3] = a.w;
        o.v[4] = c.x;
        o.v[5] = c.y;
        o.v[6] = 0.0f;
        o.v[7] = 0.0f;
        return o;
    }
}

// ------------------------------------------------- buffer-instruction I/O
// The hot streams use buffer instructions: a descriptor in SGPRs, one VGPR
// byte offset shared by every access of a node, and the per-direction shift
// in an SGPR offset, so an access costs no vector ALU work.  Bit 1 of the
// cache-policy operand is the nontemporal hint on gfx950.  Populations are
// always loaded with it; they are stored with it only when the lattice's
// populations do not fit the last-level cache (KParams::nt_store): a smaller
// lattice finds the populations written in one step there in the next.
constexpr int kNT = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, 0x00020000);
}

// The four sets (f_g, f_l, f_ag, f_al) of one direction of one node are
// adjacent in memory and move with one vector access: 16 bytes in FP32, 8 in
// FP16/BF16, 2 x 16 in FP64.
template <class T>
struct Pop4;
// (Whole vectors are bit-cast and then indexed: a bit-cast of a single
// vector element is not reliable with this compiler.)
template <>
struct Pop4<float> {
    static __device__ __forceinline__ void ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float* o,
                                              const KParams&, bool) {
        const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, kNT));
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
    template <int POL>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, const float* v,
                                              const KParams&, bool) {
        const f32x4 w = {v[0], v[1], v[2], v[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, w), r, (int)vo, (int)so, POL);
    }
};
template <>
struct Pop4<F32D> {
    static __device__ __forceinline__ void ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, double* o,
                                              const KParams&, bool) {
        const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, kNT));
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
    template <int POL>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, const double* v,
                                              const KParams&, bool) {
        const f32x4 w = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, w), r, (int)vo, (int)so, POL);
    }
};
template <>
struct Pop4<double> {
    static __device__ __forceinline__ void ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, double* o,
                                              const KParams&, bool) {
        const f64x2 a = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, kNT));
        const f64x2 b =
            __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)(so + 16), kNT));
        o[0] = a.x;
        o[1] = a.y;
        o[2] = b.x;
        o[3] = b.y;
    }
    template <int POL>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, const double* v,
                                              const KParams&, bool) {
        const f64x2 a = {v[0], v[1]}, b = {v[2], v[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, a), r, (int)vo, (int)so, POL);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, b), r, (int)vo, (int)(so + 16), POL);
    }
};
// 16-bit storage: set k sits in half-word k of the 8-byte group.  The stored
// residuals (non-equilibrium and second-order parts, see Rec8) are small, so
// FP16 holds them multiplied by a power of two per set (KParams::h16_up,
// exact): 2^20 for f_g, f_ag, f_al (residuals in [6e-11, 0.06) are normal FP16
// numbers with relative precision 2^-11) and 2^20 min(R, 64) for the moving
// populations of f_l, whose residuals shrink with the density ratio.  The
// rest population of f_l is stored unscaled: it carries the liquid density
// deviation sum f_l - 1, which no other quantity of the step uses (the liquid
// feels the pressure through Eq. (32) instead) and which drifts freely where
// liquid piles up -- at the inlet corners of the channel it passes 0.06, the
// largest residual FP16 holds at the 2^20 scale, within 4000 steps.  BF16 has the exponent range of
// FP32 and is stored unscaled.
template <class H>
struct Pop4Half {
    static constexpr bool kHalf = std::is_same<H, __half>::value;
    static __device__ __forceinline__ float to_f(unsigned short h, float down) {
        if constexpr (kHalf)
            return __half2float(__ushort_as_half(h)) * down;
        else
            return __bfloat162float(__builtin_bit_cast(__hip_bfloat16, h));
    }
    static __device__ __forceinline__ void ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float* o,
                                              const KParams& p, bool rest) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, kNT);
        o[0] = to_f((unsigned short)(v.x & 0xffffu), p.h16_down[0]);
        o[1] = to_f((unsigned short)(v.x >> 16), rest ? 1.0f : p.h16_down[1]);
        o[2] = to_f((unsigned short)(v.y & 0xffffu), p.h16_down[0]);
        o[3] = to_f((unsigned short)(v.y >> 16), p.h16_down[0]);
    }
    template <int POL>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, const float* v,
                                              const KParams& p, bool rest) {
        // (the FP16 scales are powers of two: the products are exact, so the
        // one rounding is the conversion's)
        u32x2 w;
        if constexpr (kHalf) {
            w.x = pack_f16x2(v[0] * p.h16_up[0], v[1] * (rest ? 1.0f : p.h16_up[1]));
            w.y = pack_f16x2(v[2] * p.h16_up[0], v[3] * p.h16_up[0]);
        } else {
            w.x = pack_bf16x2(v[0], v[1]);
            w.y = pack_bf16x2(v[2], v[3]);
        }
        __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)vo, (int)so, POL);
    }
};
template <>
struct Pop4<__half> : Pop4Half<__half> {};
// Mixed storage (EELBM_MIXED): f_g in FP32, f_l, f_ag, f_al in FP16 with
// the scales above, one 12-byte group per direction (the tag type is 3
// bytes, a quarter of the group).  The gas density, which carries the
// pressure delta p_k, keeps the resolution of FP32 storage; the liquid and
// volume-fraction populations take 16 bits.
struct Mix12 {
    unsigned char b[3];
};
template <>
struct Pop4<Mix12> {
    static __device__ __forceinline__ float h2f(unsigned short h, float down) {
        return __half2float(__ushort_as_half(h)) * down;
    }
    static __device__ __forceinline__ unsigned short f2h(float v, float up) {
        return __half_as_ushort(__float2half_rn(v * up));
    }
    static __device__ __forceinline__ void ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float* o,
                                              const KParams& p, bool rest) {
        const u32x3 v = __builtin_bit_cast(u32x3, __builtin_amdgcn_raw_buffer_load_b96(r, (int)vo, (int)so, kNT));
        o[0] = __builtin_bit_cast(float, v.x);
        o[1] = h2f((unsigned short)(v.y & 0xffffu), rest ? 1.0f : p.h16_down[1]);
        o[2] = h2f((unsigned short)(v.y >> 16), p.h16_down[0]);
        o[3] = h2f((unsigned short)(v.z & 0xffffu), p.h16_down[0]);
    }
    template <int POL>
    static __device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, const float* v,
                                              const KParams& p, bool rest) {
        u32x3 w;
        w.x = __builtin_bit_cast(unsigned, v[0]);
        w.y = pack_f16x2(v[1] * (rest ? 1.0f : p.h16_up[1]), v[2] * p.h16_up[0]);
        w.z = (unsigned)f2h(v[3], p.h16_up[0]);
        __builtin_amdgcn_raw_buffer_store_b96(w, r, (int)vo, (int)so, POL);
    }
};
template <>
struct Pop4<__hip_bfloat16> : Pop4Half<__hip_bfloat16> {};

// wave-uniform base + 32-bit per-lane byte offset: compiles to a global
// load/store with an SGPR base, one shared VGPR offset and an immediate
// (the host keeps every array below 4 GiB)
template <class X>
__device__ __forceinline__ const X* at(const X* base, unsigned byte_off) {
    return reinterpret_cast<const X*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <class X>
__device__ __forceinline__ X* at(X* base, unsigned byte_off) {
    return reinterpret_cast<X*>(reinterpret_cast<char*>(base) + byte_off);
}

// reciprocal and square root of the compute type, correctly rounded
template <class C>
__device__ __forceinline__ C rcp(C v) {
    return C(1) / v;
}
template <class C>
__device__ __forceinline__ C root(C v) {
    return sqrt(v);
}

template <class C>
__device__ __forceinline__ C clamp01(C v) {
    return v < C(0) ? C(0) : (v > C(1) ? C(1) : v);
}

// w_q-normalised non-rest part of the second-order equilibria:
// 3 v.u + 9/2 (v.u)^2 - 3/2 |u|^2  (c_s^2 = 1/3 in Eqs. (37), (72))
template <class C>
__device__ __forceinline__ C poly2(C cu, C usq) {
    return C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq;
}

template <class L, class C>
__device__ __forceinline__ C dotc(int q, const C* u) {
    C s = C(0);
#pragma unroll
    for (int a = 0; a < L::D; ++a) {
        if (L::c[q][a] == 1) s += u[a];
        if (L::c[q][a] == -1) s -= u[a];
    }
    return s;
}

__device__ __forceinline__ int wrap_axis(int v, int nax, int per) {
    if (v < 0) return per ? v + nax : 0;
    if (v >= nax) return per ? v - nax : nax - 1;
    return v;
}

// Source-scheme populations entering a node (Eqs. (72), (95), (97)), as
// deviations f_b - w_q - w_q P_q(c_0) from the node's own equilibrium part,
// P_q(c) = 3 v_q.c + 9/2 (v_q.c)^2 - 3/2 |c|^2, with c_0 the node's own
// imposed velocity (c_g = alpha_l du, c_l = -alpha_g du, du = u_g - u_l).
// sum_q w_q P_q(c_0) = 0, so the sources S = 1 - sum f_b are unchanged, and
// for a sender with imposed velocity c_s
//   P_q(c_s) - P_q(c_0) = 3 v.d + 9/2 (v.d)(v.(c_s + c_0)) - 3/2 d.(c_s + c_0)
// with d = c_s - c_0: every term carries the difference d, formed from the
// differences of the two records (dals = alpha_l,s - alpha_l,0, da =
// alpha_g,s - alpha_g,0, ddu = (u_g,s - u_g,0) - (u_l,s - u_l,0), each exact
// in the record's type), so the sum keeps the precision of the small source
// instead of cancelling terms of the size of c or |c|^2.
template <class L, class C>
__device__ __forceinline__ C p_diff(int q, const C* d, const C* s) {
    C ds = C(0);
#pragma unroll
    for (int a = 0; a < L::D; ++a) ds += d[a] * s[a];
    const C vd = dotc<L>(q, d);
    return C(L::w[q]) * (C(3) * vd + C(4.5) * vd * dotc<L>(q, s) - C(1.5) * ds);
}
template <class L, class C>
__device__ __forceinline__ void beta_rel(int q, C as, C als, const C* dus, C dals, C da, C al0, C a0, const C* ddu,
                                         C& dbg, C& dbl) {
    constexpr int D = L::D;
    C sg[D], sl[D], dcg[D], dcl[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        dcg[a] = dals * dus[a] + al0 * ddu[a];
        dcl[a] = -(da * dus[a] + a0 * ddu[a]);
        sg[a] = C(2) * (als * dus[a]) - dcg[a];  // c_s + c_0
        sl[a] = C(-2) * (as * dus[a]) - dcl[a];
    }
    dbg = p_diff<L>(q, dcg, sg);
    dbl = p_diff<L>(q, dcl, sl);
}

// f_b entering through an inlet/outlet face: EQ(S) with beta = 1 and the
// imposed velocity extrapolated full-way (Tables 1-2, beta read as the 1 the
// equilibria carry); through a wall: EQ(S)(1, 0) -- both as deviations from
// the node's own w_q (1 + P_q(c_0)) as in beta_rel
template <class L, class C>
__device__ __forceinline__ void beta_face(int q, const C* cgB, const C* clB, const C* c0g, const C* c0l, C& dbg,
                                          C& dbl) {
    constexpr int D = L::D;
    C dg[D], dl[D], sg[D], sl[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        dg[a] = cgB[a] - c0g[a];
        dl[a] = clB[a] - c0l[a];
        sg[a] = cgB[a] + c0g[a];
        sl[a] = clB[a] + c0l[a];
    }
    dbg = p_diff<L>(q, dg, sg);
    dbl = p_diff<L>(q, dl, sl);
}
template <class L, class C>
__device__ __forceinline__ void beta_wall(int q, const C* c0g, const C* c0l, C& dbg, C& dbl) {
    C ug2 = C(0), ul2 = C(0);
#pragma unroll
    for (int a = 0; a < L::D; ++a) {
        ug2 += c0g[a] * c0g[a];
        ul2 += c0l[a] * c0l[a];
    }
    const C wq = C(L::w[q]);
    dbg = -wq * poly2(dotc<L>(q, c0g), ug2);
    dbl = -wq * poly2(dotc<L>(q, c0l), ul2);
}

// does direction q of a node on the lattice's edge arrive through a wall or
// through the inlet/outlet plane?  (Reading R15: a wall face wins at corners.)
template <class L, class WL, class WH>
__device__ __forceinline__ void bnd_kind(int q, const bool* lo, const bool* hi, int fs, int fa, WL wall_lo,
                                         WH wall_hi, bool& wall, bool& flow) {
    wall = false;
    flow = false;
#pragma unroll
    for (int a = 0; a < L::D; ++a) {
        wall = wall || (lo[a] && L::c[q][a] == 1 && wall_lo(a)) || (hi[a] && L::c[q][a] == -1 && wall_hi(a));
    }
    if (!wall && fs >= 0) {
        const int cfa = fa == 0 ? L::c[q][0] : (fa == 1 ? L::c[q][1] : L::c[q][2]);
        flow = (fs == 0 && cfa == 1) || (fs == 1 && cfa == -1);
    }
}

// record of a node built from the initial fields (stage: alpha_g, u_g,
// u_l, dp_k as [2 + 2D][n] FP64)
template <class L, class C>
__device__ __forceinline__ Rec8<C> stage_rec(const double* stage, long long src, long long n, double a_ref) {
    constexpr int D = L::D;
    Rec8<C> r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r.v[k] = C(0);
    r.v[0] = C(stage[src] - a_ref);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        r.v[1 + a] = C(stage[(1 + a) * n + src]);
        r.v[1 + D + a] = C(stage[(1 + D + a) * n + src]);
    }
    r.v[kDe<D>] = C(3.0 * stage[(1 + 2 * D) * n + src]);
    return r;
}

// n_q = f_q - E_q(r0) for a population pulled from a sender with record rs:
// the stored residual g plus E_q(rs) - E_q(r0), written with the record
// differences (see Rec8); a0d, a0 = a_r + a0d: gas fraction of r0
template <class L, class C>
__device__ __forceinline__ void rebase(int q, const C* g, const Rec8<C>& rs, C a0d, C a0, const C* ug0, const C* ul0,
                                       C de0, C* n4) {
    constexpr int D = L::D;
    const C wq = C(L::w[q]);
    C dug[D], dul[D], ugs[D], uls[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        ugs[a] = rs.v[1 + a];
        uls[a] = rs.v[1 + D + a];
        dug[a] = ugs[a] - ug0[a];
        dul[a] = uls[a] - ul0[a];
    }
    const C cdg = dotc<L>(q, dug), cdl = dotc<L>(q, dul);
    const C dA = rs.v[0] - a0d;
    n4[0] = g[0] + wq * ((rs.v[kDe<D>] - de0) + C(3) * cdg);
    n4[1] = g[1] + wq * (C(3) * cdl);
    n4[2] = g[2] + wq * (dA + C(3) * (dA * dotc<L>(q, ugs) + a0 * cdg));
    n4[3] = g[3] + wq * (C(3) * ((C(1) - a0) * cdl - dA * dotc<L>(q, uls)) - dA);
}

// beta_rel for an upstream node with record rs (the node's own: a0d, a0 =
// a_r + a0d, al0, u_g0, u_l0); als: alpha_l of the sender, renorm: alpha_l =
// 1 - alpha_g (then alpha_l,s - alpha_l,0 = -(alpha_g,s - alpha_g,0), exact
// from the record deviations)
template <class L, class C>
__device__ __forceinline__ void beta_from(int q, const Rec8<C>& rs, bool renorm, C ar, C a0d, C a0, C al0, C als,
                                          const C* ug0, const C* ul0, C& dbg, C& dbl) {
    constexpr int D = L::D;
    C dus[D], ddu[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        dus[a] = rs.v[1 + a] - rs.v[1 + D + a];
        ddu[a] = (rs.v[1 + a] - ug0[a]) - (rs.v[1 + D + a] - ul0[a]);
    }
    const C da = rs.v[0] - a0d;
    beta_rel<L>(q, ar + rs.v[0], als, dus, renorm ? -da : als - al0, da, al0, a0, ddu, dbg, dbl);
}

// Population layout: each z-plane is a sequence of x-blocks of 64 nodes (rows
// padded to a whole number of blocks); one block holds the post-collision
// populations of its 64 nodes as [q][lane][set]: the four sets of a direction
// are one 4-wide group, and a wavefront (64 nodes of one block) reads or
// writes one contiguous run of 64 groups per direction.  Element offset of
// the group (x, y, q) within its z-plane (a plane stays below 4 GiB, so every
// access is a plane descriptor plus a 32-bit offset):
template <class L>
__device__ __forceinline__ unsigned pop_in_plane(const KParams& p, int x, int y, int q) {
    return (unsigned)(((((long long)y * p.nxb + (x >> 6)) * L::Q + q) * 64 + (x & 63)) * 4);
}

// --------------------------------------------------------------- the step
// inlet ramp of Eq. (153): (y_max - y_min) tanh(t / n_t) + y_min
__device__ __forceinline__ double ramp(double t, double ymax, double ymin, double nr) {
    if (!(nr > 0.0)) return ymax;
    return (ymax - ymin) * tanh(t / nr) + ymin;
}

// One node update of one tile: `tile` is the tile's index over all planes,
// `part` the slot of its diagnostic partial sums.  Diagnostics and the field
// read-out are written when the step's control asks for them, by the same
// instantiation that runs the steps without them: a separate instantiation
// without that code needs 3-4 fewer VGPRs (no change of occupancy) but, with
// its other basic blocks, the compiler fused other multiply-add pairs, so a
// lattice's state came to depend on the steps at which it was read.
template <class L, class T, int BC, bool INIT, bool NTS = false>
__device__ __forceinline__ void step_body(const KParams& p, const KBuffers& b, const KCtl& ctl, long long tile,
                                          long long part) {
    using C = typename Compute<T>::C;
    constexpr int D = L::D;
    constexpr int Q = L::Q;
    constexpr int NPI = L::NPI;
    // Boundary configuration: compile-time constants for a lattice periodic
    // on every axis (BC = kBcPeriodic) and for the standard column (flow
    // along the last axis, inlet at its low face, outlet at its high face,
    // walls on every other face: BC = kBcColumn); the launch parameters for
    // any other channel (kBcGeneric).  Constants keep the boundary code from
    // holding scalar registers the rest of the step needs.
    constexpr bool CH = BC != kBcPeriodic;
    auto per = [&](int a) { return BC == kBcPeriodic ? 1 : (BC == kBcColumn ? int(a >= D) : p.per[a]); };
    auto wall_lo = [&](int a) { return BC == kBcColumn ? int(a < D - 1) : p.wall_lo[a]; };
    auto wall_hi = [&](int a) { return BC == kBcColumn ? int(a < D - 1) : p.wall_hi[a]; };
    const int face_lo = BC == kBcColumn ? int(EELBM_BC_INLET) : p.face_lo;
    const int face_hi = BC == kBcColumn ? int(EELBM_BC_OUTLET) : p.face_hi;
    constexpr int NV = 2 * D + 2;  // side-buffer values per node: u_g, u_l, alpha_g, alpha_l
    constexpr int kBlk = 4 * Q * 64;  // population elements of one x-block
    const C third = C(1) / C(3);
    const long long plane_tiles = (long long)p.ntx * p.nty;
    const int z = (int)(tile / plane_tiles);
    const int rem = (int)(tile - (long long)z * plane_tiles);
    const int ty_t = rem / p.ntx;
    const int x = (rem - ty_t * p.ntx) * blockDim.x + threadIdx.x;
    const int y = ty_t * blockDim.y + threadIdx.y;
    const bool act = x < p.nx && y < p.ny;
    const long long n = p.n;
    const long long node = ((long long)z * p.ny + y) * p.nx + x;
    const unsigned rb = (unsigned)node * kRecBytes<D, C>;             // ... in the record array
    const unsigned cb = (unsigned)node * (unsigned)sizeof(C);         // ... in a scalar array
    const int co[3] = {x, y, z};
    const int nn[3] = {p.nx, p.ny, p.nz};
    const long long nxy = (long long)p.nx * p.ny;

    double dsum[kNDiag];
#pragma unroll
    for (int k = 0; k < kNDiag; ++k) dsum[k] = 0.0;

    // A wavefront issues its gather and record loads at the highest wave
    // priority and drops back to the default for its arithmetic, so a newly
    // started wave gets its loads in flight ahead of the arithmetic of older
    // waves on the same SIMD (measured: -2 to -3 % on the D2Q9 channel).
    __builtin_amdgcn_s_setprio(3);
    // The upstream records of the tile (FP32 compute): the tile's nodes and a
    // one-node halo (the neighbouring planes too in D3Q19) are loaded once
    // per workgroup into LDS with coalesced loads (periodic axes wrap, other
    // coordinates clamp: a pull from outside the lattice arrives through a
    // boundary and its record is not used), so each node's Q - 1 upstream
    // records come from LDS instead of as many scattered cache loads.
    constexpr bool kStage = !INIT && sizeof(C) == 4;
    const int wx = blockDim.x + 2, wy = blockDim.y + 2;
    if constexpr (kStage) {
        const int nwin = wx * wy * (D == 3 ? 3 : 1);
        const int x0 = x - (int)threadIdx.x - 1, y0 = y - (int)threadIdx.y - 1;
        const int nthr = blockDim.x * blockDim.y;
        const __amdgpu_buffer_rsrc_t rw = rsrc(b.cf_in);
        for (int e = threadIdx.y * blockDim.x + threadIdx.x; e < nwin; e += nthr) {
            const int i = e % wx, jk = e / wx;
            const int j = jk % wy, k = jk / wy;
            const int xs = wrap_axis(x0 + i, p.nx, per(0));
            const int ys = wrap_axis(y0 + j, p.ny, per(1));
            const int zs = D == 3 ? wrap_axis(z - 1 + k, p.nz, per(2)) : 0;
            const long long src = ((long long)zs * p.ny + ys) * p.nx + xs;
            lds_put<D>(lds_win + e, ld_rec_up<D>(rw, (unsigned)src * kRecBytes<D, float>, 0u, 0.0f));
        }
        __syncthreads();
    }
    // LDS slot of the upstream node of direction q
    auto win_at = [&](int q) {
        return ((int)threadIdx.x + 1 - L::c[q][0]) +
               wx * (((int)threadIdx.y + 1 - L::c[q][1]) + wy * (D == 3 ? 1 - L::c[q][2] : 0));
    };
    if (act) {
        const T* pin = static_cast<const T*>(b.pop_in);
        const Rec8<C>* cfin = static_cast<const Rec8<C>*>(b.cf_in);
        const C* alin = static_cast<const C*>(b.al_in);
        const C* sidein = static_cast<const C*>(b.side_in);
        const C ar = C(p.alpha_ref);


        // -------------------------------------------------- boundary layout
        bool lo[3] = {false, false, false}, hi[3] = {false, false, false};
        bool edge = false;
        int fs = -1;            // flow-axis face this node lies on (0 low, 1 high)
        int ftype = EELBM_BC_PERIODIC;
        long long fidx = 0;     // node index within that face
        const int fa = BC == kBcColumn ? D - 1 : p.flow_axis;
        if constexpr (CH) {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                lo[a] = !per(a) && co[a] == 0;
                hi[a] = !per(a) && co[a] == nn[a] - 1;
                edge = edge || lo[a] || hi[a];
            }
            if (fa >= 0) {
                fidx = fa == 0 ? (long long)z * p.ny + y : (fa == 1 ? (long long)z * p.nx + x : (long long)y * p.nx + x);
                const int cf = co[fa];
                if (cf == 0 && (face_lo == EELBM_BC_INLET || face_lo == EELBM_BC_OUTLET)) {
                    fs = 0;
                    ftype = face_lo;
                } else if (cf == nn[fa] - 1 && (face_hi == EELBM_BC_INLET || face_hi == EELBM_BC_OUTLET)) {
                    fs = 1;
                    ftype = face_hi;
                }
            }
        }

        // values on the flow face (Sec. 3.5, STEP #1)
        C uinG[D], uinL[D], ain = C(0);                 // inlet: imposed u and alpha
        C ugB[D], ulB[D], agB = C(0), alB = C(0);       // outlet: EX(hw)
        // f_b from beyond the face: EQ(S) with c extrapolated full-way and beta
        // = 1, the value every node's equilibrium carries at the start of a
        // step (beta is 1 before streaming, Eqs. (105)-(107)), so its
        // extrapolation is 1 as well
        C cgB[D], clB[D];
        // (computed where they are used -- before the initial step's gather,
        // at the edge nodes of a later step after theirs -- so that they hold
        // no registers through the gather)
        auto face_values = [&]() {
#pragma unroll
        for (int a = 0; a < D; ++a) uinG[a] = uinL[a] = ugB[a] = ulB[a] = cgB[a] = clB[a] = C(0);
        if constexpr (CH) {
            if (fs >= 0) {
                const C sgn = fs == 0 ? C(1) : C(-1);
                if (ftype == EELBM_BC_INLET) {
                    // inlet ramp at t - 1 (streaming t - 1 -> t), Eq. (153)
                    const double tr = double(ctl.t - 1);
                    const double a_in_t = ramp(tr, p.a_in_max, p.a_in_min, p.n_ramp);
                    const double ug_in_t = ramp(tr, p.ug_in_max, p.ug_in_min, p.n_ramp);
                    const double ul_in_t = ramp(tr, p.ul_in_max, p.ul_in_min, p.n_ramp);
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        uinG[a] = a == fa ? sgn * C(ug_in_t) : C(0);
                        uinL[a] = a == fa ? sgn * C(ul_in_t) : C(0);
                    }
                    ain = C(a_in_t * (b.noise ? b.noise[fidx] : 1.0));
                }
                if constexpr (INIT) {
                    // t = -1: beta = 1, c from the initial fields of the edge
                    // node and its inward neighbour
                    const long long st = fa == 0 ? 1 : (fa == 1 ? (long long)p.nx : nxy);
                    const long long e = node, nx1 = fs == 0 ? node + st : node - st;
                    const double ae = b.stage[e], an = b.stage[nx1];
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        const double due = b.stage[(1 + a) * n + e] - b.stage[(1 + D + a) * n + e];
                        const double dun = b.stage[(1 + a) * n + nx1] - b.stage[(1 + D + a) * n + nx1];
                        cgB[a] = C(2.0 * (1.0 - ae) * due - (1.0 - an) * dun);
                        clB[a] = C(2.0 * (-ae * due) - (-an * dun));
                    }
                } else {
                    auto sv = [&](int layer, int v) -> C {
                        return sidein[((long long)(fs * 2 + layer) * NV + v) * p.face_n + fidx];
                    };
                    const C ae = sv(0, 2 * D), an = sv(1, 2 * D);
                    const C ale = p.renorm ? C(1) - ae : sv(0, 2 * D + 1);
                    const C aln = p.renorm ? C(1) - an : sv(1, 2 * D + 1);
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        const C uge = sv(0, a), ugn = sv(1, a), ule = sv(0, D + a), uln = sv(1, D + a);
                        ugB[a] = C(1.5) * uge - C(0.5) * ugn;
                        ulB[a] = C(1.5) * ule - C(0.5) * uln;
                        cgB[a] = C(2) * (ale * (uge - ule)) - aln * (ugn - uln);
                        clB[a] = C(2) * (ae * (ule - uge)) - an * (uln - ugn);
                    }
                    agB = C(1.5) * ae - C(0.5) * an;
                    alB = p.renorm ? C(1) - agB : C(1.5) * ale - C(0.5) * aln;
                }
            }
        }
        };
        if constexpr (INIT) face_values();

        // ---------------------------------- the node's own record at t - 1
        // The populations are stored relative to the equilibrium part E_q(r)
        // of their sender's record r (see rec_e): what is reconstructed here
        // is n_q = f_q - E_q(r0), the pulled population minus the part the
        // node's own record r0 would give, from the stored residual plus the
        // differences between the sender's record and r0 -- so the moments
        // below add small numbers to r0's values instead of summing large
        // ones.  The initial step takes r0 from the initial fields.
        Rec8<C> r0;
        if constexpr (INIT) {
            r0 = stage_rec<L, C>(b.stage, node, n, p.alpha_ref);
        } else if constexpr (kStage) {
            r0 = lds_get<D>(lds_win + win_at(0));  // the centre of the staged window
        } else {
            r0 = ld_rec_up<D>(rsrc(cfin), rb, 0u, C(0));
        }
        const C a0d = r0.v[0], a0 = ar + a0d, de0 = r0.v[kDe<D>];
        C ug0[D], ul0[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            ug0[a] = r0.v[1 + a];
            ul0[a] = r0.v[1 + D + a];
        }
        // the node's own imposed velocities of the source schemes (Eq. (97))
        C al0 = C(1) - a0;
        if constexpr (!INIT) {
            if (!p.renorm) al0 = *at(alin, cb);
        }
        C c0g[D], c0l[D];
        auto own_c = [&]() {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const C du0 = ug0[a] - ul0[a];
                c0g[a] = al0 * du0;
                c0l[a] = -a0 * du0;
            }
        };
        if constexpr (INIT) own_c();

        // ------------------------------------------------------- gather
        C f[4][Q];              // n_q of f_g, f_l, f_ag, f_al
        C Sg = C(0), Sl = C(0);  // continuity sources from f_b (Eq. (107))
        if constexpr (INIT) {
            // local equilibria of the initial fields: n_q = f^eq_q - E_q(r0)
            C us0g = C(0), us0l = C(0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                us0g += ug0[a] * ug0[a];
                us0l += ul0[a] * ul0[a];
            }
            const C w0 = C(L::w[0]);
            const C k0 = (C(1) - w0) / w0;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const C wq = C(L::w[q]);
                const C cug = dotc<L>(q, ug0), cul = dotc<L>(q, ul0);
                const C qg = C(4.5) * cug * cug - C(1.5) * us0g, ql = C(4.5) * cul * cul - C(1.5) * us0l;
                const C el = q == 0 ? -k0 * de0 * C(p.invR) : de0 * C(p.invR);
                f[0][q] = wq * qg;
                f[1][q] = wq * (el + ql);
                f[2][q] = wq * a0 * qg;
                f[3][q] = wq * (C(1) - a0) * ql;
            }
            // f_b "as streamed" from the initial imposed velocities
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                bool wall = false, flow = false;
                if constexpr (CH) {
                    if (edge) bnd_kind<L>(q, lo, hi, fs, fa, wall_lo, wall_hi, wall, flow);
                }
                C dbg, dbl;
                if (wall) {
                    beta_wall<L>(q, c0g, c0l, dbg, dbl);
                } else if (flow) {
                    beta_face<L>(q, cgB, clB, c0g, c0l, dbg, dbl);
                } else {
                    const int xs = wrap_axis(x - L::c[q][0], p.nx, per(0));
                    const int ys = wrap_axis(y - L::c[q][1], p.ny, per(1));
                    const int zs = wrap_axis(z - L::c[q][2], p.nz, per(2));
                    const Rec8<C> rs =
                        stage_rec<L, C>(b.stage, ((long long)zs * p.ny + ys) * p.nx + xs, n, p.alpha_ref);
                    beta_from<L>(q, rs, true, ar, a0d, a0, al0, C(1) - (ar + rs.v[0]), ug0, ul0, dbg, dbl);
                }
                Sg -= dbg;
                Sl -= dbl;
            }
        } else {
            // direction q of this lane arrives through a wall or the
            // inlet/outlet plane (bit q of bmask): the boundary rules below
            // start from the node's own post-collision population of the
            // opposite direction, so the gather loads that one in place of
            // the pull (one batch of Q loads, no second, dependent load)
            unsigned bmask = 0u, wmask = 0u;
            if constexpr (CH) {
                if (edge) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        bool wall = false, flow = false;
                        bnd_kind<L>(q, lo, hi, fs, fa, wall_lo, wall_hi, wall, flow);
                        if (wall || flow) bmask |= 1u << q;
                        if (wall) wmask |= 1u << q;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const bool bnd = (bmask >> q) & 1u;
                const int xs = bnd ? x : wrap_axis(x - L::c[q][0], p.nx, per(0));
                const int ys = bnd ? y : wrap_axis(y - L::c[q][1], p.ny, per(1));
                // a pull within the node's own plane keeps the wavefront's plane
                // (uniform across the wave, so the descriptor stays scalar)
                const int zs = L::c[q][2] == 0 ? z : (bnd ? z : wrap_axis(z - L::c[q][2], p.nz, per(2)));
                C g4[4];
                Pop4<T>::ld(rsrc(pin + (long long)zs * p.plane),
                            pop_in_plane<L>(p, xs, ys, bnd ? L::opp[q] : q) * (unsigned)sizeof(T), 0, g4, p, q == 0);
#pragma unroll
                for (int s = 0; s < 4; ++s) f[s][q] = g4[s];
            }
            // The upstream records and the rebase onto the node's own
            // record, one direction at a time (staged: short LDS reads; else
            // one batch of loads); a direction that arrives through a
            // boundary keeps the loaded residual of its opposite direction.
            auto pass = [&](auto rn) {
                constexpr bool renorm = decltype(rn)::value;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const bool bnd = (bmask >> q) & 1u;
                if (kStage && bnd) continue;
                const int xs = bnd ? x : wrap_axis(x - L::c[q][0], p.nx, per(0));
                const int ys = bnd ? y : wrap_axis(y - L::c[q][1], p.ny, per(1));
                const int zs = bnd ? z : wrap_axis(z - L::c[q][2], p.nz, per(2));
                const long long src = ((long long)zs * p.ny + ys) * p.nx + xs;
                Rec8<C> rs = r0;
                if (q != 0) {
                    if constexpr (kStage)
                        rs = lds_get<D>(lds_win + win_at(q));
                    else
                        rs = ld_rec_up<D>(rsrc(cfin), (unsigned)src * kRecBytes<D, C>, 0u, C(0));
                }
                const C g4[4] = {f[0][q], f[1][q], f[2][q], f[3][q]};
                C n4[4];
                rebase<L>(q, g4, rs, a0d, a0, ug0, ul0, de0, n4);
                C als;
                if constexpr (renorm)
                    als = C(1) - (ar + rs.v[0]);
                else
                    als = *at(alin, (unsigned)src * (unsigned)sizeof(C));
                C dbg, dbl;
                beta_from<L>(q, rs, renorm, ar, a0d, a0, al0, als, ug0, ul0, dbg, dbl);
#pragma unroll
                for (int s = 0; s < 4; ++s) f[s][q] = bnd ? g4[s] : n4[s];  // bnd: residual of the opposite direction
                Sg -= bnd ? C(0) : dbg;
                Sl -= bnd ? C(0) : dbl;
            }
            };
            if (p.renorm)
                pass(std::true_type{});
            else
                pass(std::false_type{});
            if constexpr (CH) {
                if (edge) {
                    face_values();
                    own_c();
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        if (!((bmask >> q) & 1u)) continue;
                        const bool wall = (wmask >> q) & 1u;
                        C fo[4];  // residual of the node's own post-collision population of the opposite direction
#pragma unroll
                        for (int s = 0; s < 4; ++s) fo[s] = f[s][q];
                        const C wq = C(L::w[q]);
                        const C cg0 = dotc<L>(q, ug0), cl0 = dotc<L>(q, ul0);
                        if (wall) {
                            // half-way bounce-back, zero wall velocity
                            f[0][q] = fo[0] - C(6) * wq * cg0;
                            f[1][q] = fo[1] - C(6) * wq * cl0;
                            f[2][q] = fo[2] - C(6) * wq * a0 * cg0;
                            f[3][q] = fo[3] - C(6) * wq * (C(1) - a0) * cl0;
                            C dbg, dbl;
                            beta_wall<L>(q, c0g, c0l, dbg, dbl);
                            Sg -= dbg;
                            Sl -= dbl;
                        } else {
                            if (ftype == EELBM_BC_INLET) {
                                C usg = C(0), usl = C(0);
#pragma unroll
                                for (int a = 0; a < D; ++a) {
                                    usg += uinG[a] * uinG[a];
                                    usl += uinL[a] * uinL[a];
                                }
                                const C cug = dotc<L>(q, uinG), cul = dotc<L>(q, uinL);
                                // BB(I), Eq. (163): + f_I(-u) - f_I(u) at q* = 6 w v_q.u
                                f[0][q] = fo[0] + C(6) * wq * (cug - cg0);
                                f[1][q] = fo[1] + C(6) * wq * (cul - cl0);
                                // EQ(S) with the imposed alpha and velocity
                                f[2][q] = wq * (((ain - ar) - a0d) + ain * poly2(cug, usg) - C(3) * a0 * cg0);
                                f[3][q] = wq * (((ar - ain) + a0d) + (C(1) - ain) * poly2(cul, usl) -
                                                C(3) * (C(1) - a0) * cl0);
                            } else {
                                C usg = C(0), usl = C(0);
#pragma unroll
                                for (int a = 0; a < D; ++a) {
                                    usg += ugB[a] * ugB[a];
                                    usl += ulB[a] * ulB[a];
                                }
                                const C cug = dotc<L>(q, ugB), cul = dotc<L>(q, ulB);
                                const C eg = C(4.5) * cug * cug - C(1.5) * usg, el = C(4.5) * cul * cul - C(1.5) * usl;
                                // ABB(I), Eq. (164), eps = phi = 1
                                f[0][q] = -fo[0] + C(2) * wq * (eg - de0);
                                f[1][q] = -fo[1] + C(2) * wq * el;
                                // ABB(S)
                                f[2][q] = -fo[2] + C(2) * wq * (((agB - ar) - a0d) + agB * eg);
                                f[3][q] = -fo[3] + C(2) * wq * (((alB - (C(1) - ar)) + a0d) + alB * el);
                            }
                            C dbg, dbl;
                            beta_face<L>(q, cgB, clB, c0g, c0l, dbg, dbl);
                            Sg -= dbg;
                            Sl -= dbl;
                        }
                    }
                }
            }
        }

        if (ctl.write_diag) {
            int bad = 0;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int q = 0; q < Q; ++q) bad += !isfinite(f[s][q]);
            bad += !isfinite(Sg) + !isfinite(Sl);
            dsum[16] = double(bad);
        }

        __builtin_amdgcn_s_setprio(0);
        // ------------------------------------------------------- moments
        // the moments of E(r0) (Eqs. (40)-(41), (73)-(74)) plus those of the
        // residuals: sum_q w_q v_q = 0, sum_q w_q v_q v_q = c_s^2 I and the
        // third moment of the weights vanishes
        C sdeg = C(0), del = C(0), sag = a0d, sal = -a0d;
        C sug[D], sul[D], Jg[D], Jl[D], Pg[NPI], Pl[NPI];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            sug[a] = C(0);
            sul[a] = C(0);
            Jg[a] = a0 * ug0[a];
            Jl[a] = (C(1) - a0) * ul0[a];
        }
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
            for (int bb = a; bb < D; ++bb) {
                Pg[sym<D>(a, bb)] = a == bb ? third * de0 : C(0);
                Pl[sym<D>(a, bb)] = C(0);
            }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            sdeg += f[0][q];  // Eq. (40), deviation from 1
            del += f[1][q];
            sag += f[2][q];  // Eq. (73), deviation from alpha_r
            sal += f[3][q];  // deviation from 1 - alpha_r
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int ca = L::c[q][a];
                if (ca != 0) {  // Eqs. (41), (74)
                    sug[a] += ca * f[0][q];
                    sul[a] += ca * f[1][q];
                    Jg[a] += ca * f[2][q];
                    Jl[a] += ca * f[3][q];
                }
#pragma unroll
                for (int bb = a; bb < D; ++bb) {
                    const int cab = ca * L::c[q][bb];
                    if (cab != 0) {  // second moment minus c_s^2 I (sum_q w_q v v = c_s^2 I)
                        Pg[sym<D>(a, bb)] += cab * f[0][q];
                        Pl[sym<D>(a, bb)] += cab * f[1][q];
                    }
                }
            }
        }
        // The phase velocities and the gas density deviation are the
        // record's values plus the residual moments.  The sum is taken in
        // FP64 (exact for two FP32 terms); the step continues with its FP32
        // value, and the rounding remainder (eug, eul, ede) is kept in the
        // stored residuals (see the collisions), so that carrying u and
        // eps_g - 1 in the FP32 record loses nothing from step to step.
        using A = double;
        A ugA[D], ulA[D];
        C ug[D], ul[D], eug[D], eul[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            ugA[a] = A(ug0[a]) + A(sug[a]);
            ulA[a] = A(ul0[a]) + A(sul[a]);
            ug[a] = C(ugA[a]);
            ul[a] = C(ulA[a]);
            eug[a] = C(ugA[a] - A(ug[a]));
            eul[a] = C(ulA[a] - A(ul[a]));
        }
        const A degA = A(de0) + A(sdeg);
        const C deg = C(degA);
        const C ede = C(degA - A(deg));
        const C ag = ar + sag;               // raw zeroth moments
        const C al_raw = (C(1) - ar) + sal;

        // ------------------------------- Spalding renormalisation, Eq. (93)
        C alg, all, dag;  // dag = alpha_g - alpha_r
        if (p.renorm) {
            if (ag >= C(0) && ag <= C(1) && al_raw >= C(0) && al_raw <= C(1)) {
                // B is the identity: alpha_g = a_g / (a_g + a_l), written around
                // a_g + a_l = 1 so that FP32 keeps the small correction exactly
                const C e = sag + sal;  // a_g + a_l - 1
                const C corr = ag * e * rcp(C(1) + e);
                dag = sag - corr;
            } else {
                const C Bg = clamp01(ag), Bl = clamp01(al_raw);
                const C den = Bg + Bl;
                dag = (den > C(0) ? Bg * rcp(den) : C(0)) - ar;
            }
            // alpha_g from its deviation, the value the record carries (the
            // stored populations are relative to it)
            alg = ar + dag;
            all = C(1) - alg;
        } else {
            alg = ag;
            all = al_raw;
            dag = sag;
        }
        // alpha_l - (1 - alpha_r)
        const C dal = p.renorm ? -dag : sal;

        // ---------------------- sources, dashpots (Eqs. (128), (131)), lag
        C usg = C(0), usl = C(0);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            usg += ug[a] * ug[a];
            usl += ul[a] * ul[a];
        }
        const C R = C(p.R), invR = C(p.invR);
        const C dphiel = deg * invR;  // phi eps_l - 1 = (eps_g - 1)/R, Eq. (32)
        const C Spg = Sg - C(p.gamma) * usg * deg;
        const C Spl = Sl - C(p.gamma) * usl * dphiel;
        const C Lam = alg * all * (alg + all * R);  // Eq. (136)
        C S2g = Spg, S2l = Spl, Laml = Lam;
        if (p.use_lag) {
            Rec2<C>* lag = static_cast<Rec2<C>*>(b.lag);
            C* lagl = static_cast<C*>(b.lag_lam);
            if (ctl.refresh) {
                Rec2<C> r;
                r.v[0] = Spg;
                r.v[1] = Spl;
                *at(lag, (unsigned)node * (unsigned)sizeof(Rec2<C>)) = r;
                *at(lagl, cb) = Lam;
            } else {
                const Rec2<C> r = *at(lag, (unsigned)node * (unsigned)sizeof(Rec2<C>));
                S2g = r.v[0];
                S2l = r.v[1];
                Laml = *at(lagl, cb);
            }
        }

        // ---------------- volume-fraction gradient, Eqs. (91) and (94)
        C grad[D];
        const C og3 = C(3) * C(p.omega_ag), ol3 = C(3) * C(p.omega_al);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const C gg = og3 * (ag * ug[a] - Jg[a]);
            const C gl = ol3 * (al_raw * ul[a] - Jl[a]);
            grad[a] = C(0.5) * (gg - gl);  // grad alpha_g; grad alpha_l = -grad
        }

        // ------------------------------------------ stresses, Eq. (70)
        C sg[NPI], sl[NPI];
        {
            const C kg = C(1) - C(0.5) * C(p.omega_g), kl = C(1) - C(0.5) * C(p.omega_l);
            const C pg = third * C(p.psi_g) * C(0.5) * S2g, pl = third * C(p.psi_l) * C(0.5) * S2l;
#pragma unroll
            for (int a = 0; a < D; ++a) {
#pragma unroll
                for (int bb = a; bb < D; ++bb) {
                    const int k = sym<D>(a, bb);
                    const C dg = a == bb ? third * deg : C(0);
                    const C dl = a == bb ? third * dphiel : C(0);
                    sg[k] = kg * (dg + ug[a] * ug[bb] - Pg[k]) - (a == bb ? pg : C(0));
                    sl[k] = kl * (dl + ul[a] * ul[bb] - Pl[k]) - (a == bb ? pl : C(0));
                }
            }
        }

        // ------------------------------------------- forces, Eqs. (24), (26)
        const C agf = alg > C(p.alpha_min) ? alg : C(p.alpha_min);
        const C alf = all > C(p.alpha_min) ? all : C(p.alpha_min);
        C du[D], dun2 = C(0);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            du[a] = ul[a] - ug[a];
            dun2 += du[a] * du[a];
        }
        const C dun = root(dun2);
        const C uln = root(usl);
        const C K = p.cgw ? C(p.kappa_I) * Laml : C(p.K_I);
        C Gg[D], Gl[D];
        const C inv_agf = rcp(agf), inv_alf = rcp(alf), inv_alfR = inv_alf * invR;
        // slope limiter of sigma . grad(alpha) / alpha: |grad alpha_phi| is
        // capped at max(alpha_phi, alpha_min) per lattice spacing (a steeper
        // log-gradient is not resolved, and where the clamp of Eq. (93) has
        // emptied a phase the flux-based gradient would meet alpha_min), so
        // the factor grad / alpha becomes grad / |grad| there
        C kgg = inv_agf, kgl = inv_alf;
        if (p.sigma_grad) {
            C g2 = C(0);
#pragma unroll
            for (int a = 0; a < D; ++a) g2 += grad[a] * grad[a];
            if (g2 > agf * agf || g2 > alf * alf) {
                const C ig = rcp(root(g2));
                if (g2 > agf * agf) kgg = ig;
                if (g2 > alf * alf) kgl = ig;
            }
        }
#pragma unroll
        for (int a = 0; a < D; ++a) {
            C sgg = C(0), sgl = C(0);
            if (p.sigma_grad) {
#pragma unroll
                for (int bb = 0; bb < D; ++bb) {
                    sgg += sg[sym<D>(a, bb)] * grad[bb];
                    sgl -= sl[sym<D>(a, bb)] * grad[bb];
                }
                sgg = sgg * kgg;
                sgl = sgl * kgl;
            }
            const C bg = a == p.up ? C(p.b_g) : C(0);
            const C bl = a == p.up ? C(p.b_l) : C(0);
            Gg[a] = S2g * ug[a] + sgg + bg + K * dun * du[a] * inv_agf;
            Gl[a] = S2l * ul[a] + sgl + bl + (-K * dun * du[a] - C(p.K_W) * uln * ul[a]) * inv_alfR;
        }

        // ---------------------------------------------------- collisions
        T* pout = static_cast<T*>(b.pop_out);
        // the node's own block: plane descriptor, plus the block offset
        // (uniform across the wave) and the lane offset in the per-lane offset
        const __amdgpu_buffer_rsrc_t ro = rsrc(pout + (long long)z * p.plane);
        const long long oblk = ((long long)y * p.nxb + (x >> 6)) * kBlk;
        const unsigned vl = (unsigned)((x & 63) * 4 * (int)sizeof(T));
        {
            // BGK relaxation plus forcing, f* = f + omega (f^eq - f) + f^L,
            // stored as the residual f* - E_q(r) against this node's new
            // record r: with f = E_q(r0) + n_q,
            //   f* - E_q(r) = (1 - omega) [n_q + E_q(r0) - E_q(r)]
            //               + omega [f^eq_q - E_q(r)] + f^L_q,
            // where E_q(r0) - E_q(r) depends only on the differences between
            // the old and new record and f^eq - E(r) holds only the
            // second-order and rest-population parts plus the FP32 rounding
            // remainders of r -- every term is small, so neither the
            // arithmetic nor the storage rounds a large value.
            const C w0 = C(L::w[0]);
            const C k0 = (C(1) - w0) / w0;
            const C el0 = del + k0 * (del - dphiel);  // eps_l eta_0(phi) - 1, Eq. (38)
            const C eg0 = C(1) + k0 * (C(1) - C(p.psi_g));
            const C el0p = C(1) + k0 * (C(1) - C(p.psi_l));
            const C og = C(p.omega_g), ol = C(p.omega_l), oag = C(p.omega_ag), oal = C(p.omega_al);
            const C kog = C(1) - og, kol = C(1) - ol, koa = C(1) - oag, kob = C(1) - oal;
            // rest and non-rest parts of f^eq - E(r) and f^L, Eqs. (37), (42)
            const C Bg = S2g * C(p.psi_g), Bg0 = S2g * eg0;
            const C Bl = ol * dphiel + S2l * C(p.psi_l), Bl0 = ol * el0 + S2l * el0p;
            // old minus new record values
            const C dA = a0d - dag;
            const C alE = C(1) - alg;  // f_al reference of the new record
            const C xl = all - alE;    // 0 with the renormalisation
            // every direction-dependent term is linear in v_q apart from the
            // second-order equilibria: the per-set vectors V collect them
            // (the record differences, the rounding remainders and 3 F),
            // A the direction-independent parts
            const C Ag = kog * (de0 - deg) + og * ede, A2 = koa * dA, A3 = oal * xl - kob * dA;
            C Vg[D], Vl[D], V2[D], V3[D];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const C dug = ug0[a] - ug[a], dul = ul0[a] - ul[a];
                Vg[a] = C(3) * (kog * dug + og * eug[a] + Gg[a]);
                Vl[a] = C(3) * (kol * dul + ol * eul[a] + Gl[a]);
                V2[a] = C(3) * koa * (dA * ug0[a] + alg * dug);
                V3[a] = C(3) * (kob * (alE * dul - dA * ul0[a]) + oal * xl * ul[a]);
            }
            const C ogA = oag * alg, olA = oal * all;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const C wq = C(L::w[q]);
                const C cug = dotc<L>(q, ug), cul = dotc<L>(q, ul);
                const C qg = C(4.5) * cug * cug - C(1.5) * usg, ql = C(4.5) * cul * cul - C(1.5) * usl;
                const C o0 = kog * f[0][q] + wq * ((Ag + (q == 0 ? Bg0 : Bg)) + dotc<L>(q, Vg) + og * qg);
                const C o1 = kol * f[1][q] + wq * ((q == 0 ? Bl0 : Bl) + dotc<L>(q, Vl) + ol * ql);
                const C o2 = koa * f[2][q] + wq * (A2 + dotc<L>(q, V2) + ogA * qg);
                const C o3 = kob * f[3][q] + wq * (A3 + dotc<L>(q, V3) + olA * ql);
                const C o4[4] = {o0, o1, o2, o3};
                const unsigned vq = vl + (unsigned)((oblk + q * 256) * (long long)sizeof(T));
                Pop4<T>::template st<NTS ? kNT : 0>(ro, vq, 0u, o4, p, q == 0);
            }
        }

        // ------------ imposed-velocity record of the source schemes (Eq. (97))
        // and reference of the stored populations (rec_e)
        {
            Rec8<C> r;
            r.v[0] = dag;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                r.v[1 + a] = ug[a];
                r.v[1 + D + a] = ul[a];
            }
            r.v[kDe<D>] = deg;
            st_rec<D>(rsrc(b.cf_out), rb, r);
            if (!p.renorm) *at(static_cast<C*>(b.al_out), cb) = all;
        }

        // -------------------- side buffers for the next step's face values
        if constexpr (CH) {
            if (fa >= 0) {
                const int cf = co[fa];
                int side = -1, layer = 0;
                const bool lo_open = face_lo == EELBM_BC_INLET || face_lo == EELBM_BC_OUTLET;
                const bool hi_open = face_hi == EELBM_BC_INLET || face_hi == EELBM_BC_OUTLET;
                if (lo_open && cf <= 1) {
                    side = 0;
                    layer = cf;
                }
                if (hi_open && cf >= nn[fa] - 2) {
                    if (side < 0 || cf == nn[fa] - 1) {
                        side = 1;
                        layer = nn[fa] - 1 - cf;
                    }
                }
                if (side >= 0) {
                    C* so = static_cast<C*>(b.side_out);
                    auto put = [&](int v, C val) {
                        so[((long long)(side * 2 + layer) * NV + v) * p.face_n + fidx] = val;
                    };
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        put(a, ug[a]);
                        put(D + a, ul[a]);
                    }
                    put(2 * D, alg);
                    put(2 * D + 1, all);
                }
            }
        }

        // ------------------------------------------------ output fields
        if (ctl.write_macro) {
            double* m = b.macro;
            m[node] = double(alg);
            m[n + node] = double(all);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                m[(2 + a) * n + node] = double(ugA[a]);
                m[(2 + D + a) * n + node] = double(ulA[a]);
            }
            m[(2 + 2 * D) * n + node] = double(degA) / 3.0;
        }
        if (ctl.write_diag) {
            dsum[0] = double(ar) + double(sag);
            dsum[1] = (1.0 - double(ar)) + double(sal);
            dsum[2] = double(alg);
            dsum[3] = double(all);
            dsum[4] = double(degA);
            dsum[5] = double(del);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                dsum[6 + a] = double(ugA[a]);
                dsum[9 + a] = double(ulA[a]);
                dsum[12 + a] = p.rho_g * double(alg) * double(ugA[a]) + p.rho_l * double(all) * double(ulA[a]);
            }
            dsum[15] = double(dag) - double(sag);
        }
    }

    // ---------------- FP64 wavefront -> block reduction of the diagnostics
    if (ctl.write_diag) {
        __shared__ double red[kNDiag][4];
        // block sizes are whole wavefronts (checked on the host)
        const int tid = threadIdx.y * blockDim.x + threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int k = 0; k < kNDiag; ++k) {
            double v = dsum[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) red[k][wave] = v;
        }
        __syncthreads();
        if (tid < kNDiag) {
            const int nw = (blockDim.x * blockDim.y + 63) >> 6;
            double v = 0.0;
            for (int w = 0; w < nw; ++w) v += red[tid][w];
            b.partials[part * kNDiag + tid] = v;
        }
    }
}

// Single-lattice step: one workgroup per tile.  Workgroups are dispatched to
// the 8 XCDs round-robin; with the XCD remap, XCD k receives one contiguous
// run of tiles, so the rows a pull reads from neighbouring tiles are mostly
// already in that XCD's L2.
__device__ __forceinline__ long long xcd_tile(long long id, long long nb, int remap) {
    if (!remap) return id;
    const long long per = nb >> 3;
    return id < per * 8 ? (id & 7) * per + (id >> 3) : id;
}


// Waves per SIMD the compiler must leave room for.  The periodic D3Q19 FP16
// step needs 174 VGPRs (2 waves); held to 168 (3 waves) it spills 9 values
// to scratch and runs 5-8 % faster (128^3 / 256^3 columns).  The other D3Q19
// steps spill 32 (BF16), 71 (FP32) or more values at 168 and ran slower, the
// FP16 channel steps spill 41-61, and the D2Q9 steps fit 4 waves without
// the hint.
template <class L, class T, int BC>
constexpr int kMinWaves = (L::D == 3 && BC == kBcPeriodic && std::is_same<T, __half>::value) ? 3 : 1;

template <class L, class T, int BC, bool INIT, bool NTS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMinWaves<L, T, BC>)))
k_step(const KParams p, const KBuffers b, const KCtl ctl) {
    if constexpr (INIT) {
        // a gated rebuild: the whole grid skips it when the device flag is 0
        if (ctl.gate && *ctl.gate == 0) return;
    }
    step_body<L, T, BC, INIT, NTS>(p, b, ctl, xcd_tile(blockIdx.x, gridDim.x, p.xcd_remap), blockIdx.x);
}

// Batched step: one launch advances every lattice of a batch by one step.
// Work item w = (lattice, tile); each lattice brings its own parameters and
// both ping-pong buffer sets; the step's time is the batch clock + k + 1, so
// a captured sequence of launches replays correctly at any time.  count
// (device, NULL: the whole grid): only the first *count work items are
// taken -- the work list of the active lattices, compacted on the device
// before the steps -- so that the active lattices' tiles spread over all
// XCDs whatever lattices are left out; the other workgroups return at once.
template <class L, class T, int BC, bool NTS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kMinWaves<L, T, BC>)))
k_step_batch(const BatchLattice* lat, const uint2* work, const long long* clock, int k, int write_last,
             const int* count) {
    const long long nb = count ? (long long)*count : (long long)gridDim.x;
    if ((long long)blockIdx.x >= nb) return;
    const uint2 w = work[xcd_tile(blockIdx.x, nb, 1)];
    const BatchLattice& d = lat[w.x];
    const KParams p = d.p;
    KCtl c;
    c.t = *clock + k + 1;
    c.refresh = c.t % p.n_gamma == 0;
    c.write_macro = write_last;
    c.write_diag = write_last;
    c.gate = nullptr;
    const KBuffers bb = d.buf[(c.t - 1) & 1];
    step_body<L, T, BC, false, NTS>(p, bb, c, w.y, w.y);
}

__global__ void k_clock_add(long long* clock, long long add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) clock[0] += add;
}

// Work list of the active lattices of a batch: aoff[i] = first position of
// lattice i's tiles in the compacted list (the tiles of the active lattices
// before it), *count = all active tiles.  moff[i] .. moff[i + 1] are lattice
// i's positions in the full list.  One thread (a few hundred lattices).
__global__ void k_batch_active_prefix(const int* __restrict__ active, const int* __restrict__ moff, int n,
                                      int* __restrict__ aoff, int* __restrict__ count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int s = 0;
        for (int i = 0; i < n; ++i) {
            aoff[i] = s;
            if (active[i]) s += moff[i + 1] - moff[i];
        }
        *count = s;
    }
}
__global__ void k_batch_active_copy(const int* __restrict__ active, const int* __restrict__ moff,
                                    const int* __restrict__ aoff, const uint2* __restrict__ work, long long nwork,
                                    uint2* __restrict__ awork) {
    for (long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x; j < nwork;
         j += (long long)gridDim.x * blockDim.x) {
        const uint2 w = work[j];
        if (active[w.x]) awork[aoff[w.x] + (j - moff[w.x])] = w;
    }
}

// ---------------------------------------------------- small reductions
__global__ void __launch_bounds__(256) k_block_sum(const double* x, long long n, double* partials) {
    __shared__ double red[256];
    double v = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        v += x[i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// column sums of a [nrows][ncols] array in a fixed order (deterministic)
__global__ void __launch_bounds__(256) k_col_sum(const double* a, int nrows, int ncols, double* out) {
    __shared__ double red[256];
    for (int c = 0; c < ncols; ++c) {
        double v = 0.0;
        for (int r = threadIdx.x; r < nrows; r += blockDim.x) v += a[(long long)r * ncols + c];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = red[0];
        __syncthreads();
    }
}

// Diagnostics finalize, first pass: workgroup g sums the rows
// [g * chunk, (g + 1) * chunk) of the [nrows][kNDiag] block partials, each
// thread a fixed subset of rows into registers (a row is 18 consecutive
// doubles, so neighbouring threads read neighbouring rows), then a fixed
// LDS tree per column.  Second pass: one workgroup sums the workgroup rows in
// order.  The result depends only on nrows: bitwise reproducible.
__global__ void __launch_bounds__(256) k_diag_rows(const double* a, int nrows, int chunk, double* out2) {
    __shared__ double red[kNDiag][256];
    const int r0 = blockIdx.x * chunk;
    const int r1 = min(r0 + chunk, nrows);
    double acc[kNDiag];
#pragma unroll
    for (int c = 0; c < kNDiag; ++c) acc[c] = 0.0;
    for (int r = r0 + (int)threadIdx.x; r < r1; r += blockDim.x) {
        const double* row = a + (long long)r * kNDiag;
#pragma unroll
        for (int c = 0; c < kNDiag; ++c) acc[c] += row[c];
    }
#pragma unroll
    for (int c = 0; c < kNDiag; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < kNDiag; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        }
        __syncthreads();
    }
    if ((int)threadIdx.x < kNDiag) out2[(long long)blockIdx.x * kNDiag + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(64) k_diag_final(const double* out2, int g, double* out) {
    if ((int)threadIdx.x < kNDiag) {
        double v = 0.0;
        for (int k = 0; k < g; ++k) v += out2[(long long)k * kNDiag + threadIdx.x];
        out[threadIdx.x] = v;
    }
}

__global__ void __launch_bounds__(256) k_convert(const double* src, void* dst, int dtype, long long n, double add,
                                                 double scale) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double v = src[i] * scale + add;
        if (dtype == EELBM_DTYPE_F64)
            static_cast<double*>(dst)[i] = v;
        else
            static_cast<float*>(dst)[i] = float(v);
    }
}

// ------------------------------------------------------------ launchers
// LDS bytes of the staged record window of a tile (0: records read from
// memory -- the initial step and FP64 compute)
template <class L, class T, bool INIT>
static unsigned window_bytes(dim3 bl) {
    if (INIT || sizeof(typename Compute<T>::C) != 4) return 0u;
    return (bl.x + 2) * (bl.y + 2) * (L::D == 3 ? 3u : 1u) * (unsigned)sizeof(Rec8<float>);
}

template <class L, class T, int BC, bool INIT, bool NTS = false>
static hipError_t go(const KParams& p, const KBuffers& b, const KCtl& c, dim3 g, dim3 bl, hipStream_t s) {
    const unsigned lds = window_bytes<L, T, INIT>(bl);
    hipLaunchKernelGGL((k_step<L, T, BC, INIT, NTS>), g, bl, lds, s, p, b, c);
    return hipGetLastError();
}

// the initial step (the standard column's uses the generic channel
// instantiation); every later step of a lattice runs one instantiation
template <class L, class T, int BC>
static hipError_t go3(bool init, const KParams& p, const KBuffers& b, const KCtl& c, dim3 g, dim3 bl,
                      hipStream_t s) {
    if (init) return go<L, T, BC == kBcColumn ? kBcGeneric : BC, true>(p, b, c, g, bl, s);
    // a lattice whose populations exceed the last-level cache stores them
    // with the nontemporal hint
    return p.nt_store ? go<L, T, BC, false, true>(p, b, c, g, bl, s) : go<L, T, BC, false, false>(p, b, c, g, bl, s);
}

template <class L, class T>
static hipError_t go2(int bc, bool init, const KParams& p, const KBuffers& b, const KCtl& c, dim3 g, dim3 bl,
                      hipStream_t s) {
    switch (bc) {
        case kBcPeriodic: return go3<L, T, kBcPeriodic>(init, p, b, c, g, bl, s);
        case kBcGeneric: return go3<L, T, kBcGeneric>(init, p, b, c, g, bl, s);
        case kBcColumn: return go3<L, T, kBcColumn>(init, p, b, c, g, bl, s);
    }
    return hipErrorInvalidValue;
}

template <class L>
static hipError_t go1(int storage, int bc, bool init, const KParams& p, const KBuffers& b, const KCtl& c, dim3 g,
                      dim3 bl, hipStream_t s) {
    switch (storage) {
        case EELBM_FP64: return go2<L, double>(bc, init, p, b, c, g, bl, s);
        case EELBM_FP32: return go2<L, float>(bc, init, p, b, c, g, bl, s);
        case EELBM_FP32_F64: return go2<L, F32D>(bc, init, p, b, c, g, bl, s);
        case EELBM_MIXED: return go2<L, Mix12>(bc, init, p, b, c, g, bl, s);
        case EELBM_FP16: return go2<L, __half>(bc, init, p, b, c, g, bl, s);
        case EELBM_BF16: return go2<L, __hip_bfloat16>(bc, init, p, b, c, g, bl, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(int lattice, int storage, int bc, bool init, const KParams& p, const KBuffers& b,
                       const KCtl& c, dim3 grid, dim3 block, hipStream_t s) {
    if (lattice == EELBM_D2Q9) return go1<D2Q9>(storage, bc, init, p, b, c, grid, block, s);
    if (lattice == EELBM_D3Q19) return go1<D3Q19>(storage, bc, init, p, b, c, grid, block, s);
    return hipErrorInvalidValue;
}

template <class L, class T, bool NTS>
static hipError_t gob_out(int bc, const BatchLattice* lat, const uint2* work, long long nwork,
                          const long long* clock, int k, int write_last, const int* count, dim3 block,
                          hipStream_t s) {
    const dim3 g((unsigned)nwork);
    const unsigned lds = window_bytes<L, T, false>(block);
    switch (bc) {
        case kBcPeriodic:
            hipLaunchKernelGGL((k_step_batch<L, T, kBcPeriodic, NTS>), g, block, lds, s, lat, work, clock, k, write_last, count);
            break;
        case kBcGeneric:
            hipLaunchKernelGGL((k_step_batch<L, T, kBcGeneric, NTS>), g, block, lds, s, lat, work, clock, k, write_last, count);
            break;
        case kBcColumn:
            hipLaunchKernelGGL((k_step_batch<L, T, kBcColumn, NTS>), g, block, lds, s, lat, work, clock, k, write_last, count);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class L, class T>
static hipError_t gob(int bc, bool nts, const BatchLattice* lat, const uint2* work, long long nwork,
                      const long long* clock, int k, int write_last, const int* count, dim3 block, hipStream_t s) {
    if (nts) return gob_out<L, T, true>(bc, lat, work, nwork, clock, k, write_last, count, block, s);
    return gob_out<L, T, false>(bc, lat, work, nwork, clock, k, write_last, count, block, s);
}

template <class L>
static hipError_t gob1(int storage, int bc, bool nts, const BatchLattice* lat, const uint2* work, long long nwork,
                       const long long* clock, int k, int write_last, const int* count, dim3 block, hipStream_t s) {
    switch (storage) {
        case EELBM_FP64: return gob<L, double>(bc, nts, lat, work, nwork, clock, k, write_last, count, block, s);
        case EELBM_FP32: return gob<L, float>(bc, nts, lat, work, nwork, clock, k, write_last, count, block, s);
        case EELBM_FP16: return gob<L, __half>(bc, nts, lat, work, nwork, clock, k, write_last, count, block, s);
        case EELBM_BF16:
            return gob<L, __hip_bfloat16>(bc, nts, lat, work, nwork, clock, k, write_last, count, block, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batch_step(int lattice, int storage, int bc, bool nts, const BatchLattice* lat, const uint2* work,
                             long long nwork, const long long* clock, int k, int write_last, const int* count,
                             dim3 block, hipStream_t s) {
    if (lattice == EELBM_D2Q9)
        return gob1<D2Q9>(storage, bc, nts, lat, work, nwork, clock, k, write_last, count, block, s);
    if (lattice == EELBM_D3Q19)
        return gob1<D3Q19>(storage, bc, nts, lat, work, nwork, clock, k, write_last, count, block, s);
    return hipErrorInvalidValue;
}

hipError_t launch_batch_compact(const int* active, const int* moff, int n, int* aoff, int* count, const uint2* work,
                                long long nwork, uint2* awork, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_active_prefix, dim3(1), dim3(64), 0, s, active, moff, n, aoff, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    long long g = (nwork + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_batch_active_copy, dim3((unsigned)(g < 1 ? 1 : g)), dim3(256), 0, s, active, moff, aoff,
                       work, nwork, awork);
    return hipGetLastError();
}

hipError_t launch_clock_add(long long* clock, long long add, hipStream_t s) {
    hipLaunchKernelGGL(k_clock_add, dim3(1), dim3(64), 0, s, clock, add);
    return hipGetLastError();
}

hipError_t launch_sum(const double* x, long long n, double* partials, int nblocks, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_block_sum, dim3(nblocks), dim3(256), 0, s, x, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_col_sum, dim3(1), dim3(256), 0, s, partials, nblocks, 1, out);
    return hipGetLastError();
}

hipError_t launch_diag_finalize(const double* partials, int nblocks, double* scratch, double* out, hipStream_t s) {
    if (nblocks < 1) return hipErrorInvalidValue;
    int g = (nblocks + kDiagRowsPerGroup - 1) / kDiagRowsPerGroup;
    if (g > kDiagGroups) g = kDiagGroups;
    const int chunk = (nblocks + g - 1) / g;
    hipLaunchKernelGGL(k_diag_rows, dim3(g), dim3(256), 0, s, partials, nblocks, chunk, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, scratch, g, out);
    return hipGetLastError();
}

hipError_t launch_convert(const double* src, void* dst, int dst_dtype, long long n, double add, double scale,
                          hipStream_t s) {
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_convert, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, dst_dtype, n, add, scale);
    return hipGetLastError();
}

}  // namespace eelbm
