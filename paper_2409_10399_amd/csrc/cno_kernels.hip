// HIP kernels of the learned surrogate: a convolutional neural operator
// (U-Net of 3x3 convolutions, 2x2 average pooling, nearest 2x upsampling,
// skip concatenations, leaky-ReLU) that maps the macroscopic fields of a D2Q9
// channel to their change over a fixed number of LBM steps.
//
// Tensors are NHWC, FP32 in memory; every channel count is a multiple of 16.
// A 3x3 convolution is an implicit GEMM, M = pixels, N = output channels,
// K = 9 * input channels ordered (tap, channel), evaluated with the 16x16x16
// BF16 matrix-core instruction and FP32 accumulation: each wavefront owns 16
// consecutive pixels of one image row and all output channels of its N-tile
// group; operands are converted to BF16 as they are loaded.  Operand layout
// of v_mfma_f32_16x16x16_bf16 (lane l, element t = 0..3):
//   A[m = l % 16][k = 4 (l / 16) + t],  B[k = 4 (l / 16) + t][n = l % 16],
//   D[m = 4 (l / 16) + t][n = l % 16].
// Weights: master FP32 W[tap][ci][co]; the forward pass reads the BF16 copy
// Wf[co][tap][ci] and the input-gradient pass the BF16 copy Wd[ci][8 - tap][co],
// so that the four K-consecutive values a lane needs are adjacent.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <atomic>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "eelbm.h"
#include "eelbm_internal.hpp"

namespace cno {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_bits(float f) {
    const unsigned u = __builtin_bit_cast(unsigned, f);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short h) { return __builtin_bit_cast(float, (unsigned)h << 16); }

// four FP32 values to BF16 (round to nearest even) with the packed hardware
// conversion of gfx950
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ s16x4 pack4(const f32x4& v) {
    return __builtin_bit_cast(s16x4, __builtin_convertvector(v, bf16x4));
}

__device__ __forceinline__ f32x4 mfma(const s16x4& a, const s16x4& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}


// --------------------------------------------------------------- forward
// out[b, y, x, co] = bias[co] + sum_{tap, ci} in[b, y + dy, x + dx, ci] Wf[co][tap][ci]
// (zero padding), then leaky-ReLU with slope `slope` if act != 0.
//
// A workgroup of four wavefronts owns kRows output rows (one per wavefront)
// x 16 MT pixels x 16 NT output channels.  The K loop runs over chunks of 32
// input channels; for each chunk the workgroup stages in LDS, as BF16,
//   * the input window: kRows + 2 rows x 16 MT + 2 pixels x 32 channels (zero
//     outside the image and beyond the input channels),
//   * the weights: 9 taps x 16 NT output channels x 32 input channels,
// and every wavefront takes its operands of the nine taps from there (one
// 16-byte LDS read per M-tile and per N-tile and tap) into the 16x16x32 BF16
// matrix-core instruction of gfx950.  All global loads of a chunk are issued
// together, and those of the next chunk are in flight while the current one
// is multiplied (one LDS buffer, refilled between two barriers).  Operand
// layout of v_mfma_f32_16x16x32_bf16 (lane l, element t):
//   A[m = l % 16][k = 8 (l / 16) + t] (t < 8),  B[k = 8 (l / 16) + t][n = l % 16] (t < 8),
//   D[m = 4 (l / 16) + t][n = l % 16] (t < 4).
// The input may be the concatenation [src0 | src1] along channels, and src0
// may be read with nearest 2x upsampling from an image of half the size (the
// decoder's upsampling and skip concatenation, fused into the load).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f32x4 mfma32(const bf16x8& a, const bf16x8& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
constexpr int kRows = 4;  // output rows of a workgroup, one per wavefront
constexpr int kKc = 32;   // input channels per staged chunk
constexpr int kPix = 40;  // LDS stride of one staged pixel or weight row in BF16 values (32 + 8 padding: 80 bytes)

template <int MT, int NT>
struct ConvTile {
    static constexpr int TW = 16 * MT;                    // output pixels of a row in the tile
    static constexpr int LW = TW + 2;                     // staged pixels of a row
    static constexpr int kA = (kRows + 2) * LW * (kKc / 4);  // 4-channel groups of the input window
    static constexpr int kAi = (kA + 255) / 256;          // ... per thread
    static constexpr int kB = 9 * 16 * NT * (kKc / 8);    // 8-channel groups of the weights
    static constexpr int kBi = (kB + 255) / 256;
    static constexpr int kLdsA = (kRows + 2) * LW * kPix;  // BF16 values
    static constexpr int kLdsB = 9 * 16 * NT * kPix;
};

// Activation storage: FP32, or BF16 (the bits of the rounded value; the
// products round their operands to BF16 anyway, so a BF16 activation between
// two convolutions is the value the next one would have used).
struct ActF32 {
    using S = float;
    using V = f32x4;  // four channels as loaded
};
struct ActBF16 {
    using S = unsigned short;
    using V = uint2;
};

template <int MT, int NT, class AI, class AO>
__global__ void __launch_bounds__(256) k_conv2(const typename AI::S* __restrict__ src0, int C0, int up0,
                                              const typename AI::S* __restrict__ src1, int C1, int B, int H, int W,
                                              const unsigned short* __restrict__ wf, const float* __restrict__ bias,
                                              int Cout, typename AO::S* __restrict__ out, int act, float slope) {
    constexpr bool kInBf16 = std::is_same<AI, ActBF16>::value;
    constexpr bool kOutBf16 = std::is_same<AO, ActBF16>::value;
    using T = ConvTile<MT, NT>;
    constexpr int LW = T::LW;
    __shared__ __attribute__((aligned(16))) unsigned short atile[T::kLdsA];
    __shared__ __attribute__((aligned(16))) unsigned short btile[T::kLdsB];
    const int Cin = C0 + C1;
    const int K = 9 * Cin;
    const int nch = (Cin + kKc - 1) / kKc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int gx = (W + T::TW - 1) / T::TW, gy = (H + kRows - 1) / kRows;
    const int ntiles = B * gx * gy;  // < 2^24 (host check)
    const int n0 = blockIdx.y * 16 * NT;  // the host launches Cout / (16 NT) groups exactly
    const int Hs = up0 ? H / 2 : H, Ws = up0 ? W / 2 : W;
    const int kh = 8 * (lane >> 4);  // this lane's K offset within a chunk

    typename AI::V av[T::kAi];
    u32x4 bv[T::kBi];
    // this thread's pixels of the staged window (tile-invariant): pixel
    // (e >> 3) of the window, e = threadIdx.x + 256 i, as ly << 16 | lx
    int lxy[T::kAi];
#pragma unroll
    for (int i = 0; i < T::kAi; ++i) {
        const int pix = (int)(threadIdx.x >> 3) + 32 * i;
        lxy[i] = (pix / LW) << 16 | (pix % LW);
    }
    const int g4 = 4 * (int)(threadIdx.x & 7);  // this thread's channel group within a chunk
    // tile coordinates, advanced by gridDim.x tiles at a time without
    // division: G = gridDim.x = (Gb gy + Gy) gx + Gx
    const int G = (int)gridDim.x;
    const int Gx = G % gx, Gy = (G / gx) % gy, Gb = G / (gx * gy);
    struct TileXY {
        int x, y, b;
    };
    auto next_tile = [&](TileXY t) {
        t.x += Gx;
        int cy = 0;
        if (t.x >= gx) {
            t.x -= gx;
            cy = 1;
        }
        t.y += Gy + cy;
        int cb = 0;
        if (t.y >= gy) {
            t.y -= gy;
            cb = 1;
        }
        t.b += Gb + cb;
        return t;
    };
    // issue every global load of chunk c0 of tile t (the values land in av
    // and, if withb, bv); element offsets fit in 32 bits (host check)
    auto load = [&](TileXY t, int c0, bool withb) {
        const int x0 = t.x * T::TW - 1, y0 = t.y * kRows - 1;
        const int c = c0 + g4;
        const bool in0 = c < C0, inc = c < Cin;
        const typename AI::S* base = in0 ? src0 + c : (inc ? src1 + (c - C0) : src0);
        const int cs = in0 ? C0 : C1;
#pragma unroll
        for (int i = 0; i < T::kAi; ++i) {
            const int e = (int)threadIdx.x + 256 * i;
            const int yy = y0 + (lxy[i] >> 16), xx = x0 + (lxy[i] & 0xffff);
            av[i] = typename AI::V{};
            if ((T::kA % 256 == 0 || i + 1 < T::kAi || e < T::kA) && (unsigned)yy < (unsigned)H &&
                (unsigned)xx < (unsigned)W && inc) {
                const int q = (in0 && up0) ? (t.b * Hs + (yy >> 1)) * Ws + (xx >> 1) : (t.b * H + yy) * W + xx;
                av[i] = *reinterpret_cast<const typename AI::V*>(base + q * cs);
            }
        }
        if (!withb) return;
#pragma unroll
        for (int i = 0; i < T::kBi; ++i) {
            const int e = threadIdx.x + 256 * i;
            const int g = e & 3, rr = e >> 2;  // rr = tap * 16 NT + column
            const int tap = rr / (16 * NT), col = rr % (16 * NT);
            const int k = c0 + 8 * g;
            bv[i] = u32x4{0u, 0u, 0u, 0u};
            if (e < T::kB && k < Cin)
                bv[i] = *reinterpret_cast<const u32x4*>(wf + (n0 + col) * K + tap * Cin + k);
        }
    };
    // write the loaded chunk to LDS
    auto store = [&](bool withb) {
#pragma unroll
        for (int i = 0; i < T::kAi; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (e < T::kA) {
                if constexpr (kInBf16)
                    *reinterpret_cast<uint2*>(atile + (e >> 3) * kPix + 4 * (e & 7)) = av[i];
                else
                    *reinterpret_cast<s16x4*>(atile + (e >> 3) * kPix + 4 * (e & 7)) = pack4(av[i]);
            }
        }
        if (!withb) return;
#pragma unroll
        for (int i = 0; i < T::kBi; ++i) {
            const int e = threadIdx.x + 256 * i;
            if (e < T::kB) *reinterpret_cast<u32x4*>(btile + (e >> 2) * kPix + 8 * (e & 3)) = bv[i];
        }
    };

    // Each workgroup takes tiles blockIdx.x, blockIdx.x + gridDim.x, ...; the
    // loads of the next (tile, chunk) are in flight while the current one is
    // multiplied.  With a single chunk the weights stay in LDS for all tiles.
    int tile = blockIdx.x, ch = 0;
    if (tile >= ntiles) return;
    TileXY cur{tile % gx, (tile / gx) % gy, tile / (gx * gy)};
    load(cur, 0, true);
    f32x4 acc[MT][NT];
    for (bool first = true;; first = false) {
        if (ch == 0) {
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        __syncthreads();  // the previous chunk's LDS reads are done
        store(nch > 1 || first);
        __syncthreads();
        int ntile = tile, nc = ch + 1;
        TileXY nxt = cur;
        if (nc == nch) {
            nc = 0;
            ntile += G;
            nxt = next_tile(cur);
        }
        const bool more = ntile < ntiles;
        if (more) load(nxt, nc * kKc, nch > 1);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
            bf16x8 a[MT], bw[NT];
#pragma unroll
            for (int m = 0; m < MT; ++m)
                a[m] = *reinterpret_cast<const bf16x8*>(atile + ((wave + dy) * LW + 16 * m + (lane & 15) + dx) * kPix + kh);
#pragma unroll
            for (int j = 0; j < NT; ++j)
                bw[j] = *reinterpret_cast<const bf16x8*>(btile + (tap * 16 * NT + 16 * j + (lane & 15)) * kPix + kh);
#pragma unroll
            for (int j = 0; j < NT; ++j)
#pragma unroll
                for (int m = 0; m < MT; ++m) acc[m][j] = mfma32(a[m], bw[j], acc[m][j]);
        }
        if (ch == nch - 1) {
            const int y = cur.y * kRows + wave;
            if (y < H) {
                const int px0 = cur.x * T::TW + 4 * (lane >> 4);
                const int row = ((cur.b * H + y) * W + px0) * Cout + n0 + (lane & 15);
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const float bc = bias ? bias[n0 + 16 * j + (lane & 15)] : 0.f;
#pragma unroll
                    for (int m = 0; m < MT; ++m) {
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            float v = acc[m][j][t] + bc;
                            v = (act && v < 0.f) ? slope * v : v;
                            if (px0 + 16 * m + t < W) {
                                const int o = row + (16 * m + t) * Cout + 16 * j;
                                if constexpr (kOutBf16)
                                    out[o] = bf16_bits(v);
                                else
                                    out[o] = v;
                            }
                        }
                    }
                }
            }
        }
        cur = nxt;
        if (!more) break;
        tile = ntile;
        ch = nc;
    }
}

// ----------------------------------------------------- gradient wrt input
// din[b, y, x, ci] = sum_{tap, co} dout[b, y - dy, x - dx, co] W[tap][ci][co]
//                  = sum_{tap', co} dout[b, y + dy', x + dx', co] Wd[ci][tap'][co]
// with the taps reversed (tap' = 8 - tap, dy' = -dy, dx' = -dx): a forward
// convolution of dout with Wd, run by k_conv2.

// ---------------------------------------------------- gradient wrt weights
// part[z][tap][ci][co] = sum_p in[p + d_tap][ci] dout[p][co] over chunk z of
// `chunk` pixels (M = (tap, ci), N = co, K = pixels); one wavefront per
// 16 x 16 tile of dW and chunk.  k_sum_parts then adds the chunks in their
// order, so the gradient does not depend on the launch (no atomics).
__global__ void __launch_bounds__(64) k_conv_bwd_weight(const float* __restrict__ in, const float* __restrict__ dout,
                                                       int B, int H, int W, int Cin, int Cout, int chunk,
                                                       float* __restrict__ part) {
    const int lane = threadIdx.x;
    const int mt = blockIdx.x;  // M tile over 9 * Cin
    const int nt = blockIdx.y;  // N tile over Cout
    const int P = B * H * W;    // < 2^31 (host check)
    const int p0 = blockIdx.z * chunk;
    const int m = mt * 16 + (lane & 15);
    const int tap = m / Cin, ci = m - tap * Cin;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int co = nt * 16 + (lane & 15);
    const int kq = 4 * (lane >> 4);
    // image coordinates of this lane's four pixels p = pk + kq + t, advanced
    // by 16 pixels per step (no division in the loop)
    int px[4], py[4], pb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int p = p0 + kq + t;
        px[t] = p % W;
        const int r = p / W;
        py[t] = r % H;
        pb[t] = r / H;
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int pend = min(p0 + chunk, P);
    for (int pk = p0; pk < pend; pk += 16) {
        f32x4 av, bv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int p = pk + kq + t;
            const int yy = py[t] + dy, xx = px[t] + dx;
            const bool okp = p < pend;
            const bool ok = okp && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
            const long long src = ok ? ((long long)pb[t] * H + yy) * W + xx : 0;
            const float a = in[src * Cin + ci];
            const float bb = dout[(long long)(okp ? p : 0) * Cout + co];
            av[t] = ok ? a : 0.f;
            bv[t] = okp ? bb : 0.f;
            px[t] += 16;
            while (px[t] >= W) {
                px[t] -= W;
                if (++py[t] == H) {
                    py[t] = 0;
                    ++pb[t];
                }
            }
        }
        acc = mfma(pack4(av), pack4(bv), acc);
    }
    float* pz = part + (long long)blockIdx.z * 9 * Cin * Cout;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int mm = mt * 16 + 4 * (lane >> 4) + t;  // row of D
        pz[(long long)mm * Cout + co] = acc[t];
    }
}

__global__ void k_bias_grad(const float* __restrict__ dout, long long P, int C, float* __restrict__ part) {
    // one workgroup per 256-pixel chunk, one thread per channel (C <= 256):
    // part[chunk][c]
    const int c = threadIdx.x;
    if (c >= C) return;
    const long long p0 = (long long)blockIdx.x * 256;
    float s = 0.f;
    for (long long p = p0; p < p0 + 256 && p < P; ++p) s += dout[p * C + c];
    part[(long long)blockIdx.x * C + c] = s;
}

// acc[i] += sum_z part[z][i], z in order
__global__ void k_sum_parts(const float* __restrict__ part, int nz, long long n, float* __restrict__ acc) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < nz; ++z) s += part[(long long)z * n + i];
        acc[i] += s;
    }
}

__global__ void k_act_bwd(const float* __restrict__ y, const float* __restrict__ dy, long long n, float slope,
                          float* __restrict__ dx) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dx[i] = y[i] > 0.f ? dy[i] : slope * dy[i];
}

// 2x2 average pooling, (B, H, W, C) -> (B, H/2, W/2, C)
__global__ void k_pool_fwd(const float* __restrict__ in, int B, int H, int W, int C, float* __restrict__ out) {
    const long long n = (long long)B * (H / 2) * (W / 2) * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        long long r = i / C;
        const int x = (int)(r % (W / 2));
        r /= (W / 2);
        const int y = (int)(r % (H / 2));
        const int b = (int)(r / (H / 2));
        const float* s = in + (((long long)b * H + 2 * y) * W + 2 * x) * C + c;
        out[i] = 0.25f * (s[0] + s[C] + s[(long long)W * C] + s[(long long)W * C + C]);
    }
}
// the same pooling of BF16 activations (sum in FP32 in the order above,
// rounded to BF16)
__global__ void k_pool_fwd_bf16(const unsigned short* __restrict__ in, int B, int H, int W, int C,
                                unsigned short* __restrict__ out) {
    const long long n = (long long)B * (H / 2) * (W / 2) * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        long long r = i / C;
        const int x = (int)(r % (W / 2));
        r /= (W / 2);
        const int y = (int)(r % (H / 2));
        const int b = (int)(r / (H / 2));
        const unsigned short* s = in + (((long long)b * H + 2 * y) * W + 2 * x) * C + c;
        out[i] = bf16_bits(0.25f * (bf16_float(s[0]) + bf16_float(s[C]) + bf16_float(s[(long long)W * C]) +
                                    bf16_float(s[(long long)W * C + C])));
    }
}
__global__ void k_pool_bwd(const float* __restrict__ dout, int B, int H, int W, int C, float* __restrict__ din) {
    const long long n = (long long)B * H * W * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        long long r = i / C;
        const int x = (int)(r % W);
        r /= W;
        const int y = (int)(r % H);
        const int b = (int)(r / H);
        din[i] = 0.25f * dout[(((long long)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c];
    }
}
// nearest 2x upsampling, (B, H, W, C) -> (B, 2H, 2W, C)
__global__ void k_up_fwd(const float* __restrict__ in, int B, int H, int W, int C, float* __restrict__ out) {
    const long long n = (long long)B * 2 * H * 2 * W * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        long long r = i / C;
        const int x = (int)(r % (2 * W));
        r /= (2 * W);
        const int y = (int)(r % (2 * H));
        const int b = (int)(r / (2 * H));
        out[i] = in[(((long long)b * H + y / 2) * W + x / 2) * C + c];
    }
}
__global__ void k_up_bwd(const float* __restrict__ dout, int B, int H, int W, int C, float* __restrict__ din) {
    const long long n = (long long)B * H * W * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        long long r = i / C;
        const int x = (int)(r % W);
        r /= W;
        const int y = (int)(r % H);
        const int b = (int)(r / H);
        const long long W2 = 2LL * W;
        const float* s = dout + (((long long)b * 2 * H + 2 * y) * W2 + 2 * x) * C + c;
        din[i] = s[0] + s[C] + s[W2 * C] + s[W2 * C + C];
    }
}
// channel concatenation [a | b] and its split, P pixels
__global__ void k_concat(const float* __restrict__ a, int Ca, const float* __restrict__ b, int Cb, long long P,
                         float* __restrict__ out) {
    const int C = Ca + Cb;
    const long long n = P * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long p = i / C;
        const int c = (int)(i - p * C);
        out[i] = c < Ca ? a[p * Ca + c] : b[p * Cb + (c - Ca)];
    }
}
__global__ void k_split_add(const float* __restrict__ d, int Ca, int Cb, long long P, float* __restrict__ da,
                            float* __restrict__ db) {
    // da = d[:, :Ca] (overwrite), db += d[:, Ca:] (the skip branch already holds a gradient)
    const int C = Ca + Cb;
    const long long n = P * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long p = i / C;
        const int c = (int)(i - p * C);
        if (c < Ca)
            da[p * Ca + c] = d[i];
        else
            db[p * Cb + (c - Ca)] += d[i];
    }
}

// mean squared error over the first Cu of C channels: partial sums per
// workgroup (FP64) and the gradient 2 (pred - target) / count
__global__ void k_mse(const float* __restrict__ pred, const float* __restrict__ target, long long P, int C, int Cu,
                      double* __restrict__ partial, float* __restrict__ dpred) {
    __shared__ double red[256];
    const double inv = 1.0 / ((double)P * Cu);
    double s = 0.0;
    const long long n = P * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        float g = 0.f;
        if (c < Cu) {
            const double d = (double)pred[i] - (double)target[i];
            s += d * d;
            g = (float)(2.0 * d * inv);
        }
        if (dpred) dpred[i] = g;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] * inv;
}

// total of the per-workgroup partial sums, in index order (one thread: the
// result does not depend on the launch)
__global__ void k_sum_in_order(const double* __restrict__ partial, int n, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += partial[i];
        *out = s;
    }
}

// Adam on the FP32 master weights W[tap][ci][co] (n = 9 Cin Cout) and biases,
// then the two BF16 operand copies Wf[co][tap][ci] and Wd[ci][tap][co]
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1, float c2,
                       float wdecay) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wdecay * w[i]);
    }
}
__global__ void k_pack_weights(const float* __restrict__ w, int Cin, int Cout, unsigned short* __restrict__ wf,
                               unsigned short* __restrict__ wd) {
    const long long n = 9LL * Cin * Cout;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int co = (int)(i % Cout);
        const long long r = i / Cout;
        const int ci = (int)(r % Cin);
        const int tap = (int)(r / Cin);
        const unsigned short h = bf16_bits(w[i]);
        wf[((long long)co * 9 + tap) * Cin + ci] = h;
        wd[((long long)ci * 9 + (8 - tap)) * Cout + co] = h;
    }
}

// network input from stacked field planes soa[b][f][p] (f < nf): the
// normalised fields, then nc per-image conditioning values, zero padding to C
__global__ void k_pack(const float* __restrict__ soa, long long P, int nf, const float* __restrict__ mean,
                       const float* __restrict__ inv_scale, const float* __restrict__ cond, int nc, int B, int C,
                       float clip, float* __restrict__ out) {
    const long long n = (long long)B * P * C;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(i % C);
        const long long bp = i / C;
        const long long p = bp % P;
        const int b = (int)(bp / P);
        float v = 0.f;
        if (c < nf) {
            v = (soa[((long long)b * nf + c) * P + p] - mean[c]) * inv_scale[c];
            if (clip > 0.f) v = fminf(fmaxf(v, -clip), clip);
        }
        else if (c < nf + nc)
            v = cond[b * nc + (c - nf)];
        out[i] = v;
    }
}
// fields after the jump: soa_out[b][f][p] = soa_in[b][f][p] + net[b][p][f] * dscale[f]
__global__ void k_unpack(const float* __restrict__ soa_in, const float* __restrict__ net, long long P, int nf, int C,
                         const float* __restrict__ dscale, int B, float* __restrict__ soa_out) {
    const long long n = (long long)B * nf * P;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long p = i % P;
        const long long bf = i / P;
        const int f = (int)(bf % nf);
        const int b = (int)(bf / nf);
        soa_out[i] = soa_in[i] + net[((long long)b * P + p) * C + f] * dscale[f];
    }
}
__global__ void k_axpy(const float* __restrict__ x, long long n, float a, float* __restrict__ y) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

__global__ void k_fill(float* __restrict__ p, long long n, float v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Gas-volume defect of a jump f0 -> f1 per lattice (the surrogate's
// acceptance test): f (N, 6, ny, nx) field planes, plane 0 alpha_g, plane 2
// u_g,y; rows 0 (inlet) .. ny - 1 (outlet).  Net inflow per step = inlet-row
// flux - outlet-row flux, each sum_x alpha u_y - chi d(alpha)/dy (one-sided
// between the end row and its neighbour); defect = |V1 - V0 - jump (in0 +
// in1) / 2| / |V0|, V = sum of alpha_g.  One workgroup of 1024 threads per
// lattice (16-byte loads when the plane allows, four loads in flight per
// thread), FP64 sums reduced in a fixed tree: the result does not depend on
// the launch.
constexpr int kDefThreads = 1024;
__global__ void __launch_bounds__(kDefThreads) k_volume_defect(const float* __restrict__ f0,
                                                               const float* __restrict__ f1, int ny, int nx,
                                                               double jump, const float* __restrict__ chi,
                                                               double* __restrict__ defect) {
    __shared__ double red[3][kDefThreads];
    const int n = blockIdx.x;
    const long long plane = (long long)ny * nx;
    const float* a0 = f0 + (long long)n * 6 * plane;
    const float* a1 = f1 + (long long)n * 6 * plane;
    const float* v0 = a0 + 2 * plane;
    const float* v1 = a1 + 2 * plane;
    const double c = chi[n];
    double s0 = 0.0, s1 = 0.0, net = 0.0;
    long long done = 0;
    if ((plane & 3) == 0) {
        // f0, f1 16-byte aligned (host check), plane a multiple of 4 values
        const float4* b0 = reinterpret_cast<const float4*>(a0);
        const float4* b1 = reinterpret_cast<const float4*>(a1);
        const long long n4 = plane >> 2;
        long long i = threadIdx.x;
        for (; i + 3 * kDefThreads < n4; i += 4 * kDefThreads) {
            float4 x[4], y[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                x[u] = b0[i + u * kDefThreads];
                y[u] = b1[i + u * kDefThreads];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                s0 += ((double)x[u].x + x[u].y) + ((double)x[u].z + x[u].w);
                s1 += ((double)y[u].x + y[u].y) + ((double)y[u].z + y[u].w);
            }
        }
        for (; i < n4; i += kDefThreads) {
            const float4 x = b0[i], y = b1[i];
            s0 += ((double)x.x + x.y) + ((double)x.z + x.w);
            s1 += ((double)y.x + y.y) + ((double)y.z + y.w);
        }
        done = plane;
    }
    for (long long i = done + threadIdx.x; i < plane; i += kDefThreads) {
        s0 += a0[i];
        s1 += a1[i];
    }
    const long long top = (long long)(ny - 1) * nx, below = (long long)(ny - 2) * nx;
    for (int x = threadIdx.x; x < nx; x += kDefThreads) {
        double in0 = (double)a0[x] * v0[x] - c * ((double)a0[nx + x] - a0[x]);
        double out0 = (double)a0[top + x] * v0[top + x] - c * ((double)a0[top + x] - a0[below + x]);
        double in1 = (double)a1[x] * v1[x] - c * ((double)a1[nx + x] - a1[x]);
        double out1 = (double)a1[top + x] * v1[top + x] - c * ((double)a1[top + x] - a1[below + x]);
        net += (in0 - out0) + (in1 - out1);
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = net;
    __syncthreads();
    for (int k = kDefThreads / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double budget = 0.5 * jump * red[2][0];
        defect[n] = fabs(red[1][0] - red[0][0] - budget) / fabs(red[0][0]);
    }
}

// Re-anchoring decision of a rollout jump, on the device: mask[i] = the jump
// of lattice i is redone on the LBM (defect above defect_max or not finite,
// or every lattice when force != 0); rebuild[i] = mask[i] and the lattice's
// LBM state is not the current one (valid[i] == 0), i.e. it must be rebuilt
// from the fields first; then valid[i] = mask[i] (the re-anchored lattices
// hold the LBM state of the next time) and count += the masked lattices.
__global__ void k_reanchor_policy(const double* __restrict__ defect, int N, double defect_max, int force,
                                  int* __restrict__ valid, int* __restrict__ mask, int* __restrict__ rebuild,
                                  long long* __restrict__ count) {
    __shared__ int nm;
    if (threadIdx.x == 0) nm = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double d = defect[i];
        const int m = (force != 0 || !(d <= defect_max)) ? 1 : 0;  // NaN compares false: masked
        mask[i] = m;
        rebuild[i] = m && !valid[i];
        valid[i] = m;
        if (m) atomicAdd(&nm, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) count[0] += nm;
}

// out[i] = mask[i / per] ? a[i] : b[i] over N blocks of per values
__global__ void k_select(const int* __restrict__ mask, long long n, long long per, const float* __restrict__ a,
                         const float* __restrict__ b, float* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = mask[i / per] ? a[i] : b[i];
}

// ------------------------------------------------------------- launchers
inline unsigned grid_for(long long n) {
    long long g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace cno

using namespace cno;

namespace {
int last_rc(hipError_t e) { return e == hipSuccess ? EELBM_OK : EELBM_E_HIP; }

// compute units of the current device (cached per device; 256 if unknown)
std::atomic<int> g_cus[64];
int cu_count() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = g_cus[dev].load();
    if (n <= 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        g_cus[dev].store(n);
    }
    return n;
}

// forward tiling: MT M-tiles of 16 pixels per wavefront (1, 2 or 4) and NT
// output tiles of 16 channels per workgroup (1 to 4, dividing Cout / 16)
template <int MT, int NT, class AI, class AO>
void conv2_mn(const typename AI::S* src0, int C0, int up0, const typename AI::S* src1, int C1, int B, int H, int W,
              const unsigned short* wf, const float* bias, int Cout, typename AO::S* out, int act, float slope,
              hipStream_t s) {
    // at most as many workgroups as fit on the chip at once (LDS-bound), each
    // looping over its share of the tiles
    const long long tiles = (long long)B * ((H + kRows - 1) / kRows) * ((W + 16 * MT - 1) / (16 * MT));
    const int ngroups = Cout / (16 * NT);
    static std::atomic<int> per_cu{0};  // workgroups of this kernel one compute unit holds (LDS, registers)
    int pc = per_cu.load();
    if (pc <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &pc, reinterpret_cast<const void*>(&k_conv2<MT, NT, AI, AO>), 256, 0) != hipSuccess ||
            pc <= 0)
            pc = 1;
        per_cu.store(pc);
    }
    const long long resident = std::max(1ll, (long long)cu_count() * pc / ngroups);
    const dim3 g((unsigned)std::min(tiles, resident), (unsigned)ngroups);
    hipLaunchKernelGGL((k_conv2<MT, NT, AI, AO>), g, dim3(256), 0, s, src0, C0, up0, src1, C1, B, H, W, wf, bias,
                       Cout, out, act, slope);
}
template <int MT, class AI, class AO>
void conv2_m(int nt, const typename AI::S* src0, int C0, int up0, const typename AI::S* src1, int C1, int B, int H,
             int W, const unsigned short* wf, const float* bias, int Cout, typename AO::S* out, int act, float slope,
             hipStream_t s) {
    switch (nt) {
        case 1: conv2_mn<MT, 1, AI, AO>(src0, C0, up0, src1, C1, B, H, W, wf, bias, Cout, out, act, slope, s); break;
        case 2: conv2_mn<MT, 2, AI, AO>(src0, C0, up0, src1, C1, B, H, W, wf, bias, Cout, out, act, slope, s); break;
        case 3: conv2_mn<MT, 3, AI, AO>(src0, C0, up0, src1, C1, B, H, W, wf, bias, Cout, out, act, slope, s); break;
        default: conv2_mn<MT, 4, AI, AO>(src0, C0, up0, src1, C1, B, H, W, wf, bias, Cout, out, act, slope, s); break;
    }
}
template <class AI, class AO>
void conv2_launch(int mt, int nt, const void* src0, int C0, int up0, const void* src1, int C1, int B, int H, int W,
                  const unsigned short* wf, const float* bias, int Cout, void* out, int act, float slope,
                  hipStream_t s) {
    using SI = typename AI::S;
    using SO = typename AO::S;
    const SI* a = static_cast<const SI*>(src0);
    const SI* b = static_cast<const SI*>(src1);
    SO* o = static_cast<SO*>(out);
    if (mt == 4)
        conv2_m<4, AI, AO>(nt, a, C0, up0, b, C1, B, H, W, wf, bias, Cout, o, act, slope, s);
    else if (mt == 2)
        conv2_m<2, AI, AO>(nt, a, C0, up0, b, C1, B, H, W, wf, bias, Cout, o, act, slope, s);
    else
        conv2_m<1, AI, AO>(nt, a, C0, up0, b, C1, B, H, W, wf, bias, Cout, o, act, slope, s);
}
// Automatic tile, from a sweep of every tile over the layers of two U-Nets
// (widths 32/48/96/192 and 16/32/64/128, batch 8 x 256^2) on the MI355X:
// two M-tiles per wavefront once a row holds them (one below 64 pixels) and
// two N-tiles, else three, else one.  Four M-tiles were never faster: their
// larger LDS window and registers leave too few workgroups per compute unit
// to cover the load latency.
std::atomic<int> g_tile_mt{0}, g_tile_nt{0};  // eelbm_cno_conv_set_tile; 0: automatic
void conv2_tile(int W, int Cout, int* mt, int* nt) {
    const int n = Cout / 16;
    *mt = W >= 64 ? 2 : 1;
    *nt = n % 2 == 0 ? 2 : n % 3 == 0 ? 3 : 1;
}

// Partial-sum workspace of the weight and bias gradients, held by the library
// per device (grown on demand, kept until the process ends): calls on one
// device and stream run in order and reuse it; calls that overlap on one
// device from different streams race on it.
constexpr long long kWgradParts = 4096;  // tile-chunks of 16 x 16 weights
std::mutex g_ws_mu;
float* g_ws[64] = {};
size_t g_ws_n[64] = {};
int workspace_for_current_device(size_t n, float** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return EELBM_E_HIP;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (g_ws_n[dev] < n) {
        // a kernel still in flight may use the old one
        if (g_ws[dev] && (hipDeviceSynchronize() != hipSuccess || hipFree(g_ws[dev]) != hipSuccess))
            return EELBM_E_HIP;
        g_ws[dev] = nullptr;
        g_ws_n[dev] = 0;
        if (hipMalloc(reinterpret_cast<void**>(&g_ws[dev]), n * sizeof(float)) != hipSuccess) return EELBM_E_HIP;
        g_ws_n[dev] = n;
    }
    *out = g_ws[dev];
    return EELBM_OK;
}

bool shape_ok(int B, int H, int W, int Cin, int Cout) {
    return B > 0 && H > 0 && W > 0 && Cin > 0 && Cout > 0 && Cin % 16 == 0 && Cout % 16 == 0 && Cout <= 16 * 16 * 12 &&
           Cin <= 4096 && Cout <= 4096;
}
}  // namespace

extern "C" {

int eelbm_cno_conv_fwd_cat_dt(const void* src0, int32_t C0, int32_t up0, const void* src1, int32_t C1, int32_t B,
                              int32_t H, int32_t W, const uint16_t* wf, const float* bias, int32_t Cout, void* out,
                              int32_t act, float slope, int32_t in_bf16, int32_t out_bf16, void* stream) {
    if (!src0 || !wf || !out || C0 <= 0 || C0 % 16 != 0 || C1 < 0 || C1 % 16 != 0 || (C1 > 0 && !src1) ||
        !shape_ok(B, H, W, C0 + C1, Cout))
        return EELBM_E_PARAM;
    if (up0 && (H % 2 != 0 || W % 2 != 0)) return EELBM_E_PARAM;
    const int Cin = C0 + C1;
    // workgroups of 256 threads along x: their threads must number < 2^32;
    // element offsets of the tensors and of the weight copy fit in 32 bits
    if ((long long)B * ((H + kRows - 1) / kRows) * ((W + 15) / 16) >= (1ll << 24) ||
        (long long)Cout * 9 * Cin >= (1ll << 31) || (long long)B * H * W * std::max(Cin, Cout) >= (1ll << 31))
        return EELBM_E_PARAM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned short* w = reinterpret_cast<const unsigned short*>(wf);
    int mt = g_tile_mt.load(), nt = g_tile_nt.load();
    if (mt == 0)
        conv2_tile(W, Cout, &mt, &nt);
    else if ((Cout / 16) % nt != 0)
        return EELBM_E_PARAM;
    if (in_bf16 && out_bf16)
        conv2_launch<ActBF16, ActBF16>(mt, nt, src0, C0, up0, src1, C1, B, H, W, w, bias, Cout, out, act, slope, s);
    else if (in_bf16)
        conv2_launch<ActBF16, ActF32>(mt, nt, src0, C0, up0, src1, C1, B, H, W, w, bias, Cout, out, act, slope, s);
    else if (out_bf16)
        conv2_launch<ActF32, ActBF16>(mt, nt, src0, C0, up0, src1, C1, B, H, W, w, bias, Cout, out, act, slope, s);
    else
        conv2_launch<ActF32, ActF32>(mt, nt, src0, C0, up0, src1, C1, B, H, W, w, bias, Cout, out, act, slope, s);
    return last_rc(hipGetLastError());
}

int eelbm_cno_conv_fwd_cat(const float* src0, int32_t C0, int32_t up0, const float* src1, int32_t C1, int32_t B,
                           int32_t H, int32_t W, const uint16_t* wf, const float* bias, int32_t Cout, float* out,
                           int32_t act, float slope, void* stream) {
    return eelbm_cno_conv_fwd_cat_dt(src0, C0, up0, src1, C1, B, H, W, wf, bias, Cout, out, act, slope, 0, 0, stream);
}

int eelbm_cno_pool_bf16(const uint16_t* in, int32_t B, int32_t H, int32_t W, int32_t C, uint16_t* out,
                        void* stream) {
    if (!in || !out || B < 1 || H < 2 || W < 2 || C < 1 || (H & 1) || (W & 1)) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_pool_fwd_bf16, dim3(grid_for((long long)B * H * W * C / 4)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), reinterpret_cast<const unsigned short*>(in), B, H, W, C,
                       reinterpret_cast<unsigned short*>(out));
    return last_rc(hipGetLastError());
}

int eelbm_cno_conv_set_tile(int32_t mt, int32_t nt) {
    if (!((mt == 0 && nt == 0) || ((mt == 1 || mt == 2 || mt == 4) && nt >= 1 && nt <= 4))) return EELBM_E_PARAM;
    g_tile_nt.store(nt);
    g_tile_mt.store(mt);
    return EELBM_OK;
}

int eelbm_cno_conv_fwd(const float* in, int32_t B, int32_t H, int32_t W, int32_t Cin, const uint16_t* wf,
                       const float* bias, int32_t Cout, float* out, int32_t act, float slope, void* stream) {
    return eelbm_cno_conv_fwd_cat(in, Cin, 0, nullptr, 0, B, H, W, wf, bias, Cout, out, act, slope, stream);
}

int eelbm_cno_conv_bwd_data(const float* dout, int32_t B, int32_t H, int32_t W, int32_t Cout, const uint16_t* wd,
                            int32_t Cin, float* din, void* stream) {
    if (!dout || !wd || !din || !shape_ok(B, H, W, Cout, Cin)) return EELBM_E_PARAM;
    // a forward convolution of dout (Cout channels) into Cin channels with
    // the tap-reversed weights Wd, no bias, no activation
    return eelbm_cno_conv_fwd(dout, B, H, W, Cout, wd, nullptr, Cin, din, 0, 0.f, stream);
}

int eelbm_cno_conv_bwd_weight(const float* in, const float* dout, int32_t B, int32_t H, int32_t W, int32_t Cin,
                              int32_t Cout, float* dw, float* dbias, void* stream) {
    if (!in || !dout || !dw || !shape_ok(B, H, W, Cin, Cout) || Cout > 256) return EELBM_E_PARAM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long P = (long long)B * H * W;
    if (P >= (1ll << 31) - 4096) return EELBM_E_PARAM;
    // pixel chunks: enough workgroups to fill the GPU, at most kWgradParts
    // tile-chunks in the workspace
    const long long tiles = (long long)(9 * Cin / 16) * (Cout / 16);
    long long nk = std::max(1ll, std::min((P + 255) / 256, kWgradParts / tiles));
    const int chunk = (int)(((P + nk - 1) / nk + 15) / 16 * 16);
    nk = (P + chunk - 1) / chunk;
    const long long nw = 9ll * Cin * Cout;
    const long long nb = (P + 255) / 256;
    float* ws = nullptr;
    int rc = workspace_for_current_device((size_t)std::max(nk * nw, dbias ? nb * Cout : 0ll), &ws);
    if (rc) return rc;
    hipLaunchKernelGGL(k_conv_bwd_weight, dim3((unsigned)(9 * Cin / 16), (unsigned)(Cout / 16), (unsigned)nk),
                       dim3(64), 0, s, in, dout, B, H, W, Cin, Cout, chunk, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return EELBM_E_HIP;
    hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)std::min(4096ll, (nw + 255) / 256)), dim3(256), 0, s, ws, (int)nk,
                       nw, dw);
    e = hipGetLastError();
    if (e != hipSuccess) return EELBM_E_HIP;
    if (dbias) {
        // the bias partials reuse the workspace once the weight sums have read it (same stream)
        hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)nb), dim3(256), 0, s, dout, P, Cout, ws);
        e = hipGetLastError();
        if (e != hipSuccess) return EELBM_E_HIP;
        hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)std::min(4096ll, ((long long)Cout + 255) / 256)), dim3(256), 0,
                           s, ws, (int)nb, (long long)Cout, dbias);
        e = hipGetLastError();
    }
    return last_rc(e);
}

int eelbm_cno_volume_defect(const float* f0, const float* f1, int32_t N, int32_t ny, int32_t nx, int32_t jump,
                            const float* chi, double* defect, void* stream) {
    if (!f0 || !f1 || !chi || !defect || N < 1 || ny < 3 || nx < 1 || jump < 0) return EELBM_E_PARAM;
    if ((reinterpret_cast<uintptr_t>(f0) & 15) || (reinterpret_cast<uintptr_t>(f1) & 15)) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_volume_defect, dim3(N), dim3(kDefThreads), 0, static_cast<hipStream_t>(stream), f0, f1, ny,
                       nx, (double)jump, chi, defect);
    return last_rc(hipGetLastError());
}

int eelbm_cno_reanchor_policy(const double* defect, int32_t N, double defect_max, int32_t force, int32_t* valid,
                              int32_t* mask, int32_t* rebuild, int64_t* count, void* stream) {
    if (!defect || !valid || !mask || !rebuild || !count || N < 1) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_reanchor_policy, dim3(1), dim3(256), 0, static_cast<hipStream_t>(stream), defect, N,
                       defect_max, force, valid, mask, rebuild, reinterpret_cast<long long*>(count));
    return last_rc(hipGetLastError());
}

int eelbm_cno_select(const int32_t* mask, int32_t N, int64_t per, const float* a, const float* b, float* out,
                     void* stream) {
    if (!mask || !a || !b || !out || N < 1 || per < 1) return EELBM_E_PARAM;
    const long long n = (long long)N * per;
    hipLaunchKernelGGL(k_select, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), mask, n, per, a,
                       b, out);
    return last_rc(hipGetLastError());
}

int eelbm_cno_act_bwd(const float* y, const float* dy, int64_t n, float slope, float* dx, void* stream) {
    if (!y || !dy || !dx || n < 0) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_act_bwd, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), y, dy, n, slope,
                       dx);
    return last_rc(hipGetLastError());
}

int eelbm_cno_pool(const float* in, int32_t B, int32_t H, int32_t W, int32_t C, float* out, int32_t backward,
                   void* stream) {
    if (!in || !out || B < 1 || H < 2 || W < 2 || C < 1 || (H & 1) || (W & 1)) return EELBM_E_PARAM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (backward)
        hipLaunchKernelGGL(k_pool_bwd, dim3(grid_for((long long)B * H * W * C)), dim3(256), 0, s, in, B, H, W, C, out);
    else
        hipLaunchKernelGGL(k_pool_fwd, dim3(grid_for((long long)B * H * W * C / 4)), dim3(256), 0, s, in, B, H, W, C,
                           out);
    return last_rc(hipGetLastError());
}

int eelbm_cno_up(const float* in, int32_t B, int32_t H, int32_t W, int32_t C, float* out, int32_t backward,
                 void* stream) {
    if (!in || !out || B < 1 || H < 1 || W < 1 || C < 1) return EELBM_E_PARAM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // forward: (H, W) -> (2H, 2W); backward: gradient of (2H, 2W) -> (H, W)
    if (backward)
        hipLaunchKernelGGL(k_up_bwd, dim3(grid_for((long long)B * H * W * C)), dim3(256), 0, s, in, B, H, W, C, out);
    else
        hipLaunchKernelGGL(k_up_fwd, dim3(grid_for((long long)B * 4 * H * W * C)), dim3(256), 0, s, in, B, H, W, C,
                           out);
    return last_rc(hipGetLastError());
}

int eelbm_cno_concat(const float* a, int32_t Ca, const float* b, int32_t Cb, int64_t P, float* out, void* stream) {
    if (!a || !b || !out || Ca < 1 || Cb < 1 || P < 1) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_concat, dim3(grid_for(P * (Ca + Cb))), dim3(256), 0, static_cast<hipStream_t>(stream), a, Ca,
                       b, Cb, P, out);
    return last_rc(hipGetLastError());
}

int eelbm_cno_split_add(const float* d, int32_t Ca, int32_t Cb, int64_t P, float* da, float* db, void* stream) {
    if (!d || !da || !db || Ca < 1 || Cb < 1 || P < 1) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_split_add, dim3(grid_for(P * (Ca + Cb))), dim3(256), 0, static_cast<hipStream_t>(stream), d,
                       Ca, Cb, P, da, db);
    return last_rc(hipGetLastError());
}

int eelbm_cno_mse(const float* pred, const float* target, int64_t P, int32_t C, int32_t Cused, double* partial,
                  int32_t nblocks, float* dpred, void* stream) {
    if (!pred || !target || !partial || P < 1 || C < 1 || Cused < 1 || Cused > C || nblocks < 1) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, static_cast<hipStream_t>(stream), pred, target, P, C, Cused,
                       partial, dpred);
    return last_rc(hipGetLastError());
}

}  // extern "C"

// Workgroup partial sums of eelbm_cno_mse_noalloc, in the library's own device
// memory (one copy per GPU, held until the process ends).  Host code never
// uses the name itself (a host-side stand-in, not a device address): it takes
// each device's address with hipGetSymbolAddress once, with that device
// current, and passes that address to the kernels.
static __device__ __align__(256) double scratch[EELBM_CNO_MSE_MAX_BLOCKS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// this device's address of `scratch`, taken at the first call on the device
int scratch_for_current_device(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return eelbm::set_error(EELBM_E_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return eelbm::set_error(EELBM_E_PARAM, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return eelbm::set_error(EELBM_E_HIP, "hipGetSymbolAddress(scratch) failed");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return EELBM_OK;
}
}  // namespace

extern "C" {

int eelbm_cno_mse_noalloc(const float* pred, const float* target, int64_t P, int32_t C, int32_t Cused,
                          int32_t nblocks, double* loss, float* dpred, void* stream) {
    if (!pred || !target || !loss) return eelbm::set_error(EELBM_E_PARAM, "NULL pointer");
    if (P < 1 || C < 1 || Cused < 1 || Cused > C || nblocks < 1)
        return eelbm::set_error(EELBM_E_PARAM, "need P, C, nblocks >= 1 and 1 <= Cused <= C");
    if (nblocks > EELBM_CNO_MSE_MAX_BLOCKS)
        return eelbm::set_error(EELBM_E_SIZE, "nblocks exceeds EELBM_CNO_MSE_MAX_BLOCKS (the size of the built-in scratch)");
    double* part = nullptr;
    int rc = scratch_for_current_device(&part);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // every one of the nblocks workgroups writes its own partial sum: nothing
    // left in the scratch by an earlier call is read
    hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, s, pred, target, P, C, Cused, part, dpred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return eelbm::set_error(EELBM_E_HIP, "k_mse launch failed");
    hipLaunchKernelGGL(k_sum_in_order, dim3(1), dim3(64), 0, s, part, nblocks, loss);
    e = hipGetLastError();
    if (e != hipSuccess) return eelbm::set_error(EELBM_E_HIP, "k_sum_in_order launch failed");
    return EELBM_OK;
}

int eelbm_cno_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                   int64_t step, float weight_decay, void* stream) {
    if (!w || !g || !m || !v || n < 1 || step < 1) return EELBM_E_PARAM;
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), w, g, m, v, n, lr, b1,
                       b2, eps, c1, c2, weight_decay);
    return last_rc(hipGetLastError());
}

int eelbm_cno_pack_weights(const float* w, int32_t Cin, int32_t Cout, uint16_t* wf, uint16_t* wd, void* stream) {
    if (!w || !wf || !wd || Cin < 1 || Cout < 1) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_pack_weights, dim3(grid_for(9LL * Cin * Cout)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), w, Cin, Cout, wf, wd);
    return last_rc(hipGetLastError());
}

int eelbm_cno_pack(const float* soa, int64_t P, int32_t nf, const float* mean, const float* inv_scale,
                   const float* cond, int32_t nc, int32_t B, int32_t C, float clip, float* out, void* stream) {
    if (!soa || !mean || !inv_scale || !out || (nc > 0 && !cond) || P < 1 || nf < 1 || nc < 0 || B < 1 ||
        nf + nc > C)
        return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_pack, dim3(grid_for((long long)B * P * C)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       soa, P, nf, mean, inv_scale, cond, nc, B, C, clip, out);
    return last_rc(hipGetLastError());
}

int eelbm_cno_unpack(const float* soa_in, const float* net, int64_t P, int32_t nf, int32_t C, const float* dscale,
                     int32_t B, float* soa_out, void* stream) {
    if (!soa_in || !net || !dscale || !soa_out || P < 1 || nf < 1 || nf > C || B < 1) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_unpack, dim3(grid_for((long long)B * nf * P)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), soa_in, net, P, nf, C, dscale, B, soa_out);
    return last_rc(hipGetLastError());
}

int eelbm_cno_axpy(const float* x, int64_t n, float a, float* y, void* stream) {
    if (!x || !y || n < 0) return EELBM_E_PARAM;
    if (n == 0) return EELBM_OK;
    hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), x, n, a, y);
    return last_rc(hipGetLastError());
}

int eelbm_cno_fill(float* p, int64_t n, float value, void* stream) {
    if (!p || n < 0) return EELBM_E_PARAM;
    if (n == 0) return EELBM_OK;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), p, n, value);
    return last_rc(hipGetLastError());
}

}  // extern "C"
