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

#include <cmath>
#include <mutex>

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
// A wavefront owns MT x 16 consecutive pixels of one image row (MT M-tiles)
// and NT output tiles of 16 channels: each loaded weight fragment feeds MT
// matrix-core products and each loaded pixel fragment NT.
// Grid: x = pixel groups of 16 MT (rows padded), y = groups of NT output tiles.
template <int MT, int NT>
__global__ void __launch_bounds__(64) k_conv_fwd(const float* __restrict__ in, int B, int H, int W, int Cin,
                                                const unsigned short* __restrict__ wf, const float* __restrict__ bias,
                                                int Cout, float* __restrict__ out, int act, float slope) {
    (void)B;  // the grid covers the B * H image rows
    const int lane = threadIdx.x;
    const int gw = (W + 16 * MT - 1) / (16 * MT);
    const long long grp = blockIdx.x;
    const int xg = (int)(grp % gw);
    const long long by = grp / gw;  // b * H + y
    const int y = (int)(by % H);
    const int b = (int)(by / H);
    const int x0 = xg * 16 * MT + (lane & 15);  // pixel of this lane's A row in M-tile 0
    const int kq = 4 * (lane >> 4);              // K offset of this lane within a 16-chunk
    const int n0 = blockIdx.y * NT * 16;        // the host launches Cout / (16 NT) tiles exactly
    const int K = 9 * Cin;
    const int nc = Cin / 16;  // 16-channel chunks per tap
    f32x4 acc[MT][NT];
    float bc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        bc[j] = bias ? bias[n0 + j * 16 + (lane & 15)] : 0.f;
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const unsigned short* wrow = wf + (long long)(n0 + (lane & 15)) * K + kq;
    const float* img = in + (long long)b * H * W * Cin + kq;  // H * W * Cin < 2^31 (host check)
    // fragments of one (tap, chunk) step: loads always address a valid pixel
    // (the image's first one when the tap falls outside), the value is
    // zeroed after the load; the next step's loads are issued before this
    // step's products
    f32x4 av[MT];
    u16x4 bv[NT];
    bool ok[MT];
    auto load = [&](int tap, int c0) {
        const int yy = y + tap / 3 - 1;
        const bool oky = (unsigned)yy < (unsigned)H;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int xx = x0 + 16 * m + tap % 3 - 1;
            ok[m] = oky & ((unsigned)xx < (unsigned)W);
            const int pix = ok[m] ? yy * W + xx : 0;
            av[m] = *reinterpret_cast<const f32x4*>(img + (pix * Cin + c0));
        }
        const int k = tap * Cin + c0;
#pragma unroll
        for (int j = 0; j < NT; ++j) bv[j] = *reinterpret_cast<const u16x4*>(wrow + (j * 16 * K + k));
    };
    int tap = 0, ch = 0;
    load(0, 0);
    for (int it = 0; it < 9 * nc; ++it) {
        s16x4 a[MT], bw[NT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const s16x4 h = pack4(av[m]);
            a[m] = ok[m] ? h : s16x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) bw[j] = __builtin_bit_cast(s16x4, bv[j]);
        if (++ch == nc) {
            ch = 0;
            ++tap;
        }
        if (tap < 9) load(tap, ch * 16);
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m][j] = mfma(a[m], bw[j], acc[m][j]);
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = n0 + j * 16 + (lane & 15);
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int px = xg * 16 * MT + 16 * m + 4 * (lane >> 4) + t;
                float v = acc[m][j][t] + bc[j];
                v = (act && v < 0.f) ? slope * v : v;
                if (px < W) out[(((long long)b * H + y) * W + px) * Cout + co] = v;
            }
        }
    }
}

// ----------------------------------------------------- gradient wrt input
// din[b, y, x, ci] = sum_{tap, co} dout[b, y - dy, x - dx, co] W[tap][ci][co]
//                  = sum_{tap', co} dout[b, y + dy', x + dx', co] Wd[ci][tap'][co]
// with the taps reversed (tap' = 8 - tap, dy' = -dy, dx' = -dx): a forward
// convolution of dout with Wd, run by k_conv_fwd.

// ---------------------------------------------------- gradient wrt weights
// dW[tap][ci][co] += sum_p in[p + d_tap][ci] dout[p][co] over this
// workgroup's chunk of `chunk` pixels (M = (tap, ci), N = co, K = pixels);
// one wavefront per 16 x 16 tile of dW, partial sums added atomically.
__global__ void __launch_bounds__(64) k_conv_bwd_weight(const float* __restrict__ in, const float* __restrict__ dout,
                                                       int B, int H, int W, int Cin, int Cout, int chunk,
                                                       float* __restrict__ dw) {
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
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int mm = mt * 16 + 4 * (lane >> 4) + t;  // row of D
        atomicAdd(dw + (long long)mm * Cout + co, acc[t]);
    }
}

__global__ void k_bias_grad(const float* __restrict__ dout, long long P, int C, float* __restrict__ db) {
    // one workgroup per 256-pixel chunk, one thread per channel (C <= 256)
    const int c = threadIdx.x;
    if (c >= C) return;
    const long long p0 = (long long)blockIdx.x * 256;
    float s = 0.f;
    for (long long p = p0; p < p0 + 256 && p < P; ++p) s += dout[p * C + c];
    atomicAdd(db + c, s);
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

// forward tiling: MT M-tiles of 16 pixels (up to 4, no more than a row holds)
// and NT <= 4 output tiles per wavefront, NT dividing the output tiles
constexpr int kFwdMaxNT = 4;

template <int MT, int NT>
void fwd_mn(const float* in, int B, int H, int W, int Cin, const unsigned short* wf, const float* bias, int Cout,
            float* out, int act, float slope, hipStream_t s) {
    const dim3 g((unsigned)((long long)B * H * ((W + 16 * MT - 1) / (16 * MT))), (unsigned)(Cout / (16 * NT)));
    hipLaunchKernelGGL((k_conv_fwd<MT, NT>), g, dim3(64), 0, s, in, B, H, W, Cin, wf, bias, Cout, out, act, slope);
}

template <int MT>
bool fwd_m(int nt, const float* in, int B, int H, int W, int Cin, const unsigned short* wf, const float* bias,
           int Cout, float* out, int act, float slope, hipStream_t s) {
    switch (nt) {
        case 1: fwd_mn<MT, 1>(in, B, H, W, Cin, wf, bias, Cout, out, act, slope, s); return true;
        case 2: fwd_mn<MT, 2>(in, B, H, W, Cin, wf, bias, Cout, out, act, slope, s); return true;
        case 3: fwd_mn<MT, 3>(in, B, H, W, Cin, wf, bias, Cout, out, act, slope, s); return true;
        case 4: fwd_mn<MT, 4>(in, B, H, W, Cin, wf, bias, Cout, out, act, slope, s); return true;
    }
    return false;
}

bool shape_ok(int B, int H, int W, int Cin, int Cout) {
    return B > 0 && H > 0 && W > 0 && Cin > 0 && Cout > 0 && Cin % 16 == 0 && Cout % 16 == 0 && Cout <= 16 * 16 * 12 &&
           Cin <= 4096 && Cout <= 4096;
}
}  // namespace

extern "C" {

int eelbm_cno_conv_fwd(const float* in, int32_t B, int32_t H, int32_t W, int32_t Cin, const uint16_t* wf,
                       const float* bias, int32_t Cout, float* out, int32_t act, float slope, void* stream) {
    if (!in || !wf || !out || !shape_ok(B, H, W, Cin, Cout)) return EELBM_E_PARAM;
    int nt = 1;
    for (int d = 1; d <= kFwdMaxNT; ++d)
        if ((Cout / 16) % d == 0) nt = d;
    if ((long long)B * H * ((W + 15) / 16) >= (1ll << 32) || (long long)H * W * Cin >= (1ll << 31) ||
        (long long)Cout * 9 * Cin >= (1ll << 31))
        return EELBM_E_PARAM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool ok = W >= 64   ? fwd_m<4>(nt, in, B, H, W, Cin, wf, bias, Cout, out, act, slope, s)
                    : W >= 32 ? fwd_m<2>(nt, in, B, H, W, Cin, wf, bias, Cout, out, act, slope, s)
                              : fwd_m<1>(nt, in, B, H, W, Cin, wf, bias, Cout, out, act, slope, s);
    if (!ok) return EELBM_E_PARAM;
    return last_rc(hipGetLastError());
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
    const int chunk = 2048;
    const long long nk = (P + chunk - 1) / chunk;
    if (nk > 65535 || P + chunk >= (1ll << 31)) return EELBM_E_PARAM;
    hipLaunchKernelGGL(k_conv_bwd_weight, dim3((unsigned)(9 * Cin / 16), (unsigned)(Cout / 16), (unsigned)nk),
                       dim3(64), 0, s, in, dout, B, H, W, Cin, Cout, chunk, dw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return EELBM_E_HIP;
    if (dbias) {
        hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, dout, P, Cout, dbias);
        e = hipGetLastError();
    }
    return last_rc(e);
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
