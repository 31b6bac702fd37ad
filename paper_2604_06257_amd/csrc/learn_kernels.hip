// gfx950 kernels of the learned-compounding network (3D U-Net): BF16 MFMA
// convolutions with FP32 accumulation, and the small element-wise steps of
// training.  Volumes are channels-last [D][H][W][C]; a tensor may be a slice of
// a wider buffer (row stride `*_stride` channels, first channel `*_coff`).
//
// Convolution (3 x 3 x 3, zero padding, stride 1) as an implicit GEMM on
// v_mfma_f32_16x16x32_bf16: M = voxels, N = output channels, K = 27 * Cin with
// k = tap * Cin + c.  One wave owns 16 voxels and all output channels; per K
// step of 32 each lane loads 8 consecutive input channels of one tap (16 B)
// for its voxel (operand A) and 8 consecutive weights of one output channel
// (operand B).  With `flip`, the taps are mirrored: this is the input gradient
// of a convolution when the weights are passed transposed ([Cin][27][Cout]).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "das_learn.h"

namespace learn {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ float bf2f(uint16_t u) { return __uint_as_float((uint32_t)u << 16); }
__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest even (finite inputs)
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

struct Vol {
    int D, H, W;
};

constexpr int kMaxNT = 8;  // up to 128 output channels per launch

// out[v][n] = act(sum_{tap,c} in[v + s*off(tap)][c] * wk[n][tap*Cin + c] + bias[n]) * mask
template <bool OUT_F32>
__global__ __launch_bounds__(256) void conv3d_kernel(const uint16_t* __restrict__ in, int in_stride, int in_coff,
                                                     const uint16_t* __restrict__ wk, const float* __restrict__ bias,
                                                     void* __restrict__ out, int out_stride, int out_coff,
                                                     const uint16_t* __restrict__ mask, int mask_stride, int mask_coff,
                                                     Vol vol, int Cin, int Cout, int flip, int relu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t V = (int64_t)vol.D * vol.H * vol.W;
    const int64_t v0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    if (v0 >= V) return;  // whole wave past the end (no barriers in this kernel)
    const int K = 27 * Cin;
    const int NT = Cout / 16;
    // operand-A voxel of this lane
    const int64_t va = v0 + (lane & 15);
    const bool va_ok = va < V;
    const int aw = (int)(va % vol.W), ah = (int)((va / vol.W) % vol.H), ad = (int)(va / ((int64_t)vol.W * vol.H));
    const int s = flip ? -1 : 1;
    f32x4 acc[kMaxNT];
#pragma unroll
    for (int t = 0; t < kMaxNT; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int kc = 0; kc < K; kc += 32) {
        const int k = kc + 8 * (lane >> 4);
        bf16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
        if (k < K && va_ok) {
            const int tap = k / Cin, c = k - tap * Cin;
            const int zd = ad + s * (tap / 9 - 1), zh = ah + s * ((tap / 3) % 3 - 1), zw = aw + s * (tap % 3 - 1);
            if (zd >= 0 && zd < vol.D && zh >= 0 && zh < vol.H && zw >= 0 && zw < vol.W) {
                const int64_t nb = ((int64_t)zd * vol.H + zh) * vol.W + zw;
                a = *reinterpret_cast<const bf16x8*>(in + nb * in_stride + in_coff + c);
            }
        }
#pragma unroll
        for (int t = 0; t < kMaxNT; ++t) {
            if (t < NT) {
                bf16x8 b = {0, 0, 0, 0, 0, 0, 0, 0};
                if (k < K) b = *reinterpret_cast<const bf16x8*>(wk + (int64_t)(t * 16 + (lane & 15)) * K + k);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kMaxNT; ++t) {
        if (t >= NT) break;
        const int n = t * 16 + (lane & 15);
        const float bn = bias ? bias[n] : 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t v = v0 + 4 * (lane >> 4) + r;
            if (v >= V) continue;
            float y = acc[t][r] + bn;
            if (relu) y = fmaxf(y, 0.0f);
            if (mask && !(bf2f(mask[v * mask_stride + mask_coff + n]) > 0.0f)) y = 0.0f;
            if (OUT_F32) reinterpret_cast<float*>(out)[v * out_stride + out_coff + n] = y;
            else reinterpret_cast<uint16_t*>(out)[v * out_stride + out_coff + n] = f2bf(y);
        }
    }
}

// Weight gradient, split over voxel chunks:
//   part[b][n][k] = sum_{v in chunk b} dy[v][n] * in[v + off(tap k)][c k],  part_db[b][n] = sum_v dy[v][n]
// MFMA with M = output channel n, N = k, reduction over voxels (32 per step).
__global__ __launch_bounds__(256) void wgrad_kernel(const uint16_t* __restrict__ in, int in_stride, int in_coff,
                                                    const uint16_t* __restrict__ dy, int dy_stride, int dy_coff,
                                                    float* __restrict__ part, float* __restrict__ part_db, Vol vol,
                                                    int Cin, int Cout, int chunk) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t V = (int64_t)vol.D * vol.H * vol.W;
    const int K = 27 * Cin;
    const int NT = Cout / 16, KT = (K + 15) / 16;
    const int64_t vbeg = (int64_t)blockIdx.x * chunk;
    const int64_t vend = (vbeg + chunk < V) ? vbeg + chunk : V;
    float* pb = part + (int64_t)blockIdx.x * Cout * K;
    // output tiles (n tile, k tile) distributed over the 4 waves
    for (int tile = wave; tile < NT * KT; tile += 4) {
        const int nt = tile / KT, kt = tile - nt * KT;
        const int n = nt * 16 + (lane & 15);       // A row of this lane
        const int kb = kt * 16 + (lane & 15);      // B column of this lane
        const bool kb_ok = kb < K;
        const int tap = kb_ok ? kb / Cin : 0, c = kb_ok ? kb - tap * Cin : 0;
        const int od = tap / 9 - 1, oh = (tap / 3) % 3 - 1, ow = tap % 3 - 1;
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int64_t vc = vbeg; vc < vend; vc += 32) {
            bf16x8 a, b;
            // coordinates of this lane's first voxel, then stepped along w
            const int64_t vs = vc + 8 * (lane >> 4);
            int w = (int)(vs % vol.W), h = (int)((vs / vol.W) % vol.H), d = (int)(vs / ((int64_t)vol.W * vol.H));
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t v = vs + j;
                short av = 0, bv = 0;
                if (v < vend) {
                    av = (short)dy[v * dy_stride + dy_coff + n];
                    if (kb_ok) {
                        const int zd = d + od, zh = h + oh, zw = w + ow;
                        if (zd >= 0 && zd < vol.D && zh >= 0 && zh < vol.H && zw >= 0 && zw < vol.W)
                            bv = (short)in[(((int64_t)zd * vol.H + zh) * vol.W + zw) * in_stride + in_coff + c];
                    }
                }
                a[j] = av;
                b[j] = bv;
                if (++w == vol.W) {
                    w = 0;
                    if (++h == vol.H) {
                        h = 0;
                        ++d;
                    }
                }
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int nn = nt * 16 + 4 * (lane >> 4) + r, kk = kt * 16 + (lane & 15);
            if (kk < K) pb[(int64_t)nn * K + kk] = acc[r];
        }
    }
    // bias partial: one thread per output channel, fixed voxel order
    for (int n = threadIdx.x; n < Cout; n += 256) {
        float sacc = 0.0f;
        for (int64_t v = vbeg; v < vend; ++v) sacc += bf2f(dy[v * dy_stride + dy_coff + n]);
        part_db[(int64_t)blockIdx.x * Cout + n] = sacc;
    }
}

// dw[i] = sum_b part[b][i] in chunk order (deterministic), i over Cout * K; same for db.
__global__ void reduce_parts_kernel(const float* __restrict__ part, int nparts, int64_t n, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * n + i];
    out[i] = s;
}

// wt[ci][tap][co] = w[co][tap][ci] (bf16), the weights of the input-gradient convolution.
__global__ void transpose_w_kernel(const uint16_t* __restrict__ w, uint16_t* __restrict__ wt, int Cin, int Cout) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)Cout * 27 * Cin;
    if (i >= n) return;
    const int co = (int)(i / (27 * Cin)), rem = (int)(i % (27 * Cin)), tap = rem / Cin, ci = rem % Cin;
    wt[((int64_t)ci * 27 + tap) * Cout + co] = w[i];
}

// 2x average pooling: out[d][h][w][c] = mean of the 8 children.
__global__ void avgpool2_kernel(const uint16_t* __restrict__ in, int in_stride, int in_coff, uint16_t* __restrict__ out,
                                int out_stride, int out_coff, Vol vo, int C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)vo.D * vo.H * vo.W * C;
    if (i >= n) return;
    const int c = (int)(i % C);
    const int64_t v = i / C;
    const int w = (int)(v % vo.W), h = (int)((v / vo.W) % vo.H), d = (int)(v / ((int64_t)vo.W * vo.H));
    const int Hi = 2 * vo.H, Wi = 2 * vo.W;
    float s = 0.0f;
    for (int q = 0; q < 8; ++q) {
        const int64_t vi = ((int64_t)(2 * d + (q >> 2)) * Hi + (2 * h + ((q >> 1) & 1))) * Wi + (2 * w + (q & 1));
        s += bf2f(in[vi * in_stride + in_coff + c]);
    }
    out[v * out_stride + out_coff + c] = f2bf(0.125f * s);
}

// Gradient of the 2x average pooling: each child gets 1/8 of its parent's gradient, optionally added.
__global__ void avgpool2_bwd_kernel(const uint16_t* __restrict__ gout, int gout_stride, int gout_coff,
                                    uint16_t* __restrict__ gin, int gin_stride, int gin_coff, Vol vi, int C,
                                    int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)vi.D * vi.H * vi.W * C;
    if (i >= n) return;
    const int c = (int)(i % C);
    const int64_t v = i / C;
    const int w = (int)(v % vi.W), h = (int)((v / vi.W) % vi.H), d = (int)(v / ((int64_t)vi.W * vi.H));
    const int64_t vp = ((int64_t)(d >> 1) * (vi.H >> 1) + (h >> 1)) * (vi.W >> 1) + (w >> 1);
    float g = 0.125f * bf2f(gout[vp * gout_stride + gout_coff + c]);
    uint16_t* dst = gin + v * gin_stride + gin_coff + c;
    if (accumulate) g += bf2f(*dst);
    *dst = f2bf(g);
}

// 2x nearest upsampling (forward) into a channel slice.
__global__ void upsample2_kernel(const uint16_t* __restrict__ in, int in_stride, int in_coff, uint16_t* __restrict__ out,
                                 int out_stride, int out_coff, Vol vo, int C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)vo.D * vo.H * vo.W * C;
    if (i >= n) return;
    const int c = (int)(i % C);
    const int64_t v = i / C;
    const int w = (int)(v % vo.W), h = (int)((v / vo.W) % vo.H), d = (int)(v / ((int64_t)vo.W * vo.H));
    const int64_t vp = ((int64_t)(d >> 1) * (vo.H >> 1) + (h >> 1)) * (vo.W >> 1) + (w >> 1);
    out[v * out_stride + out_coff + c] = in[vp * in_stride + in_coff + c];
}

// Gradient of the 2x nearest upsampling: sum over the 8 children (fixed order), optionally masked by a ReLU output.
__global__ void upsample2_bwd_kernel(const uint16_t* __restrict__ gout, int gout_stride, int gout_coff,
                                     uint16_t* __restrict__ gin, int gin_stride, int gin_coff,
                                     const uint16_t* __restrict__ mask, int mask_stride, int mask_coff, Vol vi, int C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)vi.D * vi.H * vi.W * C;
    if (i >= n) return;
    const int c = (int)(i % C);
    const int64_t v = i / C;
    const int w = (int)(v % vi.W), h = (int)((v / vi.W) % vi.H), d = (int)(v / ((int64_t)vi.W * vi.H));
    const int Ho = 2 * vi.H, Wo = 2 * vi.W;
    float s = 0.0f;
    for (int q = 0; q < 8; ++q) {
        const int64_t vo = ((int64_t)(2 * d + (q >> 2)) * Ho + (2 * h + ((q >> 1) & 1))) * Wo + (2 * w + (q & 1));
        s += bf2f(gout[vo * gout_stride + gout_coff + c]);
    }
    if (mask && !(bf2f(mask[v * mask_stride + mask_coff + c]) > 0.0f)) s = 0.0f;
    gin[v * gin_stride + gin_coff + c] = f2bf(s);
}

// g[v][c] = (a[v][c] + b[v][c]) * (mask[v][c] > 0)   (bf16 slices)
__global__ void add_mask_kernel(const uint16_t* __restrict__ a, int a_stride, int a_coff, const uint16_t* __restrict__ b,
                                int b_stride, int b_coff, const uint16_t* __restrict__ mask, int m_stride, int m_coff,
                                uint16_t* __restrict__ g, int g_stride, int g_coff, int64_t V, int C) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V * C) return;
    const int c = (int)(i % C);
    const int64_t v = i / C;
    float s = bf2f(a[v * a_stride + a_coff + c]) + bf2f(b[v * b_stride + b_coff + c]);
    if (mask && !(bf2f(mask[v * m_stride + m_coff + c]) > 0.0f)) s = 0.0f;
    g[v * g_stride + g_coff + c] = f2bf(s);
}

// Residual prediction and MSE: pred = base + net (FP32 [V][2]); loss parts per block; grad = 2 (pred - target) / n
// written as BF16 into a [V][gstride] buffer (first 2 channels; the padded channels get 0).
__global__ void mse_kernel(const float* __restrict__ net, int net_stride, const float* __restrict__ base,
                           const float* __restrict__ target, int64_t V, uint16_t* __restrict__ grad, int gstride,
                           float* __restrict__ pred, float* __restrict__ loss_part) {
    __shared__ float red[256];
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.0f;
    if (v < V) {
        const float scale = 2.0f / (float)(2 * V);
        for (int c = 0; c < gstride; ++c) {
            if (c < 2) {
                const float p = base[2 * v + c] + net[v * net_stride + c];
                const float e = p - target[2 * v + c];
                if (pred) pred[2 * v + c] = p;
                l += e * e;
                if (grad) grad[v * gstride + c] = f2bf(scale * e);
            } else if (grad) {
                grad[v * gstride + c] = 0;
            }
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Adam with bias correction on FP32 master weights; refreshes the BF16 copy.
__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ vv,
                            const float* __restrict__ g, uint16_t* __restrict__ wbf, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * vv[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    vv[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    if (wbf) wbf[i] = f2bf(wi);
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}


// ---- compounding features
// part[b] = sum over the block's voxels of |sum_a y_a[v]|^2   (y complex64 [A][V])
__global__ __launch_bounds__(256) void sumsq_kernel(const float2* __restrict__ y, int A, int64_t V,
                                                    float* __restrict__ part) {
    __shared__ float red[256];
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float l = 0.0f;
    if (v < V) {
        float re = 0.0f, im = 0.0f;
        for (int a = 0; a < A; ++a) {
            const float2 z = y[(int64_t)a * V + v];
            re += z.x;
            im += z.y;
        }
        l = re * re + im * im;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// scale[0] = sqrt(sum(part) / V) (the RMS), scale[1] = 1 / scale[0] (0 for an all-zero input); one block.
__global__ __launch_bounds__(256) void rms_kernel(const float* __restrict__ part, int nparts, int64_t V,
                                                  float* __restrict__ scale) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float rms = (float)sqrt(red[0] / (double)V);
        scale[0] = rms;
        scale[1] = rms > 0.0f ? 1.0f / rms : 0.0f;
    }
}

// x[v][2a + {0,1}] = bf16(y_a[v] / rms), x[v][c >= 2A] = 0; base[v] = gain * sum_a y_a[v] / rms
__global__ __launch_bounds__(256) void features_kernel(const float2* __restrict__ y, int A, int64_t V, float gain,
                                                       const float* __restrict__ scale, uint16_t* __restrict__ x,
                                                       int cin, float* __restrict__ base) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= V) return;
    const float inv = scale[1];
    float re = 0.0f, im = 0.0f;
    for (int a = 0; a < A; ++a) {
        const float2 z = y[(int64_t)a * V + v];
        re += z.x;
        im += z.y;
        x[v * cin + 2 * a] = f2bf(z.x * inv);
        x[v * cin + 2 * a + 1] = f2bf(z.y * inv);
    }
    for (int c = 2 * A; c < cin; ++c) x[v * cin + c] = 0;
    if (base) {
        base[2 * v] = gain * re * inv;
        base[2 * v + 1] = gain * im * inv;
    }
}

// out[v] = y[v] * scale[k]: k = 1 normalises a complex64 volume, k = 0 restores physical units
__global__ void rescale_kernel(const float2* __restrict__ y, int64_t V, const float* __restrict__ scale, int k,
                               float2* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float s = scale[k];
    const float2 z = y[v];
    out[v] = make_float2(z.x * s, z.y * s);
}

// out[v] = (base[v] + net[v][0:2]) * rms: the network's estimate in the beamformer's units (complex64)
__global__ void compound_output_kernel(const float* __restrict__ net, int net_stride, const float* __restrict__ base,
                                       int64_t V, const float* __restrict__ scale, float2* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float s = scale[0];
    out[v] = make_float2((base[2 * v] + net[v * net_stride]) * s, (base[2 * v + 1] + net[v * net_stride + 1]) * s);
}

}  // namespace learn

// ------------------------------------------------------------------ C ABI
namespace {
thread_local const char* g_learn_err = "";
int lfail(int st, const char* msg) {
    g_learn_err = msg;
    return st;
}
bool al(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
bool slices_ok(int s1, int o1, int s2, int o2, int c) { return c >= 1 && o1 >= 0 && o2 >= 0 && s1 >= o1 + c && s2 >= o2 + c; }
bool even_dims(int D, int H, int W) { return D >= 2 && H >= 2 && W >= 2 && D % 2 == 0 && H % 2 == 0 && W % 2 == 0; }
int launch_status(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return lfail(DAS_EHIP, what);
    return DAS_OK;
}
}  // namespace

extern "C" {

const char* das_learn_last_error(void) { return g_learn_err; }

int das_conv3d(const void* in, int in_stride, int in_coff, const void* weight, const float* bias, void* out,
               int out_stride, int out_coff, int out_f32, const void* mask, int mask_stride, int mask_coff, int D,
               int H, int W, int cin, int cout, int flip, int relu, void* stream) {
    if (!in || !weight || !out) return lfail(DAS_EINVAL, "conv3d: null pointer");
    if (D < 1 || H < 1 || W < 1 || cin < 8 || cin % 8 || cout < 16 || cout % 16 || cout > 16 * learn::kMaxNT)
        return lfail(DAS_ESHAPE, "conv3d: need D,H,W >= 1, Cin a multiple of 8, Cout a multiple of 16 up to 128");
    if (in_stride < in_coff + cin || in_stride % 8 || in_coff % 8 || in_coff < 0 || out_stride < out_coff + cout ||
        out_coff < 0 || (mask && (mask_stride < mask_coff + cout || mask_coff < 0)))
        return lfail(DAS_ESHAPE, "conv3d: channel slice outside its buffer or not a multiple of 8");
    if (!al(in, 16) || !al(weight, 16)) return lfail(DAS_EALIGN, "conv3d: input and weights must be 16-byte aligned");
    const int64_t V = (int64_t)D * H * W;
    const learn::Vol vol{D, H, W};
    const dim3 grid(blocks_for(V, 64)), block(256);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint16_t* x = reinterpret_cast<const uint16_t*>(in);
    const uint16_t* w = reinterpret_cast<const uint16_t*>(weight);
    const uint16_t* mk = reinterpret_cast<const uint16_t*>(mask);
    if (out_f32)
        hipLaunchKernelGGL(learn::conv3d_kernel<true>, grid, block, 0, s, x, in_stride, in_coff, w, bias, out,
                           out_stride, out_coff, mk, mask_stride, mask_coff, vol, cin, cout, flip, relu);
    else
        hipLaunchKernelGGL(learn::conv3d_kernel<false>, grid, block, 0, s, x, in_stride, in_coff, w, bias, out,
                           out_stride, out_coff, mk, mask_stride, mask_coff, vol, cin, cout, flip, relu);
    return launch_status("conv3d launch failed");
}

int das_conv3d_wgrad(const void* in, int in_stride, int in_coff, const void* dy, int dy_stride, int dy_coff,
                     float* dw, float* db, float* work, int64_t work_floats, int D, int H, int W, int cin, int cout,
                     int chunk, void* stream) {
    if (!in || !dy || !dw || !db || !work) return lfail(DAS_EINVAL, "wgrad: null pointer");
    if (D < 1 || H < 1 || W < 1 || cin < 8 || cin % 8 || cout < 16 || cout % 16 || chunk < 32 || chunk % 32)
        return lfail(DAS_ESHAPE, "wgrad: bad sizes (chunk a positive multiple of 32)");
    const int64_t V = (int64_t)D * H * W;
    const int nparts = (int)((V + chunk - 1) / chunk);
    const int64_t K = 27LL * cin, nw = (int64_t)cout * K;
    if (in_stride < in_coff + cin || in_coff < 0 || dy_stride < dy_coff + cout || dy_coff < 0)
        return lfail(DAS_ESHAPE, "wgrad: channel slice outside its buffer");
    if (work_floats < (int64_t)nparts * (nw + cout)) return lfail(DAS_ESHAPE, "wgrad: work buffer too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float* part = work;
    float* part_db = work + (int64_t)nparts * nw;
    hipLaunchKernelGGL(learn::wgrad_kernel, dim3(nparts), dim3(256), 0, s, reinterpret_cast<const uint16_t*>(in),
                       in_stride, in_coff, reinterpret_cast<const uint16_t*>(dy), dy_stride, dy_coff, part, part_db,
                       learn::Vol{D, H, W}, cin, cout, chunk);
    hipLaunchKernelGGL(learn::reduce_parts_kernel, dim3(blocks_for(nw, 256)), dim3(256), 0, s, part, nparts, nw,
                       dw);
    hipLaunchKernelGGL(learn::reduce_parts_kernel, dim3(blocks_for(cout, 256)), dim3(256), 0, s, part_db, nparts,
                       (int64_t)cout, db);
    return launch_status("wgrad launch failed");
}

int64_t das_conv3d_wgrad_work(int D, int H, int W, int cin, int cout, int chunk) {
    if (chunk < 1) return -1;
    const int64_t V = (int64_t)D * H * W;
    return ((V + chunk - 1) / chunk) * ((int64_t)cout * 27 * cin + cout);
}

int das_transpose_weights(const void* w, void* wt, int cin, int cout, void* stream) {
    if (!w || !wt) return lfail(DAS_EINVAL, "transpose: null pointer");
    const int64_t n = (int64_t)cout * 27 * cin;
    hipLaunchKernelGGL(learn::transpose_w_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(w),
                       reinterpret_cast<uint16_t*>(wt), cin, cout);
    return launch_status("transpose launch failed");
}

int das_avgpool2(const void* in, int in_stride, int in_coff, void* out, int out_stride, int out_coff, int Do, int Ho,
                 int Wo, int c, void* stream) {
    if (!in || !out) return lfail(DAS_EINVAL, "avgpool2: null pointer");
    if (!slices_ok(in_stride, in_coff, out_stride, out_coff, c) || Do < 1 || Ho < 1 || Wo < 1)
        return lfail(DAS_ESHAPE, "avgpool2: bad sizes or channel slices");
    const int64_t n = (int64_t)Do * Ho * Wo * c;
    hipLaunchKernelGGL(learn::avgpool2_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(in), in_stride, in_coff,
                       reinterpret_cast<uint16_t*>(out), out_stride, out_coff, learn::Vol{Do, Ho, Wo}, c);
    return launch_status("avgpool2 launch failed");
}

int das_avgpool2_bwd(const void* gout, int gout_stride, int gout_coff, void* gin, int gin_stride, int gin_coff, int Di,
                     int Hi, int Wi, int c, int accumulate, void* stream) {
    if (!gout || !gin) return lfail(DAS_EINVAL, "avgpool2_bwd: null pointer");
    if (!slices_ok(gout_stride, gout_coff, gin_stride, gin_coff, c) || !even_dims(Di, Hi, Wi))
        return lfail(DAS_ESHAPE, "avgpool2_bwd: input dimensions must be even and positive; bad channel slices");
    const int64_t n = (int64_t)Di * Hi * Wi * c;
    hipLaunchKernelGGL(learn::avgpool2_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(gout), gout_stride,
                       gout_coff, reinterpret_cast<uint16_t*>(gin), gin_stride, gin_coff, learn::Vol{Di, Hi, Wi}, c,
                       accumulate);
    return launch_status("avgpool2_bwd launch failed");
}

int das_upsample2(const void* in, int in_stride, int in_coff, void* out, int out_stride, int out_coff, int Do, int Ho,
                  int Wo, int c, void* stream) {
    if (!in || !out) return lfail(DAS_EINVAL, "upsample2: null pointer");
    if (!slices_ok(in_stride, in_coff, out_stride, out_coff, c) || !even_dims(Do, Ho, Wo))
        return lfail(DAS_ESHAPE, "upsample2: output dimensions must be even and positive; bad channel slices");
    const int64_t n = (int64_t)Do * Ho * Wo * c;
    hipLaunchKernelGGL(learn::upsample2_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(in), in_stride, in_coff,
                       reinterpret_cast<uint16_t*>(out), out_stride, out_coff, learn::Vol{Do, Ho, Wo}, c);
    return launch_status("upsample2 launch failed");
}

int das_upsample2_bwd(const void* gout, int gout_stride, int gout_coff, void* gin, int gin_stride, int gin_coff,
                      const void* mask, int mask_stride, int mask_coff, int Di, int Hi, int Wi, int c, void* stream) {
    if (!gout || !gin) return lfail(DAS_EINVAL, "upsample2_bwd: null pointer");
    if (!slices_ok(gout_stride, gout_coff, gin_stride, gin_coff, c) || Di < 1 || Hi < 1 || Wi < 1 ||
        (mask && (mask_stride < mask_coff + c || mask_coff < 0)))
        return lfail(DAS_ESHAPE, "upsample2_bwd: bad sizes or channel slices");
    const int64_t n = (int64_t)Di * Hi * Wi * c;
    hipLaunchKernelGGL(learn::upsample2_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(gout), gout_stride,
                       gout_coff, reinterpret_cast<uint16_t*>(gin), gin_stride, gin_coff,
                       reinterpret_cast<const uint16_t*>(mask), mask_stride, mask_coff, learn::Vol{Di, Hi, Wi}, c);
    return launch_status("upsample2_bwd launch failed");
}

int das_add_mask(const void* a, int a_stride, int a_coff, const void* b, int b_stride, int b_coff, const void* mask,
                 int m_stride, int m_coff, void* g, int g_stride, int g_coff, int64_t V, int c, void* stream) {
    if (!a || !b || !g) return lfail(DAS_EINVAL, "add_mask: null pointer");
    if (V < 0 || !slices_ok(a_stride, a_coff, g_stride, g_coff, c) || b_stride < b_coff + c || b_coff < 0 ||
        (mask && (m_stride < m_coff + c || m_coff < 0)))
        return lfail(DAS_ESHAPE, "add_mask: bad sizes or channel slices");
    hipLaunchKernelGGL(learn::add_mask_kernel, dim3(blocks_for(V * c, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(a), a_stride, a_coff,
                       reinterpret_cast<const uint16_t*>(b), b_stride, b_coff, reinterpret_cast<const uint16_t*>(mask),
                       m_stride, m_coff, reinterpret_cast<uint16_t*>(g), g_stride, g_coff, V, c);
    return launch_status("add_mask launch failed");
}

int das_mse_residual(const float* net, int net_stride, const float* base, const float* target, int64_t V, void* grad,
                     int grad_stride, float* pred, float* loss_parts, void* stream) {
    if (!net || !base || !target || !loss_parts) return lfail(DAS_EINVAL, "mse: null pointer");
    if (net_stride < 2 || (grad && grad_stride < 2)) return lfail(DAS_ESHAPE, "mse: strides");
    hipLaunchKernelGGL(learn::mse_kernel, dim3(blocks_for(V, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), net, net_stride, base, target, V,
                       reinterpret_cast<uint16_t*>(grad), grad_stride, pred, loss_parts);
    return launch_status("mse launch failed");
}

int das_adam(float* w, float* m, float* v, const float* g, void* w_bf16, int64_t n, float lr, float beta1, float beta2,
             float eps, int step, void* stream) {
    if (!w || !m || !v || !g) return lfail(DAS_EINVAL, "adam: null pointer");
    if (step < 1) return lfail(DAS_EINVAL, "adam: step counts from 1");
    const float c1 = 1.0f / (1.0f - powf(beta1, (float)step)), c2 = 1.0f / (1.0f - powf(beta2, (float)step));
    hipLaunchKernelGGL(learn::adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), w, m, v, g, reinterpret_cast<uint16_t*>(w_bf16), n, lr,
                       beta1, beta2, eps, c1, c2);
    return launch_status("adam launch failed");
}

int das_f32_to_bf16(const float* x, void* y, int64_t n, void* stream) {
    if (!x || !y) return lfail(DAS_EINVAL, "cast: null pointer");
    hipLaunchKernelGGL(learn::f32_to_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), x, reinterpret_cast<uint16_t*>(y), n);
    return launch_status("cast launch failed");
}


int das_compound_features(const void* y, int n_in, int64_t V, float gain, void* x, int cin, float* base, float* work,
                          float* scale, void* stream) {
    if (!y || !x || !work || !scale) return lfail(DAS_EINVAL, "compound_features: null pointer");
    if (n_in < 1 || V < 1 || cin < 2 * n_in) return lfail(DAS_ESHAPE, "compound_features: need V >= 1, cin >= 2 n_in");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const float2* yy = reinterpret_cast<const float2*>(y);
    const unsigned nb = blocks_for(V, 256);
    hipLaunchKernelGGL(learn::sumsq_kernel, dim3(nb), dim3(256), 0, s, yy, n_in, V, work);
    hipLaunchKernelGGL(learn::rms_kernel, dim3(1), dim3(256), 0, s, work, (int)nb, V, scale);
    hipLaunchKernelGGL(learn::features_kernel, dim3(nb), dim3(256), 0, s, yy, n_in, V, gain, scale,
                       reinterpret_cast<uint16_t*>(x), cin, base);
    return launch_status("compound_features launch failed");
}

int64_t das_compound_work(int64_t V) { return V < 1 ? 0 : (V + 255) / 256; }

int das_compound_rescale(const void* y, int64_t V, const float* scale, int restore, void* out, void* stream) {
    if (!y || !scale || !out) return lfail(DAS_EINVAL, "compound_rescale: null pointer");
    if (V < 0) return lfail(DAS_ESHAPE, "compound_rescale: V < 0");
    if (V == 0) return DAS_OK;
    hipLaunchKernelGGL(learn::rescale_kernel, dim3(blocks_for(V, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const float2*>(y), V, scale,
                       restore ? 0 : 1, reinterpret_cast<float2*>(out));
    return launch_status("compound_rescale launch failed");
}

int das_compound_output(const float* net, int net_stride, const float* base, int64_t V, const float* scale, void* out,
                        void* stream) {
    if (!net || !base || !scale || !out) return lfail(DAS_EINVAL, "compound_output: null pointer");
    if (V < 0 || net_stride < 2) return lfail(DAS_ESHAPE, "compound_output: V < 0 or net_stride < 2");
    if (V == 0) return DAS_OK;
    hipLaunchKernelGGL(learn::compound_output_kernel, dim3(blocks_for(V, 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), net, net_stride, base, V, scale,
                       reinterpret_cast<float2*>(out));
    return launch_status("compound_output launch failed");
}

}  // extern "C"
