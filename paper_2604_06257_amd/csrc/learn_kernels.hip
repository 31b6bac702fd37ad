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

// Convolution on a brick of 8 (W) x 8 (H) x MT (D) output voxels per workgroup of 4 waves, for NT x 16 of the
// output channels (grid.y = channel groups).  Wave w owns the 4 x 4 (W x H) patch w of every depth slice (one
// 16-voxel MFMA row tile per slice) and the workgroup's output channels.  The input brick with its one-voxel
// halo, 10 x 10 x (MT + 2) voxels, is staged in LDS one channel chunk (CC channels) at a time, so each input
// value is read from global memory once per chunk instead of once per tap.
//
// K is ordered by in-plane offset (dx, dy) first: a K step of 32 holds 32 / CC in-plane taps of one depth offset
// dz (CC channels each).  The operand-A fragment of an in-plane offset at halo slice z (one 16-byte LDS read per
// lane) is the same for the three depth offsets, so it feeds three MFMAs: output slice z - 1 - dz for dz = -1, 0,
// 1 (the slices that exist).  Per chunk a wave reads (MT + 2) ceil(9 CC / 32) fragments for 3 MT ceil(9 CC / 32)
// MFMAs per channel tile, instead of one fragment per MFMA.  Weights (operand B) of the three depth offsets
// come from global memory (shared by all waves through the caches), one in-plane group ahead.
//
// With several channel chunks and DB the halo is double-buffered: the next chunk's loads are issued before the
// current chunk's MFMAs and written to the other buffer after them, one barrier per chunk (used for launches with
// few workgroups, in the 1 x 1 shape; elsewhere the second buffer's LDS costs more occupancy than it hides).
//
// Epilogue: bias, ReLU, then the tile goes through LDS as float [voxel][channel], and each thread writes 8
// channels of a voxel (one 16-byte store, two for float output) after the optional mask; with `vec` = 0
// (unaligned slices) the same values are stored one element at a time.
constexpr int kHaloW = 10, kHaloH = 10;

template <int MT, int NT, int CC, bool DB>
__global__ __launch_bounds__(256) void conv3d_kernel(const uint16_t* __restrict__ in, int in_stride, int in_coff,
                                                     const uint16_t* __restrict__ wk, const float* __restrict__ bias,
                                                     void* __restrict__ out, int out_stride, int out_coff, int out_f32,
                                                     const uint16_t* __restrict__ mask, int mask_stride, int mask_coff,
                                                     Vol vol, int Cin, int flip, int relu, int vec) {
    constexpr int HD = MT + 2;
    constexpr int NHALO = kHaloW * kHaloH * HD;
    constexpr int VP = CC + 8;             // LDS elements per halo voxel (padding spreads the banks)
    constexpr int TPK = 32 / CC;           // in-plane taps per K step: 1 (CC = 32), 2 (16), 4 (8)
    constexpr int NG = (9 + TPK - 1) / TPK;  // K steps per depth offset and chunk
    constexpr int CH = 16 * NT + 4;        // epilogue row (floats; the pad spreads the banks)
    constexpr int HALO_BYTES = NHALO * VP * 2 * (DB ? 2 : 1), OUT_BYTES = 64 * MT * CH * 4;
    constexpr int NITEMS = NHALO * (CC / 8), IPT = (NITEMS + 255) / 256;  // 16-byte halo items (per thread)
    __shared__ __attribute__((aligned(16))) char smem[HALO_BYTES > OUT_BYTES ? HALO_BYTES : OUT_BYTES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nbw = (vol.W + 7) / 8, nbh = (vol.H + 7) / 8;
    const int bx = blockIdx.x % nbw, by = (blockIdx.x / nbw) % nbh, bz = blockIdx.x / (nbw * nbh);
    // output channels [n0, n0 + 16 NT) of this workgroup (grid.y = channel groups)
    const int n0 = blockIdx.y * NT * 16;
    const int w0 = 8 * bx, h0 = 8 * by, d0 = MT * bz;
    const int K = 27 * Cin;
    const int s = flip ? -1 : 1;
    // this lane's operand-A voxel within its wave's patch (row lane & 15 of the MFMA tile)
    const int pw = 4 * (wave & 1), ph = 4 * (wave >> 1);
    const int rw = pw + (lane & 3), rh = ph + ((lane >> 2) & 3);
    // this lane's 8 elements of a K step: in-plane tap slot and channel offset within the chunk
    const int g = lane >> 4, slot = g / (CC / 8), cg = 8 * (g % (CC / 8));
    f32x4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // this thread's halo items: global offset (without the chunk's first channel; -1 outside the volume) and LDS
    // offset, the same for every chunk
    int64_t goff[IPT];
    int loff[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int it = threadIdx.x + 256 * i;
        const int hv = it / (CC / 8), c8 = it - hv * (CC / 8);
        const int hx = hv % kHaloW, hy = (hv / kHaloW) % kHaloH, hz = hv / (kHaloW * kHaloH);
        const int zw = w0 - 1 + hx, zh = h0 - 1 + hy, zd = d0 - 1 + hz;
        const bool inside = it < NITEMS && (unsigned)zw < (unsigned)vol.W && (unsigned)zh < (unsigned)vol.H &&
                            (unsigned)zd < (unsigned)vol.D;
        goff[i] = inside ? (((int64_t)zd * vol.H + zh) * vol.W + zw) * in_stride + in_coff + 8 * c8 : -1;
        loff[i] = it < NITEMS ? hv * VP + 8 * c8 : -1;
    }
    bf16x8 pre[IPT];
    auto fetch = [&](int cc0) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            pre[i] = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
            if (goff[i] >= 0) pre[i] = *reinterpret_cast<const bf16x8*>(in + goff[i] + cc0);
        }
    };
    auto put = [&](uint16_t* buf) {
#pragma unroll
        for (int i = 0; i < IPT; ++i)
            if (loff[i] >= 0) *reinterpret_cast<bf16x8*>(&buf[loff[i]]) = pre[i];
    };
    uint16_t* const hbuf0 = reinterpret_cast<uint16_t*>(smem);
    uint16_t* const hbuf1 = hbuf0 + (DB ? NHALO * VP : 0);
    fetch(0);
    put(hbuf0);
    __syncthreads();
    for (int cc0 = 0, ci = 0; cc0 < Cin; cc0 += CC, ++ci) {
        const uint16_t* halo = (ci & 1) ? hbuf1 : hbuf0;
        const bool more = cc0 + CC < Cin;
        if (DB && more) fetch(cc0 + CC);  // in flight during this chunk's MFMAs
        // B of in-plane group q: slot dzi holds the weights of depth offset dz with s dz = dzi - 1 (so that halo
        // slice z feeds output slice z - dzi); taps past the ninth are zero
        bf16x8 b[3][NT], bn[3][NT];
        auto load_b = [&](int q, bf16x8(&dst)[3][NT]) {
            const int idx = q * TPK + slot;
            const int dx = idx % 3 - 1, dy = idx / 3 - 1;
#pragma unroll
            for (int dzi = 0; dzi < 3; ++dzi) {
                const int dz = s * (dzi - 1);
                const int tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                const uint16_t* wp = wk + (int64_t)(n0 + (lane & 15)) * K + tap * Cin + cc0 + cg;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    dst[dzi][t] = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
                    if (idx < 9) dst[dzi][t] = *reinterpret_cast<const bf16x8*>(wp + (int64_t)t * 16 * K);
                }
            }
        };
        load_b(0, b);
        for (int q = 0; q < NG; ++q) {
            if (q + 1 < NG) load_b(q + 1, bn);
            // operand A: this lane's voxel shifted in-plane by s (dx, dy); padding slots read the centre (their
            // weights are zero)
            const int idx = q * TPK + slot, ii = idx < 9 ? idx : 4;
            const int dx = ii % 3 - 1, dy = ii / 3 - 1;
            const uint16_t* ap = &halo[((rh + 1 + s * dy) * kHaloW + (rw + 1 + s * dx)) * VP + cg];
#pragma unroll
            for (int z = 0; z < HD; ++z) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(ap + z * kHaloW * kHaloH * VP);
#pragma unroll
                for (int dzi = 0; dzi < 3; ++dzi) {
                    const int m = z - dzi;
                    if (m >= 0 && m < MT) {
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[dzi][t], acc[m][t], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int dzi = 0; dzi < 3; ++dzi)
#pragma unroll
                for (int t = 0; t < NT; ++t) b[dzi][t] = bn[dzi][t];
        }
        if (more) {
            if (DB) {
                put((ci & 1) ? hbuf0 : hbuf1);  // the other buffer: every wave finished reading it a chunk ago
            } else {
                __syncthreads();  // single buffer: all waves done with this chunk before it is overwritten
                fetch(cc0 + CC);
                put(hbuf0);
            }
        }
        __syncthreads();
    }
    // epilogue: result row 4 (lane / 16) + r of tile (m, t) is voxel (pw + r, ph + lane / 16) of slice m, channel
    // t * 16 + lane % 16; bias and ReLU here, the tile into LDS as [voxel][channel] (the loop ended on a barrier)
    float* ot = reinterpret_cast<float*>(smem);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int ch = t * 16 + (lane & 15);
        const float bn_ = bias ? bias[n0 + ch] : 0.0f;
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float y = acc[m][t][r] + bn_;
                if (relu) y = fmaxf(y, 0.0f);
                ot[((m * 8 + ph + (lane >> 4)) * 8 + pw + r) * CH + ch] = y;
            }
    }
    __syncthreads();
    for (int it = threadIdx.x; it < 64 * MT * 2 * NT; it += 256) {
        const int vl = it / (2 * NT), c8 = it - vl * (2 * NT);
        const int zw = w0 + (vl & 7), zh = h0 + ((vl >> 3) & 7), zd = d0 + (vl >> 6);
        if (zw >= vol.W || zh >= vol.H || zd >= vol.D) continue;
        const int64_t v = ((int64_t)zd * vol.H + zh) * vol.W + zw;
        const int n = n0 + 8 * c8;
        const float4 lo = *reinterpret_cast<const float4*>(&ot[vl * CH + 8 * c8]);
        const float4 hi = *reinterpret_cast<const float4*>(&ot[vl * CH + 8 * c8 + 4]);
        float y[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
        if (mask) {
            const uint16_t* mp = mask + v * mask_stride + mask_coff + n;
            if (vec) {
                const bf16x8 mk = *reinterpret_cast<const bf16x8*>(mp);
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (!(bf2f((uint16_t)mk[e]) > 0.0f)) y[e] = 0.0f;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (!(bf2f(mp[e]) > 0.0f)) y[e] = 0.0f;
            }
        }
        if (out_f32) {
            float* op = reinterpret_cast<float*>(out) + v * out_stride + out_coff + n;
            if (vec) {
                *reinterpret_cast<float4*>(op) = make_float4(y[0], y[1], y[2], y[3]);
                *reinterpret_cast<float4*>(op + 4) = make_float4(y[4], y[5], y[6], y[7]);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) op[e] = y[e];
            }
        } else {
            uint16_t* op = reinterpret_cast<uint16_t*>(out) + v * out_stride + out_coff + n;
            if (vec) {
                bf16x8 o;
#pragma unroll
                for (int e = 0; e < 8; ++e) o[e] = (short)f2bf(y[e]);
                *reinterpret_cast<bf16x8*>(op) = o;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) op[e] = f2bf(y[e]);
            }
        }
    }
}

// Weight gradient, split over voxel chunks:
//   part[b][n][k] = sum_{v in chunk b} dy[v][n] * in[v + off(tap k)][c k],  part_db[b][n] = sum_v dy[v][n]
// One wave per workgroup owns (chunk, tap, NB x 16 output channels, CB x 16 input channels).  The reduction
// runs over voxels, which are not contiguous for a fixed channel in the channels-last layout, so every
// 32-voxel step stages dy and the shifted input transposed into LDS ([channel][voxel]); both MFMA operands
// are then one 16-byte LDS read per lane.
constexpr int kWgPitch = 40;  // LDS row: 32 voxels + 8 pad (80 B: 16-byte aligned, rows spread over banks)

template <int NB, int CB>
__global__ __launch_bounds__(64) void wgrad_kernel(const uint16_t* __restrict__ in, int in_stride, int in_coff,
                                                   const uint16_t* __restrict__ dy, int dy_stride, int dy_coff,
                                                   float* __restrict__ part, float* __restrict__ part_db, Vol vol,
                                                   int Cin, int Cout, int chunk, int n_cgroups) {
    __shared__ __attribute__((aligned(16))) uint16_t dyT[NB * 16 * kWgPitch];
    __shared__ __attribute__((aligned(16))) uint16_t xT[CB * 16 * kWgPitch];
    const int lane = threadIdx.x;
    const int64_t V = (int64_t)vol.D * vol.H * vol.W;
    const int K = 27 * Cin;
    const int b = blockIdx.x, tap = blockIdx.y;
    const int ng = blockIdx.z / n_cgroups, cg = blockIdx.z - ng * n_cgroups;
    const int n0 = ng * NB * 16, c0 = cg * CB * 16;
    const int64_t vbeg = (int64_t)b * chunk;
    const int64_t vend = (vbeg + chunk < V) ? vbeg + chunk : V;
    const int dz = tap / 9 - 1, dyy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int64_t off = ((int64_t)dz * vol.H + dyy) * vol.W + dx;
    const bool do_db = (tap == 0 && cg == 0);
    f32x4 acc[NB][CB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float dbs = 0.0f;
    // staging map: lane -> (voxel = lane % 32, 8-channel group = lane / 32 + 2 r)
    const int sv = lane & 31, sg = lane >> 5;
    for (int64_t vc = vbeg; vc < vend; vc += 32) {
        const int64_t v = vc + sv;
        const bool vin = v < vend;
        int w = 0, h = 0, d = 0;
        if (vin) {  // V < 2^31: 32-bit index arithmetic
            const uint32_t vu = (uint32_t)v, q = vu / (uint32_t)vol.W;
            w = (int)(vu - q * (uint32_t)vol.W);
            h = (int)(q % (uint32_t)vol.H);
            d = (int)(q / (uint32_t)vol.H);
        }
        const bool nbr = vin && (unsigned)(d + dz) < (unsigned)vol.D && (unsigned)(h + dyy) < (unsigned)vol.H &&
                         (unsigned)(w + dx) < (unsigned)vol.W;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int g = sg + 2 * r;  // 8-channel group within the NB x 16 output channels
            bf16x8 val = {0, 0, 0, 0, 0, 0, 0, 0};
            if (vin) val = *reinterpret_cast<const bf16x8*>(dy + v * dy_stride + dy_coff + n0 + 8 * g);
#pragma unroll
            for (int j = 0; j < 8; ++j) dyT[(8 * g + j) * kWgPitch + sv] = (uint16_t)val[j];
        }
#pragma unroll
        for (int r = 0; r < CB; ++r) {
            const int g = sg + 2 * r;
            const int c = c0 + 8 * g;
            bf16x8 val = {0, 0, 0, 0, 0, 0, 0, 0};
            if (nbr && c < Cin) val = *reinterpret_cast<const bf16x8*>(in + (v + off) * in_stride + in_coff + c);
#pragma unroll
            for (int j = 0; j < 8; ++j) xT[(8 * g + j) * kWgPitch + sv] = (uint16_t)val[j];
        }
        __syncthreads();
        bf16x8 A[NB], B[CB];
#pragma unroll
        for (int i = 0; i < NB; ++i)
            A[i] = *reinterpret_cast<const bf16x8*>(&dyT[(i * 16 + (lane & 15)) * kWgPitch + 8 * (lane >> 4)]);
#pragma unroll
        for (int j = 0; j < CB; ++j)
            B[j] = *reinterpret_cast<const bf16x8*>(&xT[(j * 16 + (lane & 15)) * kWgPitch + 8 * (lane >> 4)]);
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[i], B[j], acc[i][j], 0, 0, 0);
        if (do_db && lane < NB * 16)
            for (int u = 0; u < 32; ++u) dbs += bf2f(dyT[lane * kWgPitch + u]);
    }
    float* pb = part + (int64_t)b * Cout * K;
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = n0 + i * 16 + 4 * (lane >> 4) + r, c = c0 + j * 16 + (lane & 15);
                if (c < Cin) pb[(int64_t)n * K + tap * Cin + c] = acc[i][j][r];
            }
    if (do_db && lane < NB * 16) part_db[(int64_t)b * Cout + n0 + lane] = dbs;
}

// dw[i] = sum_b part[b][i], i over Cout * K (same for db): 32 outputs per workgroup, the parts split over 8
// thread rows (row r sums parts r, r + 8, ... in order), the 8 row sums added in row order: deterministic.
__global__ __launch_bounds__(256) void reduce_parts_kernel(const float* __restrict__ part, int nparts, int64_t n,
                                                           float* __restrict__ out) {
    __shared__ float red[8][32];
    const int col = threadIdx.x & 31, row = threadIdx.x >> 5;
    const int64_t i = (int64_t)blockIdx.x * 32 + col;
    float s = 0.0f;
    if (i < n)
        for (int b = row; b < nparts; b += 8) s += part[(int64_t)b * n + i];
    red[row][col] = s;
    __syncthreads();
    if (row == 0 && i < n) {
        float t = red[0][col];
#pragma unroll
        for (int r = 1; r < 8; ++r) t += red[r][col];
        out[i] = t;
    }
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

// Vector forms of the upsampling, the pooling gradient and add_mask: 8 BF16 channels (16 bytes) per thread, for
// slices whose channel count, stride and offset are multiples of 8.  Same arithmetic in the same order per
// element, so the results are bitwise those of the scalar kernels.  Thread (x, y) of block (bx, by, d): x over
// (w, channel group), h = 4 by + y, d = depth of the volume the thread writes.
__device__ __forceinline__ void unpack8(const uint4& r, float (&f)[8]) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f[2 * j] = __uint_as_float(w[j] << 16);
        f[2 * j + 1] = __uint_as_float(w[j] & 0xffff0000u);
    }
}

__device__ __forceinline__ uint4 pack8(const float (&f)[8]) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = (uint32_t)f2bf(f[2 * j]) | ((uint32_t)f2bf(f[2 * j + 1]) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

struct V8Pos {
    int d, h, w, c;
    bool ok;
};

__device__ __forceinline__ V8Pos v8_pos(const Vol& v, int C8) {
    V8Pos p;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    p.h = blockIdx.y * blockDim.y + threadIdx.y;
    p.d = blockIdx.z;
    p.w = x / C8;
    p.c = (x - p.w * C8) * 8;
    p.ok = x < v.W * C8 && p.h < v.H;
    return p;
}

__global__ void avgpool2_bwd_v8_kernel(const uint16_t* __restrict__ gout, int gout_stride, int gout_coff,
                                       uint16_t* __restrict__ gin, int gin_stride, int gin_coff, Vol vi, int C8,
                                       int accumulate) {
    const V8Pos p = v8_pos(vi, C8);
    if (!p.ok) return;
    const int64_t v = ((int64_t)p.d * vi.H + p.h) * vi.W + p.w;
    const int64_t vp = ((int64_t)(p.d >> 1) * (vi.H >> 1) + (p.h >> 1)) * (vi.W >> 1) + (p.w >> 1);
    float g[8];
    unpack8(*reinterpret_cast<const uint4*>(gout + vp * gout_stride + gout_coff + p.c), g);
#pragma unroll
    for (int j = 0; j < 8; ++j) g[j] = 0.125f * g[j];
    uint4* dst = reinterpret_cast<uint4*>(gin + v * gin_stride + gin_coff + p.c);
    if (accumulate) {
        float a[8];
        unpack8(*dst, a);
#pragma unroll
        for (int j = 0; j < 8; ++j) g[j] += a[j];
    }
    *dst = pack8(g);
}

__global__ void upsample2_v8_kernel(const uint16_t* __restrict__ in, int in_stride, int in_coff,
                                    uint16_t* __restrict__ out, int out_stride, int out_coff, Vol vo, int C8) {
    const V8Pos p = v8_pos(vo, C8);
    if (!p.ok) return;
    const int64_t v = ((int64_t)p.d * vo.H + p.h) * vo.W + p.w;
    const int64_t vp = ((int64_t)(p.d >> 1) * (vo.H >> 1) + (p.h >> 1)) * (vo.W >> 1) + (p.w >> 1);
    *reinterpret_cast<uint4*>(out + v * out_stride + out_coff + p.c) =
        *reinterpret_cast<const uint4*>(in + vp * in_stride + in_coff + p.c);
}

__global__ void upsample2_bwd_v8_kernel(const uint16_t* __restrict__ gout, int gout_stride, int gout_coff,
                                        uint16_t* __restrict__ gin, int gin_stride, int gin_coff,
                                        const uint16_t* __restrict__ mask, int mask_stride, int mask_coff, Vol vi,
                                        int C8) {
    const V8Pos p = v8_pos(vi, C8);
    if (!p.ok) return;
    const int Ho = 2 * vi.H, Wo = 2 * vi.W;
    float s[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] = 0.0f;
    for (int q = 0; q < 8; ++q) {
        const int64_t vo = ((int64_t)(2 * p.d + (q >> 2)) * Ho + (2 * p.h + ((q >> 1) & 1))) * Wo + (2 * p.w + (q & 1));
        float f[8];
        unpack8(*reinterpret_cast<const uint4*>(gout + vo * gout_stride + gout_coff + p.c), f);
#pragma unroll
        for (int j = 0; j < 8; ++j) s[j] += f[j];
    }
    const int64_t v = ((int64_t)p.d * vi.H + p.h) * vi.W + p.w;
    if (mask) {
        float m[8];
        unpack8(*reinterpret_cast<const uint4*>(mask + v * mask_stride + mask_coff + p.c), m);
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (!(m[j] > 0.0f)) s[j] = 0.0f;
    }
    *reinterpret_cast<uint4*>(gin + v * gin_stride + gin_coff + p.c) = pack8(s);
}

// add_mask over V voxels x C8 channel groups (V * C8 < 2^31, so the index split is a 32-bit division)
__global__ void add_mask_v8_kernel(const uint16_t* __restrict__ a, int a_stride, int a_coff,
                                   const uint16_t* __restrict__ b, int b_stride, int b_coff,
                                   const uint16_t* __restrict__ mask, int m_stride, int m_coff,
                                   uint16_t* __restrict__ g, int g_stride, int g_coff, int n, int C8) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int v32 = i / C8;
    const int c = (i - v32 * C8) * 8;
    const int64_t v = v32;
    float x[8], y[8];
    unpack8(*reinterpret_cast<const uint4*>(a + v * a_stride + a_coff + c), x);
    unpack8(*reinterpret_cast<const uint4*>(b + v * b_stride + b_coff + c), y);
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] += y[j];
    if (mask) {
        float m[8];
        unpack8(*reinterpret_cast<const uint4*>(mask + v * m_stride + m_coff + c), m);
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (!(m[j] > 0.0f)) x[j] = 0.0f;
    }
    *reinterpret_cast<uint4*>(g + v * g_stride + g_coff + c) = pack8(x);
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
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
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
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
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
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
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

// The 8-channel vector kernels apply when every slice is 16-byte aligned (pointer, stride and offset) and the
// volume fits their grid (x = W * C / 8 in 64-thread blocks, y = H in blocks of 4, z = D).
bool v8_slice(const void* p, int stride, int coff) {
    return p == nullptr || (reinterpret_cast<uintptr_t>(p) % 16 == 0 && stride % 8 == 0 && coff % 8 == 0);
}

bool v8_volume(int D, int H, int W, int c) {
    return c % 8 == 0 && (int64_t)W * (c / 8) < (int64_t)1 << 30 && D <= 65535 && (H + 3) / 4 <= 65535;
}

dim3 v8_grid(int D, int H, int W, int c) {
    return dim3((unsigned)(((int64_t)W * (c / 8) + 63) / 64), (unsigned)((H + 3) / 4), (unsigned)D);
}

const dim3 kV8Block(64, 4, 1);
bool slices_ok(int s1, int o1, int s2, int o2, int c) { return c >= 1 && o1 >= 0 && o2 >= 0 && s1 >= o1 + c && s2 >= o2 + c; }
bool even_dims(int D, int H, int W) { return D >= 2 && H >= 2 && W >= 2 && D % 2 == 0 && H % 2 == 0 && W % 2 == 0; }
int launch_status(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return lfail(DAS_EHIP, what);
    return DAS_OK;
}

// Workgroup shape: MT depth slices and NT channel tiles (NT divides Cout / 16).  Candidates in order of
// decreasing work per workgroup; the first with at least 512 workgroups (two per CU) is used, else the one
// with the most workgroups (small volumes).  The input chunk is the largest of 32, 16, 8 channels dividing Cin.
template <int MT, int NT, int CC>
void launch_conv_t(int ngroups, int out_f32, const learn::Vol& vol, hipStream_t s, const uint16_t* x, int in_stride,
                   int in_coff, const uint16_t* w, const float* bias, void* out, int out_stride, int out_coff,
                   const uint16_t* mk, int mask_stride, int mask_coff, int cin, int flip, int relu) {
    const unsigned nb = (unsigned)(((vol.W + 7) / 8) * ((vol.H + 7) / 8) * ((vol.D + MT - 1) / MT));
    // 16-byte output (and mask) accesses: 8 channels of a voxel start on a 16-byte boundary
    const int ea = out_f32 ? 4 : 8;
    const bool vec = reinterpret_cast<uintptr_t>(out) % 16 == 0 && out_stride % ea == 0 && out_coff % ea == 0 &&
                     (!mk || (reinterpret_cast<uintptr_t>(mk) % 16 == 0 && mask_stride % 8 == 0 && mask_coff % 8 == 0));
    // double-buffered halo only for small launches (few workgroups: latency-bound), which take the 1 x 1 shape;
    // on large ones the second buffer costs occupancy (d0a at 96^3: 84 -> 94 us; the 24^3 and 12^3 layers gain
    // ~1 us each).  Other shapes are not instantiated double-buffered (compile time).
    if constexpr (MT == 1 && NT == 1) {
        if (cin > CC && (int64_t)nb * ngroups <= 768) {
            hipLaunchKernelGGL((learn::conv3d_kernel<MT, NT, CC, true>), dim3(nb, ngroups), dim3(256), 0, s, x,
                               in_stride, in_coff, w, bias, out, out_stride, out_coff, out_f32, mk, mask_stride,
                               mask_coff, vol, cin, flip, relu, (int)vec);
            return;
        }
    }
    hipLaunchKernelGGL((learn::conv3d_kernel<MT, NT, CC, false>), dim3(nb, ngroups), dim3(256), 0, s, x, in_stride,
                       in_coff, w, bias, out, out_stride, out_coff, out_f32, mk, mask_stride, mask_coff, vol, cin,
                       flip, relu, (int)vec);
}

template <int MT, int NT>
void launch_conv_cc(int ngroups, int out_f32, const learn::Vol& vol, hipStream_t s, const uint16_t* x,
                    int in_stride, int in_coff, const uint16_t* w, const float* bias, void* out, int out_stride,
                    int out_coff, const uint16_t* mk, int mask_stride, int mask_coff, int cin, int flip, int relu) {
    if (cin % 32 == 0)
        launch_conv_t<MT, NT, 32>(ngroups, out_f32, vol, s, x, in_stride, in_coff, w, bias, out, out_stride, out_coff,
                                  mk, mask_stride, mask_coff, cin, flip, relu);
    else if (cin % 16 == 0)
        launch_conv_t<MT, NT, 16>(ngroups, out_f32, vol, s, x, in_stride, in_coff, w, bias, out, out_stride, out_coff,
                                  mk, mask_stride, mask_coff, cin, flip, relu);
    else
        launch_conv_t<MT, NT, 8>(ngroups, out_f32, vol, s, x, in_stride, in_coff, w, bias, out, out_stride, out_coff,
                                 mk, mask_stride, mask_coff, cin, flip, relu);
}

struct ConvShape {
    int mt, nt;
};

ConvShape pick_conv_shape(int nt_total, const learn::Vol& vol) {
    // (MT, NT) instantiated below, by decreasing MT * NT
    static const ConvShape cands[] = {{1, 8}, {1, 7}, {1, 6}, {1, 5}, {2, 4}, {2, 3}, {4, 2}, {4, 1},
                                      {1, 4}, {1, 3}, {1, 2}, {1, 1}};
    auto blocks = [&](const ConvShape& c) {
        return (int64_t)((vol.W + 7) / 8) * ((vol.H + 7) / 8) * ((vol.D + c.mt - 1) / c.mt) * (nt_total / c.nt);
    };
    ConvShape best{1, 1};
    int64_t best_blocks = -1;
    int best_work = 0;
    for (const ConvShape& c : cands) {
        if (nt_total % c.nt) continue;
        const int64_t b = blocks(c);
        if (b >= 512 && c.mt * c.nt > best_work) {
            best = c;
            best_work = c.mt * c.nt;
            best_blocks = b;
        }
    }
    if (best_work > 0) return best;
    for (const ConvShape& c : cands) {
        if (nt_total % c.nt) continue;
        if (blocks(c) > best_blocks) {
            best = c;
            best_blocks = blocks(c);
        }
    }
    return best;
}

void launch_conv(int nt_total, int out_f32, const learn::Vol& vol, hipStream_t s, const uint16_t* x, int in_stride,
                 int in_coff, const uint16_t* w, const float* bias, void* out, int out_stride, int out_coff,
                 const uint16_t* mk, int mask_stride, int mask_coff, int cin, int flip, int relu) {
    const ConvShape c = pick_conv_shape(nt_total, vol);
    const int ng = nt_total / c.nt;
#define LC(M, N)                                                                                                  \
    if (c.mt == M && c.nt == N) {                                                                                 \
        launch_conv_cc<M, N>(ng, out_f32, vol, s, x, in_stride, in_coff, w, bias, out, out_stride, out_coff, mk,  \
                             mask_stride, mask_coff, cin, flip, relu);                                            \
        return;                                                                                                   \
    }
    LC(1, 8) LC(1, 7) LC(1, 6) LC(1, 5) LC(2, 4) LC(2, 3) LC(4, 2) LC(4, 1) LC(1, 4) LC(1, 3) LC(1, 2) LC(1, 1)
#undef LC
}

// Largest divisor of n that is at most 4: channel tiles per wave in the weight gradient.
int tiles_per_wave(int n) {
    for (int d = 4; d > 1; --d)
        if (n % d == 0) return d;
    return 1;
}

template <int NB, int CB>
void launch_wgrad_t(int nt, int ct, int nparts, hipStream_t s, const uint16_t* in, int in_stride, int in_coff,
                    const uint16_t* dy, int dy_stride, int dy_coff, float* part, float* part_db, learn::Vol vol,
                    int cin, int cout, int chunk) {
    const int ncg = ct / CB;
    hipLaunchKernelGGL((learn::wgrad_kernel<NB, CB>), dim3(nparts, 27, (nt / NB) * ncg), dim3(64), 0, s, in,
                       in_stride, in_coff, dy, dy_stride, dy_coff, part, part_db, vol, cin, cout, chunk, ncg);
}

void launch_wgrad(int nt, int ct, int nparts, hipStream_t s, const uint16_t* in, int in_stride, int in_coff,
                  const uint16_t* dy, int dy_stride, int dy_coff, float* part, float* part_db, learn::Vol vol,
                  int cin, int cout, int chunk) {
    const int nb = tiles_per_wave(nt), cb = tiles_per_wave(ct);
#define LW(A, B)                                                                                             \
    if (nb == A && cb == B) {                                                                                \
        launch_wgrad_t<A, B>(nt, ct, nparts, s, in, in_stride, in_coff, dy, dy_stride, dy_coff, part, part_db, \
                             vol, cin, cout, chunk);                                                         \
        return;                                                                                              \
    }
    LW(1, 1) LW(1, 2) LW(1, 3) LW(1, 4) LW(2, 1) LW(2, 2) LW(2, 3) LW(2, 4)
    LW(3, 1) LW(3, 2) LW(3, 3) LW(3, 4) LW(4, 1) LW(4, 2) LW(4, 3) LW(4, 4)
#undef LW
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
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint16_t* x = reinterpret_cast<const uint16_t*>(in);
    const uint16_t* w = reinterpret_cast<const uint16_t*>(weight);
    const uint16_t* mk = reinterpret_cast<const uint16_t*>(mask);
    (void)V;
    launch_conv(cout / 16, out_f32 != 0, vol, s, x, in_stride, in_coff, w, bias, out, out_stride, out_coff, mk,
                mask_stride, mask_coff, cin, flip, relu);
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
    if (in_stride < in_coff + cin || in_coff < 0 || dy_stride < dy_coff + cout || dy_coff < 0 || in_stride % 8 ||
        in_coff % 8 || dy_stride % 8 || dy_coff % 8)
        return lfail(DAS_ESHAPE, "wgrad: channel slices outside their buffers or not multiples of 8");
    if ((int64_t)D * H * W >= (int64_t)1 << 31) return lfail(DAS_ESHAPE, "wgrad: volume above 2^31 voxels");
    if (!al(in, 16) || !al(dy, 16)) return lfail(DAS_EALIGN, "wgrad: input and dy must be 16-byte aligned");
    if (work_floats < (int64_t)nparts * (nw + cout)) return lfail(DAS_ESHAPE, "wgrad: work buffer too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float* part = work;
    float* part_db = work + (int64_t)nparts * nw;
    launch_wgrad(cout / 16, (cin + 15) / 16, nparts, s, reinterpret_cast<const uint16_t*>(in), in_stride, in_coff,
                 reinterpret_cast<const uint16_t*>(dy), dy_stride, dy_coff, part, part_db, learn::Vol{D, H, W}, cin,
                 cout, chunk);
    hipLaunchKernelGGL(learn::reduce_parts_kernel, dim3(blocks_for(nw, 32)), dim3(256), 0, s, part, nparts, nw, dw);
    hipLaunchKernelGGL(learn::reduce_parts_kernel, dim3(blocks_for(cout, 32)), dim3(256), 0, s, part_db, nparts,
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
    // one channel per thread: the 8-channel form (8x fewer threads, eight 16-byte gathers each) measured slower
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
    if (v8_volume(Di, Hi, Wi, c) && v8_slice(gout, gout_stride, gout_coff) && v8_slice(gin, gin_stride, gin_coff)) {
        hipLaunchKernelGGL(learn::avgpool2_bwd_v8_kernel, v8_grid(Di, Hi, Wi, c), kV8Block, 0,
                           reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(gout), gout_stride,
                           gout_coff, reinterpret_cast<uint16_t*>(gin), gin_stride, gin_coff, learn::Vol{Di, Hi, Wi},
                           c / 8, accumulate);
        return launch_status("avgpool2_bwd launch failed");
    }
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
    if (v8_volume(Do, Ho, Wo, c) && v8_slice(in, in_stride, in_coff) && v8_slice(out, out_stride, out_coff)) {
        hipLaunchKernelGGL(learn::upsample2_v8_kernel, v8_grid(Do, Ho, Wo, c), kV8Block, 0,
                           reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(in), in_stride,
                           in_coff, reinterpret_cast<uint16_t*>(out), out_stride, out_coff, learn::Vol{Do, Ho, Wo},
                           c / 8);
        return launch_status("upsample2 launch failed");
    }
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
    if (v8_volume(Di, Hi, Wi, c) && v8_slice(gout, gout_stride, gout_coff) && v8_slice(gin, gin_stride, gin_coff) &&
        v8_slice(mask, mask_stride, mask_coff)) {
        hipLaunchKernelGGL(learn::upsample2_bwd_v8_kernel, v8_grid(Di, Hi, Wi, c), kV8Block, 0,
                           reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(gout), gout_stride,
                           gout_coff, reinterpret_cast<uint16_t*>(gin), gin_stride, gin_coff,
                           reinterpret_cast<const uint16_t*>(mask), mask_stride, mask_coff, learn::Vol{Di, Hi, Wi},
                           c / 8);
        return launch_status("upsample2_bwd launch failed");
    }
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
    if (c % 8 == 0 && V * (c / 8) < ((int64_t)1 << 31) && v8_slice(a, a_stride, a_coff) &&
        v8_slice(b, b_stride, b_coff) && v8_slice(mask, m_stride, m_coff) && v8_slice(g, g_stride, g_coff)) {
        const int n = (int)(V * (c / 8));
        if (n == 0) return DAS_OK;
        hipLaunchKernelGGL(learn::add_mask_v8_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                           reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const uint16_t*>(a), a_stride,
                           a_coff, reinterpret_cast<const uint16_t*>(b), b_stride, b_coff,
                           reinterpret_cast<const uint16_t*>(mask), m_stride, m_coff, reinterpret_cast<uint16_t*>(g),
                           g_stride, g_coff, n, c / 8);
        return launch_status("add_mask launch failed");
    }
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
