// gfx950 post-processing of beamformed volumes y [V][F] (complex64, frame innermost):
// B-mode log compression and Power Doppler with an SVD clutter filter.
//
// B-mode: per-frame peak of |y| (block maxima through an LDS integer max, which
// is exact and order independent for non-negative floats), then
// max(20 log10(|y| / peak), -dr).
//
// Power Doppler: the right singular vectors of the Casorati matrix C = y are the
// eigenvectors of the Gram matrix G = C^H C (F x F, Hermitian).  G is summed in
// float64 over voxel chunks (partials added in chunk order: deterministic), then
// diagonalised by one workgroup with the parallel cyclic Jacobi method (round-
// robin ordering: F/2 disjoint rotations at a time, each a complex phase
// followed by a real plane rotation).  The energy a voxel keeps after removing
// the k largest components is |c|^2 - sum_{j<k} |c . v_j|^2, evaluated in float64.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "das_post.h"

namespace post {

constexpr int kMaxF = 32;

__device__ __forceinline__ float cabs2f(float2 z) { return z.x * z.x + z.y * z.y; }

// part[b][f] = max over the block's 256 voxels of |y[v][f]|
__global__ __launch_bounds__(256) void frame_max_kernel(const float2* __restrict__ y, int64_t V, int F,
                                                        float* __restrict__ part) {
    __shared__ unsigned int mx[1024];
    for (int f = threadIdx.x; f < F; f += 256) mx[f] = 0u;
    __syncthreads();
    const int64_t v0 = (int64_t)blockIdx.x * 256;
    const int64_t nv = (V - v0 < 256) ? V - v0 : 256;
    const int64_t n = nv * F;
    const float2* base = y + v0 * F;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const float a = sqrtf(cabs2f(base[i]));
        atomicMax(&mx[(int)(i % F)], __float_as_uint(a));  // non-negative floats order as their bit patterns
    }
    __syncthreads();
    for (int f = threadIdx.x; f < F; f += 256) part[(int64_t)blockIdx.x * F + f] = __uint_as_float(mx[f]);
}

// peak[f] = max_b part[b][f]; one block per frame
__global__ __launch_bounds__(256) void frame_peak_kernel(const float* __restrict__ part, int nb, int F,
                                                         float* __restrict__ peak) {
    __shared__ float red[256];
    const int f = blockIdx.x;
    float m = 0.0f;
    for (int b = threadIdx.x; b < nb; b += 256) m = fmaxf(m, part[(int64_t)b * F + f]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) peak[f] = red[0];
}

__global__ void bmode_kernel(const float2* __restrict__ y, int64_t n, int F, const float* __restrict__ peak,
                             float floor_db, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float p = peak[i % F];
    const float a = sqrtf(cabs2f(y[i]));
    float db = floor_db;
    if (p > 0.0f && a > 0.0f) db = fmaxf(20.0f * log10f(a / p), floor_db);
    out[i] = db;
}

// part[i F + j][b] = sum over block b's voxel chunk of conj(y[v][i]) y[v][j]   (float64 complex, F <= 32)
__global__ __launch_bounds__(256) void gram_partial_kernel(const float2* __restrict__ y, int64_t V, int F,
                                                           int64_t chunk, double2* __restrict__ part) {
    __shared__ float2 tile[64 * kMaxF];
    const int64_t vb = (int64_t)blockIdx.x * chunk;
    const int64_t ve = (vb + chunk < V) ? vb + chunk : V;
    const int npair = F * F;
    double2 acc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = make_double2(0.0, 0.0);
    for (int64_t v = vb; v < ve; v += 64) {
        const int nv = (int)((ve - v < 64) ? ve - v : 64);
        __syncthreads();
        for (int i = threadIdx.x; i < nv * F; i += 256) tile[i] = y[v * F + i];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pr = threadIdx.x + 256 * r;
            if (pr < npair) {
                const int i = pr / F, j = pr % F;
                double re = acc[r].x, im = acc[r].y;
                for (int u = 0; u < nv; ++u) {
                    const float2 a = tile[u * F + i], b = tile[u * F + j];
                    // conj(a) * b
                    re += (double)a.x * b.x + (double)a.y * b.y;
                    im += (double)a.x * b.y - (double)a.y * b.x;
                }
                acc[r] = make_double2(re, im);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int pr = threadIdx.x + 256 * r;
        if (pr < npair) part[(int64_t)pr * gridDim.x + blockIdx.x] = acc[r];  // entry-major: [pair][block]
    }
}

// G[e] = sum_b part[e][b]: one wave per entry; lane l adds blocks l, l + 64, ... in order, then a fixed xor
// butterfly over the 64 lanes (deterministic)
__global__ __launch_bounds__(64) void gram_reduce_kernel(const double2* __restrict__ part, int nb,
                                                         double2* __restrict__ g) {
    const int e = blockIdx.x, lane = threadIdx.x;
    const double2* src = part + (int64_t)e * nb;
    double re = 0.0, im = 0.0;
    for (int b = lane; b < nb; b += 64) {
        const double2 x = src[b];
        re += x.x;
        im += x.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o);
        im += __shfl_xor(im, o);
    }
    if (lane == 0) g[e] = make_double2(re, im);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Round-robin position: element 0 stays, the others rotate by one place per step.
__device__ __forceinline__ int rr(int i, int s, int n) { return i == 0 ? 0 : ((i - 1 + s) % (n - 1)) + 1; }

// G = sum_b part[b]; eigenvectors by parallel cyclic Jacobi; vec[f][j] = eigenvector j (descending eigenvalues).
// NT threads (256 measured faster than one 64-lane wave: the update pass dominates a step).  The pair schedule
// and every thread's update indices are formed once, outside the sweeps.
template <int NT>
__global__ __launch_bounds__(NT) void jacobi_kernel(const double2* __restrict__ part, int nb, int F,
                                                    double2* __restrict__ vec, double* __restrict__ eval,
                                                    int max_sweeps) {
    constexpr int kQItems = (kMaxF / 2 * kMaxF + NT - 1) / NT;  // Q-update items per thread
    __shared__ double2 A[kMaxF][kMaxF + 1];
    __shared__ double2 Q[kMaxF][kMaxF + 1];
    __shared__ double2 U[kMaxF / 2][4];       // u_pp, u_pq, u_qp, u_qq per pair
    __shared__ int PT[kMaxF - 1][kMaxF / 2][2];  // round-robin pairs (p < q) of every step of a sweep
    __shared__ int order[kMaxF];
    __shared__ int rotated;
    __shared__ double floor2;  // (1e-16 trace G)^2: rounding leaves off-diagonal entries near eps * |G|
    const int n = F + (F & 1);  // even; index F is a dummy when F is odd
    const int half = n / 2;
    for (int pr = threadIdx.x; pr < n * n; pr += NT) {
        const int i = pr / n, j = pr % n;
        double2 g = make_double2(0.0, 0.0);
        if (i < F && j < F)
            for (int b = 0; b < nb; ++b) g = cadd(g, part[(int64_t)b * F * F + i * F + j]);
        A[i][j] = g;
        Q[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    for (int w = threadIdx.x; w < (n - 1) * half; w += NT) {
        const int st = w / half, k = w % half;
        int p = rr(k, st, n), q = rr(n - 1 - k, st, n);
        if (p > q) {
            const int t = p;
            p = q;
            q = t;
        }
        PT[st][k][0] = p;
        PT[st][k][1] = q;
    }
    // this thread's work in the update pass: one 2 x 2 block of pairs (bi, bj) and up to kQItems (pair, row) of Q
    const int nblk = half * half, nq = half * n;
    const bool has_blk = (int)threadIdx.x < nblk;
    const int bi = has_blk ? (int)threadIdx.x / half : 0, bj = has_blk ? (int)threadIdx.x - bi * half : 0;
    int qk[kQItems], qi[kQItems];
#pragma unroll
    for (int r = 0; r < kQItems; ++r) {
        const int w = threadIdx.x + r * NT;
        qk[r] = w < nq ? w / n : -1;
        qi[r] = w < nq ? w % n : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int i = 0; i < F; ++i) tr += fabs(A[i][i].x);
        floor2 = 1e-32 * tr * tr;
    }
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        // a sweep that rotates no pair ends the iteration (every |a_pq| is at rounding level)
        if (threadIdx.x == 0) rotated = 0;
        __syncthreads();
        for (int s = 0; s < n - 1; ++s) {
            if ((int)threadIdx.x < half) {
                const int k = threadIdx.x;
                const int p = PT[s][k][0], q = PT[s][k][1];
                double2 upp = make_double2(1.0, 0.0), upq = make_double2(0.0, 0.0), uqp = upq, uqq = upp;
                const double2 apq = A[p][q];
                const double b2 = apq.x * apq.x + apq.y * apq.y;
                const double app = A[p][p].x, aqq = A[q][q].x;
                // rotate unless |a_pq| is negligible against its diagonal pair (|a_pq| <= 1e-15 sqrt(a_pp a_qq))
                // or at the rounding floor of the whole matrix (|a_pq| <= 1e-16 trace G)
                if (q < F && b2 > floor2 && b2 > 1e-30 * fabs(app * aqq)) {
                    rotated = 1;
                    const double rb = rsqrt(b2);                       // 1 / |a_pq|
                    const double e_re = apq.x * rb, e_im = -apq.y * rb;  // e = exp(-i arg a_pq)
                    const double tau = 0.5 * (aqq - app) * rb;
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    const double c = rsqrt(1.0 + t * t), sn = t * c;
                    // U = diag(1, e) [[c, s], [-s, c]]
                    upp = make_double2(c, 0.0);
                    upq = make_double2(sn, 0.0);
                    uqp = make_double2(-sn * e_re, -sn * e_im);
                    uqq = make_double2(c * e_re, c * e_im);
                }
                U[k][0] = upp;
                U[k][1] = upq;
                U[k][2] = uqp;
                U[k][3] = uqq;
            }
            __syncthreads();
            // A <- U^H A U block by block: the 2 x 2 block of pairs (i, j) becomes U_i^H B U_j (the row update,
            // rounded, then the column update, as two separate passes would compute it); Q <- Q U
            if (has_blk) {
                const int pi = PT[s][bi][0], qi_ = PT[s][bi][1], pj = PT[s][bj][0], qj = PT[s][bj][1];
                const double2 a00 = A[pi][pj], a01 = A[pi][qj], a10 = A[qi_][pj], a11 = A[qi_][qj];
                const double2 t00 = cadd(cmul(cconj(U[bi][0]), a00), cmul(cconj(U[bi][2]), a10));
                const double2 t01 = cadd(cmul(cconj(U[bi][0]), a01), cmul(cconj(U[bi][2]), a11));
                const double2 t10 = cadd(cmul(cconj(U[bi][1]), a00), cmul(cconj(U[bi][3]), a10));
                const double2 t11 = cadd(cmul(cconj(U[bi][1]), a01), cmul(cconj(U[bi][3]), a11));
                A[pi][pj] = cadd(cmul(t00, U[bj][0]), cmul(t01, U[bj][2]));
                A[pi][qj] = cadd(cmul(t00, U[bj][1]), cmul(t01, U[bj][3]));
                A[qi_][pj] = cadd(cmul(t10, U[bj][0]), cmul(t11, U[bj][2]));
                A[qi_][qj] = cadd(cmul(t10, U[bj][1]), cmul(t11, U[bj][3]));
            }
#pragma unroll
            for (int r = 0; r < kQItems; ++r) {
                if (qk[r] < 0) continue;
                const int k = qk[r], i = qi[r], p = PT[s][k][0], q = PT[s][k][1];
                const double2 qp = Q[i][p], qq = Q[i][q];
                Q[i][p] = cadd(cmul(qp, U[k][0]), cmul(qq, U[k][2]));
                Q[i][q] = cadd(cmul(qp, U[k][1]), cmul(qq, U[k][3]));
            }
            __syncthreads();
        }
        // every thread reads the flag before thread 0 may reset it for the next sweep, so all leave together
        const bool again = rotated != 0;
        __syncthreads();
        if (!again) break;
    }
    // eigenvalues in descending order, ties in index order: each thread ranks one eigenvalue (order starts as
    // the identity so that every entry is a valid index even if a NaN makes two ranks collide)
    for (int i = threadIdx.x; i < F; i += NT) order[i] = i;
    __syncthreads();
    for (int i = threadIdx.x; i < F; i += NT) {
        const double di = A[i][i].x;
        int rank = 0;
        for (int j = 0; j < F; ++j) {
            const double dj = A[j][j].x;
            rank += (dj > di || (dj == di && j < i)) ? 1 : 0;
        }
        order[rank] = i;
    }
    __syncthreads();
    for (int pr = threadIdx.x; pr < F * F; pr += NT) {
        const int f = pr / F, j = pr % F;
        vec[pr] = Q[f][order[j]];
    }
    for (int j = threadIdx.x; j < F; j += NT) eval[j] = A[order[j]][order[j]].x;
}

// pd[v] = |c_v|^2 - sum_{j<k} |sum_f c_v[f] vec[f][j]|^2  (float64), clamped at 0
__global__ __launch_bounds__(256) void pd_kernel(const float2* __restrict__ y, int64_t V, int F, int k,
                                                 const double2* __restrict__ vec, float* __restrict__ pd) {
    __shared__ double2 sv[kMaxF * kMaxF];
    for (int i = threadIdx.x; i < F * F; i += 256) sv[i] = vec[i];
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= V) return;
    const float2* c = y + v * F;
    double e = 0.0;
    for (int f = 0; f < F; ++f) {
        const float2 z = c[f];
        e += (double)z.x * z.x + (double)z.y * z.y;
    }
    for (int j = 0; j < k; ++j) {
        double re = 0.0, im = 0.0;
        for (int f = 0; f < F; ++f) {
            const float2 z = c[f];
            const double2 w = sv[f * F + j];
            re += z.x * w.x - z.y * w.y;
            im += z.x * w.y + z.y * w.x;
        }
        e -= re * re + im * im;
    }
    pd[v] = (float)(e > 0.0 ? e : 0.0);
}

}  // namespace post

namespace {
thread_local const char* g_post_err = "";
int pfail(int st, const char* msg) {
    g_post_err = msg;
    return st;
}
int post_launch_status(const char* what) {
    return hipGetLastError() == hipSuccess ? DAS_OK : pfail(DAS_EHIP, what);
}
// voxels per Gram partial block: at most max_blocks blocks (2048 fill the chip), at least one 64-voxel tile each
int64_t gram_chunk(int64_t V, int64_t max_blocks = 2048) {
    const int64_t c = (V + max_blocks - 1) / max_blocks;
    return c < 64 ? 64 : c;
}

// Work layout of Power Doppler in double2 units: nb partial Gram matrices, their sum, the eigenvectors, then the
// F eigenvalues (doubles, rounded up to whole double2).
int64_t pd_work2(int64_t nb, int F) { return nb * F * F + 2 * (int64_t)F * F + (F + 1) / 2; }

// Allocation-free Power Doppler: its work lives in this fixed device array (one per GPU, kept until the process
// ends).  Size: the work of 2048 partial blocks at 16 frames, so that up to 16 frames the voxel chunking is the
// same as with a caller's buffer; 17-32 frames use fewer, larger chunks.
constexpr int64_t kScratch2 = 2048 * 16 * 16 + 2 * 32 * 32 + 16;  // double2 entries (8.03 MiB)
static __device__ __align__(256) double2 scratch[kScratch2];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double2* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device, looked up once per device.  The array's host-side
// name is not a device address; only this pointer is passed to kernels.
int scratch_on_current_device(double2** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return pfail(DAS_EHIP, "power_doppler_noalloc: no current HIP device");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
            return pfail(DAS_EHIP, "power_doppler_noalloc: hipGetSymbolAddress(scratch) failed");
        g_scratch_ptr[dev] = static_cast<double2*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return DAS_OK;
}

// Power Doppler on a work area of work2 double2 entries with at most max_blocks Gram partial blocks.
int power_doppler_impl(const void* y, int64_t V, int F, int n_clutter, float* pd, double2* work, int64_t max_blocks,
                       hipStream_t s) {
    const float2* yy = reinterpret_cast<const float2*>(y);
    const int64_t chunk = gram_chunk(V, max_blocks);
    const int nb = (int)((V + chunk - 1) / chunk);
    double2* part = work;
    double2* gram = part + (int64_t)nb * F * F;
    double2* vec = gram + (int64_t)F * F;
    double* eval = reinterpret_cast<double*>(vec + (int64_t)F * F);
    hipLaunchKernelGGL(post::gram_partial_kernel, dim3(nb), dim3(256), 0, s, yy, V, F, chunk, part);
    hipLaunchKernelGGL(post::gram_reduce_kernel, dim3((unsigned)(F * F)), dim3(64), 0, s, part, nb, gram);
    hipLaunchKernelGGL(post::jacobi_kernel<256>, dim3(1), dim3(256), 0, s, gram, 1, F, vec, eval, 40);
    hipLaunchKernelGGL(post::pd_kernel, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, yy, V, F, n_clutter, vec,
                       pd);
    return post_launch_status("power_doppler launch failed");
}
}  // namespace

extern "C" {

const char* das_post_last_error(void) { return g_post_err; }

int64_t das_bmode_work(int64_t V, int F) {
    if (V < 1 || F < 1) return 0;
    return ((V + 255) / 256) * F + F;
}

int das_bmode(const void* y, int64_t V, int F, float dynamic_range_db, float* out_db, float* work,
              int64_t work_floats, void* stream) {
    if (!y || !out_db || !work) return pfail(DAS_EINVAL, "bmode: null pointer");
    if (V < 1 || F < 1 || F > 1024) return pfail(DAS_ESHAPE, "bmode: need V >= 1 and 1 <= F <= 1024");
    if (!(dynamic_range_db > 0.0f) || dynamic_range_db > 1e30f)
        return pfail(DAS_EINVAL, "bmode: dynamic range must be positive and finite");
    if (work_floats < das_bmode_work(V, F)) return pfail(DAS_ESHAPE, "bmode: work buffer too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const float2* yy = reinterpret_cast<const float2*>(y);
    const int nb = (int)((V + 255) / 256);
    float* part = work;
    float* peak = work + (int64_t)nb * F;
    hipLaunchKernelGGL(post::frame_max_kernel, dim3(nb), dim3(256), 0, s, yy, V, F, part);
    hipLaunchKernelGGL(post::frame_peak_kernel, dim3(F), dim3(256), 0, s, part, nb, F, peak);
    const int64_t n = V * F;
    hipLaunchKernelGGL(post::bmode_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, yy, n, F, peak,
                       -dynamic_range_db, out_db);
    return post_launch_status("bmode launch failed");
}

int64_t das_power_doppler_work(int64_t V, int F) {
    if (V < 1 || F < 1) return 0;
    const int64_t nb = (V + gram_chunk(V) - 1) / gram_chunk(V);
    return 2 * pd_work2(nb, F);  // partial Gram matrices, the sum, eigenvectors; eigenvalues
}

int das_power_doppler(const void* y, int64_t V, int F, int n_clutter, float* pd, double* work, int64_t work_doubles,
                      void* stream) {
    if (!y || !pd || !work) return pfail(DAS_EINVAL, "power_doppler: null pointer");
    if (V < 1 || F < 1 || F > post::kMaxF) return pfail(DAS_ESHAPE, "power_doppler: need V >= 1 and 1 <= F <= 32");
    if (n_clutter < 0 || n_clutter > F) return pfail(DAS_EINVAL, "power_doppler: need 0 <= n_clutter <= F");
    if (work_doubles < das_power_doppler_work(V, F)) return pfail(DAS_ESHAPE, "power_doppler: work buffer too small");
    if (reinterpret_cast<uintptr_t>(work) % 16 != 0) return pfail(DAS_EALIGN, "power_doppler: work must be 16-byte aligned");
    return power_doppler_impl(y, V, F, n_clutter, pd, reinterpret_cast<double2*>(work), 2048,
                              reinterpret_cast<hipStream_t>(stream));
}

int das_power_doppler_noalloc(const void* y, int64_t V, int F, int n_clutter, float* pd, void* stream) {
    if (!y || !pd) return pfail(DAS_EINVAL, "power_doppler_noalloc: null pointer");
    if (V < 1 || F < 1 || F > post::kMaxF)
        return pfail(DAS_ESHAPE, "power_doppler_noalloc: need V >= 1 and 1 <= F <= 32");
    if (n_clutter < 0 || n_clutter > F) return pfail(DAS_EINVAL, "power_doppler_noalloc: need 0 <= n_clutter <= F");
    // the most Gram partial blocks the scratch array holds at F frames (F <= 32 always leaves room for 500)
    const int64_t fit = (kScratch2 - pd_work2(0, F)) / ((int64_t)F * F);
    const int64_t max_blocks = fit < 2048 ? fit : 2048;
    if (pd_work2((V + gram_chunk(V, max_blocks) - 1) / gram_chunk(V, max_blocks), F) > kScratch2)
        return pfail(DAS_ESHAPE, "power_doppler_noalloc: work exceeds the 8 MiB scratch array");
    double2* work = nullptr;
    const int st = scratch_on_current_device(&work);
    if (st != DAS_OK) return st;
    return power_doppler_impl(y, V, F, n_clutter, pd, work, max_blocks, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
