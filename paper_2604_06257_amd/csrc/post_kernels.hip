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

// part[b][i][j] = sum over the block's voxel chunk of conj(y[v][i]) y[v][j]   (float64 complex, F <= 32)
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
        if (pr < npair) part[(int64_t)blockIdx.x * npair + pr] = acc[r];
    }
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Round-robin position: element 0 stays, the others rotate by one place per step.
__device__ __forceinline__ int rr(int i, int s, int n) { return i == 0 ? 0 : ((i - 1 + s) % (n - 1)) + 1; }

// G = sum_b part[b]; eigenvectors by parallel cyclic Jacobi; vec[f][j] = eigenvector j (descending eigenvalues)
__global__ __launch_bounds__(256) void jacobi_kernel(const double2* __restrict__ part, int nb, int F,
                                                     double2* __restrict__ vec, double* __restrict__ eval,
                                                     int max_sweeps) {
    __shared__ double2 A[kMaxF][kMaxF + 1];
    __shared__ double2 Q[kMaxF][kMaxF + 1];
    __shared__ double2 U[kMaxF / 2][4];  // u_pp, u_pq, u_qp, u_qq per pair
    __shared__ int P[kMaxF / 2][2];
    __shared__ double red[256];
    __shared__ int order[kMaxF];
    __shared__ int done;
    const int n = F + (F & 1);  // even; index F is a dummy when F is odd
    const int half = n / 2;
    for (int pr = threadIdx.x; pr < n * n; pr += 256) {
        const int i = pr / n, j = pr % n;
        double2 g = make_double2(0.0, 0.0);
        if (i < F && j < F)
            for (int b = 0; b < nb; ++b) g = cadd(g, part[(int64_t)b * F * F + i * F + j]);
        A[i][j] = g;
        Q[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        // convergence: off-diagonal energy against the total
        double off = 0.0, tot = 0.0;
        for (int pr = threadIdx.x; pr < n * n; pr += 256) {
            const int i = pr / n, j = pr % n;
            const double m = A[i][j].x * A[i][j].x + A[i][j].y * A[i][j].y;
            tot += m;
            if (i != j) off += m;
        }
        red[threadIdx.x] = off;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        const double off_sum = red[0];
        __syncthreads();
        red[threadIdx.x] = tot;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) done = !(off_sum > 1e-28 * red[0]);  // off-diagonal norm below 1e-14 of the total
        __syncthreads();
        if (done) break;
        for (int s = 0; s < n - 1; ++s) {
            if ((int)threadIdx.x < half) {
                const int k = threadIdx.x;
                int p = rr(k, s, n), q = rr(n - 1 - k, s, n);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                P[k][0] = p;
                P[k][1] = q;
                double2 upp = make_double2(1.0, 0.0), upq = make_double2(0.0, 0.0), uqp = upq, uqq = upp;
                const double2 apq = A[p][q];
                const double b = sqrt(apq.x * apq.x + apq.y * apq.y);
                if (q < F && b > 0.0) {
                    const double e_re = apq.x / b, e_im = -apq.y / b;  // e = exp(-i arg a_pq)
                    const double tau = (A[q][q].x - A[p][p].x) / (2.0 * b);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
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
            // rows: A <- U^H A
            for (int w = threadIdx.x; w < half * n; w += 256) {
                const int k = w / n, j = w % n, p = P[k][0], q = P[k][1];
                const double2 ap = A[p][j], aq = A[q][j];
                A[p][j] = cadd(cmul(cconj(U[k][0]), ap), cmul(cconj(U[k][2]), aq));
                A[q][j] = cadd(cmul(cconj(U[k][1]), ap), cmul(cconj(U[k][3]), aq));
            }
            __syncthreads();
            // columns: A <- A U, Q <- Q U
            for (int w = threadIdx.x; w < half * n; w += 256) {
                const int k = w / n, i = w % n, p = P[k][0], q = P[k][1];
                const double2 ap = A[i][p], aq = A[i][q];
                A[i][p] = cadd(cmul(ap, U[k][0]), cmul(aq, U[k][2]));
                A[i][q] = cadd(cmul(ap, U[k][1]), cmul(aq, U[k][3]));
                const double2 qp = Q[i][p], qq = Q[i][q];
                Q[i][p] = cadd(cmul(qp, U[k][0]), cmul(qq, U[k][2]));
                Q[i][q] = cadd(cmul(qp, U[k][1]), cmul(qq, U[k][3]));
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {  // eigenvalues in descending order (stable: ties keep index order)
        for (int i = 0; i < F; ++i) order[i] = i;
        for (int i = 0; i < F; ++i) {
            int best = i;
            for (int j = i + 1; j < F; ++j)
                if (A[order[j]][order[j]].x > A[order[best]][order[best]].x) best = j;
            const int t = order[i];
            order[i] = order[best];
            order[best] = t;
        }
    }
    __syncthreads();
    for (int pr = threadIdx.x; pr < F * F; pr += 256) {
        const int f = pr / F, j = pr % F;
        vec[pr] = Q[f][order[j]];
    }
    for (int j = threadIdx.x; j < F; j += 256) eval[j] = A[order[j]][order[j]].x;
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
int64_t gram_chunk(int64_t V) {
    const int64_t c = (V + 511) / 512;
    return c < 1024 ? 1024 : c;
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
    return 2 * (nb * F * F + (int64_t)F * F) + F;
}

int das_power_doppler(const void* y, int64_t V, int F, int n_clutter, float* pd, double* work, int64_t work_doubles,
                      void* stream) {
    if (!y || !pd || !work) return pfail(DAS_EINVAL, "power_doppler: null pointer");
    if (V < 1 || F < 1 || F > post::kMaxF) return pfail(DAS_ESHAPE, "power_doppler: need V >= 1 and 1 <= F <= 32");
    if (n_clutter < 0 || n_clutter > F) return pfail(DAS_EINVAL, "power_doppler: need 0 <= n_clutter <= F");
    if (work_doubles < das_power_doppler_work(V, F)) return pfail(DAS_ESHAPE, "power_doppler: work buffer too small");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const float2* yy = reinterpret_cast<const float2*>(y);
    const int64_t chunk = gram_chunk(V);
    const int nb = (int)((V + chunk - 1) / chunk);
    double2* part = reinterpret_cast<double2*>(work);
    double2* vec = part + (int64_t)nb * F * F;
    double* eval = reinterpret_cast<double*>(vec + (int64_t)F * F);
    hipLaunchKernelGGL(post::gram_partial_kernel, dim3(nb), dim3(256), 0, s, yy, V, F, chunk, part);
    hipLaunchKernelGGL(post::jacobi_kernel, dim3(1), dim3(256), 0, s, part, nb, F, vec, eval, 40);
    hipLaunchKernelGGL(post::pd_kernel, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, yy, V, F, n_clutter, vec,
                       pd);
    return post_launch_status("power_doppler launch failed");
}

}  // extern "C"
