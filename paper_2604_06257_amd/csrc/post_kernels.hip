// gfx950 post-processing of beamformed volumes y [V][F] (complex64, frame innermost):
// B-mode log compression and Power Doppler with an SVD clutter filter.
//
// B-mode: per-frame peak of |y| (block maxima through an LDS integer max, which
// is exact and order independent for non-negative floats), then
// max(20 log10(|y| / peak), -dr).
//
// Power Doppler: the right singular vectors of the Casorati matrix C = y are the
// eigenvectors of the Gram matrix G = C^H C (F x F, Hermitian).  G is summed in
// float64 over voxel chunks (partials added in chunk order: deterministic).  Only
// the k eigenvectors of the largest eigenvalues are needed: one workgroup reduces
// G to a real tridiagonal matrix (Householder), finds those eigenvalues by Sturm
// multisection and their eigenvectors by twisted factorisations, and transforms
// them back; a spectrum that fails its residual or orthogonality checks takes the
// parallel cyclic Jacobi method instead.  The energy a voxel keeps after removing
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

// Gram partial sums.  Block b sums conj(y[v][i]) y[v][j] over its chunk of voxels in float64, for the upper
// triangle of 4 x 4 tiles of the 32 x 32 matrix (frames past F are zeros): 36 tiles, each owned by 7 threads that
// take every 7th voxel of the chunk; a chunk is staged in LDS in float64 in sub-chunks of kGV voxels.  The 7
// partial tiles are then added in thread order, and block b writes part[(i F + j) nb + b] for the entries of its
// tiles (i <= j, and both triangles of the diagonal tiles): entry-major, so that the reduction reads contiguously.
constexpr int kGV = 128;   // voxels per LDS stage
constexpr int kGGrp = 7;   // voxel groups
constexpr int kGTiles = 36;
__global__ __launch_bounds__(256) void gram_partial_kernel(const float2* __restrict__ y, int64_t V, int F,
                                                           int64_t chunk, double2* __restrict__ part) {
    __shared__ double2 ys[kGV][kMaxF + 1];  // 67.6 KB; also the tiles' reduction area at the end
    const int t = threadIdx.x;
    const int grp = t / kGTiles, tile = t % kGTiles;
    const bool busy = grp < kGGrp;
    int bi = 0, bj = tile;  // tile -> (bi, bj), bi <= bj, row by row
    while (bj >= 8 - bi) {
        bj -= 8 - bi;
        ++bi;
    }
    bj += bi;
    double2 acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = make_double2(0.0, 0.0);
    const int64_t vb = (int64_t)blockIdx.x * chunk;
    const int64_t ve = vb + chunk < V ? vb + chunk : V;
    for (int64_t v0 = vb; v0 < ve; v0 += kGV) {
        const int nv = (int)(ve - v0 < kGV ? ve - v0 : kGV);
        __syncthreads();
        // lane f of a 32-lane half loads frame f of voxel (t / 32) + 8 i: consecutive lanes, consecutive samples
        for (int v = t >> 5; v < kGV; v += 8) {
            const int f = t & 31;
            const float2 z = (v < nv && f < F) ? y[(v0 + v) * F + f] : make_float2(0.0f, 0.0f);
            ys[v][f] = make_double2((double)z.x, (double)z.y);
        }
        __syncthreads();
        if (busy) {
            for (int v = grp; v < nv; v += kGGrp) {
                double2 ai[4], bq[4];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    ai[p] = ys[v][4 * bi + p];
                    bq[p] = ys[v][4 * bj + p];
                }
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {  // conj(a) b
                        acc[p][q].x = fma(ai[p].x, bq[q].x, fma(ai[p].y, bq[q].y, acc[p][q].x));
                        acc[p][q].y = fma(ai[p].x, bq[q].y, fma(-ai[p].y, bq[q].x, acc[p][q].y));
                    }
            }
        }
    }
    __syncthreads();
    double2* red = &ys[0][0];  // [grp][tile][16]
    if (busy) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) red[(grp * kGTiles + tile) * 16 + p * 4 + q] = acc[p][q];
    }
    __syncthreads();
    const int nb = gridDim.x;
    for (int e = t; e < kGTiles * 16; e += 256) {
        const int tl = e >> 4, pq = e & 15;
        int ti = 0, tj = tl;
        while (tj >= 8 - ti) {
            tj -= 8 - ti;
            ++ti;
        }
        tj += ti;
        const int i = 4 * ti + (pq >> 2), j = 4 * tj + (pq & 3);
        if (i < F && j < F) {
            double2 sum = red[tl * 16 + pq];
            for (int gg = 1; gg < kGGrp; ++gg) sum = make_double2(sum.x + red[(gg * kGTiles + tl) * 16 + pq].x,
                                                                 sum.y + red[(gg * kGTiles + tl) * 16 + pq].y);
            part[(int64_t)(i * F + j) * nb + blockIdx.x] = sum;
        }
    }
}

// G[i][j] = sum_b part[e][b] with e = (i, j) for i <= j, and the conjugate of entry (j, i) below the diagonal:
// one wave per entry; lane l adds blocks l, l + 64, ... in order, then a fixed xor butterfly (deterministic)
__global__ __launch_bounds__(64) void gram_reduce_kernel(const double2* __restrict__ part, int nb, int F,
                                                         double2* __restrict__ g) {
    const int e = blockIdx.x, lane = threadIdx.x;
    const int i = e / F, j = e % F;
    const bool lower = i > j;
    const double2* src = part + (int64_t)(lower ? j * F + i : e) * nb;
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
    if (lane == 0) g[e] = make_double2(re, lower ? -im : im);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Round-robin position: element 0 stays, the others rotate by one place per step.
__device__ __forceinline__ int rr(int i, int s, int n) { return i == 0 ? 0 : ((i - 1 + s) % (n - 1)) + 1; }

// Every eigenvector of G (F x F, row-major) by parallel cyclic Jacobi; vec[f][j] = eigenvector j (descending
// eigenvalues), eval[j] its eigenvalue.  Called by all NT threads of the workgroup (256 measured faster than one
// 64-lane wave: the update pass dominates a step).  The pair schedule and every thread's update indices are formed
// once, outside the sweeps.  Robust for any spectrum (repeated eigenvalues included), but a chain of ~F/2 * 10
// dependent rotation steps: the fallback of the top-k solver below.
template <int NT>
__device__ void jacobi_solve(const double2* __restrict__ g, int F, double2* __restrict__ vec,
                             double* __restrict__ eval, int max_sweeps) {
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
        A[i][j] = (i < F && j < F) ? g[i * F + j] : make_double2(0.0, 0.0);
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
                    atomicOr(&rotated, 1);
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

__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 csel(bool c, double2 a, double2 b) { return c ? a : b; }

// Cross-lane moves of a double: DPP within rows of 16 lanes (a VALU operand modifier, no LDS round trip), the
// swizzle for the two rows of a 32-lane half.
template <int kCtrl>
__device__ __forceinline__ double dpp_d(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), kCtrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double swap16_d(double x) {  // lane i <-> lane i ^ 16
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(x), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(x), 0x401F);
    return __hiloint2double(hi, lo);
}
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kRowHalfMirror = 0x141, kRowMirror = 0x140;
// Sums over aligned groups of 8 and of 32 lanes; every lane of the group gets the same value (each step adds a
// lane's value and its partner's, which both lanes form alike).
__device__ __forceinline__ double sum8(double x) {
    x += dpp_d<kQuadXor1>(x);
    x += dpp_d<kQuadXor2>(x);
    return x + dpp_d<kRowHalfMirror>(x);
}
__device__ __forceinline__ double sum32(double x) {
    x = sum8(x);
    x += dpp_d<kRowMirror>(x);
    return x + swap16_d(x);
}

// Number of eigenvalues below sig of the symmetric tridiagonal T (diagonal d, squared off-diagonal e2[i] =
// e_{i-1}^2, e_{-1} = 0; |T| <= 1), for kP points at once: the sign changes of the Sturm sequence of leading
// principal minors p_i = (d_{i-1} - sig) p_{i-1} - e_{i-2}^2 p_{i-2}, p_0 = 1 (one eigenvalue below sig per
// negative ratio p_i / p_{i-1}).  No division: the chain is one FMA per step; every four steps both carried
// minors are rescaled by the same power of two (exact, signs kept), so no minor overflows or underflows.  The
// kP chains are independent and interleave.
template <int kP>
__device__ __forceinline__ void sturm_counts(const double (&d)[kMaxF], const double (&e2)[kMaxF],
                                             const double (&sig)[kP], int (&c)[kP]) {
    double p[kP], pp[kP];
#pragma unroll
    for (int q = 0; q < kP; ++q) {
        p[q] = 1.0;
        pp[q] = 0.0;
        c[q] = 0;
    }
#pragma unroll
    for (int i = 0; i < kMaxF; ++i) {
#pragma unroll
        for (int q = 0; q < kP; ++q) {
            const double pn = fma(d[i] - sig[q], p[q], -e2[i] * pp[q]);
            c[q] += (pn * p[q] < 0.0) ? 1 : 0;
            pp[q] = p[q];
            p[q] = pn;
            if ((i & 3) == 3) {
                const int ex = __builtin_amdgcn_frexp_exp(p[q]);
                p[q] = __builtin_ldexp(p[q], -ex);
                pp[q] = __builtin_ldexp(pp[q], -ex);
            }
        }
    }
}

constexpr int kFastK = 4, kFastIters = 24;  // fast path of the top-k solver: largest k, iterations

// One round of the top-k solver's fast path, by the 64 lanes of one wave (lanes 0-31 hold rows 0-31, lanes 32-63
// repeat them; their results are not used): X (orthonormal, xs) and Y = G X (ys) give H = X^H Y and
// R = Y - X H.  If the certificate holds, X is written out as the eigenvector basis (vec[f][j]) with eval[j] =
// H_jj and state = 1; otherwise xs <- an orthonormal basis of Y (modified Gram-Schmidt), and state = 2 when a
// column vanishes or this was the last round.
template <int K>
__device__ void fast_check(double2 (*xs)[kMaxF], double2 (*ys)[kMaxF], int n, int F, double trg, bool last,
                           double2* __restrict__ vec, double* __restrict__ eval, int& state) {
    const int lane = threadIdx.x & 63, rr = lane & 31;
    double2 x[K], y[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        x[j] = xs[j][rr];
        y[j] = ys[j][rr];
    }
    double2 h[K][K];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double2 c = cmul(cconj(x[i]), y[j]);
            h[i][j] = make_double2(sum32(c.x), sum32(c.y));
        }
    double r2 = 0.0, trh = 0.0, alo = 1.0 / 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double2 rj = y[j];
#pragma unroll
        for (int i = 0; i < K; ++i) rj = csub(rj, cmul(x[i], h[i][j]));
        r2 = fma(rj.x, rj.x, fma(rj.y, rj.y, r2));
        trh += h[j][j].x;
        double off = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i != j) off += sqrt(fma(h[i][j].x, h[i][j].x, h[i][j].y * h[i][j].y));
        alo = fmin(alo, h[j][j].x - off);
    }
    const double rn = sqrt(sum32(r2));
    const double delta = alo - (trg - trh) - 1e-13 * fabs(trg);
    if (delta > 0.0 && rn <= 1e-12 * delta) {
        if (lane < n) {
#pragma unroll
            for (int j = 0; j < K; ++j) vec[lane * F + j] = x[j];
        }
        if (lane == 0) {
#pragma unroll
            for (int j = 0; j < K; ++j) eval[j] = h[j][j].x;
            state = 1;
        }
        return;
    }
    bool ok = true;
#pragma unroll
    for (int j = 0; j < K; ++j) {
#pragma unroll
        for (int i = 0; i < j; ++i) {
            const double2 c = cmul(cconj(y[i]), y[j]);
            y[j] = csub(y[j], cmul(y[i], make_double2(sum32(c.x), sum32(c.y))));
        }
        const double nr = sum32(fma(y[j].x, y[j].x, y[j].y * y[j].y));
        ok = ok && nr > 1e-280 && nr <= 1.7e308;
        y[j] = cscale(y[j], ok ? 1.0 / sqrt(nr) : 0.0);
        if (lane < 32) xs[j][lane] = lane < n ? y[j] : make_double2(0.0, 0.0);
    }
    if (lane == 0 && (!ok || last)) state = 2;
}

// 1 / x from the hardware reciprocal and two Newton steps (within an ulp or so; x finite and nonzero)
__device__ __forceinline__ double rcp_d(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// The k eigenvectors of the largest eigenvalues of the Hermitian G (F x F, row-major), 0 < k < F <= 32, for the
// clutter filter: vec[f][j] = eigenvector j (descending eigenvalues), eval[j] its eigenvalue, j < k.  One
// workgroup of 256 threads; thread t holds entries (t / 8, t % 8 + 8u), u < 4, of G and of Q in registers, so a
// row's eight threads reduce over the row with DPP moves.
//   1. Householder reduction of G to a real symmetric tridiagonal T = Q^H G Q (one reflector per column, whose
//      coefficient makes the sub-diagonal real: H = I - tau v v^H with H^H x = beta e_1, beta real), the trailing
//      block updated as B - w v^H - v w^H with w = tau B v - (|tau|^2 / 2)(v^H B v) v, and Q as Q - tau (Q v) v^H;
//   2. the k largest eigenvalues of T by multisection on Sturm counts (a group of up to 64 lanes per eigenvalue,
//      two counts per lane and round; ballots give the new bracket) until the bracket stops shrinking;
//   3. each eigenvector of T from the twisted factorisation of T - lambda I (forward and backward pivots, the
//      twist at the smallest |gamma_r|, then the two product recurrences away from r), normalised;
//   4. checks: every residual |(T - lambda) z|_i <= 1e-11 |T| and every |z_a . z_b| <= 1e-10; then one classical
//      Gram-Schmidt pass against the vectors of larger eigenvalues;
//   5. v = Q z.
// Before that, for k <= 4, a fast path: subspace iteration X <- orth(G X) from the unit vectors of the k largest
// diagonal entries, accepted as soon as the sin-theta bound certifies it: with H = X^H G X and R = G X - X H,
// the clutter subspace is within ||R||_F / delta of span X, where delta = (a Gershgorin lower bound of the
// eigenvalues of H) - (trace G - trace H, an upper bound of the (k+1)-th eigenvalue of the positive
// semidefinite G); span X is used when ||R||_F <= 1e-12 delta (the Power Doppler needs the subspace only).
// It serves spectra whose k largest eigenvalues hold most of the energy (tissue clutter); other spectra, or 24
// iterations without a certificate, go on to steps 1-5.
// A spectrum that fails a check (eigenvalues repeated among the k largest, non-finite input) takes the Jacobi
// solver instead, for the same output.  Every reduction is in a fixed order: the result is deterministic.
__global__ __launch_bounds__(256) void eig_top_kernel(const double2* __restrict__ g, int F, int k,
                                                      double2* __restrict__ vec, double* __restrict__ eval) {
    constexpr int NT = 256;
    __shared__ double2 COL[kMaxF];  // column j of the partly reduced matrix (conjugate of row j): reflector j's input
    // The current reflector, offset by one with a zero in front and zeros past its length, so that rows and
    // columns outside the trailing block update by exact zeros: HVp[1 + i] = v_i, TVC[1 + i] = tau conj(v_i),
    // PVp[1 + i] = p_i = (B v)_i, CPp[1 + i] = conj(tau p_i); UV[r] = (Q v)_r; SW = partial sums of v^H p.
    __shared__ double2 HVp[kMaxF + 1], TVC[kMaxF + 1], PVp[kMaxF + 1], CPp[kMaxF + 1];
    __shared__ double2 UV[kMaxF];
    __shared__ double SW[NT / 32];
    __shared__ double2 TAU[kMaxF];
    __shared__ double Dg[kMaxF], Ef[kMaxF], LAM[kMaxF];
    __shared__ double PIV[2][kMaxF][kMaxF + 1];  // [0] forward pivots D+_i, [1] backward pivots D-_i per eigenvalue
    __shared__ double RAT[2][kMaxF][kMaxF + 1];  // [0] e_i / D+_i, [1] e_{i-1} / D-_i
    __shared__ double Z[kMaxF][kMaxF + 1];       // tridiagonal eigenvectors, Z[j][i]
    __shared__ double M[kMaxF][kMaxF + 1];       // Z Z^T
    __shared__ int TW[kMaxF];
    __shared__ int bad;
    __shared__ double TRG;
    const int n = F, t = threadIdx.x;
    const int r = t >> 3, l = t & 7;  // this thread's row and first column
    double2 a[4], qm[4];              // G (being reduced) and Q at (r, l + 8u)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = l + 8 * u;
        const bool in = r < n && c < n;
        a[u] = in ? g[r * n + c] : make_double2(0.0, 0.0);
        qm[u] = make_double2(in && r == c ? 1.0 : 0.0, 0.0);
    }
    // the owners of row 0 publish column 0 (the conjugate of row 0)
    if (r == 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (l + 8 * u < n) COL[l + 8 * u] = cconj(a[u]);
    }
    if (t == 0) {
        bad = 0;
        HVp[0] = TVC[0] = PVp[0] = CPp[0] = make_double2(0.0, 0.0);
    }

    // 0. fast path (see above); G in registers is left as it was for steps 1-5
    if (k <= kFastK) {
        __shared__ double2 XS[kFastK][kMaxF], YS[kFastK][kMaxF];
        __shared__ int fast_state;  // 0 iterating, 1 certified, 2 given up
        const int lane = t & 63;
        if (t < 64) {
            // trace and the start vectors e_m for the k largest diagonal entries (ties to the lower index)
            double dg = lane < n ? g[lane * (n + 1)].x : -1.0 / 0.0;
            const double tr = sum32(lane < 32 && lane < n ? g[lane * (n + 1)].x : 0.0);
            if (lane == 0) TRG = tr;
            for (int j = 0; j < k; ++j) {
                double bv = lane < 32 ? dg : -1.0 / 0.0;
                int bi = lane;
                for (int o = 16; o > 0; o >>= 1) {
                    const double ov = __shfl_xor(bv, o);
                    const int oi = __shfl_xor(bi, o);
                    if (ov > bv || (ov == bv && oi < bi)) {
                        bv = ov;
                        bi = oi;
                    }
                }
                if (lane < 32) XS[j][lane] = make_double2(lane == bi ? 1.0 : 0.0, 0.0);
                if (lane == bi) dg = -1.0 / 0.0;
            }
            if (lane == 0) fast_state = 0;
        }
        for (int i = t; i < kFastK * kMaxF; i += NT) YS[i / kMaxF][i % kMaxF] = make_double2(0.0, 0.0);
        __syncthreads();
        for (int it = 0; it < kFastIters; ++it) {
            // Y = G X: this thread's four columns, then the row's eight threads
            for (int j = 0; j < k; ++j) {
                double2 y = make_double2(0.0, 0.0);
#pragma unroll
                for (int u = 0; u < 4; ++u) y = cadd(y, cmul(a[u], XS[j][l + 8 * u]));
                y.x = sum8(y.x);
                y.y = sum8(y.y);
                if (l == 0 && r < n) YS[j][r] = y;
            }
            __syncthreads();
            if (t < 64) {
                const bool last = it + 1 == kFastIters;
                switch (k) {
                    case 1: fast_check<1>(XS, YS, n, F, TRG, last, vec, eval, fast_state); break;
                    case 2: fast_check<2>(XS, YS, n, F, TRG, last, vec, eval, fast_state); break;
                    case 3: fast_check<3>(XS, YS, n, F, TRG, last, vec, eval, fast_state); break;
                    default: fast_check<4>(XS, YS, n, F, TRG, last, vec, eval, fast_state); break;
                }
            }
            __syncthreads();
            const int st = fast_state;
            if (st == 1) return;
            if (st == 2) break;
        }
    }
    __syncthreads();

    // 1. tridiagonalisation
    for (int j = 0; j + 1 < n; ++j) {
        const int m = n - 1 - j;  // length of the column below the diagonal
        if (t < 32) {
            const double2 x = t < m ? COL[j + 1 + t] : make_double2(0.0, 0.0);
            const double sq = sum32((t >= 1 && t < m) ? fma(x.x, x.x, x.y * x.y) : 0.0);
            const double ar = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x.x)),
                                               __builtin_amdgcn_readfirstlane(__double2loint(x.x)));
            const double ai = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x.y)),
                                               __builtin_amdgcn_readfirstlane(__double2loint(x.y)));
            double2 tau = make_double2(0.0, 0.0), sc = make_double2(0.0, 0.0);
            double beta = ar;
            if (sq != 0.0 || ai != 0.0) {
                beta = -copysign(sqrt(fma(ar, ar, fma(ai, ai, sq))), ar);
                const double ib = rcp_d(beta);
                tau = make_double2((beta - ar) * ib, -ai * ib);
                const double dr = ar - beta, iden = rcp_d(fma(dr, dr, ai * ai));  // 1 / (alpha - beta)
                sc = make_double2(dr * iden, -ai * iden);
            }
            const double2 v = t < m ? (t == 0 ? make_double2(1.0, 0.0) : cmul(x, sc)) : make_double2(0.0, 0.0);
            HVp[1 + t] = v;
            TVC[1 + t] = cmul(tau, cconj(v));
            if (t == 0) {
                TAU[j] = tau;
                Ef[j] = beta;
                Dg[j] = COL[j].x;
            }
        }
        __syncthreads();
        const double2 tau = TAU[j];
        const bool live = tau.x != 0.0 || tau.y != 0.0;  // uniform; H = I otherwise
        const int cn = j + 1;                            // the next column
        if (live) {
            // p = B v and u = Q v, row by row: this thread's four columns, then the row's eight threads
            double2 pa = make_double2(0.0, 0.0), pq = pa;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = l + 8 * u;
                const double2 hv = HVp[c > j ? c - j : 0];
                pa = cadd(pa, cmul(a[u], hv));
                pq = cadd(pq, cmul(qm[u], hv));
            }
            pa.x = sum8(pa.x);
            pa.y = sum8(pa.y);
            pq.x = sum8(pq.x);
            pq.y = sum8(pq.y);
            const int ri = r > j ? r - j : 0;  // row r's slot in the padded arrays (0: outside the block)
            const double2 vr = HVp[ri];
            // v^H p (real: B is Hermitian): each half-wave's four rows, summed in a fixed order below
            const double hs = sum32(l == 0 ? fma(vr.x, pa.x, vr.y * pa.y) : 0.0);
            if ((t & 31) == 0) SW[t >> 5] = hs;
            if (l == 0) {
                UV[r] = pq;
                if (r > j) {
                    PVp[ri] = pa;
                    CPp[ri] = cconj(cmul(tau, pa));
                }
            }
            __syncthreads();
            const double sv = ((SW[0] + SW[1]) + (SW[2] + SW[3])) + ((SW[4] + SW[5]) + (SW[6] + SW[7]));
            const double h2 = fma(tau.x, tau.x, tau.y * tau.y) * sv;  // 2 h = |tau|^2 v^H p
            // B[r][c] -= w_r conj(v_c) + v_r conj(w_c) with w = tau p - h v, i.e. X_r conj(v_c) + v_r conj(tau p_c)
            // with X_r = tau p_r - 2 h v_r; Q[r][c] -= u_r tau conj(v_c)
            const double2 xr = csub(cmul(tau, PVp[ri]), cscale(vr, h2));
            const double2 ur = UV[r];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = l + 8 * u, ci = c > j ? c - j : 0;
                const double2 cv = cconj(HVp[ci]);
                a[u] = csub(a[u], cadd(cmul(xr, cv), cmul(vr, CPp[ci])));
                qm[u] = csub(qm[u], cmul(ur, TVC[ci]));
            }
        }
        // the owners of row cn publish column cn (its conjugate; the matrix is Hermitian), final from here on
        if (r == cn) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (l + 8 * u < n) COL[l + 8 * u] = cconj(a[u]);
        }
        __syncthreads();
    }
    if (t == 0) Dg[n - 1] = COL[n - 1].x;
    __syncthreads();
    // T in registers (scaled by 2^-sx, exact, so that |T| <= 1), |T| and the Gershgorin interval; alike in
    // every thread.  Rows past n are decoupled copies of the largest diagonal bound: no count changes there.
    double dv[kMaxF], e2v[kMaxF];
    double tn = 0.0, lo = 1.0 / 0.0, hi = -1.0 / 0.0;
#pragma unroll
    for (int i = 0; i < kMaxF; ++i) {
        const double di = i < n ? Dg[i] : 0.0;
        const double el = (i > 0 && i < n) ? fabs(Ef[i - 1]) : 0.0, er = i + 1 < n ? fabs(Ef[i]) : 0.0;
        dv[i] = di;
        e2v[i] = el * el;
        if (i < n) {
            lo = fmin(lo, di - el - er);
            hi = fmax(hi, di + el + er);
            tn = fmax(tn, fabs(di) + el + er);
        }
    }
    const int sx = tn > 0.0 ? __builtin_amdgcn_frexp_exp(tn) : 0;
    const double sc1 = __builtin_ldexp(1.0, -sx);  // |T| sc1 in [0.5, 1)
    lo = fma(-1e-14, tn, lo) * sc1 - 1e-300;
    hi = fma(1e-14, tn, hi) * sc1 + 1e-300;
#pragma unroll
    for (int i = 0; i < kMaxF; ++i) {
        dv[i] = i < n ? dv[i] * sc1 : 2.0;  // beyond every bracket point
        e2v[i] = i < n ? e2v[i] * sc1 * sc1 : 0.0;
    }

    // 2. the k largest eigenvalues: groups of tpe lanes (a power of two <= 64, inside one wave); lane q of a group
    // counts at the points (p tpe + q + 1) / (kP tpe + 1) of the bracket, p < kP; counts grow with the point, so
    // the points below the eigenvalue are the first `below` of the group's kP tpe points and the new bracket lies
    // between points below - 1 and below
    {
        constexpr int kP = 2;
        int tpe = 64;
        while (tpe * k > NT && tpe > 1) tpe >>= 1;
        const int grp = t / tpe, q = t % tpe, gbase = (t & 63) - q;
        const uint64_t gmask = tpe == 64 ? ~0ull : ((1ull << tpe) - 1ull);
        const bool active = grp < k;
        const int idx = active ? n - 1 - grp : 0;  // eigenvalue index in ascending order
        const int npts = kP * tpe;
        const double step = 1.0 / (double)(npts + 1);
        for (int it = 0; it < 200; ++it) {
            const double w = hi - lo;
            double sig[kP];
            int cnt[kP];
#pragma unroll
            for (int p = 0; p < kP; ++p) sig[p] = fma(w, (double)(p * tpe + q + 1) * step, lo);
            sturm_counts<kP>(dv, e2v, sig, cnt);
            int below = 0;
#pragma unroll
            for (int p = 0; p < kP; ++p) below += __popcll((__ballot(cnt[p] <= idx) >> gbase) & gmask);
            const double nlo = below > 0 ? fma(w, (double)below * step, lo) : lo;
            const double nhi = below < npts ? fma(w, (double)(below + 1) * step, lo) : hi;
            const bool done = !active || (nlo == lo && nhi == hi);
            lo = nlo;
            hi = nhi;
            if (__all(done)) break;
        }
        if (active && q == 0) LAM[grp] = __builtin_ldexp(0.5 * (lo + hi), sx);
    }
    const double pivmin = 1e-290 * fmax(1.0, tn * tn);
    __syncthreads();

    // 3. twisted factorisations: lane 2j runs the forward pivots of eigenvalue j, lane 2j + 1 the backward ones,
    // as one instruction stream (index i = s forward, n - 1 - s backward)
    if (t < 2 * k) {
        const int j = t >> 1, dir = t & 1;
        const double lam = LAM[j];
        double dpv = Dg[dir ? n - 1 : 0] - lam;
#pragma unroll
        for (int s = 0; s + 1 < kMaxF; ++s) {
            const bool live = s + 1 < n;
            const int sc = live ? s : 0, i = dir ? n - 1 - sc : sc, inext = dir ? i - 1 : i + 1;
            const double e = Ef[dir ? i - 1 : i], dn = Dg[inext];  // e: the off-diagonal between i and inext
            const double rl = e * rcp_d(dpv != 0.0 ? dpv : pivmin);
            if (live) {
                PIV[dir][j][i] = dpv;
                RAT[dir][j][i] = rl;
            }
            dpv = live ? fma(-rl, e, dn - lam) : dpv;
        }
        PIV[dir][j][dir ? 0 : n - 1] = dpv;
    }
    __syncthreads();
    // twist index: the smallest |gamma_i| = |D+_i + D-_i - (d_i - lambda)|, ties to the lower index; 32 lanes each
    for (int j = t >> 5; j < k; j += NT / 32) {
        const int i = t & 31;
        double av = 1.0 / 0.0;
        if (i < n) {
            const double gm = fabs(PIV[0][j][i] + PIV[1][j][i] - (Dg[i] - LAM[j]));
            av = gm <= 1.7e308 ? gm : 1.0 / 0.0;
        }
        int ia = i;
        for (int o = 16; o > 0; o >>= 1) {
            const double b = __shfl_xor(av, o);
            const int ib = __shfl_xor(ia, o);
            if (b < av || (b == av && ib < ia)) {
                av = b;
                ia = ib;
            }
        }
        if (i == 0) TW[j] = ia;
    }
    __syncthreads();
    if (t < 2 * k) {  // z_r = 1, then lane 2j goes up (z_i = -(e_i / D+_i) z_{i+1}), lane 2j + 1 down
        const int j = t >> 1, dir = t & 1, rt = TW[j];
        double z = 1.0;
        if (dir == 0) Z[j][rt] = 1.0;
#pragma unroll
        for (int s = 1; s < kMaxF; ++s) {
            const int i = dir ? rt + s : rt - s;
            const bool live = i >= 0 && i < n;
            const double rl = RAT[dir][j][live ? i : rt];
            z = live ? -rl * z : z;
            if (live) Z[j][i] = z;
        }
    }
    __syncthreads();
    for (int j = t >> 5; j < k; j += NT / 32) {
        const int i = t & 31;
        const double z = i < n ? Z[j][i] : 0.0;
        const double s2 = sum32(z * z);
        if (i < n) Z[j][i] = z / sqrt(s2);
    }
    __syncthreads();

    // 4. residuals and orthogonality
    const double rtol = 1e-11 * tn;
    for (int e = t; e < k * 32; e += NT) {
        const int j = e >> 5, i = e & 31;
        if (i < n) {
            double res = (Dg[i] - LAM[j]) * Z[j][i];
            if (i > 0) res = fma(Ef[i - 1], Z[j][i - 1], res);
            if (i + 1 < n) res = fma(Ef[i], Z[j][i + 1], res);
            if (!(fabs(res) <= rtol)) atomicOr(&bad, 1);
        }
    }
    for (int e = t; e < k * k; e += NT) {
        const int ja = e / k, jb = e % k;
        double d = 0.0;
#pragma unroll
        for (int i = 0; i < kMaxF; ++i) {
            const double za = Z[ja][min(i, n - 1)], zb = Z[jb][min(i, n - 1)];
            d = i < n ? fma(za, zb, d) : d;
        }
        M[ja][jb] = d;
        if (ja != jb && !(fabs(d) <= 1e-10)) atomicOr(&bad, 1);
    }
    __syncthreads();
    if (bad) {  // uniform
        jacobi_solve<NT>(g, F, vec, eval, 40);
        return;
    }
    // z_j <- (z_j - sum_{a<j} M_aj z_a) / sqrt(1 - sum_{a<j} M_aj^2), into RAT[0] (free now)
    for (int e = t; e < k * 32; e += NT) {
        const int j = e >> 5, i = e & 31;
        if (i < n) {
            double z = Z[j][i], n2 = 1.0;
            for (int ja = 0; ja < j; ++ja) {
                z = fma(-M[ja][j], Z[ja][i], z);
                n2 = fma(-M[ja][j], M[ja][j], n2);
            }
            RAT[0][j][i] = z / sqrt(n2);
        }
    }
    __syncthreads();

    // 5. v_j = Q z_j: this thread's four columns, then the row's eight threads
    for (int j = 0; j < k; ++j) {
        double2 v = make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = l + 8 * u;
            const double z = RAT[0][j][c < n ? c : 0];
            v = c < n ? make_double2(fma(qm[u].x, z, v.x), fma(qm[u].y, z, v.y)) : v;
        }
        v.x = sum8(v.x);
        v.y = sum8(v.y);
        if (l == 0 && r < n) vec[r * F + j] = v;
    }
    if (t < k) eval[t] = LAM[t];
}

// pd[v] = |c_v|^2 - sum_{j<k} |sum_f c_v[f] vec[f][j]|^2  (float64), clamped at 0; k = F gives 0.  A block
// stages kPV voxel rows through LDS (coalesced loads), then one thread per voxel.
constexpr int kPV = 128;
__global__ __launch_bounds__(256) void pd_kernel(const float2* __restrict__ y, int64_t V, int F, int k,
                                                 const double2* __restrict__ vec, float* __restrict__ pd) {
    __shared__ double2 sv[kMaxF * kMaxF];
    __shared__ float2 ys[kPV][kMaxF + 1];
    const int t = threadIdx.x;
    const int64_t v0 = (int64_t)blockIdx.x * kPV;
    const int nv = (int)(V - v0 < kPV ? V - v0 : kPV);
    for (int i = t; i < F * F; i += 256)
        if (i % F < k) sv[i] = vec[i];  // the k columns the solver wrote
    if (F == kMaxF) {
        for (int v = t >> 5; v < nv; v += 8) ys[v][t & 31] = y[(v0 + v) * kMaxF + (t & 31)];
    } else {
        for (int i = t; i < nv * F; i += 256) ys[i / F][i % F] = y[v0 * F + i];
    }
    __syncthreads();
    if (t >= nv) return;
    if (k >= F) {  // every component removed
        pd[v0 + t] = 0.0f;
        return;
    }
    double e = 0.0;
    for (int f = 0; f < F; ++f) {
        const float2 z = ys[t][f];
        e = fma((double)z.x, (double)z.x, fma((double)z.y, (double)z.y, e));
    }
    for (int j = 0; j < k; ++j) {
        double re = 0.0, im = 0.0;
        for (int f = 0; f < F; ++f) {
            const float2 z = ys[t][f];
            const double2 w = sv[f * F + j];
            re = fma((double)z.x, w.x, fma(-(double)z.y, w.y, re));
            im = fma((double)z.x, w.y, fma((double)z.y, w.x, im));
        }
        e -= re * re + im * im;
    }
    pd[v0 + t] = (float)(e > 0.0 ? e : 0.0);
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
// Gram partial blocks: at most kGramBlocks (two per CU), each at least one 128-voxel LDS stage
constexpr int64_t kGramBlocks = 512;
int64_t gram_chunk(int64_t V, int64_t max_blocks = kGramBlocks) {
    const int64_t c = (V + max_blocks - 1) / max_blocks;
    return c < post::kGV ? post::kGV : c;
}

// Work layout of Power Doppler in double2 units: nb partial Gram matrices, their sum, the eigenvectors, then the
// F eigenvalues (doubles, rounded up to whole double2).
int64_t pd_work2(int64_t nb, int F) { return nb * F * F + 2 * (int64_t)F * F + (F + 1) / 2; }

// Allocation-free Power Doppler: its work lives in this fixed device array (one per GPU, kept until the process
// ends).  Size: the work of kGramBlocks partial blocks at 32 frames, so that the voxel chunking (and the result)
// is that of a call with a caller's buffer for every frame count.
constexpr int64_t kScratch2 = kGramBlocks * 32 * 32 + 2 * 32 * 32 + 16;  // double2 entries (8.03 MiB)
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
    // no filter (k = 0) keeps every voxel's energy and k = F removes all of it: no eigenvectors are needed
    if (n_clutter > 0 && n_clutter < F) {
        hipLaunchKernelGGL(post::gram_partial_kernel, dim3(nb), dim3(256), 0, s, yy, V, F, chunk, part);
        hipLaunchKernelGGL(post::gram_reduce_kernel, dim3((unsigned)(F * F)), dim3(64), 0, s, part, nb, F, gram);
        hipLaunchKernelGGL(post::eig_top_kernel, dim3(1), dim3(256), 0, s, gram, F, n_clutter, vec, eval);
    }
    hipLaunchKernelGGL(post::pd_kernel, dim3((unsigned)((V + post::kPV - 1) / post::kPV)), dim3(256), 0, s, yy, V, F,
                       n_clutter, vec,
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
    return power_doppler_impl(y, V, F, n_clutter, pd, reinterpret_cast<double2*>(work), kGramBlocks,
                              reinterpret_cast<hipStream_t>(stream));
}

int das_power_doppler_noalloc(const void* y, int64_t V, int F, int n_clutter, float* pd, void* stream) {
    if (!y || !pd) return pfail(DAS_EINVAL, "power_doppler_noalloc: null pointer");
    if (V < 1 || F < 1 || F > post::kMaxF)
        return pfail(DAS_ESHAPE, "power_doppler_noalloc: need V >= 1 and 1 <= F <= 32");
    if (n_clutter < 0 || n_clutter > F) return pfail(DAS_EINVAL, "power_doppler_noalloc: need 0 <= n_clutter <= F");
    // the most Gram partial blocks the scratch array holds at F frames (at least kGramBlocks for F <= 32)
    const int64_t fit = (kScratch2 - pd_work2(0, F)) / ((int64_t)F * F);
    const int64_t max_blocks = fit < kGramBlocks ? fit : kGramBlocks;
    if (pd_work2((V + gram_chunk(V, max_blocks) - 1) / gram_chunk(V, max_blocks), F) > kScratch2)
        return pfail(DAS_ESHAPE, "power_doppler_noalloc: work exceeds the 8 MiB scratch array");
    double2* work = nullptr;
    const int st = scratch_on_current_device(&work);
    if (st != DAS_OK) return st;
    return power_doppler_impl(y, V, F, n_clutter, pd, work, max_blocks, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
