// Fold-in of a new patient and top-k search over the patient factor
// (Section 3.2.1, Eq. 6), on the GPU.
//
// With B, C, G fixed, a new patient's observed cells (j_t, k_t, x_t) define
// rows w_t = G x2 b_{j_t} x3 c_{k_t} = H_{k_t} b_{j_t} (J1 values).  Eq. (6)
// asks for the u minimising |x - W u|; as in the library's reading a ridge
// term lambda/2 |u|^2 is added, so u solves (W^T W + lambda I) u = W^T x.
// The server computes, per request and in FP64:
//   Q = W^T W + lambda I and r = W^T x (partial sums per workgroup over
//       contiguous nonzero ranges, then added in ascending order);
//   pg_iters projected-gradient steps from u = 0 with step 1/|Q|_F (the
//       projection is the identity: u is unconstrained);
//   one refinement u <- u + Q^{-1}(r - Q u) through a Cholesky factorisation
//       of Q, which lands on the exact minimiser;
//   cosine similarity of u with every row of A (rows of zero norm excluded)
//       and the top k rows, ties to the lower row index.
// Nothing is shared between requests, so a request's result does not depend
// on what else runs beside it.
#include <hip/hip_runtime.h>

#include "snect_internal.h"

namespace snect {

// W[(k*I2 + j)*J1 + a] = sum_b H_k[a][b] B[j][b], H_k[a][b] = sum_c G[a,b,c] C[k][c]
__global__ __launch_bounds__(256) void serve_build_w(const float* B, const float* C, const float* G, int I2, int I3,
                                                     int J1, int J2, int J3, double* W)
{
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)I3 * I2 * J1) return;
    const int a = (int)(idx % J1);
    const long long kj = idx / J1;
    const int j = (int)(kj % I2), k = (int)(kj / I2);
    double s = 0.0;
    for (int b = 0; b < J2; ++b) {
        double h = 0.0;
        for (int c = 0; c < J3; ++c) h += (double)G[(a * J2 + b) * J3 + c] * (double)C[k * J3 + c];
        s += h * (double)B[(size_t)j * J2 + b];
    }
    W[idx] = s;
}

__global__ __launch_bounds__(256) void serve_row_norms(const float* A, int I1, int J1, double* nrm)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= I1) return;
    double s = 0.0;
    for (int c = 0; c < J1; ++c) s += (double)A[(size_t)r * J1 + c] * (double)A[(size_t)r * J1 + c];
    nrm[r] = sqrt(s);
}

constexpr int kFoldBatch = 128;  // nonzeros staged per pass (34 KB of LDS)

// Partial Gram sums: workgroup g takes nonzeros [g*chunk, (g+1)*chunk)
// (at most kServeMaxParts workgroups per request).
// Entry e < J1(J1+1)/2 is Q[a][b] (a <= b, row-major upper triangle); entry
// NQ + a is r[a].
__global__ __launch_bounds__(256) void serve_gram(const int32_t* jj, const int32_t* kk, const float* xx, int n,
                                                  int chunk, const double* W, int I2, int J1, double* part)
{
    __shared__ double wb[kFoldBatch * 33];
    __shared__ double xb[kFoldBatch];
    const int tid = threadIdx.x, g = blockIdx.x;
    const int nq = J1 * (J1 + 1) / 2, ne = nq + J1;
    const int z0 = g * chunk, z1 = (z0 + chunk) < n ? (z0 + chunk) : n;
    double acc[3] = {0.0, 0.0, 0.0};  // entries tid, tid+256, tid+512 (ne <= 560)
    for (int b0 = z0; b0 < z1; b0 += kFoldBatch) {
        const int nb = (z1 - b0) < kFoldBatch ? (z1 - b0) : kFoldBatch;
        __syncthreads();
        // the batch's rows of W, every thread gathering (independent loads)
        for (int idx = tid; idx < nb * J1; idx += 256) {
            const int t = idx / J1, a = idx - t * J1, z = b0 + t;
            wb[t * 33 + a] = W[((size_t)kk[z] * I2 + jj[z]) * J1 + a];
        }
        if (tid < nb) xb[tid] = (double)xx[b0 + tid];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int e = tid + 256 * u;
            if (e >= ne) continue;
            double s = acc[u];
            if (e < nq) {
                // row a of the upper triangle starts at a*J1 - a(a-1)/2
                int a = 0, rem = e;
                while (rem >= J1 - a) {
                    rem -= J1 - a;
                    ++a;
                }
                const int b = a + rem;
                for (int t = 0; t < nb; ++t) s += wb[t * 33 + a] * wb[t * 33 + b];
            } else {
                const int a = e - nq;
                for (int t = 0; t < nb; ++t) s += xb[t] * wb[t * 33 + a];
            }
            acc[u] = s;
        }
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int e = tid + 256 * u;
        if (e < ne) part[(size_t)g * ne + e] = acc[u];
    }
}

constexpr int kScoreLds = 6144;  // patients whose scores stay in LDS during the search

// Solve and search, one workgroup per request.  out: u[J1], then for the
// top k: scores (double), then indices (int, stored as double).  SL: the
// I1 <= kScoreLds scores live in dynamic LDS, else in `scores` (global).
// Orders a wavefront's LDS exchanges between its lanes: a wavefront-scope
// barrier and a compiler memory fence (every later read is a new load).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

template <bool SL>
__global__ __launch_bounds__(256) void serve_solve(const double* part, int nparts, int J1, double lam, int pg_iters,
                                                   const float* A, const double* anrm, int I1, int topk,
                                                   double* gscores, double* out, int* status)
{
    __shared__ double Q[32 * 32];
    __shared__ double L[32 * 32];
    __shared__ double r[32], u[32], g[32], d[32];
    __shared__ double psub[576];
    __shared__ double red_s[4];
    __shared__ int red_i[4];
    __shared__ double unorm, step;
    __shared__ int bad;
    extern __shared__ double lds_scores[];
    double* scores = SL ? lds_scores : gscores;
    const int tid = threadIdx.x;
    const int nq = J1 * (J1 + 1) / 2, ne = nq + J1;
    // Q and r from the partial sums: G threads per entry each add a
    // contiguous range of workgroups in ascending order (16 loads in
    // flight), then the G range sums are added in ascending order
    const int G = ne < 256 ? 256 / ne : 1;
    for (int task = tid; task < ne * G; task += 256) {
        const int e = task / G, gsub = task - e * G;
        const int p0 = (int)(((long long)nparts * gsub) / G), p1 = (int)(((long long)nparts * (gsub + 1)) / G);
        double acc = 0.0;
        for (int pb = p0; pb < p1; pb += 16) {
            double v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = pb + q < p1 ? part[(size_t)(pb + q) * ne + e] : 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) acc += v[q];
        }
        psub[task] = acc;
    }
    __syncthreads();
    for (int e = tid; e < ne; e += 256) {
        double s = psub[e * G];
        for (int gsub = 1; gsub < G; ++gsub) s += psub[e * G + gsub];
        if (e < nq) {
            int a = 0, rem = e;
            while (rem >= J1 - a) {
                rem -= J1 - a;
                ++a;
            }
            const int b = a + rem;
            Q[a * J1 + b] = s + (a == b ? lam : 0.0);
            Q[b * J1 + a] = s + (a == b ? lam : 0.0);
        } else {
            r[e - nq] = s;
        }
    }
    if (tid < J1) u[tid] = 0.0;
    if (tid == 0) bad = 0;
    __syncthreads();
    // The J1 x J1 algebra runs in wavefront 0 alone (lane a holds row a).
    // Lanes exchange values through LDS: the wavefront executes in lockstep
    // and its LDS operations complete in order, and wave_sync() after every
    // exchange stops the compiler from reusing a value read before it.
    if (tid < 64) {
        const int a = tid;
        if (a == 0) {
            double f = 0.0;
            for (int e = 0; e < J1 * J1; ++e) f += Q[e] * Q[e];
            step = f > 0.0 ? 1.0 / sqrt(f) : 0.0;
        }
        wave_sync();
        const double stp = step;
        // projected-gradient steps (identity projection)
        for (int it = 0; it < pg_iters; ++it) {
            double s = 0.0;
            if (a < J1) {
                s = -r[a];
                for (int b = 0; b < J1; ++b) s += Q[a * J1 + b] * u[b];
            }
            wave_sync();
            if (a < J1) u[a] -= stp * s;
            wave_sync();
        }
        // refinement through Q = L L^T: residual g = r - Q u
        if (a < J1) {
            double s = r[a];
            for (int b = 0; b < J1; ++b) s -= Q[a * J1 + b] * u[b];
            g[a] = s;
        }
        for (int e = a; e < J1 * J1; e += 64) L[e] = 0.0;
        wave_sync();
        // Cholesky column by column; lane rr forms L[rr][c] for rr > c,
        // every entry in the order of the textbook row loop
        bool failed = false;
        for (int c = 0; c < J1; ++c) {
            double dd = 1.0;
            if (a == c) {
                dd = Q[c * J1 + c];
                for (int t = 0; t < c; ++t) dd -= L[c * J1 + t] * L[c * J1 + t];
                L[c * J1 + c] = dd > 0.0 ? sqrt(dd) : 1.0;
            }
            failed = __ballot(a == c && !(dd > 0.0)) != 0ull;  // uniform
            wave_sync();
            if (failed) break;
            if (a > c && a < J1) {
                double v = Q[a * J1 + c];
                for (int t = 0; t < c; ++t) v -= L[a * J1 + t] * L[c * J1 + t];
                L[a * J1 + c] = v / L[c * J1 + c];
            }
            wave_sync();
        }
        if (!failed) {
            // L y = g: y[t] final at step t, then lanes a > t subtract in
            // ascending t (the order of the row loop)
            double v = a < J1 ? g[a] : 0.0;
            for (int t = 0; t < J1; ++t) {
                if (a == t) d[t] = v / L[t * J1 + t];
                wave_sync();
                if (a > t && a < J1) v -= L[a * J1 + t] * d[t];
            }
            wave_sync();
            // L^T z = y: z[t] final at step t (descending), lanes a < t subtract
            v = a < J1 ? d[a] : 0.0;
            wave_sync();
            for (int t = J1 - 1; t >= 0; --t) {
                if (a == t) d[t] = v / L[t * J1 + t];
                wave_sync();
                if (a < t) v -= L[t * J1 + a] * d[t];
            }
            wave_sync();
            if (a < J1) u[a] += d[a];
            wave_sync();
        }
        if (a == 0) {
            double s = 0.0;
            for (int e = 0; e < J1; ++e) s += u[e] * u[e];
            unorm = sqrt(s);
            bad = failed ? 1 : 0;
            status[0] = bad;
        }
    }
    __syncthreads();
    // cosine scores; rows of zero norm are excluded (NaN), a zero u scores
    // every other row -inf
    for (int i = tid; i < I1; i += 256) {
        double s = anrm[i] > 0.0 ? -INFINITY : NAN;
        if (anrm[i] > 0.0 && unorm > 0.0) {
            double dot = 0.0;
            for (int a = 0; a < J1; ++a) dot += (double)A[(size_t)i * J1 + a] * u[a];
            s = dot / (anrm[i] * unorm);
        }
        scores[i] = s;
    }
    __syncthreads();
    // top k by repeated arg-max: larger score first, lower index on ties;
    // a taken row is marked with NaN.  Each round reduces within every
    // wavefront by lane exchanges, then over the four wavefronts.
    const int lane = tid & 63, wv = tid >> 6;
    for (int t = 0; t < topk; ++t) {
        double bs = -INFINITY;
        int bi = -1;
        for (int i = tid; i < I1; i += 256) {
            const double s = scores[i];
            if (s != s) continue;
            if (bi < 0 || s > bs) {
                bs = s;
                bi = i;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double s2 = __shfl_xor(bs, o);
            const int i2 = __shfl_xor(bi, o);
            if (i2 >= 0 && (bi < 0 || s2 > bs || (s2 == bs && i2 < bi))) {
                bs = s2;
                bi = i2;
            }
        }
        if (lane == 0) {
            red_s[wv] = bs;
            red_i[wv] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double s1 = red_s[0];
            int i1 = red_i[0];
            for (int w = 1; w < 4; ++w) {
                const double s2 = red_s[w];
                const int i2 = red_i[w];
                if (i2 >= 0 && (i1 < 0 || s2 > s1 || (s2 == s1 && i2 < i1))) {
                    s1 = s2;
                    i1 = i2;
                }
            }
            out[J1 + t] = s1;
            out[J1 + topk + t] = (double)i1;
            if (i1 >= 0) scores[i1] = NAN;
        }
        __syncthreads();
    }
    if (tid < J1) out[tid] = u[tid];
}

hipError_t launch_serve_setup(const float* A, const float* B, const float* C, const float* G, int I1, int I2, int I3,
                              int J1, int J2, int J3, double* W, double* anrm, hipStream_t st)
{
    if (I1 <= kScoreLds) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&serve_solve<true>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)(sizeof(double) * kScoreLds));
        if (e != hipSuccess) return e;
    }
    const long long nw = (long long)I3 * I2 * J1;
    hipLaunchKernelGGL(serve_build_w, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, B, C, G, I2, I3, J1, J2,
                       J3, W);
    hipLaunchKernelGGL(serve_row_norms, dim3((I1 + 255) / 256), dim3(256), 0, st, A, I1, J1, anrm);
    return hipGetLastError();
}

// Workgroups for a request of n nonzeros: about 256 nonzeros each (two
// batches), at most kServeMaxParts.
int serve_parts(int n)
{
    const int p = (n + 255) / 256;
    return p < 1 ? 1 : (p < kServeMaxParts ? p : kServeMaxParts);
}

hipError_t launch_serve_request(const int32_t* jj, const int32_t* kk, const float* xx, int n, const double* W, int I2,
                                int J1, double lam, int pg_iters, const float* A, const double* anrm, int I1,
                                int topk, double* part, double* scores, double* out, int* status, hipStream_t st)
{
    const int np = serve_parts(n);
    const int chunk = n > 0 ? (n + np - 1) / np : 1;
    hipLaunchKernelGGL(serve_gram, dim3(np), dim3(256), 0, st, jj, kk, xx, n, chunk, W, I2, J1, part);
    if (I1 <= kScoreLds)
        hipLaunchKernelGGL(serve_solve<true>, dim3(1), dim3(256), sizeof(double) * I1, st, part, np, J1, lam, pg_iters,
                           A, anrm, I1, topk, scores, out, status);
    else
        hipLaunchKernelGGL(serve_solve<false>, dim3(1), dim3(256), 0, st, part, np, J1, lam, pg_iters, A, anrm, I1,
                           topk, scores, out, status);
    return hipGetLastError();
}

}  // namespace snect
