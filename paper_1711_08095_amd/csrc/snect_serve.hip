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

// Orders a wavefront's LDS exchanges between its lanes: a wavefront-scope
// barrier and a compiler memory fence (every later read is a new load).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Solve and search, one workgroup per request.  out: u[J1], then for the
// top k: scores (double), then indices (int, stored as double); status[0]:
// 1 if Q is not positive definite.  Both are stored once, at the end (a
// store to host memory would hold up every later barrier), so out and
// status may be device mappings of pinned host memory.  SL: the I1 <= kScoreLds
// scores live in dynamic LDS, else in `scores` (global).
template <bool SL>
__global__ __launch_bounds__(256) void serve_solve(const double* part, int nparts, int J1, double lam, int pg_iters,
                                                   const float* A, const double* anrm, int I1, int topk,
                                                   double* gscores, double* out, int* status)
{
    __shared__ double Q[32 * 32];
    __shared__ double L[32 * 32];
    __shared__ double r[32], u[32], g[32], d[32];
    __shared__ double psub[576];
    __shared__ double red_s[8];  // per wavefront, two rounds
    __shared__ int red_i[8];
    __shared__ double unorm, step;
    __shared__ int bad;
    __shared__ double top_s[64];  // topk <= 64
    __shared__ int top_i[64];
    extern __shared__ double lds_scores[];
    double* scores = SL ? lds_scores : gscores;
    const int tid = threadIdx.x;
    const int nq = J1 * (J1 + 1) / 2, ne = nq + J1;
    // Q and r from the partial sums: G threads per entry each add a
    // contiguous range of workgroups in ascending order (32 loads in
    // flight), then the G range sums are added in ascending order.
    // Consecutive threads take consecutive entries of one range, so a
    // wavefront reads whole rows of the partials.
    const int G = ne < 256 ? 256 / ne : 1;
    for (int task = tid; task < ne * G; task += 256) {
        const int gsub = task / ne, e = task - gsub * ne;
        const int p0 = (int)(((long long)nparts * gsub) / G), p1 = (int)(((long long)nparts * (gsub + 1)) / G);
        double acc = 0.0;
        for (int pb = p0; pb < p1; pb += 32) {
            double v[32];
#pragma unroll
            for (int q = 0; q < 32; ++q) v[q] = pb + q < p1 ? part[(size_t)(pb + q) * ne + e] : 0.0;
#pragma unroll
            for (int q = 0; q < 32; ++q) acc += v[q];
        }
        psub[task] = acc;
    }
    __syncthreads();
    for (int e = tid; e < ne; e += 256) {
        double s = psub[e];
        for (int gsub = 1; gsub < G; ++gsub) s += psub[gsub * ne + e];
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
        }
    }
    __syncthreads();
    // cosine scores; rows of zero norm are excluded (NaN), a zero u scores
    // every other row -inf.  A thread takes kCosRows rows per pass and
    // issues the loads of kCosCols columns of each before any product, so
    // one pass waits on memory once per kCosCols columns.
    constexpr int kCosRows = 9, kCosCols = 12;
    for (int i0 = tid; i0 < I1; i0 += 256 * kCosRows) {
        const float* ar[kCosRows];
        const double* np[kCosRows];
        double nr[kCosRows], dot[kCosRows];
#pragma unroll
        for (int q = 0; q < kCosRows; ++q) {
            const int i = i0 + 256 * q < I1 ? i0 + 256 * q : I1 - 1;
            ar[q] = A + (size_t)i * J1;
            np[q] = anrm + i;
            dot[q] = 0.0;
        }
        for (int c0 = 0; c0 < J1; c0 += kCosCols) {
            float v[kCosRows][kCosCols];
#pragma unroll
            for (int q = 0; q < kCosRows; ++q)
#pragma unroll
                for (int c = 0; c < kCosCols; ++c) v[q][c] = ar[q][c0 + c < J1 ? c0 + c : J1 - 1];  // unused past J1
#pragma unroll
            for (int q = 0; q < kCosRows; ++q) nr[q] = *np[q];  // with the first columns' loads
            __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the products
#pragma unroll
            for (int c = 0; c < kCosCols; ++c) {
                if (c0 + c >= J1) break;
                const double uc = u[c0 + c];
#pragma unroll
                for (int q = 0; q < kCosRows; ++q) dot[q] += (double)v[q][c] * uc;
            }
        }
#pragma unroll
        for (int q = 0; q < kCosRows; ++q) {
            const int i = i0 + 256 * q;
            if (i >= I1) break;
            double sc = nr[q] > 0.0 ? -INFINITY : NAN;
            if (nr[q] > 0.0 && unorm > 0.0) sc = dot[q] / (nr[q] * unorm);
            scores[i] = sc;
        }
    }
    // top k by repeated arg-max: larger score first, lower index on ties;
    // a taken row is marked with NaN.  Every thread keeps the best of its
    // own rows (tid, tid + 256, ...); a round reduces these within each
    // wavefront by lane exchanges, then every thread reduces the four
    // wavefront results, and only the thread owning the winner rescans.
    const int lane = tid & 63, wv = tid >> 6;
    double bs = -INFINITY;
    int bi = -1;
    for (int i = tid; i < I1; i += 256) {
        const double sc = scores[i];
        if (sc != sc) continue;
        if (bi < 0 || sc > bs) {
            bs = sc;
            bi = i;
        }
    }
    for (int t = 0; t < topk; ++t) {
        double ws = bs;
        int wi = bi;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double s2 = __shfl_xor(ws, o);
            const int i2 = __shfl_xor(wi, o);
            if (i2 >= 0 && (wi < 0 || s2 > ws || (s2 == ws && i2 < wi))) {
                ws = s2;
                wi = i2;
            }
        }
        const int rb = (t & 1) * 4;  // a buffer is rewritten two rounds later, past one more barrier
        if (lane == 0) {
            red_s[rb + wv] = ws;
            red_i[rb + wv] = wi;
        }
        __syncthreads();
        double s1 = red_s[rb];
        int i1 = red_i[rb];
        for (int w = 1; w < 4; ++w) {
            const double s2 = red_s[rb + w];
            const int i2 = red_i[rb + w];
            if (i2 >= 0 && (i1 < 0 || s2 > s1 || (s2 == s1 && i2 < i1))) {
                s1 = s2;
                i1 = i2;
            }
        }
        if (tid == 0) {
            top_s[t] = s1;
            top_i[t] = i1;
        }
        if (i1 >= 0 && (i1 & 255) == tid) {
            scores[i1] = NAN;
            bs = -INFINITY;
            bi = -1;
            for (int i = tid; i < I1; i += 256) {
                const double sc = scores[i];
                if (sc != sc) continue;
                if (bi < 0 || sc > bs) {
                    bs = sc;
                    bi = i;
                }
            }
        }
    }
    __syncthreads();
    if (tid < J1) out[tid] = u[tid];
    if (tid < topk) {
        out[J1 + tid] = top_s[tid];
        out[J1 + topk + tid] = (double)top_i[tid];
    }
    if (tid == 0) status[0] = bad;
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
