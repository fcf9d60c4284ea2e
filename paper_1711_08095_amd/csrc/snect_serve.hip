// Fold-in of a new patient and top-k search over the patient factor
// (Section 3.2.1, Eq. 6), on the GPU.
//
// With B, C, G fixed, a new patient's observed cells (j_t, k_t, x_t) define
// rows w_t = G x2 b_{j_t} x3 c_{k_t} = H_{k_t} b_{j_t} (J1 values).  Eq. (6)
// asks for the u minimising |x - W u|; as in the library's reading a ridge
// term lambda/2 |u|^2 is added, so u solves (W^T W + lambda I) u = W^T x.
// The server computes, per request:
//   Q = W^T W + lambda I and r = W^T x in FP32 (the rows w from an FP32
//       table; partial sums per workgroup over contiguous nonzero ranges,
//       then added in ascending order);
//   pg_iters projected-gradient steps from u = 0 with step 1/|Q|_F, in FP32
//       (the projection is the identity: u is unconstrained);
//   one refinement u <- u + Q^{-1}(r - Q u) in FP64: the residual and a
//       Cholesky factorisation of Q with its two triangular solves, which
//       lands on the minimiser of the FP32-formed system;
//   cosine similarity of u with every row of A in FP32 (rows of zero norm
//       excluded) and the top k rows, ties to the lower row index.
// FP64 is used for the J1 x J1 refinement only.
// Nothing is shared between requests, so a request's result does not depend
// on what else runs beside it.
#include <hip/hip_runtime.h>

#include "snect_internal.h"

namespace snect {

// W[(k*I2 + j)*J1 + a] = sum_b H_k[a][b] B[j][b], H_k[a][b] = sum_c G[a,b,c] C[k][c]
// (FP32, ascending b and c).
__global__ __launch_bounds__(256) void serve_build_w(const float* B, const float* C, const float* G, int I2, int I3,
                                                     int J1, int J2, int J3, float* W)
{
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)I3 * I2 * J1) return;
    const int a = (int)(idx % J1);
    const long long kj = idx / J1;
    const int j = (int)(kj % I2), k = (int)(kj / I2);
    float s = 0.f;
    for (int b = 0; b < J2; ++b) {
        float h = 0.f;
        for (int c = 0; c < J3; ++c) h = fmaf(G[(a * J2 + b) * J3 + c], C[k * J3 + c], h);
        s = fmaf(h, B[(size_t)j * J2 + b], s);
    }
    W[idx] = s;
}

// Row norms of A (FP32, ascending columns) and its transpose
// At[c * I1 + r] = A[r][c], so that the cosine pass reads columns with
// consecutive threads on consecutive rows.
__global__ __launch_bounds__(256) void serve_rows(const float* A, int I1, int J1, float* nrm, float* At)
{
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= I1) return;
    float s = 0.f;
    for (int c = 0; c < J1; ++c) {
        const float v = A[(size_t)r * J1 + c];
        s = fmaf(v, v, s);
        At[(size_t)c * I1 + r] = v;
    }
    nrm[r] = sqrtf(s);
}

constexpr int kFoldBatch = 128;  // nonzeros staged per pass (17 KB of LDS)

// Partial Gram sums: workgroup g takes nonzeros [g*chunk, (g+1)*chunk)
// (at most kServeMaxParts workgroups per request).
// Entry e < J1(J1+1)/2 is Q[a][b] (a <= b, row-major upper triangle); entry
// NQ + a is r[a].  G = floor(256 / ne) threads share an entry (G = 1 when
// ne > 256, a thread then taking entries tid, tid + 256, tid + 512): slice
// s of a batch's nb nonzeros is [s*nb/G, (s+1)*nb/G), and the G sums of an
// entry are added in slice order at the end.
__global__ __launch_bounds__(256) void serve_gram(const int32_t* jj, const int32_t* kk, const float* xx, int n,
                                                  int chunk, const float* W, int I2, int J1, float* part)
{
    __shared__ float wb[kFoldBatch * 33];
    __shared__ float xb[kFoldBatch];
    __shared__ long long rbase[kFoldBatch];
    __shared__ float psum[576];
    const int tid = threadIdx.x, g = blockIdx.x;
    const int nq = J1 * (J1 + 1) / 2, ne = nq + J1;
    const int G = ne < 256 ? 256 / ne : 1;
    const int z0 = g * chunk, z1 = (z0 + chunk) < n ? (z0 + chunk) : n;
    // this thread's tasks (entry, slice) and the operands of each entry
    int ta[3], tb[3], tsl[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        const int task = tid + 256 * u;
        const int e = task % ne, sl = task / ne;
        tsl[u] = task < ne * G ? sl : -1;
        if (e < nq) {
            // row a of the upper triangle starts at a*J1 - a(a-1)/2
            int aa = 0, rem = e;
            while (rem >= J1 - aa) {
                rem -= J1 - aa;
                ++aa;
            }
            ta[u] = aa;
            tb[u] = aa + rem;
        } else {
            ta[u] = e - nq;
            tb[u] = -1;  // r[a]: the value times w_a
        }
    }
    float acc[3] = {0.f, 0.f, 0.f};
    for (int b0 = z0; b0 < z1; b0 += kFoldBatch) {
        const int nb = (z1 - b0) < kFoldBatch ? (z1 - b0) : kFoldBatch;
        __syncthreads();
        if (tid < nb) {
            const int z = b0 + tid;
            rbase[tid] = ((long long)kk[z] * I2 + jj[z]) * J1;
            xb[tid] = xx[z];
        }
        __syncthreads();
        // the batch's rows of W, every thread gathering (independent loads)
#pragma unroll 4
        for (int idx = tid; idx < nb * J1; idx += 256) {
            const int t = idx / J1, c = idx - t * J1;
            wb[t * 33 + c] = W[rbase[t] + c];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            if (tsl[u] < 0) continue;
            const int t0 = (int)(((long long)nb * tsl[u]) / G), t1 = (int)(((long long)nb * (tsl[u] + 1)) / G);
            const int aa = ta[u], bb = tb[u];
            float s = acc[u];
            if (bb >= 0) {
#pragma unroll 4
                for (int t = t0; t < t1; ++t) s = fmaf(wb[t * 33 + aa], wb[t * 33 + bb], s);
            } else {
#pragma unroll 4
                for (int t = t0; t < t1; ++t) s = fmaf(xb[t], wb[t * 33 + aa], s);
            }
            acc[u] = s;
        }
    }
#pragma unroll
    for (int u = 0; u < 3; ++u)
        if (tsl[u] >= 0) psum[tid + 256 * u] = acc[u];
    __syncthreads();
    for (int e = tid; e < ne; e += 256) {
        float s = psum[e];
        for (int sl = 1; sl < G; ++sl) s += psum[sl * ne + e];
        part[(size_t)g * ne + e] = s;
    }
}

constexpr int kRegRows = 24;  // scores per thread kept in registers: I1 <= 256 * kRegRows

// Orders a wavefront's LDS exchanges between its lanes: a wavefront-scope
// barrier and a compiler memory fence (every later read is a new load).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Value of v in lane l of the wavefront (l uniform).
__device__ inline float lane_f(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double lane_d(double v, int l)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Cosine scores (FP32) of the eight rows i0 + 256 q (q < 8): the loads of up
// to twelve columns of all eight rows are issued before any product, and
// each dot product adds its columns in ascending order.  Rows past I1 are
// computed on row I1 - 1 and must not be used.
__device__ inline void cosine8(const float* At, const float* anrm, const float* u, float un, int I1, int J1, int i0,
                               float sc[8])
{
    constexpr int kCols = 12;
    int row[8];
    float nr[8], dot[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        row[q] = i0 + 256 * q < I1 ? i0 + 256 * q : I1 - 1;
        dot[q] = 0.f;
    }
    for (int c0 = 0; c0 < J1; c0 += kCols) {
        float v[8][kCols];
#pragma unroll
        for (int c = 0; c < kCols; ++c) {
            const float* col = At + (size_t)(c0 + c < J1 ? c0 + c : J1 - 1) * I1;  // unused past J1
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q][c] = col[row[q]];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) nr[q] = anrm[row[q]];
        __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the products
#pragma unroll
        for (int c = 0; c < kCols; ++c) {
            if (c0 + c >= J1) break;
            const float uc = u[c0 + c];
#pragma unroll
            for (int q = 0; q < 8; ++q) dot[q] = fmaf(v[q][c], uc, dot[q]);
        }
    }
    // rows of zero norm are excluded (NaN); a zero u scores every other row -inf
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        float x = nr[q] > 0.f ? -INFINITY : NAN;
        if (nr[q] > 0.f && un > 0.f) x = dot[q] / (nr[q] * un);
        sc[q] = x;
    }
}

// Larger score first, lower row index on ties; an index < 0 is no candidate.
__device__ inline bool better(float s2, int i2, float s1, int i1)
{
    return i2 >= 0 && (i1 < 0 || s2 > s1 || (s2 == s1 && i2 < i1));
}

// A thread's best (bs, bi) and runner-up (cs, ci) among the rows offered.
struct Best2 {
    float bs, cs;
    int bi, ci;
};

// Best candidate of the wavefront in every lane: four DPP exchange steps
// within rows of 16 lanes (quad_perm xor 1, xor 2, row_ror 4, row_ror 8),
// then exchanges across rows.  `better` is a strict total order on
// candidates, so the order of the steps does not change the result.
template <int CTRL>
__device__ inline int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ inline void best_step_dpp(float& s, int& i)
{
    const float s2 = __int_as_float(dpp_i<CTRL>(__float_as_int(s)));
    const int i2 = dpp_i<CTRL>(i);
    if (better(s2, i2, s, i)) {
        s = s2;
        i = i2;
    }
}

__device__ inline void wave_best(float& s, int& i)
{
    best_step_dpp<0xB1>(s, i);   // quad_perm [1,0,3,2]
    best_step_dpp<0x4E>(s, i);   // quad_perm [2,3,0,1]
    best_step_dpp<0x124>(s, i);  // row_ror 4
    best_step_dpp<0x128>(s, i);  // row_ror 8
#pragma unroll
    for (int o = 16; o <= 32; o <<= 1) {
        const float s2 = __shfl_xor(s, o);
        const int i2 = __shfl_xor(i, o);
        if (better(s2, i2, s, i)) {
            s = s2;
            i = i2;
        }
    }
}

__device__ __attribute__((always_inline)) inline void offer(Best2& c, float x, int i)
{
    if (x != x) return;
    if (better(x, i, c.bs, c.bi)) {
        c.cs = c.bs;
        c.ci = c.bi;
        c.bs = x;
        c.bi = i;
    } else if (better(x, i, c.cs, c.ci)) {
        c.cs = x;
        c.ci = i;
    }
}

// Solve and search, one workgroup per request.  out: u[J1], then for the
// top k: scores, then indices (as doubles); status[0]: 1 if Q is not
// positive definite.  Both are stored once, at the end (a store to host
// memory would hold up every later barrier), so out and status may be
// device mappings of pinned host memory.  RS: a thread's scores (rows
// tid + 256 q) stay in registers (I1 <= 256 * kRegRows), else they go to
// `gscores` (global, I1 entries).
template <bool RS>
__global__ __launch_bounds__(256) void serve_solve(const float* part, int nparts, int J1, float lam, int pg_iters,
                                                   const float* At, const float* anrm, int I1, int topk,
                                                   float* gscores, double* out, int* status)
{
    __shared__ float Q[32 * 32];
    __shared__ double Lt[32 * 32];  // rows of L, read back as columns
    __shared__ float r[32], uf[32];
    __shared__ double ud[32];
    __shared__ float psub[576];
    __shared__ float red_s[8];  // per wavefront, two rounds
    __shared__ int red_i[8];
    __shared__ float unorm;
    __shared__ int bad;
    __shared__ float top_s[64];  // topk <= 64
    __shared__ int top_i[64];
    const int tid = threadIdx.x;
    const int nq = J1 * (J1 + 1) / 2, ne = nq + J1;
    // Q and r from the partial sums (FP32): G threads per entry each add a
    // contiguous range of workgroups in ascending order (32 loads in
    // flight), then the G range sums are added in ascending order.
    // Consecutive threads take consecutive entries of one range, so a
    // wavefront reads whole rows of the partials.
    const int G = ne < 256 ? 256 / ne : 1;
    for (int task = tid; task < ne * G; task += 256) {
        const int gsub = task / ne, e = task - gsub * ne;
        const int p0 = (int)(((long long)nparts * gsub) / G), p1 = (int)(((long long)nparts * (gsub + 1)) / G);
        float acc = 0.f;
        for (int pb = p0; pb < p1; pb += 32) {
            float v[32];
#pragma unroll
            for (int q = 0; q < 32; ++q) v[q] = pb + q < p1 ? part[(size_t)(pb + q) * ne + e] : 0.f;
#pragma unroll
            for (int q = 0; q < 32; ++q) acc += v[q];
        }
        psub[task] = acc;
    }
    __syncthreads();
    for (int e = tid; e < ne; e += 256) {
        float s = psub[e];
        for (int gsub = 1; gsub < G; ++gsub) s += psub[gsub * ne + e];
        if (e < nq) {
            int a = 0, rem = e;
            while (rem >= J1 - a) {
                rem -= J1 - a;
                ++a;
            }
            const int b = a + rem;
            Q[a * J1 + b] = s + (a == b ? lam : 0.f);
            Q[b * J1 + a] = s + (a == b ? lam : 0.f);
        } else {
            r[e - nq] = s;
        }
    }
    __syncthreads();
    // The J1 x J1 algebra runs in wavefront 0 alone: lane a holds row a of
    // Q (and of L) in registers and reads other lanes' values by readlane.
    if (tid < 64) {
        const int a = tid;
        const bool own = a < J1;
        float qa[32];
#pragma unroll
        for (int b = 0; b < 32; ++b) qa[b] = (own && b < J1) ? Q[a * J1 + b] : 0.f;
        // PG step 1/|Q|_F: row sums of squares, added in row order
        float fa = 0.f;
#pragma unroll
        for (int b = 0; b < 32; ++b) fa = fmaf(qa[b], qa[b], fa);
        float f = 0.f;
        for (int b = 0; b < J1; ++b) f += lane_f(fa, b);
        const float stp = f > 0.f ? 1.f / sqrtf(f) : 0.f;
        const float ra = own ? r[a] : 0.f;
        // projected-gradient steps from u = 0 (identity projection), FP32; the
        // row-times-u sum runs on four accumulators (columns b mod 4).
        // Columns J1.. and lanes J1.. hold zeros, so blocks of four need no
        // inner guard.
        float ua = 0.f;
        for (int it = 0; it < pg_iters; ++it) {
            float s0 = -ra, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
            for (int b = 0; b < 32; b += 4) {
                if (b < J1) {
                    s0 = fmaf(qa[b], lane_f(ua, b), s0);
                    s1 = fmaf(qa[b + 1], lane_f(ua, b + 1), s1);
                    s2 = fmaf(qa[b + 2], lane_f(ua, b + 2), s2);
                    s3 = fmaf(qa[b + 3], lane_f(ua, b + 3), s3);
                }
            }
            if (own) ua -= stp * ((s0 + s1) + (s2 + s3));
        }
        // refinement in FP64: residual g = r - Q u, then Q = L L^T
        double ga = (double)ra;
#pragma unroll
        for (int b = 0; b < 32; ++b)
            if (b < J1) ga -= (double)qa[b] * (double)lane_f(ua, b);
        // Cholesky column by column; every entry in the order of the
        // textbook row loop (lane c forms the pivot, lanes below it L[a][c]).
        // After a pivot <= 0 the factor is not used: the loop carries on
        // with a unit pivot, so that every loop here has a fixed trip count
        // and the register arrays keep static indices.
        double la[32];
#pragma unroll
        for (int b = 0; b < 32; ++b) la[b] = 0.0;
        bool failed = false;
#pragma unroll
        for (int c = 0; c < 32; ++c) {
            if (c < J1) {
                double v = (double)qa[c];
#pragma unroll
                for (int t = 0; t < c; ++t) v -= la[t] * lane_d(la[t], c);
                const double dd = lane_d(v, c);
                failed |= !(dd > 0.0);
                const double lcc = dd > 0.0 ? sqrt(dd) : 1.0;
                if (a == c)
                    la[c] = lcc;
                else if (a > c && own)
                    la[c] = v / lcc;
            }
        }
        double za = 0.0;
        if (!failed) {
            // L y = g: y_t final at step t, then lanes a > t subtract (ascending t)
            double va = ga, ya = 0.0;
#pragma unroll
            for (int t = 0; t < 32; ++t) {
                if (t < J1) {
                    const double yt = lane_d(va / la[t], t);
                    if (a == t) ya = yt;
                    if (a > t) va -= la[t] * yt;
                }
            }
            // L^T z = y needs column a of L in lane a: through LDS
            if (own) {
#pragma unroll
                for (int t = 0; t < 32; ++t) Lt[a * 32 + t] = la[t];
            }
            wave_sync();
            double lc[32];
#pragma unroll
            for (int t = 0; t < 32; ++t) lc[t] = (own && t < J1) ? Lt[t * 32 + a] : 0.0;
            // z_t final at step t (descending), lanes a < t subtract
            double wa = ya;
#pragma unroll
            for (int t = 31; t >= 0; --t) {
                if (t < J1) {
                    const double zt = lane_d(wa / la[t], t);
                    if (a == t) za = zt;
                    if (a < t) wa -= lc[t] * zt;
                }
            }
        }
        const double uad = (double)ua + za;
        // the search works on u rounded to FP32
        const float uaf = (float)uad;
        float s = 0.f;
        for (int e = 0; e < J1; ++e) s = fmaf(lane_f(uaf, e), lane_f(uaf, e), s);
        if (own) {
            ud[a] = uad;
            uf[a] = uaf;
        }
        if (a == 0) {
            unorm = sqrtf(s);
            bad = failed ? 1 : 0;
        }
    }
    __syncthreads();
    const float un = unorm;
    // cosine scores, then top k by repeated arg-max.  Every thread keeps the
    // best and the runner-up of its own rows (tid, tid + 256, ...); a round
    // reduces the bests within each wavefront by lane exchanges, then every
    // thread reduces the four wavefront results.  The thread owning the
    // winner promotes its runner-up, and rescans its rows only when it has
    // none (it won before).  A thread's rows go in decreasing order, so the
    // rows it has left are those worse than the last one taken.
    float sc[RS ? kRegRows : 1];
    Best2 cb{-INFINITY, -INFINITY, -1, -1};
    bool have2 = true;  // cb.cs, cb.ci is the runner-up of the remaining rows
    float lt_s = 0.f;   // the last row this thread gave up (none while lt_i < 0)
    int lt_i = -1;
    if constexpr (RS) {
#pragma unroll
        for (int p = 0; p < kRegRows / 8; ++p) {
            if (p * 2048 >= I1) break;
            cosine8(At, anrm, uf, un, I1, J1, tid + p * 2048, sc + 8 * p);
        }
#pragma unroll
        for (int q = 0; q < kRegRows; ++q)
            if (tid + 256 * q < I1) offer(cb, sc[q], tid + 256 * q);
    } else {
        for (int i0 = tid; i0 < I1; i0 += 2048) {
            float x[8];
            cosine8(At, anrm, uf, un, I1, J1, i0, x);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i = i0 + 256 * q;
                if (i >= I1) break;
                gscores[i] = x[q];
                offer(cb, x[q], i);
            }
        }
    }
    const int lane = tid & 63, wv = tid >> 6;
    for (int t = 0; t < topk; ++t) {
        float ws = cb.bs;
        int wi = cb.bi;
        wave_best(ws, wi);
        const int rb = (t & 1) * 4;  // a buffer is rewritten two rounds later, past one more barrier
        if (lane == 0) {
            red_s[rb + wv] = ws;
            red_i[rb + wv] = wi;
        }
        __syncthreads();
        float s1 = red_s[rb];
        int i1 = red_i[rb];
        for (int w = 1; w < 4; ++w) {
            if (better(red_s[rb + w], red_i[rb + w], s1, i1)) {
                s1 = red_s[rb + w];
                i1 = red_i[rb + w];
            }
        }
        if (tid == 0) {
            top_s[t] = s1;
            top_i[t] = i1;
        }
        if (i1 >= 0 && (i1 & 255) == tid) {
            lt_s = s1;
            lt_i = i1;
            if (have2) {
                cb.bs = cb.cs;
                cb.bi = cb.ci;
                have2 = false;
            } else {
                cb = Best2{-INFINITY, -INFINITY, -1, -1};
                have2 = true;
                if constexpr (RS) {
#pragma unroll
                    for (int q = 0; q < kRegRows; ++q)
                        if (tid + 256 * q < I1 && better(lt_s, lt_i, sc[q], tid + 256 * q))
                            offer(cb, sc[q], tid + 256 * q);
                } else {
                    for (int i = tid; i < I1; i += 256)
                        if (better(lt_s, lt_i, gscores[i], i)) offer(cb, gscores[i], i);
                }
            }
        }
    }
    __syncthreads();
    if (tid < J1) out[tid] = ud[tid];
    if (tid < topk) {
        out[J1 + tid] = (double)top_s[tid];
        out[J1 + topk + tid] = (double)top_i[tid];
    }
    if (tid == 0) status[0] = bad;
}

hipError_t launch_serve_setup(const float* A, const float* B, const float* C, const float* G, int I1, int I2, int I3,
                              int J1, int J2, int J3, float* W, float* anrm, float* At, hipStream_t st)
{
    const long long nw = (long long)I3 * I2 * J1;
    hipLaunchKernelGGL(serve_build_w, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, B, C, G, I2, I3, J1, J2,
                       J3, W);
    hipLaunchKernelGGL(serve_rows, dim3((I1 + 255) / 256), dim3(256), 0, st, A, I1, J1, anrm, At);
    return hipGetLastError();
}

// Workgroups for a request of n nonzeros: about 256 nonzeros each (two
// batches), at most kServeMaxParts.
int serve_parts(int n)
{
    const int p = (n + 255) / 256;
    return p < 1 ? 1 : (p < kServeMaxParts ? p : kServeMaxParts);
}

hipError_t launch_serve_request(const int32_t* jj, const int32_t* kk, const float* xx, int n, const float* W, int I2,
                                int J1, double lam, int pg_iters, const float* At, const float* anrm, int I1,
                                int topk, float* part, float* scores, double* out, int* status, hipStream_t st)
{
    const int np = serve_parts(n);
    const int chunk = n > 0 ? (n + np - 1) / np : 1;
    hipLaunchKernelGGL(serve_gram, dim3(np), dim3(256), 0, st, jj, kk, xx, n, chunk, W, I2, J1, part);
    if (I1 <= 256 * kRegRows)
        hipLaunchKernelGGL(serve_solve<true>, dim3(1), dim3(256), 0, st, part, np, J1, (float)lam, pg_iters, At, anrm,
                           I1, topk, scores, out, status);
    else
        hipLaunchKernelGGL(serve_solve<false>, dim3(1), dim3(256), 0, st, part, np, J1, (float)lam, pg_iters, At, anrm,
                           I1, topk, scores, out, status);
    return hipGetLastError();
}

}  // namespace snect
