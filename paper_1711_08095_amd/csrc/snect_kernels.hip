// gfx950 kernels of the SNeCT stratified SGD (arXiv:1711.08095, Algorithm 1
// with the gradients of Eq. 5, the network term of Eq. 4, the objective of
// Eq. 3).
//
// Block kernel: one wavefront per block (p, q) of a stratum.  The block's
// patient rows and gene rows live in LDS for the whole stratum; H_k = G x3 c_k
// for every platform k is built in LDS from the stratum's frozen C and G.
// Each tile (<= 64 nonzeros of one platform) is one wavefront step: lane t
// takes nonzero t, reads its rows from before the tile, forms
// w1 = H_k b_j, w2 = H_k^T a_i, e = x - a_i . w1, stages e*w1 and e*w2, and
// the last lane of each patient run / gene chain sums its row's terms in a
// fixed order and writes the updated row.  The block's sum of e a (x) b per
// platform, needed by the core step, accumulates on the matrix cores
// (v_mfma_f32_16x16x4f32 / 32x32x2f32) from staged pre-tile rows.
#include <hip/hip_runtime.h>

#include "snect_internal.h"

namespace snect {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

// LDS carve-up of the block kernel (floats unless noted).
struct BlockLds {
    int a_off, b_off, ra_off, rb_off, h_off, sta_off, stb_off, as_off, es_off, sk_off, mk_off, jp_off;
    int total;
};

__host__ __device__ inline BlockLds block_lds_layout(int jp, int rows1_max, int rows2_max, int I3,
                                                     int J1, int J2)
{
    const int rs = row_stride(jp), mp = mfma_dim(jp);
    BlockLds L;
    int o = 0;
    L.a_off = o;  o += rows1_max * rs;
    L.b_off = o;  o += rows2_max * rs;
    L.ra_off = o; o += rows1_max;
    L.rb_off = o; o += rows2_max;
    o = (o + 3) & ~3;
    L.h_off = o;  o += I3 * jp * jp;
    o = (o + 3) & ~3;
    L.sta_off = o; o += kTileMax * rs;
    L.stb_off = o; o += kTileMax * rs;
    L.as_off = o;  o += kTileMax * mp;
    L.es_off = o;  o += kTileMax * mp;
    L.sk_off = o;  o += I3 * J1 * J2;
    L.mk_off = o;  o += I3;          // int32 counts
    L.jp_off = o;  o += kTileMax;    // int32 chain links
    L.total = o;
    return L;
}

size_t block_lds_bytes(int jp, int rows1_max, int rows2_max, int I3, int J1, int J2)
{
    return align16(sizeof(float) * (size_t)block_lds_layout(jp, rows1_max, rows2_max, I3, J1, J2).total);
}

int jp_for(int J1, int J2)
{
    const int m = J1 > J2 ? J1 : J2;
    for (int t = 0; t < kJpCount; ++t)
        if (kJpSet[t] >= m) return kJpSet[t];
    return -1;
}

// MFMA accumulator of the per-platform S = sum_t e_t a_t (x) b_t.
template <int MP> struct SAcc;

template <> struct SAcc<16> {
    floatx4 v;
    __device__ void zero() { v = floatx4{0.f, 0.f, 0.f, 0.f}; }
    // staged operands are [64][16]: step s covers nonzeros 4s..4s+3 and lane l
    // supplies A[l%16][l/16] = a_{4s+l/16}[l%16] and B[l/16][l%16] likewise,
    // which is element 64 s + l of the staging arrays
    __device__ void accumulate(const float* As, const float* Es, int n, int lane)
    {
        const int steps = (n + 3) >> 2;
        for (int s = 0; s < steps; ++s)
            v = __builtin_amdgcn_mfma_f32_16x16x4f32(As[s * 64 + lane], Es[s * 64 + lane], v, 0, 0, 0);
    }
    // output element (row 4*(l/16)+r, column l%16) sits in register r of lane l
    __device__ void flush(float* Sk, int J1, int J2, int lane)
    {
        const int col = lane & 15, rb = (lane >> 4) * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rb + r;
            if (row < J1 && col < J2) Sk[row * J2 + col] += v[r];
        }
    }
};

template <> struct SAcc<32> {
    floatx16 v;
    __device__ void zero()
    {
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = 0.f;
    }
    // staged operands are [64][32]: step s covers nonzeros 2s, 2s+1 and lane l
    // supplies a_{2s+l/32}[l%32], i.e. element 64 s + l
    __device__ void accumulate(const float* As, const float* Es, int n, int lane)
    {
        const int steps = (n + 1) >> 1;
        for (int s = 0; s < steps; ++s)
            v = __builtin_amdgcn_mfma_f32_32x32x2f32(As[s * 64 + lane], Es[s * 64 + lane], v, 0, 0, 0);
    }
    // output element (row 8*(r/4) + 4*(l/32) + r%4, column l%32) in register r
    __device__ void flush(float* Sk, int J1, int J2, int lane)
    {
        const int col = lane & 31, rb = (lane >> 5) * 4;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = (r >> 2) * 8 + rb + (r & 3);
            if (row < J1 && col < J2) Sk[row * J2 + col] += v[r];
        }
    }
};

// ---------------------------------------------------------------------------
// Block kernel (FP32)
// ---------------------------------------------------------------------------
template <int JP>
__global__ __launch_bounds__(64) void block_fp32(BlockArgs a)
{
    constexpr int RS = row_stride(JP);
    constexpr int MP = mfma_dim(JP);
    extern __shared__ float lds[];
    const int lane = threadIdx.x;
    const int p = blockIdx.x;
    const int q = (p + a.s) % a.P;
    const BlockLds L = block_lds_layout(JP, a.rows1_max, a.rows2_max, a.I3, a.J1, a.J2);
    float* Ab = lds + L.a_off;
    float* Bb = lds + L.b_off;
    float* rA = lds + L.ra_off;
    float* rB = lds + L.rb_off;
    float* Hs = lds + L.h_off;
    float* stA = lds + L.sta_off;
    float* stB = lds + L.stb_off;
    float* As = lds + L.as_off;
    float* Es = lds + L.es_off;
    float* Sk = lds + L.sk_off;
    int* Mk = reinterpret_cast<int*>(lds + L.mk_off);
    int* Jl = reinterpret_cast<int*>(lds + L.jp_off);

    const int J1 = a.J1, J2 = a.J2, J3 = a.J3, I3 = a.I3;
    const int s1 = a.start1[p], r1 = a.start1[p + 1] - s1;
    const int s2 = a.start2[q], r2 = a.start2[q + 1] - s2;

    // gather the block's rows (zero-padded to the row stride)
    for (int idx = lane; idx < r1 * RS; idx += 64) {
        const int l = idx / RS, c = idx - l * RS;
        Ab[idx] = c < J1 ? a.A[(size_t)a.perm1[s1 + l] * J1 + c] : 0.f;
    }
    for (int idx = lane; idx < r2 * RS; idx += 64) {
        const int l = idx / RS, c = idx - l * RS;
        Bb[idx] = c < J2 ? a.B[(size_t)a.perm2[s2 + l] * J2 + c] : 0.f;
    }
    for (int l = lane; l < r1; l += 64) rA[l] = a.reg1[a.perm1[s1 + l]];
    for (int l = lane; l < r2; l += 64) rB[l] = a.reg2[a.perm2[s2 + l]];
    // H_k[x][y] = sum_c G[x,y,c] C[k,c] for every platform (zero padded)
    for (int idx = lane; idx < I3 * JP * JP; idx += 64) {
        const int k = idx / (JP * JP), xy = idx - k * JP * JP, x = xy / JP, y = xy - x * JP;
        float h = 0.f;
        if (x < J1 && y < J2)
            for (int c = 0; c < J3; ++c) h += a.G[(x * J2 + y) * J3 + c] * a.C[k * J3 + c];
        Hs[idx] = h;
    }
    for (int idx = lane; idx < I3 * J1 * J2; idx += 64) Sk[idx] = 0.f;
    for (int k = lane; k < I3; k += 64) Mk[k] = 0;
    __syncthreads();

    const uint32_t mask_i = (1u << a.bits_i) - 1u, mask_j = (1u << a.bits_j) - 1u;
    const int sh_j = a.bits_i, sh_f = a.bits_i + a.bits_j;
    const int blk = p * a.P + q;
    const int t0 = a.blk_tile[blk], t1 = a.blk_tile[blk + 1];

    SAcc<MP> acc;
    acc.zero();
    int curk = -1;
    uint2 wnext = make_uint2(0u, 0u);
    if (t0 < t1) {
        const int off = a.tile_off[t0], n = a.tile_off[t0 + 1] - off;
        if (lane < n) wnext = a.nz[off + lane];
    }
    for (int tl = t0; tl < t1; ++tl) {
        const int off = a.tile_off[tl];
        const int n = a.tile_off[tl + 1] - off;
        const int k = a.tile_k[tl];
        const uint2 wv = wnext;
        if (tl + 1 < t1) {  // prefetch the next tile's records
            const int o2 = a.tile_off[tl + 1], n2 = a.tile_off[tl + 2] - o2;
            wnext = lane < n2 ? a.nz[o2 + lane] : make_uint2(0u, 0u);
        }
        if (k != curk) {
            if (curk >= 0) acc.flush(Sk + curk * J1 * J2, J1, J2, lane);
            acc.zero();
            curk = k;
        }
        const bool act = lane < n;
        const uint32_t w = wv.x;
        const float x = __uint_as_float(wv.y);
        const int il = act ? (int)(w & mask_i) : -1;
        const int jl = act ? (int)((w >> sh_j) & mask_j) : 0;
        const int jprev = (int)((w >> sh_f) & 63u);
        const bool jlast = act && ((w >> (sh_f + kJprevBits)) & 1u);

        float av[JP], bv[JP];
#pragma unroll
        for (int c = 0; c < JP; ++c) {
            av[c] = act ? Ab[il * RS + c] : 0.f;
            bv[c] = act ? Bb[jl * RS + c] : 0.f;
        }
        const float* H = Hs + k * JP * JP;
        float w1[JP], w2[JP];
#pragma unroll
        for (int c = 0; c < JP; ++c) { w1[c] = 0.f; w2[c] = 0.f; }
#pragma unroll
        for (int x_ = 0; x_ < JP; ++x_)
#pragma unroll
            for (int y = 0; y < JP; ++y) {
                const float h = H[x_ * JP + y];
                w1[x_] = fmaf(h, bv[y], w1[x_]);
                w2[y] = fmaf(av[x_], h, w2[y]);
            }
        float xt = 0.f;
#pragma unroll
        for (int c = 0; c < JP; ++c) xt = fmaf(av[c], w1[c], xt);
        const float e = act ? x - xt : 0.f;

        // stage row terms, MFMA operands and gene-chain links
#pragma unroll
        for (int c = 0; c < JP; ++c) {
            stA[lane * RS + c] = e * w1[c];
            stB[lane * RS + c] = e * w2[c];
        }
#pragma unroll
        for (int c = 0; c < MP; ++c) {
            As[lane * MP + c] = c < JP ? av[c] : 0.f;
            Es[lane * MP + c] = c < JP ? e * bv[c] : 0.f;
        }
        Jl[lane] = jprev;
        __syncthreads();

        acc.accumulate(As, Es, n, lane);

        // patient runs are contiguous (tiles are sorted by i): the last lane
        // of a run sums the run in ascending order
        const int il_up = __shfl_up(il, 1);
        const int il_dn = __shfl_down(il, 1);
        const bool ifirst = act && (lane == 0 || il_up != il);
        const bool ilast = act && (lane == 63 || il_dn != il);
        const unsigned long long heads = __ballot(ifirst);
        if (ilast) {
            const unsigned long long m = lane == 63 ? heads : (heads & ((2ull << lane) - 1ull));
            const int head = 63 - __clzll(m);
            float sum[JP];
#pragma unroll
            for (int c = 0; c < JP; ++c) sum[c] = 0.f;
            for (int u = head; u <= lane; ++u)
#pragma unroll
                for (int c = 0; c < JP; ++c) sum[c] += stA[u * RS + c];
            const float cr = (float)(lane - head + 1) * rA[il];
#pragma unroll
            for (int c = 0; c < JP; ++c) Ab[il * RS + c] = av[c] + a.lr * (sum[c] - cr * av[c]);
        }
        // gene rows: follow the chain of earlier occurrences in the tile
        if (jlast) {
            float sum[JP];
#pragma unroll
            for (int c = 0; c < JP; ++c) sum[c] = stB[lane * RS + c];
            int u = lane, pv = jprev, cnt = 1;
            while (pv != u && cnt < kTileMax) {
#pragma unroll
                for (int c = 0; c < JP; ++c) sum[c] += stB[pv * RS + c];
                u = pv;
                pv = Jl[u];
                ++cnt;
            }
            const float cr = (float)cnt * rB[jl];
#pragma unroll
            for (int c = 0; c < JP; ++c) Bb[jl * RS + c] = bv[c] + a.lr * (sum[c] - cr * bv[c]);
        }
        if (lane == 0) Mk[k] += n;
        __syncthreads();
    }
    if (curk >= 0) acc.flush(Sk + curk * J1 * J2, J1, J2, lane);
    __syncthreads();

    // write the rows back and publish the block's core-gradient sums
    for (int idx = lane; idx < r1 * J1; idx += 64) {
        const int l = idx / J1, c = idx - l * J1;
        a.A[(size_t)a.perm1[s1 + l] * J1 + c] = Ab[l * RS + c];
    }
    for (int idx = lane; idx < r2 * J2; idx += 64) {
        const int l = idx / J2, c = idx - l * J2;
        a.B[(size_t)a.perm2[s2 + l] * J2 + c] = Bb[l * RS + c];
    }
    float* Sp = a.Spart + (size_t)p * I3 * J1 * J2;
    for (int idx = lane; idx < I3 * J1 * J2; idx += 64) Sp[idx] = Sk[idx];
    for (int k = lane; k < I3; k += 64) a.Mpart[p * I3 + k] = Mk[k];
}

// ---------------------------------------------------------------------------
// Core / platform step after a stratum: blocks' sums reduced in ascending p,
// then one mean-gradient step on C and G.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void core_step(CoreArgs a)
{
    extern __shared__ float lds[];
    const int J12 = a.J1 * a.J2, I3 = a.I3, J3 = a.J3;
    float* S = lds;                        // [I3][J12]
    float* C0 = S + I3 * J12;              // [I3][J3]
    float* G0 = C0 + I3 * J3;              // [J12][J3]
    double* mk = reinterpret_cast<double*>(lds + ((I3 * J12 + I3 * J3 + J12 * J3 + 1) & ~1));
    const int tid = threadIdx.x;
    for (int idx = tid; idx < I3 * J12; idx += blockDim.x) {
        float s = 0.f;
        for (int p = 0; p < a.P; ++p) s += a.Spart[(size_t)p * I3 * J12 + idx];
        S[idx] = s;
    }
    for (int k = tid; k < I3; k += blockDim.x) {
        long long m = 0;
        for (int p = 0; p < a.P; ++p) m += a.Mpart[p * I3 + k];
        mk[k] = (double)m;
    }
    for (int idx = tid; idx < I3 * J3; idx += blockDim.x) C0[idx] = a.C[idx];
    for (int idx = tid; idx < J12 * J3; idx += blockDim.x) G0[idx] = a.G[idx];
    __syncthreads();
    double m = 0.0;
    for (int k = 0; k < I3; ++k) m += mk[k];
    if (m <= 0.0) return;
    const float inv_m = (float)(1.0 / m);
    for (int idx = tid; idx < I3 * J3; idx += blockDim.x) {
        const int k = idx / J3, c = idx - k * J3;
        float g = 0.f;
        for (int ab = 0; ab < J12; ++ab) g -= G0[ab * J3 + c] * S[k * J12 + ab];
        if (mk[k] > 0.0) g += a.lam * (float)(mk[k] / (double)a.cnt3[k]) * C0[idx];
        a.C[idx] = C0[idx] - a.etac * g * inv_m;
    }
    const float greg = a.lam * (float)(m / a.nnz);
    for (int idx = tid; idx < J12 * J3; idx += blockDim.x) {
        const int ab = idx / J3, c = idx - ab * J3;
        float g = 0.f;
        for (int k = 0; k < I3; ++k) g -= S[k * J12 + ab] * C0[k * J3 + c];
        g += greg * G0[idx];
        a.G[idx] = G0[idx] - a.etac * g * inv_m;
    }
}

// ---------------------------------------------------------------------------
// Network step: one Jacobi application of B <- B - alpha L B.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void graph_step(GraphArgs a)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.I2 * a.J2) return;
    const int r = idx / a.J2, c = idx - r * a.J2;
    float lb = a.deg[r] * a.Bin[idx];
    for (int e = a.adj_start[r]; e < a.adj_start[r + 1]; ++e)
        lb -= a.adj_w[e] * a.Bin[(size_t)a.adj_nbr[e] * a.J2 + c];
    a.Bout[idx] = a.Bin[idx] - a.alpha * lb;
}

// ---------------------------------------------------------------------------
// Loss: per-block squared errors (FP32 model value, FP64 sums), then one
// workgroup adds the blocks in order with the L2 and network terms.
// ---------------------------------------------------------------------------
struct LossLds {
    int a_off, b_off, h_off, red_off, total;
};

__host__ __device__ inline LossLds loss_lds_layout(int jp, int rows1_max, int rows2_max, int I3)
{
    const int rs = row_stride(jp);
    LossLds L;
    int o = 0;
    L.a_off = o; o += rows1_max * rs;
    L.b_off = o; o += rows2_max * rs;
    o = (o + 3) & ~3;
    L.h_off = o; o += I3 * jp * jp;
    o = (o + 1) & ~1;
    L.red_off = o; o += 2 * 256;  // 256 doubles
    L.total = o;
    return L;
}

size_t loss_lds_bytes(int jp, int rows1_max, int rows2_max, int I3)
{
    return align16(sizeof(float) * (size_t)loss_lds_layout(jp, rows1_max, rows2_max, I3).total);
}

template <int JP>
__global__ __launch_bounds__(256) void loss_blocks(LossArgs a)
{
    constexpr int RS = row_stride(JP);
    extern __shared__ float lds[];
    const LossLds L = loss_lds_layout(JP, a.rows1_max, a.rows2_max, a.I3);
    float* Ab = lds + L.a_off;
    float* Bb = lds + L.b_off;
    float* Hs = lds + L.h_off;
    double* red = reinterpret_cast<double*>(lds + L.red_off);
    const int tid = threadIdx.x;
    const int blk = blockIdx.x, p = blk / a.P, q = blk - p * a.P;
    const int J1 = a.J1, J2 = a.J2, J3 = a.J3;
    const int s1 = a.start1[p], r1 = a.start1[p + 1] - s1;
    const int s2 = a.start2[q], r2 = a.start2[q + 1] - s2;
    const int t0 = a.blk_tile[blk], t1 = a.blk_tile[blk + 1];
    double acc = 0.0;
    if (t0 < t1) {
        for (int idx = tid; idx < r1 * RS; idx += 256) {
            const int l = idx / RS, c = idx - l * RS;
            Ab[idx] = c < J1 ? a.A[(size_t)a.perm1[s1 + l] * J1 + c] : 0.f;
        }
        for (int idx = tid; idx < r2 * RS; idx += 256) {
            const int l = idx / RS, c = idx - l * RS;
            Bb[idx] = c < J2 ? a.B[(size_t)a.perm2[s2 + l] * J2 + c] : 0.f;
        }
        for (int idx = tid; idx < a.I3 * JP * JP; idx += 256) {
            const int k = idx / (JP * JP), xy = idx - k * JP * JP, x = xy / JP, y = xy - x * JP;
            float h = 0.f;
            if (x < J1 && y < J2)
                for (int c = 0; c < J3; ++c) h += a.G[(x * J2 + y) * J3 + c] * a.C[k * J3 + c];
            Hs[idx] = h;
        }
        __syncthreads();
        const uint32_t mask_i = (1u << a.bits_i) - 1u, mask_j = (1u << a.bits_j) - 1u;
        const int z0 = a.tile_off[t0], z1 = a.tile_off[t1];
        // tiles are platform-uniform; find each nonzero's platform by its tile
        int tl = t0;
        for (int z = z0 + tid; z < z1; z += 256) {
            while (a.tile_off[tl + 1] <= z) ++tl;
            const int k = a.tile_k[tl];
            const uint2 wv = a.nz[z];
            const int il = (int)(wv.x & mask_i), jl = (int)((wv.x >> a.bits_i) & mask_j);
            const float* H = Hs + k * JP * JP;
            float xt = 0.f;
#pragma unroll
            for (int x_ = 0; x_ < JP; ++x_) {
                float w1 = 0.f;
#pragma unroll
                for (int y = 0; y < JP; ++y) w1 = fmaf(H[x_ * JP + y], Bb[jl * RS + y], w1);
                xt = fmaf(Ab[il * RS + x_], w1, xt);
            }
            const float e = __uint_as_float(wv.y) - xt;
            acc += (double)e * (double)e;
        }
    }
    red[tid] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) a.partial[blk] = red[0];
}

__global__ __launch_bounds__(1024) void loss_final(LossArgs a)
{
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    const int nb = a.P * a.P;
    double sse = 0.0;
    for (int b = tid; b < nb; b += 1024) sse += a.partial[b];
    red[tid] = sse;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    sse = red[0];
    __syncthreads();
    // L2 term over the core and the observed rows
    double reg = 0.0;
    const int ng = a.J1 * a.J2 * a.J3;
    for (int q = tid; q < ng; q += 1024) reg += (double)a.G[q] * a.G[q];
    for (int r = tid; r < a.I1; r += 1024)
        if (a.cnt1[r] > 0)
            for (int c = 0; c < a.J1; ++c) reg += (double)a.A[(size_t)r * a.J1 + c] * a.A[(size_t)r * a.J1 + c];
    for (int r = tid; r < a.I2; r += 1024)
        if (a.cnt2[r] > 0)
            for (int c = 0; c < a.J2; ++c) reg += (double)a.B[(size_t)r * a.J2 + c] * a.B[(size_t)r * a.J2 + c];
    for (int r = tid; r < a.I3; r += 1024)
        if (a.cnt3[r] > 0)
            for (int c = 0; c < a.J3; ++c) reg += (double)a.C[(size_t)r * a.J3 + c] * a.C[(size_t)r * a.J3 + c];
    red[tid] = reg;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    reg = red[0];
    __syncthreads();
    // network term: each undirected pair appears twice in the symmetric CSR
    double net = 0.0;
    if (a.lam_g > 0.0) {
        for (int r = tid; r < a.I2; r += 1024)
            for (int e = a.adj_start[r]; e < a.adj_start[r + 1]; ++e) {
                const int v = a.adj_nbr[e];
                double d2 = 0.0;
                for (int c = 0; c < a.J2; ++c) {
                    const double d = (double)a.B[(size_t)r * a.J2 + c] - (double)a.B[(size_t)v * a.J2 + c];
                    d2 += d * d;
                }
                net += (double)a.adj_w[e] * d2;
            }
    }
    red[tid] = net;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    net = 0.5 * red[0];
    if (tid == 0) {
        a.out[0] = 0.5 * sse + 0.5 * a.lam * reg + 0.5 * a.lam_g * net;
        a.out[1] = sse;
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int JP>
static hipError_t launch_block_t(const BlockArgs& a, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL(block_fp32<JP>, dim3(a.P), dim3(64), lds, st, a);
    return hipGetLastError();
}

template <int JP>
static hipError_t launch_loss_t(const LossArgs& a, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL(loss_blocks<JP>, dim3(a.P * a.P), dim3(256), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(loss_final, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

#define SNECT_JP_SWITCH(JPV, CALL) \
    switch (JPV) {                 \
    case 2: return CALL(2);        \
    case 4: return CALL(4);        \
    case 5: return CALL(5);        \
    case 8: return CALL(8);        \
    case 10: return CALL(10);      \
    case 12: return CALL(12);      \
    case 16: return CALL(16);      \
    case 20: return CALL(20);      \
    case 24: return CALL(24);      \
    case 32: return CALL(32);      \
    default: return hipErrorInvalidValue; \
    }

hipError_t launch_block_fp32(const BlockArgs& a, int jp, size_t lds, hipStream_t st)
{
#define CALL_B(J) launch_block_t<J>(a, lds, st)
    SNECT_JP_SWITCH(jp, CALL_B)
#undef CALL_B
}

hipError_t launch_loss(const LossArgs& a, int jp, size_t lds, hipStream_t st)
{
#define CALL_L(J) launch_loss_t<J>(a, lds, st)
    SNECT_JP_SWITCH(jp, CALL_L)
#undef CALL_L
}

hipError_t launch_core_step(const CoreArgs& a, hipStream_t st)
{
    const int J12 = a.J1 * a.J2;
    const size_t lds = align16(sizeof(float) * (size_t)(((a.I3 * J12 + a.I3 * a.J3 + J12 * a.J3 + 1) & ~1) +
                                                      2 * a.I3));
    hipLaunchKernelGGL(core_step, dim3(1), dim3(1024), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_graph_step(const GraphArgs& a, hipStream_t st)
{
    const int n = a.I2 * a.J2;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(graph_step, dim3((n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int JP>
static hipError_t prepare_t(size_t block_lds, size_t loss_lds)
{
    hipError_t e = hipSuccess;
    if (block_lds > 65536)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&block_fp32<JP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)block_lds);
    if (e != hipSuccess) return e;
    if (loss_lds > 65536)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&loss_blocks<JP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)loss_lds);
    return e;
}

hipError_t prepare_kernels(int jp, size_t block_lds, size_t loss_lds)
{
#define CALL_P(J) prepare_t<J>(block_lds, loss_lds)
    SNECT_JP_SWITCH(jp, CALL_P)
#undef CALL_P
}

}  // namespace snect
