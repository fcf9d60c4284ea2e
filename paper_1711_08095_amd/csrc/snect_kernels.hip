// gfx950 kernels of the SNeCT stratified SGD (arXiv:1711.08095: Algorithm 1
// with the gradients of Eq. 5, the network term of Eq. 4, the objective of
// Eq. 3).
//
// Factor rows are kept in plan (position) order, so the rows of a block are
// one contiguous range.  A block (p, q) is processed by one workgroup of NW = 8
// wavefronts (two per SIMD): its patient rows and
// gene rows sit in LDS, H_k = G x3 c_k for every platform k is built in LDS
// from the stratum's frozen C and G, and each tile (<= 64 nonzeros of one
// platform) is one step in which lane t of every wavefront stands for
// nonzero t.  Factor column c has a patient task (w1_c = (H_k b_j)_c and the
// update of column c of a_i) and a gene task (w2_c = (H_k^T a_i)_c and the
// update of column c of b_j), spread over the wavefronts:
//   1. patient tasks read the tile's b rows, gene tasks its a rows, as they
//      were before the tile; each patient-task wavefront stages its share of
//      x~ = a_i . w1 (its columns, ascending);
//   2. after a barrier every lane adds the shares in wavefront order and
//      forms e = x - x~; a segmented wavefront scan then sums the terms
//      of every patient run (contiguous: tiles are sorted by i) and every
//      gene run (contiguous in the tile's gene-sorted slot order) in a fixed
//      tree order, and the last lane of a run writes the row's column;
//      patient tasks also stage the matrix-core operands of the block's sum
//      of e a (x) b, which four wavefronts accumulate at the start of the
//      next tile, each over a fixed quarter of the nonzeros;
//   3. a barrier ends the tile.
// Every sum runs in an order fixed by the problem alone (and the core size),
// so the execution choices never change a bit of the result.  Staging arrays are
// column-major with a pitch of 66 words, which keeps the column writes and
// the matrix-core operand reads free of bank conflicts; factor rows use an
// odd stride so that the rows gathered by one tile spread over the banks.
//
// Two drivers share that block step and all of the arithmetic:
//   strata_persistent: one cooperative launch per epoch; P workgroups stay
//     resident, workgroup q keeps gene block q in LDS for the whole epoch and
//     visits patient block (q - s) mod P in stratum s; the blocks' sums are
//     reduced by all workgroups (each its share), handed over in tagged
//     words that the readers poll, after which every workgroup applies the
//     same core step to its LDS copy of C and G;
//   block_step + core_step: one launch per stratum plus one for the core step
//     (used when the persistent kernel cannot be co-resident).
// Both give bit-identical results.
#include <hip/hip_runtime.h>

#include "snect_internal.h"

namespace snect {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kTS = 66;  // pitch (words) of a staged column
constexpr int kTW = 68;  // pitch (words) of a matrix-core output column (16-byte rows of 4)
constexpr int kTB = 72;  // pitch (bf16 values) of a staged BF16 operand column
constexpr int kKB = 32;  // K of the BF16 products (J padded to 32)

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

// Compiler-only ordering point: memory accesses are not moved across it
// (bounds how many LDS values the scheduler keeps in flight).
__device__ inline void lds_order_fence() { asm volatile("" ::: "memory"); }

// wg_count call sites (each with its own slots): chunk loads, the two polls,
// the reduction passes, the prefetched chunk's tile count
constexpr int kWgSites = 5;
enum { kWgChunk = 0, kWgPoll1 = 1, kWgPoll2 = 2, kWgReduce = 3, kWgPre = 4 };

// ---------------------------------------------------------------------------
// LDS carve-up of the stratum kernels (in 4-byte words).
// ---------------------------------------------------------------------------
struct StratLds {
    int a, b, ra, rb, c, g, h, ht, as, es, xtp, stg, sk, tco, tck, red, cst, cgt, sch, rec, wgs;
    int hb, sw1, sw2, xts, esl, a16, e16;  // BF16 path only (zero-sized otherwise)
    int total;
};

__host__ __device__ inline int up4(int o) { return (o + 3) & ~3; }

__host__ __device__ inline StratLds strat_lds_layout(int jp, int P, int rows1_max, int rows2_max, int I3, int J1,
                                                     int J2, int J3, int rec_cap, int bf, int nw)
{
    const int rs = strat_row_stride(jp, bf), mp = mfma_dim(jp), j12 = J1 * J2;
    StratLds L;
    int o = 0;
    L.a = o;     o = up4(o + rows1_max * rs);
    L.b = o;     o = up4(o + rows2_max * rs);
    L.ra = o;    o = up4(o + rows1_max);
    L.rb = o;    o = up4(o + rows2_max);
    L.c = o;     o = up4(o + I3 * J3);
    L.g = o;     o = up4(o + j12 * J3);
    const int f32 = bf ? 0 : 1;
    L.h = o;     o = up4(o + f32 * I3 * jp * jp);        // FP32 H_k (FP32 path)
    const int tr = (!bf && jp > 12) ? 1 : 0;
    L.ht = o;    o = up4(o + tr * I3 * jp * jp);         // H_k^T (FP32 path, JP > 12)
    L.as = o;    o = up4(o + f32 * mp * kTS);
    L.es = o;    o = up4(o + f32 * mp * kTS);
    L.xtp = o;   o = up4(o + f32 * nw * kTileMax);          // each patient-task wavefront's share of x~
    L.hb = o;    o = up4(o + bf * I3 * mp * kKB);        // 2 x I3 x mp x 32 bf16
    L.sw1 = o;   o = up4(o + bf * mp * kTW);
    L.sw2 = o;   o = up4(o + bf * mp * kTW);
    L.xts = o;   o = up4(o + bf * kTileMax);
    L.esl = o;   o = up4(o + bf * kTileMax);
    L.a16 = o;   o = up4(o + bf * mp * kTB / 2);
    L.e16 = o;   o = up4(o + bf * mp * kTB / 2);
    L.stg = o;   o = up4(o + kMfmaWaves * j12);
    L.sk = o;    o = up4(o + I3 * j12);
    L.tco = o;   o = up4(o + kTileCache + 1);
    L.tck = o;   o = up4(o + kTileCache);
    L.red = o;   o = up4(o + 64 * nw);
    L.cst = o;   o = up4(o + kCstHead + I3);        // core-step constants of the stratum
    L.cgt = o;   o = up4(o + I3 * J3 + j12 * J3);
    L.sch = o;   o = up4(o + 7 * P);                // the epoch's schedule of this workgroup
    L.rec = o;   o = up4(o + 2 * rec_cap);
    L.wgs = o;   o = up4(o + kWgSites * kDefaultWaves);  // slots of wg_count
    L.total = o;
    return L;
}

size_t strata_lds_bytes(int jp, int P, int rows1_max, int rows2_max, int I3, int J1, int J2, int J3, int rec_cap,
                        int bf, int nw)
{
    return align16(4 * (size_t)strat_lds_layout(jp, P, rows1_max, rows2_max, I3, J1, J2, J3, rec_cap, bf, nw).total);
}

int jp_for(int J1, int J2)
{
    const int m = J1 > J2 ? J1 : J2;
    for (int t = 0; t < kJpCount; ++t)
        if (kJpSet[t] >= m) return kJpSet[t];
    return -1;
}

// ---------------------------------------------------------------------------
// Shared arithmetic (identical instruction sequence in every driver)
// ---------------------------------------------------------------------------

// H_k[x][y] = sum_c G[x,y,c] C[k,c], zero padded to JP x JP, into any of:
// Hs (FP32, row x), Ht (FP32 H_k^T, row y) and Hb, the BF16 B operands of
// the matrix-core products W1 = B_tile H_k^T and W2 = A_tile H_k: for
// platform k, Hb[(2k)(MP)(32)] holds H_k[c][y] at (c, y) and
// Hb[(2k+1)(MP)(32)] holds H_k[x][c] at (c, x) (row c is read as 8 values
// per lane).  Hb's entries beyond JP (in c or in the other index) are never
// written here: clear_hb_pad zeroes them once.
template <int JP>
__device__ void build_h(float* Hs, const float* Cs, const float* Gs, int I3, int J1, int J2, int J3, int tid,
                        int nthr, float* Ht = nullptr, __bf16* Hb = nullptr)
{
    constexpr int MP = mfma_dim(JP);
    for (int idx = tid; idx < I3 * JP * JP; idx += nthr) {
        const int k = idx / (JP * JP), xy = idx - k * JP * JP, x = xy / JP, y = xy - x * JP;
        float h = 0.f;
        if (x < J1 && y < J2)
            for (int c = 0; c < J3; ++c) h = fmaf(Gs[(x * J2 + y) * J3 + c], Cs[k * J3 + c], h);
        if (Hs) Hs[idx] = h;
        if (Ht) Ht[(k * JP + y) * JP + x] = h;  // H_k^T, row y
        if (Hb) {
            Hb[((2 * k) * MP + x) * kKB + y] = (__bf16)h;
            Hb[((2 * k + 1) * MP + y) * kKB + x] = (__bf16)h;
        }
    }
}

// Zeroes the entries of the BF16 operands Hb (see build_h) that lie beyond
// JP in either index.
template <int JP>
__device__ void clear_hb_pad(__bf16* Hb, int I3, int tid, int nthr)
{
    constexpr int MP = mfma_dim(JP);
    if constexpr (MP > JP || kKB > JP) {
        for (int idx = tid; idx < I3 * 2 * MP * kKB; idx += nthr) {
            const int y = idx % kKB, c = (idx / kKB) % MP;
            if (c >= JP || y >= JP) Hb[idx] = (__bf16)0.f;
        }
    }
}

// Device-coherent accesses, for data that other workgroups of the same
// launch write or read: agent-scope relaxed atomics, which bypass the
// non-coherent L2 of the accessing XCD (global_load / global_store with sc1).
// With them the persistent kernel's exchanges need no L2 writeback or
// invalidation.
__device__ inline float ld_coh(const float* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void st_coh(float* p, float v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Waits until this wavefront's stores have been performed (s_waitcnt
// vmcnt(0), the other counters left alone; gfx9 encoding); memory accesses
// are not moved across it.
__device__ inline void coh_stores_done()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Stratum sum of one item of S over the blocks: chunks of kRedChunk
// consecutive blocks are summed in ascending order, then the chunk sums in
// ascending order.  The partial sums are read device-coherently.
__device__ inline float chunk_sum(const float* Spart, int ni, int item, int p0, int p1)
{
    float v[kRedChunk];
#pragma unroll
    for (int u = 0; u < kRedChunk; ++u) v[u] = p0 + u < p1 ? ld_coh(Spart + (size_t)(p0 + u) * ni + item) : 0.f;
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < kRedChunk; ++u) s += v[u];
    return s;
}

// Sums items [i0, i1) of the stratum into dst[item - i0] using the whole
// workgroup (red: nthr floats of LDS).
__device__ void reduce_items(const float* Spart, int P, int ni, int i0, int i1, float* dst, float* red, int tid,
                             int nthr)
{
    const int nch = (P + kRedChunk - 1) / kRedChunk;
    const int per_pass = nthr / nch > 0 ? nthr / nch : 1;
    for (int base = i0; base < i1; base += per_pass) {
        const int items = (i1 - base) < per_pass ? (i1 - base) : per_pass;
        __syncthreads();
        if (tid < items * nch) {
            const int it = tid / nch, ch = tid - it * nch;
            const int p0 = ch * kRedChunk, p1 = (p0 + kRedChunk) < P ? (p0 + kRedChunk) : P;
            red[tid] = chunk_sum(Spart, ni, base + it, p0, p1);
        }
        __syncthreads();
        if (tid < items) {
            float s = 0.f;
            for (int ch = 0; ch < nch; ++ch) s += red[tid * nch + ch];
            dst[base + tid - i0] = s;
        }
    }
    __syncthreads();
}

// Sum over the 16 lanes of each row, returned in every lane of the row.
__device__ inline float row_sum16(float v);

// Core / platform-factor step from the stratum sums S (I3 x J1J2) with the
// stratum's constants cst (kCstHead + I3 values, see kCstHead): one
// mean-gradient step of size etac,
//   C[k][c] -= etac/m (-sum_ab G0[ab][c] S_k[ab] + lam m_k/n3[k] C0[k][c])
//   G[ab][c] -= etac/m (-sum_k S_k[ab] C0[k][c] + lam m/nnz G0[ab][c]).
// The C sum of item (k, c) runs on one 16-lane row of a wavefront: lane g
// adds ab = g, g + 16, ... in ascending order, then the 16 lanes are added by
// a fixed rotation tree.  The G sums run over ascending k.  New C goes to
// newC, new G to newG (neither may alias C0 / G0); the caller synchronises
// afterwards.  Every thread of the workgroup calls it (nthr a multiple of 64).
__device__ void core_update(const float* C0, const float* G0, const float* S, const float* cst, int I3, int J12,
                            int J3, float etac, float* newC, float* newG, int tid, int nthr)
{
    const int nc = I3 * J3;
    if (cst[0] == 0.f) {  // no nonzero in this stratum
        for (int idx = tid; idx < nc; idx += nthr) newC[idx] = C0[idx];
        for (int idx = tid; idx < J12 * J3; idx += nthr) newG[idx] = G0[idx];
        return;
    }
    const float inv_m = cst[1], greg = cst[2];
    const int g16 = tid & 15, rows = nthr >> 4;
    for (int base = 0; base < nc; base += rows) {
        const int item = base + (tid >> 4);
        float v = 0.f;
        if (item < nc) {
            const int k = item / J3, c = item - k * J3;
#pragma unroll 8
            for (int ab = g16; ab < J12; ab += 16) v = fmaf(-G0[ab * J3 + c], S[k * J12 + ab], v);
        }
        v = row_sum16(v);
        if (item < nc && g16 == 0) {
            const float cr = cst[kCstHead + item / J3];
            const float g = cr != 0.f ? fmaf(cr, C0[item], v) : v;
            newC[item] = fmaf(-etac, g * inv_m, C0[item]);
        }
    }
    for (int idx = tid; idx < J12 * J3; idx += nthr) {
        const int ab = idx / J3, c = idx - ab * J3;
        float g = 0.f;
#pragma unroll 8
        for (int k = 0; k < I3; ++k) g = fmaf(-S[k * J12 + ab], C0[k * J3 + c], g);
        g = fmaf(greg, G0[idx], g);
        newG[idx] = fmaf(-etac, g * inv_m, G0[idx]);
    }
}

// MFMA accumulator of the per-platform S = sum_t e_t a_t (x) b_t.  Staged
// operands are column-major, element (t, c) at c*kTS + t.
template <int MP> struct SAcc;

template <> struct SAcc<16> {
    floatx4 v;
    __device__ void zero() { v = floatx4{0.f, 0.f, 0.f, 0.f}; }
    // v_mfma_f32_16x16x4f32: step s covers nonzeros 4s..4s+3; lane l supplies
    // A[l%16][l/16] = a_{4s+l/16}[l%16] and B[l/16][l%16] = (e b)_{4s+l/16}[l%16].
    // Matrix-core wavefront w (0..3) takes nonzeros 16w..16w+15, i.e. steps
    // 4w..4w+3, all four (operands past the tile's end are zero); the eight
    // operand reads go out before the first product.
    __device__ void accumulate_all(const float* As, const float* Es, int w, int lane)
    {
        const int col = (lane & 15) * kTS + (lane >> 4) + 16 * w;
        float x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x[u] = As[col + 4 * u];
            y[u] = Es[col + 4 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) v = __builtin_amdgcn_mfma_f32_16x16x4f32(x[u], y[u], v, 0, 0, 0);
    }
    // output element (row 4*(l/16)+r, column l%16) sits in register r of lane l
    __device__ void store(float* St, int J1, int J2, int lane)
    {
        const int col = lane & 15, rb = (lane >> 4) * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rb + r;
            if (row < J1 && col < J2) St[row * J2 + col] = v[r];
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
    // v_mfma_f32_32x32x2f32: step s covers nonzeros 2s, 2s+1; lane l supplies
    // a_{2s+l/32}[l%32] and (e b)_{2s+l/32}[l%32].  Matrix-core wavefront w takes steps
    // 8w..8w+7, all eight (operands past the tile's end are zero).
    __device__ void accumulate_all(const float* As, const float* Es, int w, int lane)
    {
        const int col = (lane & 31) * kTS + (lane >> 5) + 16 * w;
        float x[8], y[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            x[u] = As[col + 2 * u];
            y[u] = Es[col + 2 * u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v = __builtin_amdgcn_mfma_f32_32x32x2f32(x[u], y[u], v, 0, 0, 0);
    }
    // output element (row 8*(r/4) + 4*(l/32) + r%4, column l%32) in register r
    __device__ void store(float* St, int J1, int J2, int lane)
    {
        const int col = lane & 31, rb = (lane >> 5) * 4;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = (r >> 2) * 8 + rb + (r & 3);
            if (row < J1 && col < J2) St[row * J2 + col] = v[r];
        }
    }
};

// BF16 matrix-core accumulator of S (v_mfma_f32_16x16x32_bf16): the
// operands are staged column-major, element (t, c) at c*kTB + t, and lane l
// supplies rows/columns l%16 with nonzeros 8(l/16) .. 8(l/16)+7 of a 32-wide
// K step.  MP = 32: matrix-core wavefront w (0..3) owns output block
// (w/2, w%2) and both K steps; MP = 16: matrix-core wavefronts 0 and 1 own
// K step 0 and 1 of the one block.
template <int MP> struct SAccB {
    floatx4 v;
    __device__ void zero() { v = floatx4{0.f, 0.f, 0.f, 0.f}; }
    __device__ void accumulate(const __bf16* A16, const __bf16* E16, int n, int w, int lane)
    {
        const int g = lane >> 4, m = lane & 15;
        const int mb = MP == 32 ? (w >> 1) : 0, nb = MP == 32 ? (w & 1) : 0;
        const int ks0 = MP == 32 ? 0 : w, ks1 = MP == 32 ? 2 : (w < 2 ? w + 1 : w);
        for (int ks = ks0; ks < ks1; ++ks) {
            if (kKB * ks >= n) break;
            const bf16x8 x = *reinterpret_cast<const bf16x8*>(A16 + (mb * 16 + m) * kTB + kKB * ks + 8 * g);
            const bf16x8 y = *reinterpret_cast<const bf16x8*>(E16 + (nb * 16 + m) * kTB + kKB * ks + 8 * g);
            v = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, v, 0, 0, 0);
        }
    }
    // output element (row mb*16 + 4*(l/16) + r, column nb*16 + l%16) in register r
    __device__ void store(float* St, int J1, int J2, int w, int lane)
    {
        const int mb = MP == 32 ? (w >> 1) : 0, nb = MP == 32 ? (w & 1) : 0;
        const int col = nb * 16 + (lane & 15), rb = mb * 16 + (lane >> 4) * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rb + r;
            if (row < J1 && col < J2) St[row * J2 + col] = v[r];
        }
    }
};

// Eight consecutive columns [c0, c0+8) of an LDS row (stride RS, a multiple
// of 4) as BF16; columns at or beyond RS read as zero.
template <int RS>
__device__ inline bf16x8 row8_bf16(const float* row, int c0, bool act)
{
    floatx4 lo = floatx4{0.f, 0.f, 0.f, 0.f}, hi = lo;
    if (act && c0 < RS) lo = *reinterpret_cast<const floatx4*>(row + c0);
    if (act && c0 + 4 < RS) hi = *reinterpret_cast<const floatx4*>(row + c0 + 4);
    bf16x8 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        r[i] = (__bf16)lo[i];
        r[4 + i] = (__bf16)hi[i];
    }
    return r;
}

// Contiguous rows [row0, row0+nrows) of a position-ordered factor into LDS
// rows of stride RS (padding columns are left as they are: zero).
__device__ inline void load_rows(float* dst, const float* src, int row0, int nrows, int J, int RS, int tid,
                                 int nthr)
{
    constexpr int U = 8;  // loads in flight per thread
    const float* s = src + (size_t)row0 * J;
    const int total = nrows * J;
    for (int base = tid; base < total; base += U * nthr) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * nthr;
            v[u] = idx < total ? s[idx] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * nthr;
            if (idx < total) {
                const int l = idx / J, c = idx - l * J;
                dst[l * RS + c] = v[u];
            }
        }
    }
}

__device__ inline void store_rows(float* dst, const float* src, int row0, int nrows, int J, int RS, int tid,
                                  int nthr)
{
    float* d = dst + (size_t)row0 * J;
    for (int idx = tid; idx < nrows * J; idx += nthr) {
        const int l = idx / J, c = idx - l * J;
        d[idx] = src[l * RS + c];
    }
}

// Tile metadata of tiles [base, base + kTileCache) (offsets one further).
__device__ inline void load_tile_cache(const StratArgs& a, int* tco, int* tck, int base, int t1, int tid,
                                       int nthr)
{
    for (int u = tid; u < kTileCache + 1; u += nthr) {
        const int t = base + u;
        tco[u] = t <= t1 ? a.tile_off[t] : 0;
        if (u < kTileCache) tck[u] = t < t1 ? a.tile_k[t] : 0;
    }
}

// n consecutive records into LDS, eight loads in flight per thread.
__device__ inline void load_records(uint2* dst, const uint2* src, int n, int tid, int nthr)
{
    constexpr int U = 8;
    for (int b = tid; b < n; b += U * nthr) {
        uint2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = b + u * nthr;
            v[u] = src[i < n ? i : n - 1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = b + u * nthr;
            if (i < n) dst[i] = v[u];
        }
    }
}

// Cross-lane moves on the VALU (DPP), no LDS round trip.
template <int CTRL, int ROWS>
__device__ inline float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, true));
}
template <int CTRL>
__device__ inline int dpp_move_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}
constexpr int kDppRowShr = 0x110;   // + n: lane l of a 16-lane row reads lane l-n of the row
constexpr int kDppRowBcast15 = 0x142;  // lane 15 of each row to the next row
constexpr int kDppRowBcast31 = 0x143;  // lane 31 to rows 2 and 3
constexpr int kDppWaveShr1 = 0x138;    // lane l reads lane l-1
constexpr int kDppWaveShl1 = 0x130;    // lane l reads lane l+1
constexpr int kDppRowRor = 0x120;      // + n: lane l of a row reads lane (l+n) mod 16 of the row

// Sum over the 16 lanes of each row, returned in every lane of the row.
__device__ inline float row_sum16(float v)
{
    v += dpp_move<kDppRowRor + 8, 0xf>(v);
    v += dpp_move<kDppRowRor + 4, 0xf>(v);
    v += dpp_move<kDppRowRor + 2, 0xf>(v);
    v += dpp_move<kDppRowRor + 1, 0xf>(v);
    return v;
}

// Inclusive segmented scan over the lanes of a wavefront: lane l returns the
// sum of v over lanes head..l (head <= l), added in a fixed tree order:
// Hillis-Steele steps of 1, 2, 4, 8 inside each 16-lane row, then the row
// totals carried across rows.
__device__ inline float seg_scan(float v, int lane, int head)
{
    const int r = lane & 15, row = lane >> 4;
    float t;
    t = dpp_move<kDppRowShr + 1, 0xf>(v);
    if (r >= 1 && lane - 1 >= head) v += t;
    t = dpp_move<kDppRowShr + 2, 0xf>(v);
    if (r >= 2 && lane - 2 >= head) v += t;
    t = dpp_move<kDppRowShr + 4, 0xf>(v);
    if (r >= 4 && lane - 4 >= head) v += t;
    t = dpp_move<kDppRowShr + 8, 0xf>(v);
    if (r >= 8 && lane - 8 >= head) v += t;
    // the row broadcasts write every row (lanes without a source read 0); the
    // conditions keep the add to rows 1 and 3, and to rows 2 and 3
    t = dpp_move<kDppRowBcast15, 0xf>(v);
    if ((row & 1) && head <= 16 * row - 1) v += t;
    t = dpp_move<kDppRowBcast31, 0xf>(v);
    if (row >= 2 && head <= 31) v += t;
    return v;
}

// seg_scan of N columns at once, step by step (the same additions in the
// same order for each column as seg_scan; independent steps interleave).
template <int N>
__device__ inline void seg_scan_n(float (&v)[N], int lane, int head)
{
    const int r = lane & 15, row = lane >> 4;
    float t[N];
#pragma unroll
    for (int q = 0; q < N; ++q) t[q] = dpp_move<kDppRowShr + 1, 0xf>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q)
        if (r >= 1 && lane - 1 >= head) v[q] += t[q];
#pragma unroll
    for (int q = 0; q < N; ++q) t[q] = dpp_move<kDppRowShr + 2, 0xf>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q)
        if (r >= 2 && lane - 2 >= head) v[q] += t[q];
#pragma unroll
    for (int q = 0; q < N; ++q) t[q] = dpp_move<kDppRowShr + 4, 0xf>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q)
        if (r >= 4 && lane - 4 >= head) v[q] += t[q];
#pragma unroll
    for (int q = 0; q < N; ++q) t[q] = dpp_move<kDppRowShr + 8, 0xf>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q)
        if (r >= 8 && lane - 8 >= head) v[q] += t[q];
#pragma unroll
    for (int q = 0; q < N; ++q) t[q] = dpp_move<kDppRowBcast15, 0xf>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q)
        if ((row & 1) && head <= 16 * row - 1) v[q] += t[q];
#pragma unroll
    for (int q = 0; q < N; ++q) t[q] = dpp_move<kDppRowBcast31, 0xf>(v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q)
        if (row >= 2 && head <= 31) v[q] += t[q];
}

// Lanes 0..lane as a bit mask (computed once per thread).
__device__ inline unsigned long long lanes_upto(int lane) { return lane == 63 ? ~0ull : (2ull << lane) - 1ull; }

// Position of the highest set bit of `heads` among the bits of `upto`
// (lanes_upto of the calling lane).
__device__ inline int run_head(unsigned long long heads, unsigned long long upto)
{
    const unsigned long long m = heads & upto;
    return m ? 63 - __clzll(m) : 0;
}

struct TileLds {
    float *Ab, *Bb;
    const float *rA, *rB, *Hs, *Ht;
    float *As, *Es, *xtp;
    // BF16 path: H_k and H_k^T as matrix-core B operands, raw w1 (tile order)
    // and w2 (slot order) columns, x~ per nonzero, e in slot order, staged
    // BF16 operands of the S product
    const __bf16* Hb;
    float *sW1, *sW2, *xts, *eS;
    __bf16 *A16, *E16;
    float* Sk;    // [I3*J1*J2] the block's sums of e a (x) b
    float* St;    // [kMfmaWaves][J1*J2] staged partial sums of one platform
    int *tco, *tck;
    uint2* rec;   // [rec_cap] staged records
    int* wgs;     // [kWgSites][kDefaultWaves] slots of wg_count
};

// Number of threads of the workgroup (NW wavefronts) whose pred holds, in
// every thread: one workgroup barrier; each wavefront posts the population
// count of its ballot to its own word of slots[NW].  Every call site has its
// own slots, and a workgroup barrier separates the reads of one call from
// the writes of the next at the same site.
template <int NW>
__device__ inline int wg_count(bool pred, int* slots)
{
    const unsigned long long b = __ballot(pred);
    if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    int n = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) n += slots[w];
    return n;
}

// Tile metadata and records of the chunk of tiles starting at `base` (up to
// kTileCache tiles whose records fit in rec_cap) into LDS; returns the
// chunk's tile count.  Every thread of the workgroup calls it.
__device__ inline int load_chunk(const StratArgs& a, const TileLds& L, int base, int t1, int tid, int nthr)
{
    load_tile_cache(a, L.tco, L.tck, base, t1, tid, nthr);
    __syncthreads();
    const int ntc = (t1 - base) < kTileCache ? (t1 - base) : kTileCache;
    const int cend =
        wg_count<kDefaultWaves>(tid < ntc && L.tco[tid + 1] - L.tco[0] <= a.rec_cap, L.wgs + kWgChunk * kDefaultWaves);
    const int z0 = L.tco[0], nrec = L.tco[cend] - z0;
    load_records(L.rec, a.nz + z0, nrec, tid, nthr);
    __syncthreads();
    return cend;
}

// The block's S of one platform is staged: each matrix-core wavefront
// stores its partial sums (St, kMfmaWaves x J1J2), and after the next
// workgroup barrier every thread adds them up, wavefront 0 first, so the
// block's sum is ((S_0 + S_1) + S_2) + S_3 whatever the timing.  covers()
// names the wavefronts that produce entry (row, col): all four in the FP32
// step (each over a quarter of the nonzeros); in the BF16 step the owner of
// the entry's 16x16 block (MP = 32) or wavefronts 0 and 1 (MP = 16).
template <bool BF, int MP>
__device__ inline bool covers(int w, int row, int col)
{
    if (!BF) return true;
    if (MP == 32) return w == 2 * (row >> 4) + (col >> 4);
    return w < 2;
}

template <bool BF, int MP>
__device__ inline void stage_sum(const float* St, float* Skk, int J1, int J2, int tid, int nthr)
{
    const int J12 = J1 * J2;
    for (int e = tid; e < J12; e += nthr) {
        const int row = e / J2, col = e - row * J2;
        float sum = 0.f;
#pragma unroll
        for (int ww = 0; ww < kMfmaWaves; ++ww)
            if (covers<BF, MP>(ww, row, col)) sum += St[ww * J12 + e];
        Skk[e] = sum;
    }
}

// Work split of a tile's factor columns between the NW wavefronts.  Column
// c has a patient task (w1_c, its share a_c w1_c of x~, the S operands of
// column c and the patient-run sums of e w1_c) and a gene task (w2_c and the
// gene-run sums of e w2_c through the slot-ordered buffer); the two cost
// about the same.  For cores up to JP = 20 wavefronts [0, NJ) take the
// gene tasks and [NJ, NW) the patient tasks, each kind round robin, NJ
// minimising the largest load, so a wavefront reads only one of the two
// rows.  Larger cores keep both tasks of column c on wavefront c mod NW
// (fewer registers per wavefront).  The four wavefronts with the fewest
// tasks (the lower index first among equals) accumulate S.
template <int JP, int NW> struct TileSplit {
    static constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }
    static constexpr int cost(int nj)
    {
        return cdiv(JP, NW - nj) > cdiv(JP, nj) ? cdiv(JP, NW - nj) : cdiv(JP, nj);
    }
    static constexpr int pick()
    {
        int b = 1;
        for (int nj = 2; nj < NW; ++nj)
            if (cost(nj) < cost(b)) b = nj;
        return b;
    }
    static constexpr bool kSplit = JP <= 20;
    static constexpr int NJ = kSplit ? pick() : NW;  // gene-task wavefronts [0, NJ)
    static constexpr int OI = kSplit ? NJ : 0;       // patient-task wavefronts [OI, OI + NI)
    static constexpr int NI = NW - OI;
    static constexpr int QI = cdiv(JP, NI), QJ = cdiv(JP, NJ), QH = QI > QJ ? QI : QJ;
    // tasks of wavefront w
    static constexpr int tasks(int w)
    {
        const int tj = w < NJ ? cdiv(JP - w, NJ) : 0;
        const int ti = w >= OI ? cdiv(JP - (w - OI), NI) : 0;
        return (tj > 0 ? tj : 0) + (ti > 0 ? ti : 0);
    }
    // rank of wavefront w among the matrix-core wavefronts, or -1
    static constexpr int mfma_rank(int w)
    {
        int r = 0;
        for (int v = 0; v < NW; ++v)
            if (tasks(v) < tasks(w) || (tasks(v) == tasks(w) && v < w)) ++r;
        return r < kMfmaWaves ? r : -1;
    }
};

// The tiles [t0, t1) of one block, run by the whole workgroup (NW wavefronts).
// L.Ab/L.Bb hold the block's rows; L.Sk (zeroed by the caller) receives
// the block's per-platform sums through the staged partials of the four
// matrix-core wavefronts.  Every sum is taken in a fixed order (x~ over the
// patient-task wavefronts' shares, S over four fixed nonzero ranges).
//
// Two workgroup barriers per tile:
//   1. patient tasks read the tile's b rows and form w1_c and their share of
//      x~ (to LDS); gene tasks read the a rows and form w2_c (all values
//      from before the tile);
//   -- barrier --
//   2. every wavefront adds the shares of x~ and forms e; patient
//      tasks stage the S operands and sum their runs of e w1_c in
//      registers; gene tasks push e w2_c to slot order within the
//      wavefront (ds_permute) and sum their runs there; the last lane of a
//      run writes the row;
//   -- barrier --
// The matrix-core wavefronts add a tile's S operands at the start of the
// next tile, so the product overlaps the next tile's row
// reads.  Products are not contracted into fused multiply-adds beyond the
// explicit fmaf.
template <int JP, int NW>
__device__ void block_tiles(const StratArgs& a, int t0, int t1, const TileLds& L, int tid, int pre_cend)
{
#pragma clang fp contract(off)
    using SP = TileSplit<JP, NW>;
    constexpr int NJ = SP::NJ, NI = SP::NI, OI = SP::OI, QI = SP::QI, QJ = SP::QJ, QH = SP::QH;
    constexpr int RS = strat_row_stride(JP, 0);
    constexpr int MP = mfma_dim(JP);
    constexpr int NT = 64 * NW;
    const int lane = tid & 63, w = tid >> 6;
    const unsigned long long upto = lanes_upto(lane);
    const bool hj = w < NJ, hi = w >= OI;  // has gene tasks / patient tasks
    const int rj = w, ri = w - OI;         // columns rj + NJ q, ri + NI q
    const int J1 = a.J1, J2 = a.J2, J12 = J1 * J2;
    const uint32_t mask_i = (1u << a.bits_i) - 1u, mask_j = (1u << a.bits_j) - 1u;
    const int sh_j = a.bits_i, sh_r = a.bits_i + a.bits_j;
    if (t0 >= t1) return;

    // operand columns beyond the factor columns stay zero
    for (int idx = tid; idx < (MP - JP) * kTS; idx += NT) {
        L.As[JP * kTS + idx] = 0.f;
        L.Es[JP * kTS + idx] = 0.f;
    }

    SAcc<MP> acc;
    acc.zero();
    const int mw = SP::mfma_rank(w);  // matrix-core wavefronts: mw = 0..3
    const bool mfw = mw >= 0;
    int curk = -1;   // platform of the tiles whose operands acc holds
    int pend = -1;   // platform whose partial S waits in L.St
    int prev = 0;    // a tile's S operands wait in L.As/L.Es
    // small cores (JP <= 12, one task kind per wavefront): the wavefront's
    // rows (patient tasks) or columns (gene tasks) of H_k stay in registers
    // while consecutive tiles share k; larger ones read H_k and H_k^T from LDS
    constexpr bool kHreg = SP::kSplit && JP <= 12;
    // small cores request every LDS value of a task before its first
    // product; larger ones keep fewer values in flight
    constexpr bool kHoist = kHreg;
    float hh[kHreg ? QH : 1][kHreg ? JP : 1];
    int tl = t0;
    while (tl < t1) {
        // a chunk: up to kTileCache tiles whose records fit in rec_cap,
        // metadata and records brought into LDS with many loads in flight
        // (the first chunk may already be there: pre_cend tiles)
        const int cend = (pre_cend > 0 && tl == t0) ? pre_cend : load_chunk(a, L, tl, t1, tid, NT);
        const int z0 = L.tco[0];
        // each tile's records, size and platform are read from LDS during
        // the previous tile
        int n_next = L.tco[1] - z0, k_next = L.tck[0];
        uint2 wv_next = lane < n_next ? L.rec[lane] : make_uint2(0u, 0u);
        for (int u = 0; u < cend; ++u, ++tl) {
        const int n = n_next;
        const int k = k_next;
        const uint2 wv = wv_next;
        // S of the previous tile (its platform is curk); staged operands of
        // nonzeros past the tile's end are zero
        if (mfw && prev) acc.accumulate_all(L.As, L.Es, mw, lane);
        if (k != curk) {
            if (curk >= 0) {
                if (mfw) acc.store(L.St + mw * J12, J1, J2, lane);
                pend = curk;
            }
            acc.zero();
            curk = k;
            if constexpr (kHreg) {
                const float* Hk = L.Hs + k * JP * JP;
#pragma unroll
                for (int qq = 0; qq < QH; ++qq) {
                    const int c0 = hj ? rj + NJ * qq : ri + NI * qq;
                    const int c = c0 < JP ? c0 : 0;
#pragma unroll
                    for (int y = 0; y < JP; ++y) hh[qq][y] = hj ? Hk[y * JP + c] : Hk[c * JP + y];
                }
            }
        }
        const bool act = lane < n;
        const uint32_t wd = wv.x;
        const float x = __uint_as_float(wv.y);
        // lanes past the tile's end: patient -1 for the run logic, row 0 for
        // reads (their values are never used: e = 0 there)
        const int il = act ? (int)(wd & mask_i) : -1;
        const int ilc = act ? (int)(wd & mask_i) : 0;
        const int jl = act ? (int)((wd >> sh_j) & mask_j) : 0;
        const int jrank = (int)(wd >> sh_r);

        // 1. the rows from before the tile: b_j for patient tasks
        //    (w1 = H_k b), a_i for gene tasks (w2 = H_k^T a)
        const float* H = L.Hs + k * JP * JP;
        float w1q[QI], aq[QI], bq[QI], w2q[QJ];
        float rai = 0.f;  // regularisation weight of the nonzero's patient row
        if (hi) {
            float xp = 0.f;  // this wavefront's share of x~: its columns, ascending
            // every LDS value of the task is requested before the first
            // product (columns past the core read column JP - 1, unused;
            // lanes past the tile's end read row 0, unused)
            float bv[JP], ar[QI], br[QI];
#pragma unroll
            for (int c = 0; c < JP; ++c) bv[c] = L.Bb[jl * RS + c];
            if constexpr (kHoist) {
#pragma unroll
                for (int qq = 0; qq < QI; ++qq) {
                    const int c = ri + NI * qq, cc = c < JP ? c : JP - 1;
                    ar[qq] = L.Ab[ilc * RS + cc];
                    br[qq] = L.Bb[jl * RS + cc];
                }
                rai = L.rA[ilc];
            }
#pragma unroll
            for (int qq = 0; qq < QI; ++qq) {
                const int c = ri + NI * qq;
                float t = 0.f, ac = 0.f, bc = 0.f;
                if (c < JP) {
                    if constexpr (kHreg) {
#pragma unroll
                        for (int y = 0; y < JP; ++y) t = fmaf(hh[qq][y], bv[y], t);
                    } else {
                        // row c of H_k, four values per read
                        const floatx4* H4 = reinterpret_cast<const floatx4*>(H + c * JP);
#pragma unroll
                        for (int y4 = 0; y4 < JP / 4; ++y4) {
                            const floatx4 h4 = H4[y4];
#pragma unroll
                            for (int r = 0; r < 4; ++r) t = fmaf(h4[r], bv[4 * y4 + r], t);
                        }
                    }
                    if constexpr (kHoist) {
                        ac = act ? ar[qq] : 0.f;
                        bc = act ? br[qq] : 0.f;
                    } else {
                        ac = act ? L.Ab[ilc * RS + c] : 0.f;
                        bc = act ? L.Bb[jl * RS + c] : 0.f;
                    }
                    xp = qq == 0 ? ac * t : fmaf(ac, t, xp);
                }
                w1q[qq] = t;
                aq[qq] = ac;
                bq[qq] = bc;
                if constexpr (JP > 16) lds_order_fence();
            }
            L.xtp[ri * kTileMax + lane] = xp;
        }
        // gene runs, in the tile's gene-sorted slot order: slot s learns its
        // gene row from the lane that holds it (inactive lanes push to their
        // own slot, so the 64 pushes form a permutation), then the run heads,
        // the regularisation weights and the rows' values before the tile
        const int jr = act ? jrank : lane;
        int sj = -1, jhead = 0;
        bool jlast = false;
        float jcr = 0.f, bp[QJ];
        if (hj) {
            float av[JP];
            if constexpr (kHoist) {
#pragma unroll
                for (int c = 0; c < JP; ++c) av[c] = L.Ab[ilc * RS + c];
            }
            sj = __builtin_amdgcn_ds_permute(jr << 2, act ? jl : -1);
            const bool sact = lane < n;
            const int sjc = sact ? sj : 0;
            const float rbj = L.rB[sjc];
#pragma unroll
            for (int qq = 0; qq < QJ; ++qq) {
                const int c = rj + NJ * qq, cc = c < JP ? c : JP - 1;
                bp[qq] = L.Bb[sjc * RS + cc];
            }
            if constexpr (!kHoist) {
                // the slot work first (fewer values live across the products)
                const int sj_up = dpp_move_i<kDppWaveShr1>(sj), sj_dn = dpp_move_i<kDppWaveShl1>(sj);
                const bool jfirst = sact && (lane == 0 || sj_up != sj);
                jlast = sact && (lane == 63 || sj_dn != sj);
                jhead = run_head(__ballot(jfirst), upto);
                jcr = sact ? (float)(lane - jhead + 1) * rbj : 0.f;
#pragma unroll
                for (int c = 0; c < JP; ++c) av[c] = L.Ab[ilc * RS + c];
            }
#pragma unroll
            for (int qq = 0; qq < QJ; ++qq) {
                const int c = rj + NJ * qq;
                float t = 0.f;
                if (c < JP) {
                    if constexpr (kHreg) {
#pragma unroll
                        for (int x_ = 0; x_ < JP; ++x_) t = fmaf(av[x_], hh[qq][x_], t);
                    } else {
                        // column c of H_k: row c of H_k^T, four values per read
                        const floatx4* H4 = reinterpret_cast<const floatx4*>(L.Ht + (k * JP + c) * JP);
#pragma unroll
                        for (int x4 = 0; x4 < JP / 4; ++x4) {
                            const floatx4 h4 = H4[x4];
#pragma unroll
                            for (int r = 0; r < 4; ++r) t = fmaf(av[4 * x4 + r], h4[r], t);
                        }
                    }
                }
                w2q[qq] = t;
            }
            if constexpr (kHoist) {
                const int sj_up = dpp_move_i<kDppWaveShr1>(sj), sj_dn = dpp_move_i<kDppWaveShl1>(sj);
                const bool jfirst = sact && (lane == 0 || sj_up != sj);
                jlast = sact && (lane == 63 || sj_dn != sj);
                jhead = run_head(__ballot(jfirst), upto);
                jcr = sact ? (float)(lane - jhead + 1) * rbj : 0.f;
            }
#pragma unroll
            for (int qq = 0; qq < QJ; ++qq) {
                const int c = rj + NJ * qq;
                bp[qq] = (sact && c < JP) ? bp[qq] : 0.f;
            }
        }
        // patient runs (the tile is sorted by patient): heads and the
        // regularisation weight of each run (patient tasks only)
        bool ilast = false;
        int ihead = 0;
        float icr = 0.f;
        if (hi) {
            const int il_up = dpp_move_i<kDppWaveShr1>(il), il_dn = dpp_move_i<kDppWaveShl1>(il);
            const bool ifirst = act && (lane == 0 || il_up != il);
            ilast = act && (lane == 63 || il_dn != il);
            ihead = run_head(__ballot(ifirst), upto);
            if constexpr (!kHoist) rai = L.rA[ilc];
            icr = act ? (float)(lane - ihead + 1) * rai : 0.f;
        }
        __syncthreads();
        if (pend >= 0) {
            stage_sum<false, MP>(L.St, L.Sk + pend * J12, J1, J2, tid, NT);
            pend = -1;
        }
        if (u + 1 < cend) {
            const int o2 = L.tco[u + 1];
            n_next = L.tco[u + 2] - o2;
            k_next = L.tck[u + 1];
            wv_next = lane < n_next ? L.rec[o2 - z0 + lane] : make_uint2(0u, 0u);
        }

        // 2. residual (x~: the patient-task wavefronts' shares in wavefront
        // order); the tasks' run sums
        float xt;
        if constexpr (kHoist) {
            float xs[NI];
#pragma unroll
            for (int ww = 0; ww < NI; ++ww) xs[ww] = L.xtp[ww * kTileMax + lane];
            xt = xs[0];
#pragma unroll
            for (int ww = 1; ww < NI; ++ww) xt += xs[ww];
        } else {
            xt = L.xtp[lane];
#pragma unroll
            for (int ww = 1; ww < NI; ++ww) xt += L.xtp[ww * kTileMax + lane];
        }
        const float e = act ? x - xt : 0.f;
        if (hi) {
            if constexpr (kHoist) {
                // the columns' scans interleaved
                float v[QI];
#pragma unroll
                for (int qq = 0; qq < QI; ++qq) {
                    const int c = ri + NI * qq;
                    if (c < JP) {
                        L.As[c * kTS + lane] = aq[qq];
                        L.Es[c * kTS + lane] = e * bq[qq];
                    }
                    v[qq] = e * w1q[qq];
                }
                seg_scan_n<QI>(v, lane, ihead);
#pragma unroll
                for (int qq = 0; qq < QI; ++qq) {
                    const int c = ri + NI * qq;
                    if (c < JP && ilast) L.Ab[il * RS + c] = fmaf(a.lr, v[qq] - icr * aq[qq], aq[qq]);
                }
            } else {
#pragma unroll
                for (int qq = 0; qq < QI; ++qq) {
                    const int c = ri + NI * qq;
                    if (c < JP) {
                        L.As[c * kTS + lane] = aq[qq];
                        L.Es[c * kTS + lane] = e * bq[qq];
                        const float v = seg_scan(e * w1q[qq], lane, ihead);
                        if (ilast) L.Ab[il * RS + c] = fmaf(a.lr, v - icr * aq[qq], aq[qq]);
                    }
                }
            }
        }
        if (hj) {
            // e w2 of the wavefront's columns pushed to slot order
            if constexpr (kHoist) {
                float v[QJ];
#pragma unroll
                for (int qq = 0; qq < QJ; ++qq)
                    v[qq] = __int_as_float(__builtin_amdgcn_ds_permute(jr << 2, __float_as_int(e * w2q[qq])));
                seg_scan_n<QJ>(v, lane, jhead);
#pragma unroll
                for (int qq = 0; qq < QJ; ++qq) {
                    const int c = rj + NJ * qq;
                    if (c < JP && jlast) L.Bb[sj * RS + c] = fmaf(a.lr, v[qq] - jcr * bp[qq], bp[qq]);
                }
            } else {
#pragma unroll
                for (int qq = 0; qq < QJ; ++qq) {
                    const int c = rj + NJ * qq;
                    if (c < JP) {
                        const float ws =
                            __int_as_float(__builtin_amdgcn_ds_permute(jr << 2, __float_as_int(e * w2q[qq])));
                        const float v = seg_scan(ws, lane, jhead);
                        if (jlast) L.Bb[sj * RS + c] = fmaf(a.lr, v - jcr * bp[qq], bp[qq]);
                    }
                }
            }
        }
        prev = 1;
        __syncthreads();
        }
    }
    if (mfw && prev) acc.accumulate_all(L.As, L.Es, mw, lane);
    if (mfw) acc.store(L.St + mw * J12, J1, J2, lane);
    __syncthreads();
    stage_sum<false, MP>(L.St, L.Sk + curk * J12, J1, J2, tid, NT);
    __syncthreads();
}

// The tiles [t0, t1) of one block with BF16 matrix-core contractions (FP32
// accumulation; factor rows, residuals and updates stay FP32).  Per tile:
//   1. row block b = 0..3 (nonzeros 16b..16b+15) forms W1 = B_tile H_k^T
//      and W2 = A_tile H_k on the matrix cores (BF16 operands, one K step
//      of 32): W1 in tile order, W2 in the tile's gene-sorted slot order;
//      the W1 wavefront also forms x~ = a . w1 (FP32 row sums) and
//      e = x - x~ for its nonzeros, in tile order and in slot order.  With
//      eight wavefronts, wavefronts 0..3 take W1 and 4..7 take W2 (and add
//      the previous tile's S operands); with four, each takes both;
//   -- barrier --
//   2. patient tasks stage the BF16 operands a_i and e b_j of the S product
//      for their columns and sum the patient runs of e*w1, gene tasks sum
//      the gene runs of e*w2, with the segmented scans of the FP32 path
//      (with eight wavefronts gene tasks on 0..3, patient tasks on 4..7);
//   -- barrier --
template <int JP, int NW>
__device__ void block_tiles_bf(const StratArgs& a, int t0, int t1, const TileLds& L, int tid, int pre_cend)
{
#pragma clang fp contract(off)
    constexpr int RS = strat_row_stride(JP, 1);
    constexpr int MP = mfma_dim(JP);
    constexpr int NB = MP / 16;
    constexpr int NT = 64 * NW;
    constexpr bool kTwo = NW >= 2 * kMfmaWaves;  // W1 and W2 on different wavefronts
    // column tasks: with eight wavefronts the gene tasks go to wavefronts
    // 0..3 and the patient tasks (with the S operands of their columns) to
    // 4..7; with four, each wavefront takes both tasks of its columns
    constexpr int NJ = kTwo ? NW / 2 : NW, OI = kTwo ? NW / 2 : 0, NI = NW - OI;
    constexpr int QI = (JP + NI - 1) / NI, QJ = (JP + NJ - 1) / NJ;
    const int lane = tid & 63, w = tid >> 6, g = lane >> 4, m = lane & 15;
    const unsigned long long upto = lanes_upto(lane);
    const int J1 = a.J1, J2 = a.J2, J12 = J1 * J2;
    const uint32_t mask_i = (1u << a.bits_i) - 1u, mask_j = (1u << a.bits_j) - 1u;
    const int sh_j = a.bits_i, sh_r = a.bits_i + a.bits_j;
    if (t0 >= t1) return;
    const bool hj = w < NJ, hi = w >= OI;
    const int rj = w, ri = w - OI;

    // operand columns beyond the factor columns stay zero
    for (int idx = tid; idx < (MP - JP) * kTB; idx += NT) {
        L.A16[JP * kTB + idx] = (__bf16)0.f;
        L.E16[JP * kTB + idx] = (__bf16)0.f;
    }

    SAccB<MP> acc;
    acc.zero();
    // the last four wavefronts accumulate S (mw = 0..3) and form W2; W1 and
    // x~ fall to wavefronts 0..3
    const int mw = w - (NW - kMfmaWaves);
    const bool mfw = mw >= 0;
    const bool do1 = kTwo ? w < kMfmaWaves : true, do2 = mfw;
    const int rb = kTwo ? (w & (kMfmaWaves - 1)) : mw;  // row block of W1 / W2
    float* eT = L.xts;  // e in tile order
    float* eS = L.eS;   // e in slot order
    int curk = -1;
    int pend = -1;    // platform whose partial S waits in L.St
    int prev_n = 0;   // nonzeros of the tile whose S operands wait in L.A16/L.E16
    bf16x8 hb[NB];    // H_k^T (W1) or H_k (W2) operand of this wavefront
    int tl = t0;
    while (tl < t1) {
        const int cend = (pre_cend > 0 && tl == t0) ? pre_cend : load_chunk(a, L, tl, t1, tid, NT);
        const int z0 = L.tco[0];
        for (int u = 0; u < cend; ++u, ++tl) {
        const int off = L.tco[u];
        const int n = L.tco[u + 1] - off;
        const int k = L.tck[u];
        const uint2* rec = L.rec + (off - z0);
        // S of the previous tile (its platform is curk)
        if (mfw && prev_n > 0) acc.accumulate(L.A16, L.E16, prev_n, mw, lane);
        if (k != curk) {
            if (curk >= 0) {
                if (mfw) acc.store(L.St + mw * J12, J1, J2, mw, lane);
                pend = curk;
            }
            acc.zero();
            curk = k;
        }
        const bool act = lane < n;
        const uint2 wv = act ? rec[lane] : make_uint2(0u, 0u);
        const uint32_t wd = wv.x;
        const int il = act ? (int)(wd & mask_i) : -1;
        const int ilc = act ? il : 0;
        const int jl = act ? (int)((wd >> sh_j) & mask_j) : 0;
        const int jrank = (int)(wd >> sh_r);

        // the values of the wavefront's own run task, requested first: the
        // patient rows' regularisation weights and the a, b values of its
        // columns (patient tasks); the slot order, the gene rows' weights
        // and b values (gene tasks).  Columns past the core read column
        // JP - 1 and lanes past the tile's end row 0: neither value is used.
        float aq[QI], bq[QI], bp[QJ], rai = 0.f, rbj = 0.f;
        int sj = -1;
        if (hi) {
            rai = L.rA[ilc];
#pragma unroll
            for (int qq = 0; qq < QI; ++qq) {
                const int c = ri + NI * qq, cc = c < JP ? c : JP - 1;
                aq[qq] = L.Ab[ilc * RS + cc];
                bq[qq] = L.Bb[jl * RS + cc];
            }
        } else {
#pragma unroll
            for (int qq = 0; qq < QI; ++qq) aq[qq] = bq[qq] = 0.f;
        }
        if (hj) {
            // slot s learns its gene row from the lane that holds it
            // (inactive lanes push to their own slot)
            sj = __builtin_amdgcn_ds_permute((act ? jrank : lane) << 2, act ? jl : -1);
            const int sjc = act ? sj : 0;
            rbj = L.rB[sjc];
#pragma unroll
            for (int qq = 0; qq < QJ; ++qq) {
                const int c = rj + NJ * qq, cc = c < JP ? c : JP - 1;
                bp[qq] = L.Bb[sjc * RS + cc];
            }
        } else {
#pragma unroll
            for (int qq = 0; qq < QJ; ++qq) bp[qq] = 0.f;
        }

        // 1. W1 with x~ and e, W2, for nonzeros 16 rb .. 16 rb + 15
        if (do1 || do2) {
            const int to = 16 * rb + m;
            const bool ao = to < n;
            const uint32_t wo = ao ? rec[to].x : 0u;
            const floatx4 zero4 = floatx4{0.f, 0.f, 0.f, 0.f};
            if (do1) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    hb[nb] = *reinterpret_cast<const bf16x8*>(L.Hb + ((2 * k) * MP + nb * 16 + m) * kKB + 8 * g);
                const bf16x8 opb = row8_bf16<RS>(L.Bb + ((wo >> sh_j) & mask_j) * RS, 8 * g, ao);
                int ilr[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int tr = 16 * rb + 4 * g + r;
                    ilr[r] = tr < n ? (int)(rec[tr].x & mask_i) : 0;
                }
                // the a values of x~ requested before the products
                float ax[NB][4];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int c = nb * 16 + m, cc = c < JP ? c : JP - 1;
#pragma unroll
                    for (int r = 0; r < 4; ++r) ax[nb][r] = L.Ab[ilr[r] * RS + cc];
                }
                float xp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const floatx4 o1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(opb, hb[nb], zero4, 0, 0, 0);
                    const int c = nb * 16 + m;
                    *reinterpret_cast<floatx4*>(L.sW1 + c * kTW + 16 * rb + 4 * g) = o1;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (c < JP) xp[r] = fmaf(ax[nb][r], o1[r], xp[r]);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) xp[r] = row_sum16(xp[r]);
                // lane (g, m < 4) finishes nonzero 16 rb + 4 g + m
                const int te = 16 * rb + 4 * g + m;
                if (m < 4 && te < n) {
                    const uint2 we = rec[te];
                    const float xt = m == 0 ? xp[0] : (m == 1 ? xp[1] : (m == 2 ? xp[2] : xp[3]));
                    const float ee = __uint_as_float(we.y) - xt;
                    eT[te] = ee;
                    eS[we.x >> sh_r] = ee;
                }
            }
            if (do2) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    hb[nb] = *reinterpret_cast<const bf16x8*>(L.Hb + ((2 * k + 1) * MP + nb * 16 + m) * kKB + 8 * g);
                const bf16x8 opa = row8_bf16<RS>(L.Ab + (wo & mask_i) * RS, 8 * g, ao);
                int jrr[4];
                bool actr[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int tr = 16 * rb + 4 * g + r;
                    actr[r] = tr < n;
                    jrr[r] = actr[r] ? (int)(rec[tr].x >> sh_r) : 0;
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const floatx4 o2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(opa, hb[nb], zero4, 0, 0, 0);
                    const int c = nb * 16 + m;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (actr[r]) L.sW2[c * kTW + jrr[r]] = o2[r];
                }
            }
        }
        // patient runs (patient tasks): heads and regularisation weights
        bool ilast = false;
        int ihead = 0;
        float icr = 0.f;
        if (hi) {
            const int il_up = dpp_move_i<kDppWaveShr1>(il), il_dn = dpp_move_i<kDppWaveShl1>(il);
            const bool ifirst = act && (lane == 0 || il_up != il);
            ilast = act && (lane == 63 || il_dn != il);
            ihead = run_head(__ballot(ifirst), upto);
            icr = act ? (float)(lane - ihead + 1) * rai : 0.f;
#pragma unroll
            for (int qq = 0; qq < QI; ++qq) {
                const int c = ri + NI * qq;
                aq[qq] = (c < JP && act) ? aq[qq] : 0.f;
                bq[qq] = (c < JP && act) ? bq[qq] : 0.f;
            }
        }
        // gene runs in slot order (gene tasks): heads, regularisation
        // weights and the rows' values before the tile
        bool jlast = false;
        int jhead = 0;
        float jcr = 0.f;
        if (hj) {
            const int sj_up = dpp_move_i<kDppWaveShr1>(sj), sj_dn = dpp_move_i<kDppWaveShl1>(sj);
            const bool jfirst = act && (lane == 0 || sj_up != sj);
            jlast = act && (lane == 63 || sj_dn != sj);
            jhead = run_head(__ballot(jfirst), upto);
            jcr = act ? (float)(lane - jhead + 1) * rbj : 0.f;
#pragma unroll
            for (int qq = 0; qq < QJ; ++qq) {
                const int c = rj + NJ * qq;
                bp[qq] = (c < JP && act) ? bp[qq] : 0.f;
            }
        }
        __syncthreads();
        if (pend >= 0) {
            stage_sum<true, MP>(L.St, L.Sk + pend * J12, J1, J2, tid, NT);
            pend = -1;
        }


        // 2. BF16 S operands; fixed-order run sums; owned columns
        const float e = act ? eT[lane] : 0.f;
        const float es = act ? eS[lane] : 0.f;
        if (hi) {
            // the columns' e w1 read at once, their scans interleaved
            float v[QI];
#pragma unroll
            for (int qq = 0; qq < QI; ++qq) {
                const int c = ri + NI * qq, cc = c < JP ? c : JP - 1;
                v[qq] = e * L.sW1[cc * kTW + lane];
            }
#pragma unroll
            for (int qq = 0; qq < QI; ++qq) {
                const int c = ri + NI * qq;
                if (c < JP) {
                    L.A16[c * kTB + lane] = (__bf16)aq[qq];
                    L.E16[c * kTB + lane] = (__bf16)(e * bq[qq]);
                }
            }
            seg_scan_n<QI>(v, lane, ihead);
#pragma unroll
            for (int qq = 0; qq < QI; ++qq) {
                const int c = ri + NI * qq;
                if (c < JP && ilast) L.Ab[il * RS + c] = fmaf(a.lr, v[qq] - icr * aq[qq], aq[qq]);
            }
        }
        if (hj) {
            float v[QJ];
#pragma unroll
            for (int qq = 0; qq < QJ; ++qq) {
                const int c = rj + NJ * qq, cc = c < JP ? c : JP - 1;
                v[qq] = es * L.sW2[cc * kTW + lane];
            }
            seg_scan_n<QJ>(v, lane, jhead);
#pragma unroll
            for (int qq = 0; qq < QJ; ++qq) {
                const int c = rj + NJ * qq;
                if (c < JP && jlast) L.Bb[sj * RS + c] = fmaf(a.lr, v[qq] - jcr * bp[qq], bp[qq]);
            }
        }
        prev_n = n;
        __syncthreads();
        }
    }
    if (mfw && prev_n > 0) acc.accumulate(L.A16, L.E16, prev_n, mw, lane);
    if (mfw) acc.store(L.St + mw * J12, J1, J2, mw, lane);
    __syncthreads();
    stage_sum<true, MP>(L.St, L.Sk + curk * J12, J1, J2, tid, NT);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Tagged exchange of the persistent kernel.  What workgroups hand to each
// other within a stratum (the blocks' sums, the reduced stratum sums and a
// "rows stored" word per patient block) travels in 64-bit words: the float's
// bits in the low half and the stratum's tag in the high half, written by
// one device-coherent 64-bit store, so a reader that sees the tag sees the
// value.  Readers poll the words they need (reloading only those that still
// carry an older tag) instead of meeting at a grid barrier: no writer waits
// for its stores to be performed before it goes on, and a reader's wait and
// its load are one round trip.  Tags are unique per stratum and launch (the
// host hands every launch a fresh range), and every word is rewritten in
// every stratum, so an old word never carries a current tag.  A word is
// rewritten only after everyone who reads it has read it: block sums of the
// next stratum follow their writer's read of all stratum sums, which follow
// every reducer's read of the block sums; stratum sums of the next stratum
// follow every workgroup's next block sums.
//
// Patient rows are plain device-coherent stores; their writer stores the
// block's "rows stored" word only after its rows have been performed
// (coh_stores_done, after the reduction, when they long have been), and the
// next stratum's reader loads them only after it has seen that word.
//
// Every poll is bounded: after kSpinLimit rounds (far longer than any
// stratum can take; the host may set fewer, to test this path) the poller
// sets the error word and gives up, and every poller gives up once it sees
// the error word set (checked every 128 rounds); the workgroup then leaves
// the launch.
// ---------------------------------------------------------------------------
constexpr unsigned kSpinLimit = 1u << 25;
constexpr int kSumPoll = 4;  // stratum sums each thread polls per round
constexpr int kRowPre = 2;   // patient-row values per thread requested before the core step

__device__ inline void st_tag(unsigned long long* p, float v, unsigned tag)
{
    __hip_atomic_store(p, ((unsigned long long)tag << 32) | __float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long ld_tag(unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline float tag_value(unsigned long long x) { return __uint_as_float((unsigned)x); }

// Polls the words x[u] = p[u * stride] (u < n <= N, bit u of skip clear)
// and xe = *pe (unless pe is null) until each carries `tag`; the others
// read as 0.0 with the tag.  Every round reloads, in flight together, the
// words still behind.  False if the poll gave up after `limit` rounds or
// saw the error word set (see above).
template <int N>
__device__ bool poll_tagged(unsigned long long (&x)[N], unsigned long long* p, int stride, int n, unsigned skip,
                            unsigned long long& xe, unsigned long long* pe, unsigned tag, GridBar* bar,
                            unsigned limit)
{
    const unsigned long long fresh = (unsigned long long)tag << 32;
#pragma unroll
    for (int u = 0; u < N; ++u) x[u] = u < n && !((skip >> u) & 1u) ? ld_tag(p + (size_t)u * stride) : fresh;
    xe = pe ? ld_tag(pe) : fresh;
    unsigned spins = 0;
    for (;;) {
        bool done = (unsigned)(xe >> 32) == tag;
#pragma unroll
        for (int u = 0; u < N; ++u) done = done && (unsigned)(x[u] >> 32) == tag;
        if (done) return true;
        if (++spins > limit) {
            atomicOr(&bar->err, 1u);
            return false;
        }
        if ((spins & 127u) == 0u &&
            __hip_atomic_load(&bar->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
            return false;
#pragma unroll
        for (int u = 0; u < N; ++u)
            if ((unsigned)(x[u] >> 32) != tag) x[u] = ld_tag(p + (size_t)u * stride);
        if ((unsigned)(xe >> 32) != tag) xe = ld_tag(pe);
    }
}

// Items [i0, i1) of the stratum sums from the tagged block sums Sx ([P][ni])
// into dst (tagged, device-coherent) and own[i0..i1), in the order of
// reduce_items, using the whole workgroup (red: nthr floats of LDS, slots:
// those of a wg_count site, kDefaultWaves wavefronts).  The
// sums of block pown are not polled but read from own (this workgroup's
// block).  False (for every thread) if a poll gave up.
__device__ bool reduce_items_tagged(unsigned long long* Sx, int P, int ni, int i0, int i1, unsigned long long* dst,
                                    float* own, int pown, unsigned tag, GridBar* bar, unsigned limit, float* red,
                                    int* slots, int tid, int nthr)
{
    const int nch = (P + kRedChunk - 1) / kRedChunk;
    const int per_pass = nthr / nch > 0 ? nthr / nch : 1;
    for (int base = i0; base < i1; base += per_pass) {
        const int items = (i1 - base) < per_pass ? (i1 - base) : per_pass;
        const bool act = tid < items * nch;
        const int it = act ? tid / nch : 0, ch = act ? tid - it * nch : 0;
        const int p0 = ch * kRedChunk;
        // four words per poll (this path serves large cores only)
        float s = 0.f;
        bool ok = true;
        for (int g = 0; g < kRedChunk; g += 4) {
            const int n = act ? (P - p0 - g < 4 ? (P - p0 - g > 0 ? P - p0 - g : 0) : 4) : 0;
            const int so = pown - p0 - g;  // the own block's word in this group
            const unsigned skip = so >= 0 && so < 4 ? 1u << so : 0u;
            unsigned long long x[4], xe;
            ok = ok &&
                 poll_tagged<4>(x, Sx + (size_t)(p0 + g) * ni + base + it, ni, n, skip, xe, nullptr, tag, bar, limit);
#pragma unroll
            for (int u = 0; u < 4; ++u) s += u == so && u < n ? own[base + it] : tag_value(x[u]);
        }
        if (wg_count<kDefaultWaves>(!ok, slots) != 0) return false;
        if (act) red[tid] = s;
        __syncthreads();
        if (tid < items) {
            float s = 0.f;
            for (int c = 0; c < nch; ++c) s += red[tid * nch + c];
            st_tag(dst + base + tid - i0, s, tag);
            own[base + tid] = s;
        }
    }
    __syncthreads();
    return true;
}

// Workgroups are dispatched to the XCDs round-robin (workgroup q runs on XCD
// q mod 8).  xcd_slot numbers the workgroups XCD by XCD: a bijection of
// [0, n) that gives the workgroups of one XCD consecutive slots.
constexpr int kXcds = 8;
__device__ inline int xcd_slot(int q, int n)
{
    const int x = q % kXcds, per = n / kXcds, extra = n % kXcds;
    return x * per + (x < extra ? x : extra) + q / kXcds;
}

template <int JP>
__device__ inline TileLds tile_lds(float* lds, const StratLds& S)
{
    TileLds L;
    L.Ab = lds + S.a;
    L.Bb = lds + S.b;
    L.rA = lds + S.ra;
    L.rB = lds + S.rb;
    L.Hs = lds + S.h;
    L.Ht = lds + S.ht;
    L.As = lds + S.as;
    L.Es = lds + S.es;
    L.xtp = lds + S.xtp;
    L.Hb = reinterpret_cast<const __bf16*>(lds + S.hb);
    L.sW1 = lds + S.sw1;
    L.sW2 = lds + S.sw2;
    L.xts = lds + S.xts;
    L.eS = lds + S.esl;
    L.A16 = reinterpret_cast<__bf16*>(lds + S.a16);
    L.E16 = reinterpret_cast<__bf16*>(lds + S.e16);
    L.Sk = lds + S.sk;
    L.St = lds + S.stg;
    L.tco = reinterpret_cast<int*>(lds + S.tco);
    L.tck = reinterpret_cast<int*>(lds + S.tck);
    L.rec = reinterpret_cast<uint2*>(lds + S.rec);
    L.wgs = reinterpret_cast<int*>(lds + S.wgs);
    return L;
}

// Contiguous rows [row0, row0+nrows) of a position-ordered factor written
// by other workgroups of this launch, into LDS rows of stride RS
// (device-coherent loads, eight in flight per thread).
__device__ inline void load_rows_coh(float* dst, const float* src, int row0, int nrows, int J, int RS, int tid,
                                     int nthr, int from = 0)
{
    constexpr int U = 8;
    const float* s = src + (size_t)row0 * J;
    const int total = nrows * J;
    for (int base = from + tid; base < total; base += U * nthr) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * nthr;
            v[u] = idx < total ? ld_coh(s + idx) : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * nthr;
            if (idx < total) {
                const int l = idx / J, c = idx - l * J;
                dst[l * RS + c] = v[u];
            }
        }
    }
}

__device__ inline void store_rows_coh(float* dst, const float* src, int row0, int nrows, int J, int RS, int tid,
                                      int nthr)
{
    float* d = dst + (size_t)row0 * J;
    for (int idx = tid; idx < nrows * J; idx += nthr) {
        const int l = idx / J, c = idx - l * J;
        st_coh(d + idx, src[l * RS + c]);
    }
}

// ---------------------------------------------------------------------------
// Persistent driver: every stratum of one epoch in one launch.
// ---------------------------------------------------------------------------
// Every stratum of one epoch of one problem, run by its workgroup q (gene
// block q) of the problem's P co-resident workgroups.  The epoch's schedule
// (stratum order, and for each stratum the block's tile range, record range
// and patient rows) is read into LDS once.  Per stratum (exchanges tagged,
// see poll_tagged):
//   H_k from the current C, G; the block's tiles (its first record chunk and
//   tile metadata already in LDS); its patient rows (coherent stores) and
//   sums of e a (x) b (tagged) out; the next block's tile metadata and first
//   record chunk requested (read-only data, in flight during the waits);
//   this workgroup's share of the stratum sums: the blocks' sums polled, then
//   added in a fixed order; the prefetched chunk and the stratum's core-step
//   constants into LDS; the share (tagged) and, once this workgroup's rows
//   have been performed, its "rows stored" word out;
//   every stratum sum and the next block's "rows stored" word polled; that
//   block's patient rows in (coherent loads); the same C/G step in every
//   workgroup, on its LDS copy.
template <int JP, bool BF, int NW>
__device__ void strata_body(const StratArgs& a, int q, float* lds)
{
    constexpr int RS = strat_row_stride(JP, BF ? 1 : 0);
    constexpr int NT = 64 * NW;
    const int tid0 = threadIdx.x;
    const int P = a.P, I3 = a.I3, J1 = a.J1, J2 = a.J2, J3 = a.J3, J12 = J1 * J2;
    const int ni = I3 * J12;
    const StratLds S = strat_lds_layout(JP, P, a.rows1_max, a.rows2_max, I3, J1, J2, J3, a.rec_cap, BF ? 1 : 0, NW);
    const TileLds L = tile_lds<JP>(lds, S);
    float* Cs = lds + S.c;
    float* Gs = lds + S.g;
    float* Hs = lds + S.h;
    float* Sk = lds + S.sk;
    float* red = lds + S.red;
    float* cst = lds + S.cst;
    float* cgt = lds + S.cgt;
    float* Cn = cgt;            // C and G after the stratum's core step
    float* Gn = cgt + I3 * J3;
    // schedule of stratum index si: [0] first tile, [1] tile end, [2] first
    // record, [3] record end, [4] first patient row, [5] patient row end,
    // [6] the stratum s (at sch[x * P + si])
    int* sch = reinterpret_cast<int*>(lds + S.sch);

    for (int idx = tid0; idx < a.rows1_max * RS; idx += NT) lds[S.a + idx] = 0.f;
    for (int idx = tid0; idx < a.rows2_max * RS; idx += NT) lds[S.b + idx] = 0.f;
    if constexpr (BF) clear_hb_pad<JP>(reinterpret_cast<__bf16*>(lds + S.hb), I3, tid0, NT);
    for (int si = tid0; si < P; si += NT) {
        const int s = a.order[si], p = (q - s + P) % P, b = p * P + q;
        sch[si] = a.blk_tile[b];
        sch[P + si] = a.blk_tile[b + 1];
        sch[2 * P + si] = a.blk_rec[b];
        sch[3 * P + si] = a.blk_rec[b + 1];
        sch[4 * P + si] = a.start1[p];
        sch[5 * P + si] = a.start1[p + 1];
        sch[6 * P + si] = s;
    }
    __syncthreads();
    const int s2 = a.start2[q], r2 = a.start2[q + 1] - s2;
    load_rows(L.Bb, a.Bp, s2, r2, J2, RS, tid0, NT);
    for (int l = tid0; l < r2; l += NT) lds[S.rb + l] = a.reg2[s2 + l];
    for (int idx = tid0; idx < I3 * J3; idx += NT) Cs[idx] = a.C[idx];
    for (int idx = tid0; idx < J12 * J3; idx += NT) Gs[idx] = a.G[idx];
    {
        const int s1 = sch[4 * P], r1 = sch[5 * P] - s1;
        load_rows_coh(L.Ab, a.Ap, s1, r1, J1, RS, tid0, NT);
        for (int l = tid0; l < r1; l += NT) lds[S.ra + l] = a.reg1[s1 + l];
    }
    __syncthreads();
    // tagged exchange words: the blocks' sums [P][ni], the stratum sums [ni],
    // the "rows stored" word of each patient block [P]
    unsigned long long* Xpart = a.Sx;
    unsigned long long* Xsum = a.Sx + (size_t)P * ni;
    unsigned long long* Xrows = Xsum + ni;
    const unsigned wlim = a.spin_limit ? a.spin_limit : kSpinLimit;  // poll rounds before a wait gives up

    // this workgroup's share of the stratum reduction: consecutive shares go
    // to workgroups on the same XCD, so each XCD fetches its own contiguous
    // slice of the per-block sums
    const int r = xcd_slot(q, P);
    const int i0 = (int)(((long long)ni * r) / P), i1 = (int)(((long long)ni * (r + 1)) / P);
    const int nchr = (P + kRedChunk - 1) / kRedChunk;
    const int nitems = i1 - i0 > 0 ? i1 - i0 : 1;
    const bool one = (i1 - i0) * nchr <= NT;
    // the next stratum's first chunk is requested by wavefronts 2.. (the
    // reduction share is polled by its first (i1 - i0) * nchr threads:
    // wavefronts 0 and 1 at the PanCan-sized cores)
    constexpr int kPreRec = (kMaxRecCap + NT - 129) / (NT - 128);  // records per thread
    constexpr int kPreTc = (kTileCache + NT - 128) / (NT - 128);    // tile entries per thread (of kTileCache + 1)
    int pre_cend = 0;  // tiles of this stratum's first chunk already in LDS

    for (int si = 0; si < P; ++si) {
        // the thread index, opaque to the compiler in every stratum: what is
        // derived from it is formed here, not hoisted out of the loop and
        // held (spilled) across the tiles (the BF16 tile step, measured
        // faster with its values hoisted, takes the plain index)
        int tid = tid0;
        asm volatile("" : "+v"(tid));
        // item and chunk of this thread's share of the reduction: consecutive
        // lanes take consecutive items of one chunk (coalesced loads)
        const int rch = tid / nitems, rit = tid - rch * nitems;
        const int pt = tid - 128;
        const int s = sch[6 * P + si];
        const int p = (q - s + P) % P;
        const int s1 = sch[4 * P + si], r1 = sch[5 * P + si] - s1;
        const unsigned tg = a.tag0 + (unsigned)si + 1u;  // this stratum's tag
        if constexpr (BF)
            build_h<JP>(nullptr, Cs, Gs, I3, J1, J2, J3, tid, NT, nullptr, reinterpret_cast<__bf16*>(lds + S.hb));
        else
            build_h<JP>(Hs, Cs, Gs, I3, J1, J2, J3, tid, NT, JP > 12 ? lds + S.ht : nullptr);
        for (int idx = tid; idx < ni; idx += NT) Sk[idx] = 0.f;
        __syncthreads();
        if constexpr (BF)
            block_tiles_bf<JP, NW>(a, sch[si], sch[P + si], L, tid0, pre_cend);
        else
            block_tiles<JP, NW>(a, sch[si], sch[P + si], L, tid, pre_cend);
        pre_cend = 0;
        store_rows_coh(a.Ap, L.Ab, s1, r1, J1, RS, tid, NT);
        unsigned long long* Xp = Xpart + (size_t)p * ni;
        for (int idx = tid; idx < ni; idx += NT) st_tag(Xp + idx, Sk[idx], tg);
        // the next stratum's tile metadata (as load_tile_cache lays it out) and
        // first record chunk: read-only, requested now, used after the polls
        const bool more = si + 1 < P;
        const int tn0 = more ? sch[si + 1] : 0, tn1 = more ? sch[P + si + 1] : 0;
        const int zn0 = more ? sch[2 * P + si + 1] : 0, zn1 = more ? sch[3 * P + si + 1] : 0;
        const int ntc = (tn1 - tn0) < kTileCache ? (tn1 - tn0) : kTileCache;
        const int nrec = (zn1 - zn0) < a.rec_cap ? (zn1 - zn0) : a.rec_cap;
        int tov[kPreTc], tkv[kPreTc];
        uint2 rr[kPreRec];
#pragma unroll
        for (int h = 0; h < kPreTc; ++h) {
            const int u = pt + h * (NT - 128);
            tov[h] = pt >= 0 && u <= ntc ? a.tile_off[tn0 + u] : 0;
            tkv[h] = pt >= 0 && u < ntc ? a.tile_k[tn0 + u] : 0;
        }
#pragma unroll
        for (int h = 0; h < kPreRec; ++h) {
            const int i = pt + h * (NT - 128);
            rr[h] = pt >= 0 && i < nrec ? a.nz[zn0 + i] : make_uint2(0u, 0u);
        }
        float cv = tid < kCstHead + I3 ? a.ccst[(size_t)s * (kCstHead + I3) + tid] : 0.f;

        // this workgroup's share of the stratum sums: with one chunk of
        // kRedChunk blocks per thread when the share allows, all blocks'
        // sums polled in one round
        float rv[kRedChunk];
        if (one) {
            const bool rt = tid < (i1 - i0) * nchr;
            const int p0 = rch * kRedChunk;
            const int n = rt ? (P - p0 < kRedChunk ? P - p0 : kRedChunk) : 0;
            // this workgroup's own block sums come from LDS
            const int so = p - p0;
            const unsigned skip = so >= 0 && so < kRedChunk ? 1u << so : 0u;
            unsigned long long x[kRedChunk], xe;
            const bool ok = poll_tagged<kRedChunk>(x, Xpart + (rt ? p0 * ni + i0 + rit : 0), ni, n, skip, xe,
                                                   nullptr, tg, a.bar, wlim);
            const float mine = rt && skip ? Sk[i0 + rit] : 0.f;
#pragma unroll
            for (int u = 0; u < kRedChunk; ++u) rv[u] = u == so ? mine : tag_value(x[u]);
            if (wg_count<NW>(!ok, L.wgs + kWgPoll1 * kDefaultWaves) != 0) return;
        }
        // this wavefront's patient rows (stored before the polls) have been
        // performed; once every wavefront has passed this, the block's "rows
        // stored" word goes out with the share
        coh_stores_done();
        if (one) {
            // the order of reduce_items: each chunk's blocks ascending, then
            // the chunks ascending
            if (tid < (i1 - i0) * nchr) {
                float cs = 0.f;
#pragma unroll
                for (int u = 0; u < kRedChunk; ++u) cs += rv[u];
                red[rit * nchr + rch] = cs;
            }
            __syncthreads();
            if (tid == 0) st_tag(Xrows + p, 0.f, tg);
            if (tid < i1 - i0) {
                float t = 0.f;
#pragma unroll 8
                for (int ch = 0; ch < nchr; ++ch) t += red[tid * nchr + ch];
                st_tag(Xsum + i0 + tid, t, tg);
                Sk[i0 + tid] = t;
            }
        } else {
            if (!reduce_items_tagged(Xpart, P, ni, i0, i1, Xsum + i0, Sk, p, tg, a.bar, wlim, red,
                                     L.wgs + kWgReduce * kDefaultWaves, tid, NT))
                return;
            if (tid == 0) st_tag(Xrows + p, 0.f, tg);
        }
        // the tiles of the prefetched chunk whose records fit in it, from the
        // offsets in registers (tile u + 1 starts at tov of thread u + 1; the
        // chunk starts at the block's first record zn0)
        static_assert(kPreTc == 1, "one prefetched tile offset per thread");
        pre_cend = wg_count<NW>(pt >= 1 && pt <= ntc && tov[0] - zn0 <= a.rec_cap, L.wgs + kWgPre * kDefaultWaves);
        // the prefetched chunk and the stratum's core-step constants into LDS
        // (read after the next workgroup barrier)
        if (pt >= 0) {
#pragma unroll
            for (int h = 0; h < kPreTc; ++h) {
                const int u = pt + h * (NT - 128);
                if (u <= kTileCache) L.tco[u] = tov[h];
                if (u < kTileCache) L.tck[u] = tkv[h];
            }
#pragma unroll
            for (int h = 0; h < kPreRec; ++h) {
                const int i = pt + h * (NT - 128);
                if (i < nrec) L.rec[i] = rr[h];
            }
        }
        if (tid < kCstHead + I3) cst[tid] = cv;
        for (int idx = tid + NT; idx < kCstHead + I3; idx += NT) cst[idx] = a.ccst[(size_t)s * (kCstHead + I3) + idx];

        // every stratum sum (this workgroup's own share is in Sk already),
        // and the "rows stored" word of the patient block the next stratum
        // visits (stored in this stratum by the workgroup that visited it),
        // kSumPoll sums per thread and round
        {
            const int pn = more ? (q - sch[6 * P + si + 1] + P) % P : 0;
            bool ok = true;
            for (int base = 0; base < ni; base += kSumPoll * NT) {
                const int i = base + tid;
                const int n = i < ni ? ((ni - i + NT - 1) / NT < kSumPoll ? (ni - i + NT - 1) / NT : kSumPoll) : 0;
                unsigned skip = 0u;
#pragma unroll
                for (int u = 0; u < kSumPoll; ++u)
                    if (i + u * NT >= i0 && i + u * NT < i1) skip |= 1u << u;
                unsigned long long x[kSumPoll], xe;
                ok = ok && poll_tagged<kSumPoll>(x, Xsum + i, NT, n, skip, xe,
                                                 more && base == 0 && tid == NT - 1 ? Xrows + pn : nullptr, tg,
                                                 a.bar, wlim);
#pragma unroll
                for (int u = 0; u < kSumPoll; ++u)
                    if (u < n && !((skip >> u) & 1u)) Sk[i + u * NT] = tag_value(x[u]);
            }
            if (wg_count<NW>(!ok, L.wgs + kWgPoll2 * kDefaultWaves) != 0) return;
        }
        // the next block's patient rows: the first kRowPre values per thread
        // requested before the core step, stored after it
        const int s1n = more ? sch[4 * P + si + 1] : 0, r1n = more ? sch[5 * P + si + 1] - s1n : 0;
        const int nrv = r1n * J1;
        const float* rsrc = a.Ap + (size_t)s1n * J1;
        float rwv[kRowPre];
#pragma unroll
        for (int u = 0; u < kRowPre; ++u) rwv[u] = tid + u * NT < nrv ? ld_coh(rsrc + tid + u * NT) : 0.f;
        const float rg = tid < r1n ? a.reg1[s1n + tid] : 0.f;
        core_update(Cs, Gs, Sk, cst, I3, J12, J3, a.etac, Cn, Gn, tid, NT);
#pragma unroll
        for (int u = 0; u < kRowPre; ++u) {
            const int idx = tid + u * NT;
            if (idx < nrv) {
                const int l = idx / J1, c = idx - l * J1;
                L.Ab[l * RS + c] = rwv[u];
            }
        }
        if (tid < r1n) lds[S.ra + tid] = rg;
        if (nrv > kRowPre * NT) load_rows_coh(L.Ab, a.Ap, s1n, r1n, J1, RS, tid, NT, kRowPre * NT);
        for (int l = tid + NT; l < r1n; l += NT) lds[S.ra + l] = a.reg1[s1n + l];
        __syncthreads();
        // the new C and G become current; the old buffers take the next step
        float* t = Cs;
        Cs = Cn;
        Cn = t;
        t = Gs;
        Gs = Gn;
        Gn = t;
    }
    store_rows(a.Bp, L.Bb, s2, r2, J2, RS, tid0, NT);
    if (q == 0) {
        for (int idx = tid0; idx < I3 * J3; idx += NT) a.C[idx] = Cs[idx];
        for (int idx = tid0; idx < J12 * J3; idx += NT) a.G[idx] = Gs[idx];
    }
}

template <int JP, bool BF, int NW>
__global__ __launch_bounds__(64 * NW) void strata_persistent(StratArgs a)
{
    extern __shared__ float lds[];
    strata_body<JP, BF, NW>(a, blockIdx.x, lds);
}

// Batched sweep: the workgroups [wg_start[i], wg_start[i+1]) of one
// cooperative launch run problem i with the code of its own core size
// (a.jp), exactly as the single-problem kernel would; each problem
// exchanges through its own tagged words.
template <bool BF>
__global__ __launch_bounds__(64 * kDefaultWaves) void strata_sweep(const StratArgs* args, const int32_t* wg_start,
                                                                   int n)
{
    constexpr int NW = kDefaultWaves;
    extern __shared__ float lds[];
    const int b = blockIdx.x;
    int i = 0;
    while (i + 1 < n && b >= wg_start[i + 1]) ++i;
    const StratArgs a = args[i];
    const int q = b - wg_start[i];
    switch (a.jp) {
    case 2: strata_body<2, BF, NW>(a, q, lds); break;
    case 4: strata_body<4, BF, NW>(a, q, lds); break;
    case 5: strata_body<5, BF, NW>(a, q, lds); break;
    case 8: strata_body<8, BF, NW>(a, q, lds); break;
    case 10: strata_body<10, BF, NW>(a, q, lds); break;
    case 12: strata_body<12, BF, NW>(a, q, lds); break;
    case 16: strata_body<16, BF, NW>(a, q, lds); break;
    case 20: strata_body<20, BF, NW>(a, q, lds); break;
    case 24: strata_body<24, BF, NW>(a, q, lds); break;
    case 32: strata_body<32, BF, NW>(a, q, lds); break;
    default: break;
    }
}

// ---------------------------------------------------------------------------
// Multi-launch driver: one block step per stratum, then one core step.
// ---------------------------------------------------------------------------
template <int JP, bool BF, int NW>
__global__ __launch_bounds__(64 * NW) void block_step(StratArgs a)
{
    constexpr int RS = strat_row_stride(JP, BF ? 1 : 0);
    constexpr int NT = 64 * NW;
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    const int p = blockIdx.x, P = a.P;
    const int q = (p + a.s) % P;
    const int I3 = a.I3, J1 = a.J1, J2 = a.J2, J3 = a.J3, J12 = J1 * J2, ni = I3 * J12;
    const StratLds S = strat_lds_layout(JP, P, a.rows1_max, a.rows2_max, I3, J1, J2, J3, a.rec_cap, BF ? 1 : 0, NW);
    const TileLds L = tile_lds<JP>(lds, S);
    float* Cs = lds + S.c;
    float* Gs = lds + S.g;
    float* Hs = lds + S.h;
    float* Sk = lds + S.sk;
    for (int idx = tid; idx < a.rows1_max * RS; idx += NT) lds[S.a + idx] = 0.f;
    for (int idx = tid; idx < a.rows2_max * RS; idx += NT) lds[S.b + idx] = 0.f;
    __syncthreads();
    const int s1 = a.start1[p], r1 = a.start1[p + 1] - s1;
    const int s2 = a.start2[q], r2 = a.start2[q + 1] - s2;
    load_rows(L.Ab, a.Ap, s1, r1, J1, RS, tid, NT);
    load_rows(L.Bb, a.Bp, s2, r2, J2, RS, tid, NT);
    for (int l = tid; l < r1; l += NT) lds[S.ra + l] = a.reg1[s1 + l];
    for (int l = tid; l < r2; l += NT) lds[S.rb + l] = a.reg2[s2 + l];
    for (int idx = tid; idx < I3 * J3; idx += NT) Cs[idx] = a.C[idx];
    for (int idx = tid; idx < J12 * J3; idx += NT) Gs[idx] = a.G[idx];
    for (int idx = tid; idx < ni; idx += NT) Sk[idx] = 0.f;
    __syncthreads();
    if constexpr (BF) {
        clear_hb_pad<JP>(reinterpret_cast<__bf16*>(lds + S.hb), I3, tid, NT);
        build_h<JP>(nullptr, Cs, Gs, I3, J1, J2, J3, tid, NT, nullptr, reinterpret_cast<__bf16*>(lds + S.hb));
    } else {
        build_h<JP>(Hs, Cs, Gs, I3, J1, J2, J3, tid, NT, JP > 12 ? lds + S.ht : nullptr);
    }
    __syncthreads();
    const int t0 = a.blk_tile[p * P + q], t1 = a.blk_tile[p * P + q + 1];
    if constexpr (BF)
        block_tiles_bf<JP, NW>(a, t0, t1, L, tid, 0);
    else
        block_tiles<JP, NW>(a, t0, t1, L, tid, 0);
    store_rows(a.Ap, L.Ab, s1, r1, J1, RS, tid, NT);
    store_rows(a.Bp, L.Bb, s2, r2, J2, RS, tid, NT);
    __syncthreads();
    float* Sp = a.Spart + (size_t)p * ni;
    for (int idx = tid; idx < ni; idx += NT) Sp[idx] = Sk[idx];
}

struct CoreLds {
    int s, c, cgt, red, cst, total;
};

__host__ __device__ inline CoreLds core_lds_layout(int I3, int J1, int J2, int J3, int threads)
{
    CoreLds L;
    int o = 0;
    L.s = o;    o = up4(o + I3 * J1 * J2);
    L.c = o;    o = up4(o + I3 * J3);
    L.cgt = o;  o = up4(o + I3 * J3);
    L.red = o;  o = up4(o + threads);
    L.cst = o;  o = up4(o + kCstHead + I3);
    L.total = o;
    return L;
}

size_t core_lds_bytes(int I3, int J1, int J2, int J3, int threads)
{
    return align16(4 * (size_t)core_lds_layout(I3, J1, J2, J3, threads).total);
}

// One workgroup: the stratum reduction and the core step on C, G in HBM.
// New G values go to Gtmp first so that every C item still reads the old G.
__global__ __launch_bounds__(kCoreThreads) void core_step(StratArgs a, float* Gtmp)
{
    extern __shared__ float lds[];
    constexpr int NT = kCoreThreads;
    const int tid = threadIdx.x;
    const int P = a.P, I3 = a.I3, J1 = a.J1, J2 = a.J2, J3 = a.J3, J12 = J1 * J2, ni = I3 * J12;
    const CoreLds L = core_lds_layout(I3, J1, J2, J3, NT);
    float* S = lds + L.s;
    float* C0 = lds + L.c;
    float* cgt = lds + L.cgt;
    float* red = lds + L.red;
    float* cst = lds + L.cst;
    for (int idx = tid; idx < kCstHead + I3; idx += NT) cst[idx] = a.ccst[(size_t)a.s * (kCstHead + I3) + idx];
    for (int idx = tid; idx < I3 * J3; idx += NT) C0[idx] = a.C[idx];
    reduce_items(a.Spart, P, ni, 0, ni, S, red, tid, NT);
    core_update(C0, a.G, S, cst, I3, J12, J3, a.etac, cgt, Gtmp, tid, NT);
    __syncthreads();
    for (int idx = tid; idx < I3 * J3; idx += NT) a.C[idx] = cgt[idx];
    for (int idx = tid; idx < J12 * J3; idx += NT) a.G[idx] = Gtmp[idx];
}

// ---------------------------------------------------------------------------
// Network: one wavefront per gene row (position order).
//   mode 0: Bout[r] = Bin[r] - alpha (deg[r] Bin[r] - sum_nbr w Bin[nbr])
//   mode 1: net_part[r] = sum_nbr w |Bin[r] - Bin[nbr]|^2   (FP64)
// Lanes stride over the neighbours; a butterfly reduction (fixed order)
// combines the lanes.
// ---------------------------------------------------------------------------
template <int JP>
__global__ __launch_bounds__(256) void graph_rows(GraphArgs g, int mode)
{
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= g.I2) return;
    const int J2 = g.J2;
    const int e0 = g.adj_start[r], e1 = g.adj_start[r + 1];
    if (mode == 0) {
        float acc[JP];
#pragma unroll
        for (int c = 0; c < JP; ++c) acc[c] = 0.f;
        for (int e = e0 + lane; e < e1; e += 64) {
            const float w = g.adj_w[e];
            const float* bn = g.Bin + (size_t)g.adj_nbr[e] * J2;
#pragma unroll
            for (int c = 0; c < JP; ++c)
                if (c < J2) acc[c] = fmaf(w, bn[c], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < JP; ++c)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o);
        float mine = 0.f;
#pragma unroll
        for (int c = 0; c < JP; ++c)
            if (c == lane) mine = acc[c];
        if (lane < J2) {
            const float b = g.Bin[(size_t)r * J2 + lane];
            g.Bout[(size_t)r * J2 + lane] = fmaf(-g.alpha, fmaf(g.deg[r], b, -mine), b);
        }
    } else {
        double d = 0.0;
        const float* br = g.Bin + (size_t)r * J2;
        for (int e = e0 + lane; e < e1; e += 64) {
            const float* bn = g.Bin + (size_t)g.adj_nbr[e] * J2;
            double s = 0.0;
            for (int c = 0; c < J2; ++c) {
                const double t = (double)br[c] - (double)bn[c];
                s += t * t;
            }
            d += (double)g.adj_w[e] * s;
        }
        for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
        if (lane == 0) g.net_part[r] = d;
    }
}

// ---------------------------------------------------------------------------
// Loss: squared errors per block (FP32 model value, FP64 sums), L2 terms per
// row group, network term per gene row, then one workgroup adds each list in
// a fixed order.
// ---------------------------------------------------------------------------
struct LossLds {
    int a, b, c, g, h, red, total;
};

__host__ __device__ inline LossLds loss_lds_layout(int jp, int rows1_max, int rows2_max, int I3, int J1, int J2,
                                                   int J3)
{
    const int rs = row_stride(jp);
    LossLds L;
    int o = 0;
    L.a = o;   o = up4(o + rows1_max * rs);
    L.b = o;   o = up4(o + rows2_max * rs);
    L.c = o;   o = up4(o + I3 * J3);
    L.g = o;   o = up4(o + J1 * J2 * J3);
    L.h = o;   o = up4(o + I3 * jp * jp);
    L.red = o; o = up4(o + 2 * 256);
    L.total = o;
    return L;
}

size_t loss_lds_bytes(int jp, int rows1_max, int rows2_max, int I3, int J1, int J2, int J3)
{
    return align16(4 * (size_t)loss_lds_layout(jp, rows1_max, rows2_max, I3, J1, J2, J3).total);
}

// Sum over a 256-thread workgroup in a fixed order: a butterfly within each
// wavefront (both partners of a step add the same two values, so every lane
// ends with the same bits), then (w0 + w1) + (w2 + w3).
__device__ inline double block_sum_256(double v, double* red, int tid)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return r;
}

template <int JP>
__global__ __launch_bounds__(256) void loss_blocks(LossArgs a)
{
    constexpr int RS = row_stride(JP);
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    const int blk = blockIdx.x, p = blk / a.P, q = blk - p * a.P;
    const int t0 = a.blk_tile[blk], t1 = a.blk_tile[blk + 1];
    if (t0 >= t1) {
        if (tid == 0) a.sse_part[blk] = 0.0;
        return;
    }
    const int J1 = a.J1, J2 = a.J2, J3 = a.J3;
    const LossLds L = loss_lds_layout(JP, a.rows1_max, a.rows2_max, a.I3, J1, J2, J3);
    float* Ab = lds + L.a;
    float* Bb = lds + L.b;
    float* Cs = lds + L.c;
    float* Gs = lds + L.g;
    float* Hs = lds + L.h;
    double* red = reinterpret_cast<double*>(lds + L.red);
    for (int idx = tid; idx < (a.rows1_max + a.rows2_max) * RS; idx += 256) lds[L.a + idx] = 0.f;
    for (int idx = tid; idx < a.I3 * J3; idx += 256) Cs[idx] = a.C[idx];
    for (int idx = tid; idx < J1 * J2 * J3; idx += 256) Gs[idx] = a.G[idx];
    __syncthreads();
    const int s1 = a.start1[p], r1 = a.start1[p + 1] - s1;
    const int s2 = a.start2[q], r2 = a.start2[q + 1] - s2;
    load_rows(Ab, a.Ap, s1, r1, J1, RS, tid, 256);
    load_rows(Bb, a.Bp, s2, r2, J2, RS, tid, 256);
    build_h<JP>(Hs, Cs, Gs, a.I3, J1, J2, J3, tid, 256);
    __syncthreads();
    const uint32_t mask_i = (1u << a.bits_i) - 1u, mask_j = (1u << a.bits_j) - 1u;
    // one wavefront per tile: the tile's platform is uniform
    const int wave = tid >> 6, lane = tid & 63;
    double acc = 0.0;
    for (int tl = t0 + wave; tl < t1; tl += 4) {
        const int off = a.tile_off[tl], n = a.tile_off[tl + 1] - off, k = a.tile_k[tl];
        if (lane < n) {
            const uint2 wv = a.nz[off + lane];
            const int il = (int)(wv.x & mask_i), jl = (int)((wv.x >> a.bits_i) & mask_j);
            const float* H = Hs + k * JP * JP;
            float bv[JP];
#pragma unroll
            for (int y = 0; y < JP; ++y) bv[y] = Bb[jl * RS + y];
            float xt = 0.f;
#pragma unroll
            for (int x_ = 0; x_ < JP; ++x_) {
                float w1 = 0.f;
#pragma unroll
                for (int y = 0; y < JP; ++y) w1 = fmaf(H[x_ * JP + y], bv[y], w1);
                xt = fmaf(Ab[il * RS + x_], w1, xt);
            }
            const float e = __uint_as_float(wv.y) - xt;
            acc += (double)e * (double)e;
        }
    }
    const double s = block_sum_256(acc, red, tid);
    if (tid == 0) a.sse_part[blk] = s;
}

// The same sums of squared residuals, column by column: workgroup (q, part)
// keeps gene block q and first forms w1 = H_k b_j for every gene row of the
// block and every platform k (the values loss_blocks forms per nonzero, in
// the same operation order), then visits patient blocks p0..p1-1.  Per
// nonzero only x~ = a_i . w1 remains (JP instead of JP^2 + JP fused
// multiply-adds).  Tiles go to wavefronts and lanes as in loss_blocks and
// each block's sum is the same tree, so sse_part is bit-identical.
constexpr int kLossChunkTiles = 16;  // tiles whose records are staged at once

struct LossColLds {
    int w, a, u, b, h, g, c, to, tk, rec, red, total;
};

__host__ __device__ inline LossColLds loss_col_layout(int jp, int rows1_max, int rows2_max, int I3, int J1, int J2,
                                                      int J3)
{
    const int rl = up4(jp);  // row pitch: whole 16-byte vectors
    LossColLds L;
    int o = 0;
    L.w = o;   o = up4(o + rows2_max * I3 * rl);      // w1 per gene row and platform
    L.a = o;   o = up4(o + rows1_max * rl);           // patient rows of the current block
    L.c = o;   o = up4(o + I3 * J3);
    L.red = o; o = up4(o + 2 * 256);
    L.to = o;  o = up4(o + kLossChunkTiles + 1);      // the chunk's tile offsets
    L.tk = o;  o = up4(o + kLossChunkTiles);          // and platforms
    // set-up only (gene rows, H_k, G) and then the staged records
    const int setup = up4(rows2_max * jp) + up4(I3 * jp * jp) + up4(J1 * J2 * J3);
    const int recs = 2 * kLossChunkTiles * kTileMax;
    L.u = o;
    L.b = o;
    L.h = L.b + up4(rows2_max * jp);
    L.g = L.h + up4(I3 * jp * jp);
    L.rec = o;
    o = up4(o + (setup > recs ? setup : recs));
    L.total = o;
    return L;
}

size_t loss_cols_lds_bytes(int jp, int rows1_max, int rows2_max, int I3, int J1, int J2, int J3)
{
    return align16(4 * (size_t)loss_col_layout(jp, rows1_max, rows2_max, I3, J1, J2, J3).total);
}

template <int JP>
__global__ __launch_bounds__(256) void loss_cols(LossArgs a)
{
    constexpr int NT = 256;
    constexpr int RL = (JP + 3) & ~3;  // pitch of the w1 and patient rows (float4 reads)
    extern __shared__ float lds[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int P = a.P, q = blockIdx.x % P, part = blockIdx.x / P, nparts = gridDim.x / P;
    const int p0 = (int)(((long long)P * part) / nparts), p1 = (int)(((long long)P * (part + 1)) / nparts);
    const int I3 = a.I3, J1 = a.J1, J2 = a.J2, J3 = a.J3;
    const LossColLds L = loss_col_layout(JP, a.rows1_max, a.rows2_max, I3, J1, J2, J3);
    float* W = lds + L.w;
    float* Ab = lds + L.a;
    float* Bt = lds + L.b;
    float* Hs = lds + L.h;
    float* Gs = lds + L.g;
    float* Cs = lds + L.c;
    uint2* rec = reinterpret_cast<uint2*>(lds + L.rec);
    double* red = reinterpret_cast<double*>(lds + L.red);
    int* toff = reinterpret_cast<int*>(lds + L.to);
    int* tkk = reinterpret_cast<int*>(lds + L.tk);

    // set-up: gene rows (zero beyond J2), H_k, then w1 for every (row, k)
    for (int idx = tid; idx < a.rows1_max * RL; idx += NT) Ab[idx] = 0.f;
    for (int idx = tid; idx < a.rows2_max * JP; idx += NT) Bt[idx] = 0.f;
    for (int idx = tid; idx < I3 * J3; idx += NT) Cs[idx] = a.C[idx];
    for (int idx = tid; idx < J1 * J2 * J3; idx += NT) Gs[idx] = a.G[idx];
    __syncthreads();
    const int s2 = a.start2[q], r2 = a.start2[q + 1] - s2;
    load_rows(Bt, a.Bp, s2, r2, J2, JP, tid, NT);
    build_h<JP>(Hs, Cs, Gs, I3, J1, J2, J3, tid, NT);
    __syncthreads();
    for (int idx = tid; idx < r2 * I3 * JP; idx += NT) {
        const int l = idx / (I3 * JP), kx = idx - l * (I3 * JP), k = kx / JP, x = kx - k * JP;
        const float* H = Hs + (k * JP + x) * JP;
        const float* bv = Bt + l * JP;
        float w1 = 0.f;
#pragma unroll
        for (int y = 0; y < JP; ++y) w1 = fmaf(H[y], bv[y], w1);
        W[(l * I3 + k) * RL + x] = w1;
    }
    __syncthreads();

    const uint32_t mask_i = (1u << a.bits_i) - 1u, mask_j = (1u << a.bits_j) - 1u;
    for (int p = p0; p < p1; ++p) {
        const int blk = p * P + q;
        const int t0 = a.blk_tile[blk], t1 = a.blk_tile[blk + 1];
        if (t0 >= t1) {
            if (tid == 0) a.sse_part[blk] = 0.0;
            continue;
        }
        const int s1 = a.start1[p], r1 = a.start1[p + 1] - s1;
        // the block's patient rows and its first chunk's records in one
        // round of loads
        constexpr int kRowRegs = 4, kRecRegs = kLossChunkTiles * kTileMax / NT;
        const int nrow = r1 * J1;
        const bool rows_fit = nrow <= kRowRegs * NT;
        float rowv[kRowRegs];
        uint2 recv[kRecRegs];
        int tov = 0, tkv = 0;
        {
            const float* src = a.Ap + (size_t)s1 * J1;
#pragma unroll
            for (int h = 0; h < kRowRegs; ++h) {
                const int idx = tid + h * NT;
                rowv[h] = rows_fit && idx < nrow ? src[idx] : 0.f;
            }
            const int c1 = t0 + kLossChunkTiles < t1 ? t0 + kLossChunkTiles : t1;
            const int z0 = a.tile_off[t0], nrec = a.tile_off[c1] - z0;
#pragma unroll
            for (int h = 0; h < kRecRegs; ++h) {
                const int i = tid + h * NT;
                recv[h] = i < nrec ? a.nz[z0 + i] : make_uint2(0u, 0u);
            }
            if (tid <= c1 - t0) tov = a.tile_off[t0 + tid];
            if (tid < c1 - t0) tkv = a.tile_k[t0 + tid];
            if (rows_fit) {
#pragma unroll
                for (int h = 0; h < kRowRegs; ++h) {
                    const int idx = tid + h * NT;
                    if (idx < nrow) {
                        const int l = idx / J1, c = idx - l * J1;
                        Ab[l * RL + c] = rowv[h];
                    }
                }
            } else {
                load_rows(Ab, a.Ap, s1, r1, J1, RL, tid, NT);
            }
#pragma unroll
            for (int h = 0; h < kRecRegs; ++h) {
                const int i = tid + h * NT;
                if (i < nrec) rec[i] = recv[h];
            }
            if (tid <= c1 - t0) toff[tid] = tov;
            if (tid < c1 - t0) tkk[tid] = tkv;
        }
        double acc = 0.0;
        // wavefront w takes the tiles t0 + w, t0 + w + 4, ... (chunks hold a
        // multiple of four tiles)
        for (int c0 = t0; c0 < t1; c0 += kLossChunkTiles) {
            const int c1 = c0 + kLossChunkTiles < t1 ? c0 + kLossChunkTiles : t1;
            const int z0 = a.tile_off[c0], nrec = a.tile_off[c1] - z0;
            if (c0 > t0) {
                // the chunk's tile offsets and platforms in the same round as its records
                const int to_ = tid <= c1 - c0 ? a.tile_off[c0 + tid] : 0;
                const int tk_ = tid < c1 - c0 ? a.tile_k[c0 + tid] : 0;
                load_records(rec, a.nz + z0, nrec, tid, NT);
                if (tid <= c1 - c0) toff[tid] = to_;
                if (tid < c1 - c0) tkk[tid] = tk_;
            }
            __syncthreads();
            for (int tl = c0 + wave; tl < c1; tl += 4) {
                const int off = toff[tl - c0], n = toff[tl - c0 + 1] - off, k = tkk[tl - c0];
                if (lane < n) {
                    const uint2 wv = rec[off - z0 + lane];
                    const int il = (int)(wv.x & mask_i), jl = (int)((wv.x >> a.bits_i) & mask_j);
                    const float4* w4 = reinterpret_cast<const float4*>(W + (jl * I3 + k) * RL);
                    const float4* a4 = reinterpret_cast<const float4*>(Ab + il * RL);
                    float w1[RL], av[RL];
#pragma unroll
                    for (int v = 0; v < RL / 4; ++v) {
                        const float4 wq = w4[v], aq = a4[v];
                        w1[4 * v] = wq.x; w1[4 * v + 1] = wq.y; w1[4 * v + 2] = wq.z; w1[4 * v + 3] = wq.w;
                        av[4 * v] = aq.x; av[4 * v + 1] = aq.y; av[4 * v + 2] = aq.z; av[4 * v + 3] = aq.w;
                    }
                    float xt = 0.f;
#pragma unroll
                    for (int x_ = 0; x_ < JP; ++x_) xt = fmaf(av[x_], w1[x_], xt);
                    const float e = __uint_as_float(wv.y) - xt;
                    acc += (double)e * (double)e;
                }
            }
            __syncthreads();
        }
        const double s = block_sum_256(acc, red, tid);
        if (tid == 0) a.sse_part[blk] = s;
    }
}

// L2 terms: workgroups [0, nA) take patient rows, [nA, nA+nB) gene rows, the
// last one the platform rows and the core.
__global__ __launch_bounds__(256) void loss_reg(LossArgs a)
{
    __shared__ double red[256];
    const int tid = threadIdx.x, wg = blockIdx.x;
    const int nA = (a.I1 + 255) / 256, nB = (a.I2 + 255) / 256;
    double v = 0.0;
    if (wg < nA) {
        const int r = wg * 256 + tid;
        if (r < a.I1 && a.cnt1[r] > 0)
            for (int c = 0; c < a.J1; ++c) v += (double)a.Ap[(size_t)r * a.J1 + c] * a.Ap[(size_t)r * a.J1 + c];
    } else if (wg < nA + nB) {
        const int r = (wg - nA) * 256 + tid;
        if (r < a.I2 && a.cnt2[r] > 0)
            for (int c = 0; c < a.J2; ++c) v += (double)a.Bp[(size_t)r * a.J2 + c] * a.Bp[(size_t)r * a.J2 + c];
    } else {
        const int ng = a.J1 * a.J2 * a.J3;
        for (int t = tid; t < ng; t += 256) v += (double)a.G[t] * a.G[t];
        for (int r = tid; r < a.I3; r += 256)
            if (a.cnt3[r] > 0)
                for (int c = 0; c < a.J3; ++c) v += (double)a.C[(size_t)r * a.J3 + c] * a.C[(size_t)r * a.J3 + c];
    }
    const double s = block_sum_256(v, red, tid);
    if (tid == 0) a.reg_part[wg] = s;
}

__device__ double ordered_sum(const double* x, int n, double* red, int tid)
{
    double v = 0.0;
    for (int t = tid; t < n; t += 1024) v += x[t];
    red[tid] = v;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(1024) void loss_final(LossArgs a)
{
    __shared__ double red[1024];
    const int tid = threadIdx.x;
    const double sse = ordered_sum(a.sse_part, a.P * a.P, red, tid);
    const double reg = ordered_sum(a.reg_part, a.n_reg_wg, red, tid);
    const double net = a.lam_g > 0.0 ? 0.5 * ordered_sum(a.net_part, a.I2, red, tid) : 0.0;
    if (tid == 0) {
        a.out[0] = 0.5 * sse + 0.5 * a.lam * reg + 0.5 * a.lam_g * net;
        a.out[1] = sse;
    }
}

// Row permutation: gather dst[r] = src[perm[r]] or scatter dst[perm[r]] = src[r].
__global__ __launch_bounds__(256) void permute_rows(const float* src, float* dst, const int32_t* perm, int rows,
                                                    int cols, int gather)
{
    const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long long)rows * cols) return;
    const int r = (int)(idx / cols), c = (int)(idx - (long long)r * cols);
    const size_t pr = (size_t)perm[r] * cols + c;
    if (gather)
        dst[idx] = src[pr];
    else
        dst[pr] = src[idx];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
#define SNECT_JP_SWITCH(JPV, CALL)            \
    switch (JPV) {                            \
    case 2: return CALL(2);                   \
    case 4: return CALL(4);                   \
    case 5: return CALL(5);                   \
    case 8: return CALL(8);                   \
    case 10: return CALL(10);                 \
    case 12: return CALL(12);                 \
    case 16: return CALL(16);                 \
    case 20: return CALL(20);                 \
    case 24: return CALL(24);                 \
    case 32: return CALL(32);                 \
    default: return hipErrorInvalidValue;     \
    }

// Instantiation of a (JP, BF16?, wavefronts) variant of a stratum-kernel helper.
#define SNECT_VARIANT(F, J, ...) (bf ? F<J, true, kDefaultWaves>(__VA_ARGS__) : F<J, false, kDefaultWaves>(__VA_ARGS__))

template <int JP, bool BF, int NW>
static hipError_t launch_persistent_t(const StratArgs& a, size_t lds, hipStream_t st)
{
    StratArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&strata_persistent<JP, BF, NW>), dim3(a.P),
                                      dim3(64 * NW), args, (unsigned)lds, st);
}

hipError_t launch_strata_persistent(const StratArgs& a, int jp, int bf, int nw, size_t lds, hipStream_t st)
{
#define CALL_P(J) SNECT_VARIANT(launch_persistent_t, J, a, lds, st)
    SNECT_JP_SWITCH(jp, CALL_P)
#undef CALL_P
}

template <bool BF>
static hipError_t launch_sweep_t(const StratArgs* args, const int32_t* wg_start, int n, int nwg, size_t lds,
                                 hipStream_t st)
{
    void* kargs[] = {&args, &wg_start, &n};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&strata_sweep<BF>), dim3(nwg),
                                      dim3(64 * kDefaultWaves), kargs, (unsigned)lds, st);
}

hipError_t launch_strata_sweep(const StratArgs* args, const int32_t* wg_start, int n, int nwg, int bf, size_t lds,
                               hipStream_t st)
{
    return bf ? launch_sweep_t<true>(args, wg_start, n, nwg, lds, st)
              : launch_sweep_t<false>(args, wg_start, n, nwg, lds, st);
}

template <int JP, bool BF, int NW>
static hipError_t launch_block_t(const StratArgs& a, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL((block_step<JP, BF, NW>), dim3(a.P), dim3(64 * NW), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_block(const StratArgs& a, int jp, int bf, int nw, size_t lds, hipStream_t st)
{
#define CALL_B(J) SNECT_VARIANT(launch_block_t, J, a, lds, st)
    SNECT_JP_SWITCH(jp, CALL_B)
#undef CALL_B
}

hipError_t launch_core_step(const StratArgs& a, size_t lds, hipStream_t st)
{
    hipLaunchKernelGGL(core_step, dim3(1), dim3(kCoreThreads), lds, st, a, a.Ssum);
    return hipGetLastError();
}

template <int JP>
static hipError_t launch_graph_t(const GraphArgs& g, int mode, hipStream_t st)
{
    if (g.I2 == 0) return hipSuccess;
    hipLaunchKernelGGL(graph_rows<JP>, dim3((g.I2 + 3) / 4), dim3(256), 0, st, g, mode);
    return hipGetLastError();
}

hipError_t launch_graph_step(const GraphArgs& g, int jp, hipStream_t st)
{
#define CALL_G(J) launch_graph_t<J>(g, 0, st)
    SNECT_JP_SWITCH(jp, CALL_G)
#undef CALL_G
}

template <int JP>
static hipError_t launch_loss_t(const LossArgs& a, const GraphArgs& g, size_t lds, size_t lds_cols, int nparts,
                                hipStream_t st)
{
    if (lds_cols > 0)
        hipLaunchKernelGGL(loss_cols<JP>, dim3(a.P * nparts), dim3(256), lds_cols, st, a);
    else
        hipLaunchKernelGGL(loss_blocks<JP>, dim3(a.P * a.P), dim3(256), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(loss_reg, dim3(a.n_reg_wg), dim3(256), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.lam_g > 0.0) {
        e = launch_graph_t<JP>(g, 1, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(loss_final, dim3(1), dim3(1024), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_loss(const LossArgs& a, const GraphArgs& g, int jp, size_t lds, size_t lds_cols, int nparts,
                       hipStream_t st)
{
#define CALL_L(J) launch_loss_t<J>(a, g, lds, lds_cols, nparts, st)
    SNECT_JP_SWITCH(jp, CALL_L)
#undef CALL_L
}

hipError_t launch_permute(const float* src, float* dst, const int32_t* perm, int rows, int cols, int gather,
                          hipStream_t st)
{
    const long long n = (long long)rows * cols;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(permute_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, perm, rows,
                       cols, gather);
    return hipGetLastError();
}

template <int JP, bool BF, int NW>
static hipError_t prepare_strata_t(size_t slds)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&strata_persistent<JP, BF, NW>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)slds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&block_step<JP, BF, NW>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)slds);
    return e;
}

hipError_t prepare_sweep(int bf, size_t lds)
{
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(bf ? reinterpret_cast<const void*>(&strata_sweep<true>)
                                  : reinterpret_cast<const void*>(&strata_sweep<false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t prepare_strata(int jp, int bf, int nw, size_t slds)
{
    if (slds <= 65536) return hipSuccess;
#define CALL_S(J) SNECT_VARIANT(prepare_strata_t, J, slds)
    SNECT_JP_SWITCH(jp, CALL_S)
#undef CALL_S
}

template <int JP>
static hipError_t prepare_t(size_t llds, size_t clds, size_t lcols)
{
    hipError_t e = hipSuccess;
    const int limit = 65536;
    if (llds > (size_t)limit)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&loss_blocks<JP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)llds);
    if (e == hipSuccess && lcols > (size_t)limit)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&loss_cols<JP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lcols);
    if (e == hipSuccess && clds > (size_t)limit)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&core_step), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)clds);
    return e;
}

hipError_t prepare_kernels(int jp, size_t llds, size_t clds, size_t lcols)
{
#define CALL_R(J) prepare_t<J>(llds, clds, lcols)
    SNECT_JP_SWITCH(jp, CALL_R)
#undef CALL_R
}

template <int JP, bool BF, int NW>
static int capacity_t(size_t lds)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu,
                                                     reinterpret_cast<const void*>(&strata_persistent<JP, BF, NW>),
                                                     64 * NW, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * cus;
}

int sweep_capacity(int bf, size_t lds)
{
    int per_cu = 0;
    const void* fn = bf ? reinterpret_cast<const void*>(&strata_sweep<true>)
                        : reinterpret_cast<const void*>(&strata_sweep<false>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kDefaultWaves, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return per_cu * cus;
}

int persistent_capacity(int jp, int bf, int nw, size_t lds)
{
#define CALL_C(J) SNECT_VARIANT(capacity_t, J, lds)
    SNECT_JP_SWITCH(jp, CALL_C)
#undef CALL_C
}

}  // namespace snect
