// Internal declarations shared by the host runtime (snect_host.cpp) and the
// gfx950 kernels (snect_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

// The opaque context of the C ABI.
struct snect_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    size_t max_lds = 65536;
    int num_cu = 0;
    int coop = 0;
    int live_problems = 0;  // problems and servers still referring to this context
    void* qr_static = nullptr;  // this device's fixed QR scratch (device address)
};

namespace snect {

// Nonzero record in plan order: .x = packed word, .y = float bits of x.
// Packed word, from bit 0 up:
//   i_local  (bits_i)   row of the patient block
//   j_local  (bits_j)   row of the gene block
//   jrank    (6)        slot of this nonzero in the tile's order by
//                       (j_local, position)
constexpr int kSlotBits = 6;
constexpr int kMaxLocalBits = 32 - kSlotBits;
constexpr int kTileMax = 64;    // one tile = one wavefront
constexpr int kTileCache = 256; // tile metadata entries cached in LDS
constexpr int kMaxRecCap = 2048; // largest record chunk staged in LDS
constexpr int kRedChunk = 16;   // blocks summed per chunk in the stratum reduce

// Core-size instantiations of the kernels: the smallest JP >= max(J1, J2).
constexpr int kJpSet[] = {2, 4, 5, 8, 10, 12, 16, 20, 24, 32};
constexpr int kJpCount = sizeof(kJpSet) / sizeof(kJpSet[0]);

__host__ __device__ constexpr int row_stride(int jp) { return (jp + 3) & ~3; }
// LDS row stride of the stratum kernels' factor rows: odd in the FP32 step,
// so that rows gathered by the lanes of a tile fall in different banks; a
// multiple of four in the BF16 step, whose operands are read 16 bytes at a
// time.
__host__ __device__ constexpr int strat_row_stride(int jp, int bf) { return bf ? ((jp + 3) & ~3) : (jp | 1); }
__host__ __device__ constexpr int mfma_dim(int jp) { return jp <= 16 ? 16 : 32; }

// Error word of the persistent kernel's exchange (zeroed before each launch;
// nonzero once a workgroup gave up waiting).
struct GridBar {
    unsigned int err;
    unsigned int pad[3];
};

// Everything the stratum kernels read or write.  Factor rows are in plan
// (position) order: row r of Ap is patient perm1[r]; block p owns rows
// start1[p] .. start1[p+1]-1.
struct StratArgs {
    const uint2* nz;
    const int32_t* tile_off;   // [ntiles+1]
    const int32_t* tile_k;     // [ntiles]
    const int32_t* blk_tile;   // [P*P+1]
    const int32_t* start1;     // [P+1]
    const int32_t* start2;     // [P+1]
    const float* reg1;         // lambda / n1, position order (0 for empty rows)
    const float* reg2;
    const int32_t* cnt3;       // n3[k]
    float* Ap;                 // [I1][J1] position order
    float* Bp;                 // [I2][J2] position order
    float* C;                  // [I3][J3]
    float* G;                  // [J1][J2][J3]
    float* Spart;              // [P][I3*J1*J2] per-block sums of e a (x) b
    const int32_t* blk_rec;    // [P*P+1] first record of each block (and nnz at the end)
    const float* ccst;         // [P][I3+3] core-step constants of each stratum (fixed by the plan)
    float* Ssum;               // [max(I3*J1*J2, J1*J2*J3)] the multi-launch core step's new G
    // persistent kernel: tagged exchange words (high half the stratum's tag,
    // low half a float): [P][I3*J1*J2] block sums, [I3*J1*J2] stratum sums,
    // [P] "rows stored" word of each patient block; stratum si of the launch
    // writes tag tag0 + si + 1
    unsigned long long* Sx;
    const int32_t* order;      // [P] stratum order of this epoch
    GridBar* bar;
    uint32_t tag0;
    uint32_t spin_limit;       // poll rounds before a wait gives up (0: the kernel's default)
    int32_t jp;                // kernel instantiation of this problem's core
    int32_t P, s, I3, J1, J2, J3;
    int32_t rows1_max, rows2_max;
    int32_t bits_i, bits_j;
    int32_t rec_cap;           // records staged in LDS per chunk (>= kTileMax)
    float lr, lam, etac;
    double nnz;
};

struct LossArgs {
    const uint2* nz;
    const int32_t* tile_off;
    const int32_t* tile_k;
    const int32_t* blk_tile;
    const int32_t* start1;
    const int32_t* start2;
    const int32_t* cnt1;       // position order
    const int32_t* cnt2;
    const int32_t* cnt3;
    const float* Ap;
    const float* Bp;
    const float* C;
    const float* G;
    const int32_t* adj_start;  // position order CSR
    const int32_t* adj_nbr;
    const float* adj_w;
    double* sse_part;          // [P*P]
    double* reg_part;          // [n_reg_wg]
    double* net_part;          // [I2]
    double* out;               // [2]: f_opt, sum of squared errors
    int32_t P, I1, I2, I3, J1, J2, J3;
    int32_t rows1_max, rows2_max;
    int32_t bits_i, bits_j;
    int32_t n_reg_wg;
    double lam, lam_g;
};

struct GraphArgs {
    const float* Bin;
    float* Bout;
    const int32_t* adj_start;
    const int32_t* adj_nbr;
    const float* adj_w;
    const float* deg;
    double* net_part;
    int32_t I2, J2;
    float alpha;
};

size_t strata_lds_bytes(int jp, int P, int rows1_max, int rows2_max, int I3, int J1, int J2, int J3, int rec_cap,
                        int bf, int nw);
// Per-stratum constants of the core step, from the counts m_k of the
// stratum's nonzeros on each platform k and m = sum_k m_k: [0] 1 if m > 0
// else 0, [1] (float)(1 / m), [2] lambda (float)(m / nnz),
// [3 + k] lambda (float)(m_k / n3[k]) (0 when m_k = 0).
constexpr int kCstHead = 3;
size_t loss_lds_bytes(int jp, int rows1_max, int rows2_max, int I3, int J1, int J2, int J3);
size_t loss_cols_lds_bytes(int jp, int rows1_max, int rows2_max, int I3, int J1, int J2, int J3);
size_t core_lds_bytes(int I3, int J1, int J2, int J3, int threads);
int jp_for(int J1, int J2);

// Persistent: one cooperative launch runs every stratum of one epoch.
hipError_t launch_strata_persistent(const StratArgs& a, int jp, int bf, int nw, size_t lds, hipStream_t st);
// Batched sweep: n problems in one cooperative launch of nwg workgroups of
// kDefaultWaves wavefronts (args and wg_start in device memory).
hipError_t launch_strata_sweep(const StratArgs* args, const int32_t* wg_start, int n, int nwg, int bf, size_t lds,
                               hipStream_t st);
hipError_t prepare_sweep(int bf, size_t lds);
// Fallback: one launch per stratum plus one core-step launch.  bf selects
// the BF16 matrix-core contractions of the tile step.
hipError_t launch_block(const StratArgs& a, int jp, int bf, int nw, size_t lds, hipStream_t st);
hipError_t launch_core_step(const StratArgs& a, size_t lds, hipStream_t st);
hipError_t launch_graph_step(const GraphArgs& a, int jp, hipStream_t st);
// lds_cols > 0: the column-wise loss kernel on P * nparts workgroups
hipError_t launch_loss(const LossArgs& a, const GraphArgs& g, int jp, size_t lds, size_t lds_cols, int nparts,
                       hipStream_t st);
hipError_t launch_permute(const float* src, float* dst, const int32_t* perm, int rows, int cols, int gather,
                          hipStream_t st);
hipError_t prepare_kernels(int jp, size_t loss_lds, size_t core_lds, size_t loss_cols_lds);
// Allows the stratum kernels of one variant more than 64 KB of LDS.
hipError_t prepare_strata(int jp, int bf, int nw, size_t strata_lds);
// Orthonormalisation of one mode (FP64 CholeskyQR2); see snect_qr.hip.
// Scratch of one mode (independent of the factor's row count).
size_t qr_scratch_bytes();
hipError_t launch_qr_mode(float* U, int I, int J, float* G, int J1, int J2, int J3, int mode, void* scratch,
                          int* status, hipStream_t st);
hipError_t launch_qr_clear(int* status, int n, hipStream_t st);
// The fixed per-device scratch of the allocation-free variant: its size
// (one mode's scratch plus 256 bytes of status words) and its address on the
// current device.
size_t qr_static_scratch_bytes();
hipError_t qr_static_scratch_address(void** ptr);
// Largest number of co-resident workgroups of the persistent kernel.
int persistent_capacity(int jp, int bf, int nw, size_t lds);
// Largest number of co-resident workgroups of the batched sweep kernel.
int sweep_capacity(int bf, size_t lds);

// Wavefronts per stratum workgroup (4 or 8; factor columns are shared
// among them); four of them accumulate the block's S on the matrix cores.
constexpr int kDefaultWaves = 8;
constexpr int kMfmaWaves = 4;
// Workgroups that share one fold-in request's Gram sums (at most).
constexpr int kServeMaxParts = 256;
// The batched sweep launch (snect_sweep_train) is switched off: after the
// LDS layout lost its per-wavefront S partials, its first run took a GPU
// memory-aperture fault that single-problem launches of the same stratum
// code never showed, and no cause has been established.  The sweep kernel
// calls the stratum body as a function (its LDS accesses are flat), which
// the single-problem kernels inline; that difference is a suspicion only.
constexpr bool kSweepEnabled = false;
constexpr int kCoreThreads = 1024;

}  // namespace snect
