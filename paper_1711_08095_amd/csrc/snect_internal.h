// Internal declarations shared by the host runtime (snect_host.cpp) and the
// gfx950 kernels (snect_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snect {

// Nonzero record in plan order: .x = packed word, .y = float bits of x.
// Packed word, from bit 0 up:
//   i_local  (bits_i)   row of the patient block
//   j_local  (bits_j)   row of the gene block
//   jprev    (6)        tile position of the previous nonzero with the same
//                       gene row, or its own position when there is none
//   jlast    (1)        this is the last nonzero of its gene row in the tile
constexpr int kJprevBits = 6;
constexpr int kWordFlagBits = kJprevBits + 1;
constexpr int kMaxLocalBits = 32 - kWordFlagBits;
constexpr int kTileMax = 64;  // one tile = one wavefront

// Core-size instantiations of the kernels: the smallest JP >= max(J1, J2).
constexpr int kJpSet[] = {2, 4, 5, 8, 10, 12, 16, 20, 24, 32};
constexpr int kJpCount = sizeof(kJpSet) / sizeof(kJpSet[0]);

__host__ __device__ constexpr int row_stride(int jp) { return (jp + 3) & ~3; }
__host__ __device__ constexpr int mfma_dim(int jp) { return jp <= 16 ? 16 : 32; }

// Arguments of the per-stratum block kernel.
struct BlockArgs {
    const uint2* nz;
    const int32_t* tile_off;   // [ntiles+1]
    const int32_t* tile_k;     // [ntiles]
    const int32_t* blk_tile;   // [P*P+1]
    const int32_t* perm1;      // position -> patient row
    const int32_t* start1;     // [P+1] first position of each patient block
    const int32_t* perm2;
    const int32_t* start2;
    const float* reg1;         // lambda / n1[row] (0 for empty rows)
    const float* reg2;
    float* A;
    float* B;
    const float* C;
    const float* G;
    float* Spart;              // [P][I3][J1*J2] per-block sums of e a (x) b
    int32_t* Mpart;            // [P][I3] per-block nonzero counts
    int32_t P, s, I3, J1, J2, J3;
    int32_t rows1_max, rows2_max;
    int32_t bits_i, bits_j;
    float lr;
};

// Arguments of the per-stratum core / platform step.
struct CoreArgs {
    float* C;
    float* G;
    const float* Spart;
    const int32_t* Mpart;
    const int32_t* cnt3;
    int32_t P, I3, J1, J2, J3;
    float lam, etac;
    double nnz;
};

// Arguments of the loss kernels.
struct LossArgs {
    const uint2* nz;
    const int32_t* tile_off;
    const int32_t* tile_k;
    const int32_t* blk_tile;
    const int32_t* perm1;
    const int32_t* start1;
    const int32_t* perm2;
    const int32_t* start2;
    const int32_t* cnt1;
    const int32_t* cnt2;
    const int32_t* cnt3;
    const float* A;
    const float* B;
    const float* C;
    const float* G;
    const int32_t* adj_start;
    const int32_t* adj_nbr;
    const float* adj_w;
    double* partial;           // [P*P]
    double* out;               // [2]: f_opt, sum of squared errors
    int32_t P, I1, I2, I3, J1, J2, J3;
    int32_t rows1_max, rows2_max;
    int32_t bits_i, bits_j;
    double lam, lam_g;
};

struct GraphArgs {
    const float* Bin;
    float* Bout;
    const int32_t* adj_start;
    const int32_t* adj_nbr;
    const float* adj_w;
    const float* deg;
    int32_t I2, J2;
    float alpha;
};

// LDS bytes of the block kernel for a given shape.
size_t block_lds_bytes(int jp, int rows1_max, int rows2_max, int I3, int J1, int J2);
size_t loss_lds_bytes(int jp, int rows1_max, int rows2_max, int I3);
int jp_for(int J1, int J2);

hipError_t launch_block_fp32(const BlockArgs& a, int jp, size_t lds, hipStream_t st);
hipError_t launch_core_step(const CoreArgs& a, hipStream_t st);
hipError_t launch_graph_step(const GraphArgs& a, hipStream_t st);
hipError_t launch_loss(const LossArgs& a, int jp, size_t lds, hipStream_t st);
hipError_t prepare_kernels(int jp, size_t block_lds, size_t loss_lds);

}  // namespace snect
