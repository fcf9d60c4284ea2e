// Orthonormalisation post-step of Algorithm 1 (last step: U(n) = Q R,
// U(n) <- Q, G <- G x_n R for every mode) on the GPU, in FP64 arithmetic on
// FP32 storage.
//
// Each tall factor U (I x J, J <= 32) is factored by CholeskyQR2: the Gram
// matrix W1 = U^T U is summed in FP64, its Cholesky factor R1 (upper,
// positive diagonal) gives Q1 = U R1^{-1}; a second pass on Q1 gives
// Q = Q1 R2^{-1} and R = R2 R1.  R has a positive diagonal, which makes
// (Q, R) the unique QR factorisation of a full-rank U.  The core then takes
// G <- G x_n R.
//
// Q1 is never stored: the second Gram pass and the final pass recompute the
// rows of U R1^{-1} in FP64 from U, block by block.  The scratch a mode
// needs is therefore independent of I: kQrParts partial Gram matrices, the
// triangular factors and the new core (qr_scratch_bytes).
#include <hip/hip_runtime.h>

#include "snect_internal.h"

namespace snect {

constexpr int kQrParts = 256;  // partial Gram matrices (row ranges) per pass
constexpr int kQrRows = 64;    // rows staged in LDS at a time
constexpr int kQrPad = 33;     // LDS row pitch (doubles)

// Rows [r0, r0 + nr) of U into LDS as FP64 (row pitch kQrPad); with Ri set,
// each row is replaced by its product with the upper-triangular Ri
// (q_c = sum_{i <= c} u_i Ri[i][c], ascending i).  tmp: kQrRows * kQrPad
// doubles of LDS.
__device__ void qr_stage_rows(const float* U, const double* Ri, int r0, int nr, int J, double* rows, double* tmp,
                              int tid)
{
    double* dst = Ri ? tmp : rows;
    for (int idx = tid; idx < nr * J; idx += 256) {
        const int r = idx / J, c = idx - r * J;
        dst[r * kQrPad + c] = (double)U[(size_t)(r0 + r) * J + c];
    }
    __syncthreads();
    if (Ri) {
        for (int idx = tid; idx < nr * J; idx += 256) {
            const int r = idx / J, c = idx - r * J;
            double s = 0.0;
            for (int i = 0; i <= c; ++i) s += tmp[r * kQrPad + i] * Ri[i * J + c];
            rows[r * kQrPad + c] = s;
        }
        __syncthreads();
    }
}

// Partial Gram matrices: workgroup b of the kQrParts sums the rows
// [b I / kQrParts, (b+1) I / kQrParts) of U (Ri == nullptr) or of U Ri,
// ascending, in FP64.  part[b][x][y] receives the sum.
__global__ __launch_bounds__(256) void qr_gram_partial(const float* U, const double* Ri, int I, int J, double* part)
{
    __shared__ double rows[kQrRows * kQrPad];
    __shared__ double tmp[kQrRows * kQrPad];
    __shared__ double ri[32 * 32];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int r0 = (int)(((long long)I * b) / kQrParts), r1 = (int)(((long long)I * (b + 1)) / kQrParts);
    if (Ri)
        for (int e = tid; e < J * J; e += 256) ri[e] = Ri[e];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // entries tid, tid + 256, ... of the J x J Gram
    for (int c0 = r0; c0 < r1; c0 += kQrRows) {
        const int nr = (r1 - c0) < kQrRows ? (r1 - c0) : kQrRows;
        __syncthreads();
        qr_stage_rows(U, Ri ? ri : nullptr, c0, nr, J, rows, tmp, tid);
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int e = tid + 256 * h;
            if (e < J * J) {
                const int x = e / J, y = e - x * J;
                double s = acc[h];
                for (int r = 0; r < nr; ++r) s += rows[r * kQrPad + x] * rows[r * kQrPad + y];
                acc[h] = s;
            }
        }
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        const int e = tid + 256 * h;
        if (e < J * J) part[(size_t)b * J * J + e] = acc[h];
    }
}

// Sum of the partial Gram matrices (ascending), Cholesky W = R^T R (R upper,
// positive diagonal) and the inverse of R, in one workgroup.  status[0] = 1
// when W is not positive definite, 0 otherwise.
__global__ __launch_bounds__(256) void qr_chol(const double* part, int J, double* R, double* Rinv, int* status)
{
    __shared__ double W[32 * 32];
    __shared__ double Rs[32 * 32];
    __shared__ double Ri[32 * 32];
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int e = tid; e < J * J; e += 256) {
        double s = 0.0;
        for (int b = 0; b < kQrParts; ++b) s += part[(size_t)b * J * J + e];
        W[e] = s;
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    if (tid == 0) {
        // Cholesky, row by row: R[k][k] = sqrt(W[k][k] - sum_i R[i][k]^2),
        // R[k][j] = (W[k][j] - sum_i R[i][k] R[i][j]) / R[k][k]
        for (int e = 0; e < J * J; ++e) Rs[e] = 0.0;
        for (int k = 0; k < J && !bad; ++k) {
            double d = W[k * J + k];
            for (int i = 0; i < k; ++i) d -= Rs[i * J + k] * Rs[i * J + k];
            if (!(d > 0.0)) {
                bad = 1;
                break;
            }
            const double rk = sqrt(d);
            Rs[k * J + k] = rk;
            for (int j = k + 1; j < J; ++j) {
                double v = W[k * J + j];
                for (int i = 0; i < k; ++i) v -= Rs[i * J + k] * Rs[i * J + j];
                Rs[k * J + j] = v / rk;
            }
        }
        // inverse of the upper-triangular R by back substitution, column by column
        for (int e = 0; e < J * J; ++e) Ri[e] = 0.0;
        if (!bad)
            for (int c = 0; c < J; ++c)
                for (int r = c; r >= 0; --r) {
                    double v = (r == c) ? 1.0 : 0.0;
                    for (int i = r + 1; i <= c; ++i) v -= Rs[r * J + i] * Ri[i * J + c];
                    Ri[r * J + c] = v / Rs[r * J + r];
                }
        status[0] = bad;
    }
    __syncthreads();
    for (int e = tid; e < J * J; e += 256) {
        R[e] = Rs[e];
        Rinv[e] = Ri[e];
    }
}

// Q = (U R1^{-1}) R2^{-1}, kQrRows rows per workgroup, in FP64, stored to U
// as FP32 (each workgroup reads and writes only its own rows).
__global__ __launch_bounds__(256) void qr_apply(float* U, const double* R1i, const double* R2i, int I, int J)
{
    __shared__ double rows[kQrRows * kQrPad];
    __shared__ double tmp[kQrRows * kQrPad];
    __shared__ double r1[32 * 32];
    __shared__ double r2[32 * 32];
    const int tid = threadIdx.x;
    for (int e = tid; e < J * J; e += 256) {
        r1[e] = R1i[e];
        r2[e] = R2i[e];
    }
    const int r0 = blockIdx.x * kQrRows, nr = (I - r0) < kQrRows ? (I - r0) : kQrRows;
    __syncthreads();
    qr_stage_rows(U, r1, r0, nr, J, rows, tmp, tid);
    for (int idx = tid; idx < nr * J; idx += 256) {
        const int r = idx / J, c = idx - r * J;
        double s = 0.0;
        for (int i = 0; i <= c; ++i) s += rows[r * kQrPad + i] * r2[i * J + c];
        U[(size_t)(r0 + r) * J + c] = (float)s;
    }
}

// R = R2 R1 (upper triangular products), then G <- G x_n R:
// G'[..., j, ...] = sum_i G[..., i, ...] R[j, i].  One workgroup.
__global__ __launch_bounds__(256) void qr_core(const double* R1, const double* R2, float* G, int J1, int J2, int J3,
                                              int mode, double* gtmp)
{
    __shared__ double R[32 * 32];
    const int tid = threadIdx.x;
    const int Jn = mode == 0 ? J1 : (mode == 1 ? J2 : J3);
    for (int e = tid; e < Jn * Jn; e += 256) {
        const int j = e / Jn, i = e - j * Jn;
        double s = 0.0;
        for (int t = 0; t < Jn; ++t) s += R2[j * Jn + t] * R1[t * Jn + i];
        R[e] = s;
    }
    __syncthreads();
    const int ng = J1 * J2 * J3;
    for (int e = tid; e < ng; e += 256) {
        const int a = e / (J2 * J3), b = (e / J3) % J2, c = e % J3;
        double s = 0.0;
        if (mode == 0)
            for (int i = 0; i < J1; ++i) s += (double)G[(i * J2 + b) * J3 + c] * R[a * J1 + i];
        else if (mode == 1)
            for (int i = 0; i < J2; ++i) s += (double)G[(a * J2 + i) * J3 + c] * R[b * J2 + i];
        else
            for (int i = 0; i < J3; ++i) s += (double)G[(a * J2 + b) * J3 + i] * R[c * J3 + i];
        gtmp[e] = s;
    }
    __syncthreads();
    for (int e = tid; e < ng; e += 256) G[e] = (float)gtmp[e];
}

// Clears the status words (a kernel, not a memset, so that the whole
// sequence can be captured in a graph).
__global__ void qr_clear_status(int* status, int n)
{
    if ((int)threadIdx.x < n) status[threadIdx.x] = 0;
}

// Scratch of one mode's factorisation: kQrParts partial Gram matrices,
// R1, R1^{-1}, R2, R2^{-1} (32 x 32 each) and the new core (32^3), FP64;
// independent of I.
size_t qr_scratch_bytes()
{
    return sizeof(double) * ((size_t)kQrParts * 32 * 32 + 4 * 32 * 32 + 32 * 32 * 32);
}

hipError_t launch_qr_clear(int* status, int n, hipStream_t st)
{
    hipLaunchKernelGGL(qr_clear_status, dim3(1), dim3(64), 0, st, status, n);
    return hipGetLastError();
}

// One mode: U (I x J, device FP32) replaced by Q, G by G x_n R.  scratch
// holds qr_scratch_bytes(); status[0..1] (device ints, cleared by the
// caller) are set to 1 when a pass finds the Gram matrix not positive
// definite (a rank-deficient factor).
hipError_t launch_qr_mode(float* U, int I, int J, float* G, int J1, int J2, int J3, int mode, void* scratch,
                          int* status, hipStream_t st)
{
    double* part = static_cast<double*>(scratch);
    double* R1 = part + (size_t)kQrParts * 32 * 32;
    double* R1i = R1 + 32 * 32;
    double* R2 = R1i + 32 * 32;
    double* R2i = R2 + 32 * 32;
    double* gtmp = R2i + 32 * 32;
    const unsigned gapply = (unsigned)((I + kQrRows - 1) / kQrRows);
    hipLaunchKernelGGL(qr_gram_partial, dim3(kQrParts), dim3(256), 0, st, U, nullptr, I, J, part);
    hipLaunchKernelGGL(qr_chol, dim3(1), dim3(256), 0, st, part, J, R1, R1i, status);
    hipLaunchKernelGGL(qr_gram_partial, dim3(kQrParts), dim3(256), 0, st, U, R1i, I, J, part);
    hipLaunchKernelGGL(qr_chol, dim3(1), dim3(256), 0, st, part, J, R2, R2i, status + 1);
    hipLaunchKernelGGL(qr_apply, dim3(gapply), dim3(256), 0, st, U, R1i, R2i, I, J);
    hipLaunchKernelGGL(qr_core, dim3(1), dim3(256), 0, st, R1, R2, G, J1, J2, J3, mode, gtmp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free orthonormalisation: one copy
// per device, kept until the process ends.  Host code never passes the
// symbol itself to a kernel; it takes the address hipGetSymbolAddress gives
// for the current device.
// ---------------------------------------------------------------------------
constexpr size_t kQrStaticBytes = sizeof(double) * ((size_t)kQrParts * 32 * 32 + 4 * 32 * 32 + 32 * 32 * 32) + 256;
static __device__ __align__(256) unsigned char scratch[kQrStaticBytes];

size_t qr_static_scratch_bytes() { return kQrStaticBytes; }

hipError_t qr_static_scratch_address(void** ptr)
{
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

}  // namespace snect
