// Orthonormalisation post-step of Algorithm 1 (last step: U(n) = Q R,
// U(n) <- Q, G <- G x_n R for every mode) on the GPU, in FP64 arithmetic on
// FP32 storage.
//
// Each tall factor U (I x J, J <= 32) is factored by CholeskyQR2: the Gram
// matrix W = U^T U is summed in FP64 over row blocks (fixed order), its
// Cholesky factor R1 (upper, positive diagonal) gives Q1 = U R1^{-1}; a
// second pass on Q1 gives Q = Q1 R2^{-1} and R = R2 R1.  R has a positive
// diagonal, which makes (Q, R) the unique QR factorisation of a full-rank U.
// The core then takes G <- G x_n R.
#include <hip/hip_runtime.h>

#include "snect_internal.h"

namespace snect {

constexpr int kQrRows = 128;  // rows per Gram block

// Partial Gram matrices: block b sums rows [b*kQrRows, ...) of U (or of the
// double-precision Q1 when U1 != nullptr), U^T U in FP64.
__global__ __launch_bounds__(256) void qr_gram_partial(const float* U, const double* U1, int I, int J,
                                                       double* part)
{
    __shared__ double rows[kQrRows * 33];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int r0 = b * kQrRows, nr = (I - r0) < kQrRows ? (I - r0) : kQrRows;
    for (int idx = tid; idx < nr * J; idx += 256) {
        const int r = idx / J, c = idx - r * J;
        rows[r * 33 + c] = U1 ? U1[(size_t)(r0 + r) * J + c] : (double)U[(size_t)(r0 + r) * J + c];
    }
    __syncthreads();
    for (int e = tid; e < J * J; e += 256) {
        const int x = e / J, y = e - x * J;
        double s = 0.0;
        for (int r = 0; r < nr; ++r) s += rows[r * 33 + x] * rows[r * 33 + y];
        part[(size_t)b * J * J + e] = s;
    }
}

// Sum of the partial Gram matrices (ascending block order), Cholesky
// W = R^T R (R upper, positive diagonal) and the inverse of R, in one
// workgroup.  status[0] = 1 when W is not positive definite.
__global__ __launch_bounds__(256) void qr_chol(const double* part, int nb, int J, double* R, double* Rinv,
                                              int* status)
{
    __shared__ double W[32 * 32];
    __shared__ double Rs[32 * 32];
    __shared__ double Ri[32 * 32];
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int e = tid; e < J * J; e += 256) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[(size_t)b * J * J + e];
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

// Q = U Rinv row by row (FP64); the result goes to Q64 (pass 1) or to the
// FP32 factor (pass 2).
__global__ __launch_bounds__(256) void qr_apply(const float* U, const double* U1, const double* Rinv, int I, int J,
                                               double* Q64, float* Q32)
{
    __shared__ double Ri[32 * 32];
    const int tid = threadIdx.x;
    for (int e = tid; e < J * J; e += 256) Ri[e] = Rinv[e];
    __syncthreads();
    const long long idx = (long long)blockIdx.x * 256 + tid;
    if (idx >= (long long)I * J) return;
    const int r = (int)(idx / J), c = (int)(idx - (long long)r * J);
    double s = 0.0;
    for (int i = 0; i <= c; ++i) {
        const double u = U1 ? U1[(size_t)r * J + i] : (double)U[(size_t)r * J + i];
        s += u * Ri[i * J + c];
    }
    if (Q64) Q64[idx] = s;
    if (Q32) Q32[idx] = (float)s;
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

size_t qr_scratch_bytes(int I, int J, int J1, int J2, int J3)
{
    const int nb = (I + kQrRows - 1) / kQrRows;
    return sizeof(double) * ((size_t)nb * J * J + 4 * (size_t)J * J + (size_t)I * J + (size_t)J1 * J2 * J3) + 64;
}

// One mode: U (I x J, device FP32) replaced by Q, G by G x_n R.  scratch
// holds qr_scratch_bytes(I, J, ...); status (device int) is set to 1 on a
// rank-deficient factor.
hipError_t launch_qr_mode(float* U, int I, int J, float* G, int J1, int J2, int J3, int mode, void* scratch,
                          int* status, hipStream_t st)
{
    const int nb = (I + kQrRows - 1) / kQrRows;
    double* part = static_cast<double*>(scratch);
    double* R1 = part + (size_t)nb * J * J;
    double* R1i = R1 + J * J;
    double* R2 = R1i + J * J;
    double* R2i = R2 + J * J;
    double* Q1 = R2i + J * J;
    double* gtmp = Q1 + (size_t)I * J;
    const unsigned gapply = (unsigned)(((long long)I * J + 255) / 256);
    hipLaunchKernelGGL(qr_gram_partial, dim3(nb), dim3(256), 0, st, U, nullptr, I, J, part);
    hipLaunchKernelGGL(qr_chol, dim3(1), dim3(256), 0, st, part, nb, J, R1, R1i, status);
    hipLaunchKernelGGL(qr_apply, dim3(gapply), dim3(256), 0, st, U, nullptr, R1i, I, J, Q1, nullptr);
    hipLaunchKernelGGL(qr_gram_partial, dim3(nb), dim3(256), 0, st, nullptr, Q1, I, J, part);
    hipLaunchKernelGGL(qr_chol, dim3(1), dim3(256), 0, st, part, nb, J, R2, R2i, status + 1);
    hipLaunchKernelGGL(qr_apply, dim3(gapply), dim3(256), 0, st, nullptr, Q1, R2i, I, J, nullptr, U);
    hipLaunchKernelGGL(qr_core, dim3(1), dim3(256), 0, st, R1, R2, G, J1, J2, J3, mode, gtmp);
    return hipGetLastError();
}

}  // namespace snect
