// Host runtime of the SNeCT engine: input validation, the stratified plan,
// device residency, the epoch launch sequence and the C ABI of snect.h.
//
// Plan (Algorithm 1's random order replaced by a seeded, deterministic
// schedule): SplitMix64 streams (Steele, Lea & Flood 2014) drive Fisher-Yates
// shuffles of the patient rows (stream 0), the gene rows (stream 1) and, for
// epoch e, the P strata (stream 2 + e).  Stream t of a seed starts from the
// t-th output of SplitMix64 seeded with that seed; a shuffle of n items walks
// r = n-1 .. 1 and swaps item r with item floor(u (r+1) / 2^64) for the next
// 64-bit draw u.  Position r of a permutation belongs to block
// floor(r P / I).  Each block's nonzeros are sorted by (k, i, j) and cut into
// tiles of at most T entries within one platform.
//
// On the device the factor rows live in plan (position) order for the whole
// of a training call, so every block's rows are one contiguous range; they
// are gathered from and scattered back to the caller's row order at the
// start and the end of the call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/snect.h"
#include "snect_internal.h"

using namespace snect;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

int set_err(snect_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

uint64_t sm64_next(uint64_t& s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

// Output number n (0-based) of SplitMix64 seeded with `seed`: the state
// after n + 1 steps is seed + (n + 1) * gamma, then the finaliser.
uint64_t sm64_at(uint64_t seed, uint64_t n)
{
    uint64_t s = seed + n * 0x9e3779b97f4a7c15ULL;
    return sm64_next(s);
}

// Stream t of a seed starts from output t of SplitMix64(seed).
uint64_t stream_start(uint64_t seed, uint64_t stream) { return sm64_at(seed, stream); }

// Stream of the default random initialisation (far from the plan's streams
// 0, 1 and 2 + epoch).
constexpr uint64_t kInitStream = uint64_t(1) << 40;

void seeded_shuffle(std::vector<int32_t>& v, uint64_t seed, uint64_t stream)
{
    uint64_t s = stream_start(seed, stream);
    for (int64_t r = (int64_t)v.size() - 1; r >= 1; --r) {
        const uint64_t u = sm64_next(s);
        const int64_t j = (int64_t)(((unsigned __int128)u * (unsigned __int128)(uint64_t)(r + 1)) >> 64);
        std::swap(v[r], v[j]);
    }
}

std::vector<int32_t> stratum_order(int P, uint64_t seed, int64_t epoch)
{
    std::vector<int32_t> o(P);
    for (int s = 0; s < P; ++s) o[s] = s;
    seeded_shuffle(o, seed, 2 + (uint64_t)epoch);
    return o;
}

int ceil_log2(int64_t n)
{
    int b = 0;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

template <class F>
void parallel_for(int64_t n, F&& f)
{
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<int64_t>(std::max(1u, std::min(hw, 16u)), std::max<int64_t>(1, n));
    if (nt <= 1 || n < 64) {
        for (int64_t t = 0; t < n; ++t) f(t, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    const int64_t chunk = std::max<int64_t>(1, n / (nt * 16));
    for (int w = 0; w < nt; ++w)
        th.emplace_back([&, w]() {
            for (;;) {
                const int64_t s = next.fetch_add(chunk);
                if (s >= n) break;
                const int64_t e = std::min(n, s + chunk);
                for (int64_t t = s; t < e; ++t) f(t, w);
            }
        });
    for (auto& t : th) t.join();
}

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct snect_problem {
    snect_ctx* ctx = nullptr;
    // shape and parameters
    int32_t I1 = 0, I2 = 0, I3 = 0, J1 = 0, J2 = 0, J3 = 0, P = 1, T = 1, jp = 0, bf = 0;
    int64_t nnz = 0, ntiles = 0, ecsr = 0;
    double lam = 0, lam_g = 0, lr = 0, cls = 1;
    uint64_t seed = 0;
    int32_t rows1_max = 0, rows2_max = 0, bits_i = 0, bits_j = 0, n_sub = 0, n_reg_wg = 0;
    double dmax = 0;
    size_t strata_lds = 0, block_lds = 0, loss_lds = 0, core_lds = 0;
    size_t loss_cols_lds = 0;  // column-wise loss kernel (0: per-block kernel)
    int loss_parts = 1;        // workgroups per gene block of the column-wise loss kernel
    int capacity = 0;
    int rec_cap = kMaxRecCap;       // records staged per LDS chunk
    int rec_cap_max = kMaxRecCap;   // the largest that fits
    int sweep_rec_cap = 0;    // record chunk inside a batched sweep (0: rec_cap_max)
    int nw = kDefaultWaves;   // wavefronts per stratum workgroup
    double plan_s = 0, upload_s = 0;
    std::vector<int32_t> perm1, perm2;  // host copies kept for export
    // device buffers
    std::vector<DevBuf> bufs;
    uint2* d_nz = nullptr;
    int32_t *d_tile_off = nullptr, *d_tile_k = nullptr, *d_blk_tile = nullptr;
    int32_t *d_perm1 = nullptr, *d_start1 = nullptr, *d_perm2 = nullptr, *d_start2 = nullptr;
    float *d_reg1 = nullptr, *d_reg2 = nullptr;
    int32_t *d_cnt1 = nullptr, *d_cnt2 = nullptr, *d_cnt3 = nullptr;
    int32_t *d_adj_start = nullptr, *d_adj_nbr = nullptr;
    float *d_adj_w = nullptr, *d_deg = nullptr;
    float *d_Ap = nullptr, *d_Bp = nullptr, *d_Btmp = nullptr;
    float *d_Spart = nullptr, *d_Ssum = nullptr;
    unsigned long long* d_Sx = nullptr;  // the persistent kernel's tagged exchange words
    uint32_t tag_next = 0;               // tags handed out so far (see take_tags)
    int32_t wait_limit = 0;              // snect_exec.wait_limit
    int32_t* d_blk_rec = nullptr;  // [P*P+1] first record of each block
    float* d_ccst = nullptr;       // [P][kCstHead+I3] core-step constants per stratum
    int32_t* d_order = nullptr;  // [P]
    GridBar* d_bar = nullptr;
    double *d_sse = nullptr, *d_regp = nullptr, *d_net = nullptr, *d_lossout = nullptr;
    // Per-epoch state comes in two slots (epoch parity), so that the next
    // epoch can be queued before the previous one is checked.
    double* h_lossout = nullptr;  // pinned [2][2]: f_opt, sum of squared errors
    GridBar* h_bar = nullptr;     // pinned [2]: the exchange's error word after the epoch
    int32_t* h_order = nullptr;   // pinned [2][P]
    float *d_bakA = nullptr, *d_bakB = nullptr, *d_bakC = nullptr, *d_bakG = nullptr;  // [2] each
    // execution
    int path = SNECT_PATH_AUTO;
    bool per_launch = false;
    hipStream_t stream_override = nullptr;  // a sweep's per-problem stream (else the context's)
    hipEvent_t ev[2][4] = {{nullptr, nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr, nullptr}};
    std::vector<hipEvent_t> evl;  // per-launch timing events, [2][2 * launches]
    double t_ms[5] = {0, 0, 0, 0, 0};

    template <class T_>
    T_* alloc(size_t count, int& rc)
    {
        DevBuf b;
        b.bytes = std::max<size_t>(count * sizeof(T_), 16);
        if (hipMalloc(&b.p, b.bytes) != hipSuccess) {
            rc = SNECT_E_OOM;
            (void)hipGetLastError();
            return nullptr;
        }
        bufs.push_back(b);
        return static_cast<T_*>(b.p);
    }
    ~snect_problem()
    {
        for (auto& b : bufs) (void)hipFree(b.p);
        if (h_lossout) (void)hipHostFree(h_lossout);
        if (h_bar) (void)hipHostFree(h_bar);
        if (h_order) (void)hipHostFree(h_order);
        for (auto& es : ev)
            for (auto& e : es)
                if (e) (void)hipEventDestroy(e);
        for (auto& e : evl)
            if (e) (void)hipEventDestroy(e);
    }
    bool persistent_ok() const { return ctx->coop && capacity >= P && strata_lds <= ctx->max_lds; }
    int chosen_path() const
    {
        if (path == SNECT_PATH_MULTI) return SNECT_PATH_MULTI;
        if (path == SNECT_PATH_PERSISTENT) return SNECT_PATH_PERSISTENT;
        return persistent_ok() ? SNECT_PATH_PERSISTENT : SNECT_PATH_MULTI;
    }
};

// Wavefronts per workgroup and records per LDS chunk of the stratum kernels
// (execution choices: results do not depend on them).  Sets the LDS size,
// allows it for the chosen variant and counts the co-resident workgroups.
static hipError_t configure_exec(snect_problem* pr, int nw, int rec_cap)
{
    const size_t slds = strata_lds_bytes(pr->jp, pr->P, pr->rows1_max, pr->rows2_max, pr->I3, pr->J1, pr->J2,
                                         pr->J3, rec_cap, pr->bf, nw);
    if (slds > pr->ctx->max_lds) return hipErrorInvalidValue;
    const hipError_t e = prepare_strata(pr->jp, pr->bf, nw, slds);
    if (e != hipSuccess) return e;
    pr->nw = nw;
    pr->rec_cap = rec_cap;
    pr->strata_lds = pr->block_lds = slds;
    pr->capacity = pr->ctx->coop ? persistent_capacity(pr->jp, pr->bf, nw, slds) : 0;
    return hipSuccess;
}

#define HIP_TRY_CTX(C, call)                                                                  \
    do {                                                                                       \
        hipError_t _e = (call);                                                                \
        if (_e != hipSuccess)                                                                  \
            return set_err((C), SNECT_E_HIP, std::string(#call ": ") + hipGetErrorString(_e)); \
    } while (0)

#define HIP_TRY(call)                                                                          \
    do {                                                                                       \
        hipError_t _e = (call);                                                                \
        if (_e != hipSuccess)                                                                  \
            return set_err(ctx, SNECT_E_HIP, std::string(#call ": ") + hipGetErrorString(_e)); \
    } while (0)

// Device address of the fixed QR scratch on each device, looked up once per
// device (with that device current) by the first snect_create on it.
static std::mutex g_qr_mu;
static void* g_qr_static[256] = {};

static hipError_t qr_static_for(int device, void** ptr)
{
    std::lock_guard<std::mutex> lk(g_qr_mu);
    if (device < 0 || device >= 256) return hipErrorInvalidDevice;
    if (!g_qr_static[device]) {
        void* p = nullptr;
        const hipError_t e = qr_static_scratch_address(&p);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_qr_static[device] = p;
    }
    *ptr = g_qr_static[device];
    return hipSuccess;
}

extern "C" {

int snect_create(snect_ctx** out, int device, void* stream)
{
    if (!out) return SNECT_E_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return SNECT_E_ARG;
    }
    snect_ctx* c = new (std::nothrow) snect_ctx();
    if (!c) return SNECT_E_OOM;
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return SNECT_E_HIP;
    }
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && v > 0)
        c->max_lds = (size_t)v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess) c->num_cu = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, device) == hipSuccess) c->coop = v;
    if (qr_static_for(device, &c->qr_static) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return SNECT_E_HIP;
    }
    *out = c;
    return SNECT_OK;
}

int snect_destroy(snect_ctx* ctx)
{
    if (!ctx) return SNECT_E_ARG;
    if (ctx->live_problems > 0) return set_err(ctx, SNECT_E_BUSY, "destroy the context's problems first");
    delete ctx;
    return SNECT_OK;
}

const char* snect_last_error(const snect_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int snect_problem_create(snect_ctx* ctx, const snect_tensor* X, const snect_graph* Y, const snect_params* pa,
                         snect_problem** out)
{
    if (!ctx) return SNECT_E_ARG;
    ctx->err.clear();
    if (!X || !pa || !out) return set_err(ctx, SNECT_E_ARG, "null argument");
    *out = nullptr;
    const double t_plan0 = now_s();
    // ---------------- validation ----------------
    if (X->I1 <= 0 || X->I2 <= 0 || X->I3 <= 0) return set_err(ctx, SNECT_E_ARG, "tensor dims must be positive");
    if (X->nnz < 0 || X->nnz >= (int64_t(1) << 31)) return set_err(ctx, SNECT_E_ARG, "nnz out of range");
    if (X->nnz > 0 && (!X->i || !X->j || !X->k || !X->x)) return set_err(ctx, SNECT_E_ARG, "null tensor array");
    if (pa->J1 < 1 || pa->J2 < 1 || pa->J3 < 1 || pa->J1 > SNECT_MAX_RANK || pa->J2 > SNECT_MAX_RANK ||
        pa->J3 > SNECT_MAX_RANK)
        return set_err(ctx, SNECT_E_RANK, "core size must be in 1..32");
    if (!(pa->lambda >= 0) || !(pa->lambda_g >= 0) || !(pa->lr > 0) || !(pa->core_lr_scale >= 0) ||
        !std::isfinite(pa->lambda) || !std::isfinite(pa->lambda_g) || !std::isfinite(pa->lr) ||
        !std::isfinite(pa->core_lr_scale))
        return set_err(ctx, SNECT_E_ARG, "lambda, lambda_g, core_lr_scale must be >= 0 and lr > 0");
    if (pa->strata_P < 1 || pa->strata_P > X->I1 || pa->strata_P > X->I2)
        return set_err(ctx, SNECT_E_ARG, "strata_P must be in 1..min(I1, I2)");
    if (pa->tile_T < 1 || pa->tile_T > SNECT_MAX_TILE) return set_err(ctx, SNECT_E_ARG, "tile_T must be in 1..64");
    if (pa->precision != SNECT_PRECISION_FP32 && pa->precision != SNECT_PRECISION_BF16)
        return set_err(ctx, SNECT_E_ARG, "unknown precision");
    const int64_t E = Y ? Y->E : 0;
    if (E < 0 || E >= (int64_t(1) << 30)) return set_err(ctx, SNECT_E_ARG, "edge count out of range");
    if (E > 0 && (!Y->u || !Y->v)) return set_err(ctx, SNECT_E_ARG, "null edge array");
    const int32_t I1 = X->I1, I2 = X->I2, I3 = X->I3;
    const int64_t nnz = X->nnz;
    for (int64_t t = 0; t < nnz; ++t) {
        if (X->i[t] < 0 || X->i[t] >= I1 || X->j[t] < 0 || X->j[t] >= I2 || X->k[t] < 0 || X->k[t] >= I3)
            return set_err(ctx, SNECT_E_INDEX, "nonzero " + std::to_string(t) + " has a coordinate out of range");
        if (!std::isfinite(X->x[t])) return set_err(ctx, SNECT_E_ARG, "non-finite value at nonzero " + std::to_string(t));
    }
    for (int64_t e = 0; e < E; ++e) {
        if (Y->u[e] < 0 || Y->u[e] >= I2 || Y->v[e] < 0 || Y->v[e] >= I2)
            return set_err(ctx, SNECT_E_INDEX, "edge " + std::to_string(e) + " endpoint out of range");
        if (Y->u[e] == Y->v[e]) return set_err(ctx, SNECT_E_ARG, "self-loop at edge " + std::to_string(e));
        if (Y->w && (!(Y->w[e] >= 0) || !std::isfinite(Y->w[e])))
            return set_err(ctx, SNECT_E_ARG, "edge weights must be finite and >= 0");
    }
    const int P = pa->strata_P, T = pa->tile_T;
    const int J1 = pa->J1, J2 = pa->J2, J3 = pa->J3;
    const int jp = jp_for(J1, J2);
    if (jp < 0) return set_err(ctx, SNECT_E_RANK, "no kernel for this core size");
    const int rows1_max = (I1 + P - 1) / P, rows2_max = (I2 + P - 1) / P;
    const int bits_i = std::max(1, ceil_log2(rows1_max)), bits_j = std::max(1, ceil_log2(rows2_max));
    if (bits_i + bits_j > kMaxLocalBits)
        return set_err(ctx, SNECT_E_UNSUPPORTED, "blocks too large to pack; raise strata_P");
    if (I3 > 4096) return set_err(ctx, SNECT_E_UNSUPPORTED, "at most 4096 platforms");
    if ((int64_t)P * P * I3 >= (int64_t(1) << 31)) return set_err(ctx, SNECT_E_UNSUPPORTED, "too many blocks");
    const int bf = pa->precision == SNECT_PRECISION_BF16 ? 1 : 0;
    // the largest record chunk that still fits in LDS
    int rec_cap = kMaxRecCap;
    while (rec_cap > kTileMax &&
           strata_lds_bytes(jp, P, rows1_max, rows2_max, I3, J1, J2, J3, rec_cap, bf, 8) > ctx->max_lds)
        rec_cap /= 2;
    const size_t slds = strata_lds_bytes(jp, P, rows1_max, rows2_max, I3, J1, J2, J3, rec_cap, bf, 8);
    const size_t blds = slds;
    const size_t llds = loss_lds_bytes(jp, rows1_max, rows2_max, I3, J1, J2, J3);
    const size_t clds = core_lds_bytes(I3, J1, J2, J3, kCoreThreads);
    if (blds > ctx->max_lds || llds > ctx->max_lds || clds > ctx->max_lds)
        return set_err(ctx, SNECT_E_UNSUPPORTED,
                       "a block's rows and the core do not fit in LDS (" + std::to_string(blds) +
                           " bytes); raise strata_P");

    snect_problem* pr = new (std::nothrow) snect_problem();
    if (!pr) return set_err(ctx, SNECT_E_OOM, "host allocation");
    pr->ctx = ctx;
    pr->I1 = I1; pr->I2 = I2; pr->I3 = I3;
    pr->J1 = J1; pr->J2 = J2; pr->J3 = J3;
    pr->P = P; pr->T = T; pr->jp = jp; pr->bf = bf; pr->nnz = nnz;
    pr->lam = pa->lambda; pr->lam_g = pa->lambda_g; pr->lr = pa->lr; pr->cls = pa->core_lr_scale;
    pr->seed = pa->seed;
    pr->rows1_max = rows1_max; pr->rows2_max = rows2_max; pr->bits_i = bits_i; pr->bits_j = bits_j;
    pr->strata_lds = slds; pr->block_lds = blds; pr->loss_lds = llds; pr->core_lds = clds;
    {
        // the column-wise loss kernel when a gene block's w1 table fits
        // comfortably in LDS; as many workgroups as are resident at once (at
        // most 4 per CU, 1,024 in all), so each gene block's table is built
        // no more often than the workgroups can run together
        const size_t lc = loss_cols_lds_bytes(jp, rows1_max, rows2_max, I3, J1, J2, J3);
        pr->loss_cols_lds = (lc <= (size_t)96 * 1024 && lc <= ctx->max_lds) ? lc : 0;
        const int per_cu = lc > 0 ? std::max(1, std::min(4, (int)(ctx->max_lds / lc))) : 4;
        const int resident = ctx->num_cu > 0 ? std::min(1024, ctx->num_cu * per_cu) : 1024;
        pr->loss_parts = std::max(1, std::min(P, resident / P));
    }
    pr->rec_cap = rec_cap;
    pr->rec_cap_max = rec_cap;
    pr->n_reg_wg = (I1 + 255) / 256 + (I2 + 255) / 256 + 1;

    int rc = SNECT_OK;
    try {
        // ---------------- slice counts ----------------
        std::vector<int32_t> cnt1(I1, 0), cnt2(I2, 0), cnt3(I3, 0);
        for (int64_t t = 0; t < nnz; ++t) {
            cnt1[X->i[t]]++;
            cnt2[X->j[t]]++;
            cnt3[X->k[t]]++;
        }
        // ---------------- permutations and blocks ----------------
        pr->perm1.resize(I1);
        pr->perm2.resize(I2);
        for (int r = 0; r < I1; ++r) pr->perm1[r] = r;
        for (int r = 0; r < I2; ++r) pr->perm2[r] = r;
        seeded_shuffle(pr->perm1, pa->seed, 0);
        seeded_shuffle(pr->perm2, pa->seed, 1);
        std::vector<int32_t> pos1(I1), pos2(I2), blk1(I1), blk2(I2), start1(P + 1), start2(P + 1);
        for (int p = 0; p <= P; ++p) {
            start1[p] = (int32_t)(((int64_t)p * I1 + P - 1) / P);
            start2[p] = (int32_t)(((int64_t)p * I2 + P - 1) / P);
        }
        for (int64_t r = 0; r < I1; ++r) {
            pos1[pr->perm1[r]] = (int32_t)r;
            blk1[pr->perm1[r]] = (int32_t)(r * P / I1);
        }
        for (int64_t r = 0; r < I2; ++r) {
            pos2[pr->perm2[r]] = (int32_t)r;
            blk2[pr->perm2[r]] = (int32_t)(r * P / I2);
        }
        // per-row data in position order
        std::vector<float> reg1p(I1), reg2p(I2);
        std::vector<int32_t> cnt1p(I1), cnt2p(I2);
        for (int r = 0; r < I1; ++r) {
            const int32_t row = pr->perm1[r];
            cnt1p[r] = cnt1[row];
            reg1p[r] = cnt1[row] ? (float)(pa->lambda / cnt1[row]) : 0.f;
        }
        for (int r = 0; r < I2; ++r) {
            const int32_t row = pr->perm2[r];
            cnt2p[r] = cnt2[row];
            reg2p[r] = cnt2[row] ? (float)(pa->lambda / cnt2[row]) : 0.f;
        }
        // ---------------- bucket by (block, k), sort by (i, j) ----------------
        const int64_t nb = (int64_t)P * P * I3;
        std::vector<int64_t> bstart(nb + 1, 0);
        std::vector<int32_t> ord(nnz);
        {
            std::vector<int32_t> bucket(nnz);
            for (int64_t t = 0; t < nnz; ++t) {
                const int64_t b = ((int64_t)blk1[X->i[t]] * P + blk2[X->j[t]]) * I3 + X->k[t];
                bucket[t] = (int32_t)b;
                bstart[b + 1]++;
            }
            for (int64_t b = 0; b < nb; ++b) bstart[b + 1] += bstart[b];
            std::vector<int64_t> fill(bstart.begin(), bstart.end() - 1);
            for (int64_t t = 0; t < nnz; ++t) ord[fill[bucket[t]]++] = (int32_t)t;
        }
        std::atomic<int> dup{0};
        parallel_for(nb, [&](int64_t b, int) {
            const int64_t s = bstart[b], e = bstart[b + 1];
            if (e - s < 2) return;
            std::vector<std::pair<int64_t, int32_t>> kv(e - s);
            for (int64_t t = s; t < e; ++t) kv[t - s] = {(int64_t)X->i[ord[t]] * I2 + X->j[ord[t]], ord[t]};
            std::sort(kv.begin(), kv.end());
            for (size_t u = 1; u < kv.size(); ++u)
                if (kv[u].first == kv[u - 1].first) dup.store(1);
            for (int64_t t = s; t < e; ++t) ord[t] = kv[t - s].second;
        });
        if (dup.load()) {
            delete pr;
            return set_err(ctx, SNECT_E_DUPLICATE, "duplicate (i,j,k) coordinate");
        }
        // ---------------- tiles ----------------
        std::vector<int64_t> tiles_in_bucket(nb + 1, 0);
        for (int64_t b = 0; b < nb; ++b)
            tiles_in_bucket[b + 1] = tiles_in_bucket[b] + (bstart[b + 1] - bstart[b] + T - 1) / T;
        const int64_t ntiles = tiles_in_bucket[nb];
        if (ntiles >= (int64_t(1) << 31)) {
            delete pr;
            return set_err(ctx, SNECT_E_UNSUPPORTED, "too many tiles");
        }
        std::vector<int32_t> tile_off(ntiles + 1), tile_k(ntiles), blk_tile((size_t)P * P + 1);
        for (int64_t b = 0; b < nb; ++b) {
            const int k = (int)(b % I3);
            for (int64_t u = 0; u < tiles_in_bucket[b + 1] - tiles_in_bucket[b]; ++u) {
                tile_off[tiles_in_bucket[b] + u] = (int32_t)(bstart[b] + u * T);
                tile_k[tiles_in_bucket[b] + u] = k;
            }
        }
        tile_off[ntiles] = (int32_t)nnz;
        for (int64_t blk = 0; blk <= (int64_t)P * P; ++blk) blk_tile[blk] = (int32_t)tiles_in_bucket[blk * I3];
        // nonzeros of stratum s (blocks (p, (p + s) mod P)) on each platform
        std::vector<int32_t> scount((size_t)P * I3, 0);
        for (int p = 0; p < P; ++p)
            for (int q = 0; q < P; ++q) {
                const int s = (q - p + P) % P;
                const int64_t blk = (int64_t)p * P + q;
                for (int64_t tl = blk_tile[blk]; tl < blk_tile[blk + 1]; ++tl)
                    scount[(size_t)s * I3 + tile_k[tl]] += tile_off[tl + 1] - tile_off[tl];
            }
        // core-step constants of each stratum (see kCstHead), in the precision
        // the step uses them
        const int ncst = kCstHead + I3;
        std::vector<float> ccst((size_t)P * ncst, 0.f);
        const float lamf = (float)pa->lambda;
        for (int s = 0; s < P; ++s) {
            double m = 0.0;
            for (int k = 0; k < I3; ++k) m += (double)scount[(size_t)s * I3 + k];
            float* c = &ccst[(size_t)s * ncst];
            if (m > 0.0) {
                c[0] = 1.f;
                c[1] = (float)(1.0 / m);
                c[2] = lamf * (float)(m / (double)nnz);
                for (int k = 0; k < I3; ++k) {
                    const int32_t mk = scount[(size_t)s * I3 + k];
                    c[kCstHead + k] = mk > 0 ? lamf * (float)((double)mk / (double)cnt3[k]) : 0.f;
                }
            }
        }
        // first record of each block
        std::vector<int32_t> blk_rec((size_t)P * P + 1);
        for (int64_t blk = 0; blk <= (int64_t)P * P; ++blk) blk_rec[blk] = tile_off[blk_tile[blk]];
        // ---------------- pack records with the tile's gene-slot order ----------------
        std::vector<uint2> nz(nnz);
        const int sh_f = bits_i + bits_j;
        parallel_for(ntiles, [&](int64_t tl, int) {
            const int32_t s = tile_off[tl], e = tile_off[tl + 1], n = e - s;
            int32_t jl[kTileMax], slot_of[kTileMax], at_slot[kTileMax];
            for (int t = 0; t < n; ++t) {
                const int32_t id = ord[s + t];
                jl[t] = pos2[X->j[id]] - start2[blk2[X->j[id]]];
                at_slot[t] = t;
            }
            // stable order by gene row: slot -> position
            std::stable_sort(at_slot, at_slot + n, [&](int32_t u, int32_t v) { return jl[u] < jl[v]; });
            for (int sl = 0; sl < n; ++sl) slot_of[at_slot[sl]] = sl;
            for (int t = 0; t < n; ++t) {
                const int32_t id = ord[s + t];
                const uint32_t il = (uint32_t)(pos1[X->i[id]] - start1[blk1[X->i[id]]]);
                nz[s + t].x = il | ((uint32_t)jl[t] << bits_i) | ((uint32_t)slot_of[t] << sh_f);
                std::memcpy(&nz[s + t].y, &X->x[id], 4);
            }
        });
        // ---------------- network: symmetric CSR over gene positions ----------------
        std::vector<std::pair<int64_t, float>> ed;
        ed.reserve(2 * E);
        for (int64_t e = 0; e < E; ++e) {
            const float w = Y->w ? Y->w[e] : 1.f;
            const int64_t a = pos2[Y->u[e]], b = pos2[Y->v[e]];
            ed.push_back({a * I2 + b, w});
            ed.push_back({b * I2 + a, w});
        }
        std::sort(ed.begin(), ed.end(), [](const std::pair<int64_t, float>& a, const std::pair<int64_t, float>& b) {
            return a.first < b.first;
        });
        std::vector<int32_t> adj_start(I2 + 1, 0), adj_nbr;
        std::vector<float> adj_w;
        for (size_t e = 0; e < ed.size(); ++e) {
            if (e > 0 && ed[e].first == ed[e - 1].first) {
                adj_w.back() += ed[e].second;
            } else {
                adj_nbr.push_back((int32_t)(ed[e].first % I2));
                adj_w.push_back(ed[e].second);
                adj_start[ed[e].first / I2 + 1]++;
            }
        }
        for (int r = 0; r < I2; ++r) adj_start[r + 1] += adj_start[r];
        std::vector<float> deg(I2, 0.f);
        double dmax = 0.0;
        for (int r = 0; r < I2; ++r) {
            double d = 0.0;
            for (int e = adj_start[r]; e < adj_start[r + 1]; ++e) d += (double)adj_w[e];
            deg[r] = (float)d;
            dmax = std::max(dmax, d);
        }
        pr->dmax = dmax;
        pr->ecsr = (int64_t)adj_nbr.size();
        pr->n_sub = 0;
        if (pa->lambda_g > 0 && E > 0) pr->n_sub = std::max(1, (int)std::ceil(2.0 * pa->lr * pa->lambda_g * dmax));
        pr->ntiles = ntiles;
        pr->plan_s = now_s() - t_plan0;

        // ---------------- upload ----------------
        const double t_up0 = now_s();
        HIP_TRY(hipSetDevice(ctx->device));
        const size_t ni = (size_t)I3 * J1 * J2, ng = (size_t)J1 * J2 * J3;
        pr->d_nz = pr->alloc<uint2>(nnz, rc);
        pr->d_tile_off = pr->alloc<int32_t>(ntiles + 1, rc);
        pr->d_tile_k = pr->alloc<int32_t>(ntiles, rc);
        pr->d_blk_tile = pr->alloc<int32_t>((size_t)P * P + 1, rc);
        pr->d_perm1 = pr->alloc<int32_t>(I1, rc);
        pr->d_perm2 = pr->alloc<int32_t>(I2, rc);
        pr->d_start1 = pr->alloc<int32_t>(P + 1, rc);
        pr->d_start2 = pr->alloc<int32_t>(P + 1, rc);
        pr->d_reg1 = pr->alloc<float>(I1, rc);
        pr->d_reg2 = pr->alloc<float>(I2, rc);
        pr->d_cnt1 = pr->alloc<int32_t>(I1, rc);
        pr->d_cnt2 = pr->alloc<int32_t>(I2, rc);
        pr->d_cnt3 = pr->alloc<int32_t>(I3, rc);
        pr->d_adj_start = pr->alloc<int32_t>(I2 + 1, rc);
        pr->d_adj_nbr = pr->alloc<int32_t>(adj_nbr.size(), rc);
        pr->d_adj_w = pr->alloc<float>(adj_w.size(), rc);
        pr->d_deg = pr->alloc<float>(I2, rc);
        pr->d_Ap = pr->alloc<float>((size_t)I1 * J1, rc);
        pr->d_Bp = pr->alloc<float>((size_t)I2 * J2, rc);
        pr->d_Btmp = pr->alloc<float>((size_t)I2 * J2, rc);
        pr->d_Spart = pr->alloc<float>((size_t)P * ni, rc);
        pr->d_Ssum = pr->alloc<float>(std::max(ni, ng), rc);
        pr->d_Sx = pr->alloc<unsigned long long>((size_t)(P + 1) * ni + P, rc);
        pr->d_blk_rec = pr->alloc<int32_t>((size_t)P * P + 1, rc);
        pr->d_ccst = pr->alloc<float>((size_t)P * (kCstHead + I3), rc);
        pr->d_order = pr->alloc<int32_t>(P, rc);
        pr->d_bar = pr->alloc<GridBar>(1, rc);
        pr->d_sse = pr->alloc<double>((size_t)P * P, rc);
        pr->d_regp = pr->alloc<double>(pr->n_reg_wg, rc);
        pr->d_net = pr->alloc<double>(I2, rc);
        pr->d_lossout = pr->alloc<double>(2, rc);
        pr->d_bakA = pr->alloc<float>(2 * (size_t)I1 * J1, rc);
        pr->d_bakB = pr->alloc<float>(2 * (size_t)I2 * J2, rc);
        pr->d_bakC = pr->alloc<float>(2 * (size_t)I3 * J3, rc);
        pr->d_bakG = pr->alloc<float>(2 * ng, rc);
        if (rc) {
            delete pr;
            return set_err(ctx, SNECT_E_OOM, "device allocation failed");
        }
        if (hipHostMalloc((void**)&pr->h_lossout, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&pr->h_bar, 2 * sizeof(GridBar), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&pr->h_order, 2 * (size_t)P * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
            delete pr;
            return set_err(ctx, SNECT_E_OOM, "pinned host allocation failed");
        }
        hipStream_t st = ctx->stream;
        auto up = [&](void* d, const void* h, size_t bytes) -> hipError_t {
            if (bytes == 0) return hipSuccess;
            return hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st);
        };
        hipError_t he = hipSuccess;
        he = he ? he : up(pr->d_nz, nz.data(), nnz * sizeof(uint2));
        he = he ? he : up(pr->d_tile_off, tile_off.data(), tile_off.size() * 4);
        he = he ? he : up(pr->d_tile_k, tile_k.data(), tile_k.size() * 4);
        he = he ? he : up(pr->d_blk_tile, blk_tile.data(), blk_tile.size() * 4);
        he = he ? he : up(pr->d_blk_rec, blk_rec.data(), blk_rec.size() * 4);
        he = he ? he : up(pr->d_ccst, ccst.data(), ccst.size() * 4);
        he = he ? he : up(pr->d_perm1, pr->perm1.data(), (size_t)I1 * 4);
        he = he ? he : up(pr->d_perm2, pr->perm2.data(), (size_t)I2 * 4);
        he = he ? he : up(pr->d_start1, start1.data(), (size_t)(P + 1) * 4);
        he = he ? he : up(pr->d_start2, start2.data(), (size_t)(P + 1) * 4);
        he = he ? he : up(pr->d_reg1, reg1p.data(), (size_t)I1 * 4);
        he = he ? he : up(pr->d_reg2, reg2p.data(), (size_t)I2 * 4);
        he = he ? he : up(pr->d_cnt1, cnt1p.data(), (size_t)I1 * 4);
        he = he ? he : up(pr->d_cnt2, cnt2p.data(), (size_t)I2 * 4);
        he = he ? he : up(pr->d_cnt3, cnt3.data(), (size_t)I3 * 4);
        he = he ? he : up(pr->d_adj_start, adj_start.data(), (size_t)(I2 + 1) * 4);
        he = he ? he : up(pr->d_adj_nbr, adj_nbr.data(), adj_nbr.size() * 4);
        he = he ? he : up(pr->d_adj_w, adj_w.data(), adj_w.size() * 4);
        he = he ? he : up(pr->d_deg, deg.data(), (size_t)I2 * 4);
        // exchange words start with tag 0, which no stratum uses
        he = he ? he : hipMemsetAsync(pr->d_Sx, 0, ((size_t)(P + 1) * ni + P) * sizeof(unsigned long long), st);
        he = he ? he : hipStreamSynchronize(st);
        he = he ? he : prepare_kernels(jp, llds, clds, pr->loss_cols_lds);
        he = he ? he : configure_exec(pr, kDefaultWaves, rec_cap);
        for (int t = 0; t < 8 && he == hipSuccess; ++t) he = hipEventCreate(&pr->ev[t / 4][t % 4]);
        if (he != hipSuccess) {
            delete pr;
            return set_err(ctx, SNECT_E_HIP, std::string("upload: ") + hipGetErrorString(he));
        }
        pr->upload_s = now_s() - t_up0;
        ctx->live_problems++;
    } catch (const std::bad_alloc&) {
        delete pr;
        return set_err(ctx, SNECT_E_OOM, "host allocation failed while planning");
    }
    *out = pr;
    return SNECT_OK;
}

int snect_problem_destroy(snect_problem* prob)
{
    if (!prob) return SNECT_E_ARG;
    (void)hipSetDevice(prob->ctx->device);
    (void)hipStreamSynchronize(prob->ctx->stream);
    prob->ctx->live_problems--;
    delete prob;
    return SNECT_OK;
}

int snect_problem_info(const snect_problem* pr, snect_info* info)
{
    if (!pr || !info) return SNECT_E_ARG;
    info->nnz = pr->nnz;
    info->ntiles = pr->ntiles;
    info->edges_csr = pr->ecsr;
    info->P = pr->P;
    info->T = pr->T;
    info->rows1_max = pr->rows1_max;
    info->rows2_max = pr->rows2_max;
    info->bits_i = pr->bits_i;
    info->bits_j = pr->bits_j;
    info->n_sub = pr->n_sub;
    info->d_max = pr->dmax;
    int64_t b = 0;
    for (auto& x : pr->bufs) b += (int64_t)x.bytes;
    info->device_bytes = b;
    info->plan_seconds = pr->plan_s;
    info->upload_seconds = pr->upload_s;
    return SNECT_OK;
}

static int check_factors(snect_ctx* ctx, const snect_factors* f)
{
    if (!f || !f->A || !f->B || !f->C || !f->G) return set_err(ctx, SNECT_E_ARG, "null factor pointer");
    return SNECT_OK;
}

// The stream a problem's work is queued on.
static hipStream_t pstream(const snect_problem* pr)
{
    return pr->stream_override ? pr->stream_override : pr->ctx->stream;
}

static GraphArgs graph_args(const snect_problem* pr)
{
    GraphArgs ga;
    ga.Bin = pr->d_Bp;
    ga.Bout = pr->d_Btmp;
    ga.adj_start = pr->d_adj_start;
    ga.adj_nbr = pr->d_adj_nbr;
    ga.adj_w = pr->d_adj_w;
    ga.deg = pr->d_deg;
    ga.net_part = pr->d_net;
    ga.I2 = pr->I2;
    ga.J2 = pr->J2;
    ga.alpha = pr->n_sub > 0 ? (float)(pr->lr * pr->lam_g / pr->n_sub) : 0.f;
    return ga;
}

// Loss of the factors held in position order (d_Ap, d_Bp, C, G) into
// slot `slot` of pr->h_lossout (asynchronous; the caller synchronises).
static int run_loss(snect_problem* pr, const float* C, const float* G, int slot = 0)
{
    snect_ctx* ctx = pr->ctx;
    LossArgs la;
    la.nz = pr->d_nz; la.tile_off = pr->d_tile_off; la.tile_k = pr->d_tile_k; la.blk_tile = pr->d_blk_tile;
    la.start1 = pr->d_start1; la.start2 = pr->d_start2;
    la.cnt1 = pr->d_cnt1; la.cnt2 = pr->d_cnt2; la.cnt3 = pr->d_cnt3;
    la.Ap = pr->d_Ap; la.Bp = pr->d_Bp; la.C = C; la.G = G;
    la.adj_start = pr->d_adj_start; la.adj_nbr = pr->d_adj_nbr; la.adj_w = pr->d_adj_w;
    la.sse_part = pr->d_sse; la.reg_part = pr->d_regp; la.net_part = pr->d_net; la.out = pr->d_lossout;
    la.P = pr->P; la.I1 = pr->I1; la.I2 = pr->I2; la.I3 = pr->I3;
    la.J1 = pr->J1; la.J2 = pr->J2; la.J3 = pr->J3;
    la.rows1_max = pr->rows1_max; la.rows2_max = pr->rows2_max; la.bits_i = pr->bits_i; la.bits_j = pr->bits_j;
    la.n_reg_wg = pr->n_reg_wg;
    la.lam = pr->lam; la.lam_g = pr->lam_g;
    GraphArgs ga = graph_args(pr);
    HIP_TRY(launch_loss(la, ga, pr->jp, pr->loss_lds, pr->loss_cols_lds, pr->loss_parts, pstream(pr)));
    HIP_TRY(hipMemcpyAsync(pr->h_lossout + 2 * slot, pr->d_lossout, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           pstream(pr)));
    return SNECT_OK;
}

static int to_positions(snect_problem* pr, const snect_factors* f)
{
    snect_ctx* ctx = pr->ctx;
    HIP_TRY(launch_permute(f->A, pr->d_Ap, pr->d_perm1, pr->I1, pr->J1, 1, pstream(pr)));
    HIP_TRY(launch_permute(f->B, pr->d_Bp, pr->d_perm2, pr->I2, pr->J2, 1, pstream(pr)));
    return SNECT_OK;
}

static int from_positions(snect_problem* pr, snect_factors* f)
{
    snect_ctx* ctx = pr->ctx;
    HIP_TRY(launch_permute(pr->d_Ap, f->A, pr->d_perm1, pr->I1, pr->J1, 0, pstream(pr)));
    HIP_TRY(launch_permute(pr->d_Bp, f->B, pr->d_perm2, pr->I2, pr->J2, 0, pstream(pr)));
    return SNECT_OK;
}

int snect_evaluate(snect_problem* pr, const snect_factors* f, double* loss, double* rmse)
{
    if (!pr) return SNECT_E_ARG;
    snect_ctx* ctx = pr->ctx;
    ctx->err.clear();
    int rc = check_factors(ctx, f);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    if ((rc = to_positions(pr, f))) return rc;
    if ((rc = run_loss(pr, f->C, f->G))) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (loss) *loss = pr->h_lossout[0];
    if (rmse) *rmse = pr->nnz > 0 ? std::sqrt(pr->h_lossout[1] / (double)pr->nnz) : 0.0;
    return SNECT_OK;
}

// Tags of the next persistent launch of a problem: its strata write tags
// t0 + 1 .. t0 + P (returned: t0).  Consecutive launches get disjoint ranges
// and 0 is never handed out, so no exchange word left by an earlier launch
// (or by the initial clear) carries a tag of the current one.
static uint32_t take_tags(snect_problem* pr)
{
    if (pr->tag_next > UINT32_MAX - (uint32_t)pr->P) pr->tag_next = 0;
    const uint32_t t0 = pr->tag_next;
    pr->tag_next += (uint32_t)pr->P;
    return t0;
}

static StratArgs strat_args(const snect_problem* pr, const snect_factors* f)
{
    StratArgs sa;
    sa.nz = pr->d_nz; sa.tile_off = pr->d_tile_off; sa.tile_k = pr->d_tile_k; sa.blk_tile = pr->d_blk_tile;
    sa.start1 = pr->d_start1; sa.start2 = pr->d_start2;
    sa.reg1 = pr->d_reg1; sa.reg2 = pr->d_reg2; sa.cnt3 = pr->d_cnt3;
    sa.Ap = pr->d_Ap; sa.Bp = pr->d_Bp; sa.C = f->C; sa.G = f->G;
    sa.Spart = pr->d_Spart; sa.blk_rec = pr->d_blk_rec; sa.ccst = pr->d_ccst; sa.Ssum = pr->d_Ssum;
    sa.Sx = pr->d_Sx; sa.tag0 = 0; sa.spin_limit = (uint32_t)pr->wait_limit;
    sa.order = pr->d_order; sa.bar = pr->d_bar; sa.jp = pr->jp;
    sa.P = pr->P; sa.s = 0; sa.I3 = pr->I3; sa.J1 = pr->J1; sa.J2 = pr->J2; sa.J3 = pr->J3;
    sa.rows1_max = pr->rows1_max; sa.rows2_max = pr->rows2_max; sa.bits_i = pr->bits_i; sa.bits_j = pr->bits_j;
    sa.rec_cap = pr->rec_cap;
    sa.lr = (float)pr->lr; sa.lam = (float)pr->lam; sa.etac = (float)(pr->lr * pr->cls);
    sa.nnz = (double)pr->nnz;
    return sa;
}

// Start of an epoch: keep the factors (position order) for a divergence
// rollback in backup slot `slot`, then the network step (Jacobi sub-steps
// through Btmp).
static int epoch_begin(snect_problem* pr, snect_factors* f, int slot = 0)
{
    snect_ctx* ctx = pr->ctx;
    hipStream_t st = pstream(pr);
    const size_t nA = (size_t)pr->I1 * pr->J1, nB = (size_t)pr->I2 * pr->J2, nC = (size_t)pr->I3 * pr->J3,
                 nG = (size_t)pr->J1 * pr->J2 * pr->J3;
    HIP_TRY(hipMemcpyAsync(pr->d_bakA + slot * nA, pr->d_Ap, 4 * nA, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(pr->d_bakB + slot * nB, pr->d_Bp, 4 * nB, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(pr->d_bakC + slot * nC, f->C, 4 * nC, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(pr->d_bakG + slot * nG, f->G, 4 * nG, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipEventRecord(pr->ev[slot][0], st));
    GraphArgs ga = graph_args(pr);
    for (int it = 0; it < pr->n_sub; ++it) {
        const bool even = (it % 2) == 0;
        ga.Bin = even ? pr->d_Bp : pr->d_Btmp;
        ga.Bout = even ? pr->d_Btmp : pr->d_Bp;
        HIP_TRY(launch_graph_step(ga, pr->jp, st));
    }
    if (pr->n_sub % 2 == 1) HIP_TRY(hipMemcpyAsync(pr->d_Bp, pr->d_Btmp, 4 * nB, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipEventRecord(pr->ev[slot][1], st));
    return SNECT_OK;
}

// The persistent driver's per-epoch inputs: the stratum order (through
// pinned slot `slot`, whose previous upload finished before the epoch two
// back was checked) and a cleared error word.
static int persistent_inputs(snect_problem* pr, int32_t ep, int slot = 0)
{
    snect_ctx* ctx = pr->ctx;
    const std::vector<int32_t> order = stratum_order(pr->P, pr->seed, ep);
    int32_t* h = pr->h_order + (size_t)slot * pr->P;
    std::memcpy(h, order.data(), (size_t)pr->P * 4);
    HIP_TRY(hipMemcpyAsync(pr->d_order, h, (size_t)pr->P * 4, hipMemcpyHostToDevice, pstream(pr)));
    HIP_TRY(hipMemsetAsync(pr->d_bar, 0, sizeof(GridBar), pstream(pr)));
    return SNECT_OK;
}

// After the strata: the loss launch and the downloads of the loss and of the
// exchange's error word into slot `slot` (asynchronous).
static int epoch_loss(snect_problem* pr, snect_factors* f, int slot = 0)
{
    HIP_TRY_CTX(pr->ctx, hipEventRecord(pr->ev[slot][2], pstream(pr)));
    int rc = run_loss(pr, f->C, f->G, slot);
    if (rc) return rc;
    HIP_TRY_CTX(pr->ctx, hipMemcpyAsync(pr->h_bar + slot, pr->d_bar, sizeof(GridBar), hipMemcpyDeviceToHost,
                                        pstream(pr)));
    HIP_TRY_CTX(pr->ctx, hipEventRecord(pr->ev[slot][3], pstream(pr)));
    return SNECT_OK;
}

// Once the epoch in slot `slot` has finished (this waits for it): barrier
// health, timings, the epoch's loss, and the rollback of a non-finite epoch
// (SNECT_E_DIVERGED) from the slot's backup, after everything queued behind
// it has finished too.
static int epoch_finish(snect_problem* pr, snect_factors* f, int32_t ep, bool persistent, double* loss,
                        double* rmse, int slot = 0)
{
    snect_ctx* ctx = pr->ctx;
    hipStream_t st = pstream(pr);
    HIP_TRY(hipEventSynchronize(pr->ev[slot][3]));
    if (persistent && pr->h_bar[slot].err) return set_err(ctx, SNECT_E_HIP, "the stratum kernel timed out waiting for another workgroup");
    float m0 = 0, m1 = 0, m2 = 0;
    HIP_TRY(hipEventElapsedTime(&m0, pr->ev[slot][0], pr->ev[slot][1]));
    HIP_TRY(hipEventElapsedTime(&m1, pr->ev[slot][1], pr->ev[slot][2]));
    HIP_TRY(hipEventElapsedTime(&m2, pr->ev[slot][2], pr->ev[slot][3]));
    pr->t_ms[0] += m0;
    pr->t_ms[1] += m1;
    pr->t_ms[2] += m2;
    const double fl = pr->h_lossout[2 * slot];
    const double r = pr->nnz > 0 ? std::sqrt(pr->h_lossout[2 * slot + 1] / (double)pr->nnz) : 0.0;
    if (loss) *loss = fl;
    if (rmse) *rmse = r;
    if (!std::isfinite(fl) || !std::isfinite(r)) {
        const size_t nA = (size_t)pr->I1 * pr->J1, nB = (size_t)pr->I2 * pr->J2, nC = (size_t)pr->I3 * pr->J3,
                     nG = (size_t)pr->J1 * pr->J2 * pr->J3;
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipMemcpyAsync(pr->d_Ap, pr->d_bakA + slot * nA, 4 * nA, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(pr->d_Bp, pr->d_bakB + slot * nB, 4 * nB, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(f->C, pr->d_bakC + slot * nC, 4 * nC, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(f->G, pr->d_bakG + slot * nG, 4 * nG, hipMemcpyDeviceToDevice, st));
        return set_err(ctx, SNECT_E_DIVERGED, "loss not finite at epoch " + std::to_string(ep));
    }
    return SNECT_OK;
}

int snect_train(snect_problem* pr, snect_factors* f, int32_t start_epoch, int32_t epochs, double* loss,
                double* rmse)
{
    if (!pr) return SNECT_E_ARG;
    snect_ctx* ctx = pr->ctx;
    ctx->err.clear();
    int rc = check_factors(ctx, f);
    if (rc) return rc;
    if (epochs < 0 || start_epoch < 0) return set_err(ctx, SNECT_E_ARG, "negative epoch count or start");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int P = pr->P;
    const int path = pr->chosen_path();
    const bool persistent = path == SNECT_PATH_PERSISTENT;
    if (persistent && !pr->persistent_ok())
        return set_err(ctx, SNECT_E_UNSUPPORTED, "the persistent stratum kernel cannot be resident for this P");
    for (double& t : pr->t_ms) t = 0.0;
    const int nlaunch = persistent ? 1 : P;
    if (pr->per_launch && (int)pr->evl.size() < 4 * nlaunch) {
        const size_t have = pr->evl.size();
        pr->evl.resize(4 * (size_t)nlaunch, nullptr);
        for (size_t t = have; t < pr->evl.size(); ++t) HIP_TRY(hipEventCreate(&pr->evl[t]));
    }
    StratArgs sa = strat_args(pr, f);
    if ((rc = to_positions(pr, f))) return rc;
    // Epoch ep is queued before epoch ep - 1 is checked, so the host's work
    // between epochs overlaps the device's; per-epoch state alternates
    // between two slots.  A non-finite epoch rolls back to its own start once
    // the epoch queued behind it has finished.
    auto finish = [&](int32_t e) -> int {
        const int slot = e & 1;
        if (pr->per_launch) {
            hipEvent_t* el = pr->evl.data() + (size_t)slot * 2 * nlaunch;
            HIP_TRY(hipEventSynchronize(pr->ev[slot][3]));
            for (int l = 0; l < nlaunch; ++l) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, el[2 * l], el[2 * l + 1]));
                pr->t_ms[3] += ms;
            }
            pr->t_ms[4] += nlaunch;
        }
        int r = epoch_finish(pr, f, e, persistent, loss ? loss + (e - start_epoch) : nullptr,
                             rmse ? rmse + (e - start_epoch) : nullptr, slot);
        if (r) {
            const std::string msg = ctx->err;
            (void)hipStreamSynchronize(st);
            if (r == SNECT_E_DIVERGED && from_positions(pr, f) == SNECT_OK) (void)hipStreamSynchronize(st);
            ctx->err = msg;
        }
        return r;
    };
    int32_t pending = -1;
    for (int32_t ep = start_epoch; ep < start_epoch + epochs; ++ep) {
        const int slot = ep & 1;
        hipEvent_t* el = pr->per_launch ? pr->evl.data() + (size_t)slot * 2 * nlaunch : nullptr;
        if ((rc = epoch_begin(pr, f, slot))) return rc;
        if (persistent) {
            if ((rc = persistent_inputs(pr, ep, slot))) return rc;
            if (el) HIP_TRY(hipEventRecord(el[0], st));
            sa.tag0 = take_tags(pr);
            HIP_TRY(launch_strata_persistent(sa, pr->jp, pr->bf, pr->nw, pr->strata_lds, st));
            if (el) HIP_TRY(hipEventRecord(el[1], st));
        } else {
            const std::vector<int32_t> order = stratum_order(P, pr->seed, ep);
            for (int si = 0; si < P; ++si) {
                sa.s = order[si];
                if (el) HIP_TRY(hipEventRecord(el[2 * si], st));
                HIP_TRY(launch_block(sa, pr->jp, pr->bf, pr->nw, pr->block_lds, st));
                if (el) HIP_TRY(hipEventRecord(el[2 * si + 1], st));
                HIP_TRY(launch_core_step(sa, pr->core_lds, st));
            }
        }
        if ((rc = epoch_loss(pr, f, slot))) return rc;
        if (pending >= 0 && (rc = finish(pending))) return rc;
        pending = ep;
    }
    if (pending >= 0 && (rc = finish(pending))) return rc;
    if ((rc = from_positions(pr, f))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    return SNECT_OK;
}

// The sweep while its single batched launch is switched off: every problem
// on a stream of its own (default priority), with the multi-launch driver
// (a block-step launch and a core-step launch per stratum), the problems'
// epochs queued side by side so that they run concurrently; the host checks
// each epoch of every problem as snect_train does.  The results are those
// of snect_train on each problem, bit for bit.  The sweep's record chunk
// (snect_sweep_autotune) applies up to the problem's own.
static int sweep_concurrent(snect_ctx* ctx, int32_t n, snect_problem* const* probs, snect_factors* fs,
                            int32_t start_epoch, int32_t epochs, double* loss, double* rmse)
{
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<hipStream_t> sts(n, nullptr);
    hipEvent_t start_ev = nullptr;
    struct Cleanup {
        std::vector<hipStream_t>& s;
        snect_problem* const* p;
        int32_t n;
        hipEvent_t& e;
        ~Cleanup()
        {
            for (int32_t i = 0; i < n; ++i) {
                if (s[i]) (void)hipStreamSynchronize(s[i]);
                p[i]->stream_override = nullptr;
                if (s[i]) (void)hipStreamDestroy(s[i]);
            }
            if (e) (void)hipEventDestroy(e);
        }
    } cleanup{sts, probs, n, start_ev};
    // the problem streams start after the work already queued on the
    // context's stream (the callers' factors are written there)
    HIP_TRY(hipEventCreateWithFlags(&start_ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(start_ev, ctx->stream));
    std::vector<StratArgs> sa(n);
    for (int32_t i = 0; i < n; ++i) {
        HIP_TRY(hipStreamCreateWithFlags(&sts[i], hipStreamNonBlocking));
        HIP_TRY(hipStreamWaitEvent(sts[i], start_ev, 0));
        snect_problem* pr = probs[i];
        pr->stream_override = sts[i];
        for (double& t : pr->t_ms) t = 0.0;
        sa[i] = strat_args(pr, &fs[i]);
        if (pr->sweep_rec_cap) sa[i].rec_cap = std::min(pr->sweep_rec_cap, pr->rec_cap);
        int rc = to_positions(pr, &fs[i]);
        if (rc) return rc;
    }
    int rc = SNECT_OK;
    for (int32_t ep = start_epoch; ep < start_epoch + epochs && !rc; ++ep) {
        for (int32_t i = 0; i < n && !rc; ++i) {
            snect_problem* pr = probs[i];
            if ((rc = epoch_begin(pr, &fs[i]))) break;
            const std::vector<int32_t> order = stratum_order(pr->P, pr->seed, ep);
            for (int si = 0; si < pr->P; ++si) {
                sa[i].s = order[si];
                HIP_TRY(launch_block(sa[i], pr->jp, pr->bf, pr->nw, pr->block_lds, sts[i]));
                HIP_TRY(launch_core_step(sa[i], pr->core_lds, sts[i]));
            }
            rc = epoch_loss(pr, &fs[i]);
        }
        for (int32_t i = 0; i < n && !rc; ++i) {
            const size_t o = (size_t)i * epochs + (ep - start_epoch);
            rc = epoch_finish(probs[i], &fs[i], ep, false, loss ? loss + o : nullptr, rmse ? rmse + o : nullptr);
            if (rc == SNECT_E_DIVERGED) ctx->err = "problem " + std::to_string(i) + ": " + ctx->err;
        }
    }
    const std::string msg = ctx->err;
    for (int32_t i = 0; i < n; ++i) (void)from_positions(probs[i], &fs[i]);
    for (int32_t i = 0; i < n; ++i) {
        const hipError_t e = hipStreamSynchronize(sts[i]);
        if (e != hipSuccess && !rc) rc = set_err(ctx, SNECT_E_HIP, std::string("sweep: ") + hipGetErrorString(e));
    }
    if (rc != SNECT_E_HIP) ctx->err = msg;
    return rc;
}

int snect_sweep_train(snect_ctx* ctx, int32_t n, snect_problem* const* probs, snect_factors* fs, int32_t start_epoch,
                      int32_t epochs, double* loss, double* rmse)
{
    if (!ctx) return SNECT_E_ARG;
    ctx->err.clear();
    if (n < 1 || !probs || !fs || epochs < 0 || start_epoch < 0)
        return set_err(ctx, SNECT_E_ARG, "bad sweep arguments");
    int bf = -1, nwg = 0;
    for (int i = 0; i < n; ++i) {
        snect_problem* pr = probs[i];
        if (!pr || pr->ctx != ctx) return set_err(ctx, SNECT_E_ARG, "problem " + std::to_string(i) + " is not on ctx");
        int rc = check_factors(ctx, &fs[i]);
        if (rc) return rc;
        for (int t = 0; t < i; ++t)
            if (probs[t] == pr) return set_err(ctx, SNECT_E_ARG, "a problem appears twice in the sweep");
        if (bf >= 0 && pr->bf != bf) return set_err(ctx, SNECT_E_ARG, "all problems of a sweep share one precision");
        bf = pr->bf;
        nwg += pr->P;
    }
    if (!kSweepEnabled) return sweep_concurrent(ctx, n, probs, fs, start_epoch, epochs, loss, rmse);
    if (!ctx->coop) return set_err(ctx, SNECT_E_UNSUPPORTED, "cooperative launches not available");
    // one launch of kDefaultWaves-wavefront workgroups; each problem keeps
    // its own core-size code, LDS layout and largest record chunk
    std::vector<int> rcap(n);
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
        const snect_problem* pr = probs[i];
        rcap[i] = pr->sweep_rec_cap ? pr->sweep_rec_cap : pr->rec_cap_max;
        lds = std::max(lds, strata_lds_bytes(pr->jp, pr->P, pr->rows1_max, pr->rows2_max, pr->I3, pr->J1, pr->J2,
                                             pr->J3, rcap[i], bf, kDefaultWaves));
    }
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(prepare_sweep(bf, lds));
    const int cap = sweep_capacity(bf, lds);
    if (nwg > cap)
        return set_err(ctx, SNECT_E_UNSUPPORTED, "the sweep needs " + std::to_string(nwg) +
                                                     " co-resident workgroups, the device holds " + std::to_string(cap));
    hipStream_t st = ctx->stream;
    // launch arguments in device memory
    std::vector<StratArgs> args(n);
    std::vector<int32_t> wg_start(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        args[i] = strat_args(probs[i], &fs[i]);
        args[i].rec_cap = rcap[i];
        wg_start[i + 1] = wg_start[i] + probs[i]->P;
    }
    void* d_args = nullptr;
    if (hipMalloc(&d_args, sizeof(StratArgs) * n + sizeof(int32_t) * (n + 1)) != hipSuccess) {
        (void)hipGetLastError();
        return set_err(ctx, SNECT_E_OOM, "sweep argument buffer");
    }
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        (void)hipFree(d_args);
    };
    int32_t* d_wg = reinterpret_cast<int32_t*>(static_cast<char*>(d_args) + sizeof(StratArgs) * n);
    hipError_t e = hipMemcpyAsync(d_args, args.data(), sizeof(StratArgs) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d_wg, wg_start.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        cleanup();
        return set_err(ctx, SNECT_E_HIP, std::string("sweep arguments: ") + hipGetErrorString(e));
    }
    int rc = SNECT_OK;
    for (int i = 0; i < n && !rc; ++i) {
        for (double& t : probs[i]->t_ms) t = 0.0;
        rc = to_positions(probs[i], &fs[i]);
    }
    for (int32_t ep = start_epoch; ep < start_epoch + epochs && !rc; ++ep) {
        for (int i = 0; i < n && !rc; ++i) rc = epoch_begin(probs[i], &fs[i]);
        for (int i = 0; i < n && !rc; ++i) rc = persistent_inputs(probs[i], ep);
        // fresh tags: the arguments again (a pageable copy, done with the
        // host array when it returns)
        for (int i = 0; i < n; ++i) args[i].tag0 = take_tags(probs[i]);
        if (!rc && (e = hipMemcpyAsync(d_args, args.data(), sizeof(StratArgs) * n, hipMemcpyHostToDevice, st)) !=
                       hipSuccess)
            rc = set_err(ctx, SNECT_E_HIP, std::string("sweep arguments: ") + hipGetErrorString(e));
        if (!rc) {
            e = launch_strata_sweep(static_cast<const StratArgs*>(d_args), d_wg, n, nwg, bf, lds, st);
            if (e != hipSuccess) rc = set_err(ctx, SNECT_E_HIP, std::string("sweep launch: ") + hipGetErrorString(e));
        }
        for (int i = 0; i < n && !rc; ++i) rc = epoch_loss(probs[i], &fs[i]);
        if (!rc && (e = hipStreamSynchronize(st)) != hipSuccess)
            rc = set_err(ctx, SNECT_E_HIP, std::string("sweep: ") + hipGetErrorString(e));
        for (int i = 0; i < n && !rc; ++i) {
            const size_t o = (size_t)i * epochs + (ep - start_epoch);
            rc = epoch_finish(probs[i], &fs[i], ep, true, loss ? loss + o : nullptr, rmse ? rmse + o : nullptr);
            if (rc == SNECT_E_DIVERGED) ctx->err = "problem " + std::to_string(i) + ": " + ctx->err;
        }
    }
    const std::string msg = ctx->err;
    for (int i = 0; i < n; ++i) (void)from_positions(probs[i], &fs[i]);
    cleanup();
    ctx->err = msg;
    return rc;
}

// Device copies of a problem's factors (scratch for the autotuners).
struct FactorCopy {
    snect_factors f{nullptr, nullptr, nullptr, nullptr};
    size_t sz[4] = {0, 0, 0, 0};
    ~FactorCopy()
    {
        (void)hipFree(f.A);
        (void)hipFree(f.B);
        (void)hipFree(f.C);
        (void)hipFree(f.G);
    }
    hipError_t alloc(const snect_problem* pr)
    {
        sz[0] = (size_t)pr->I1 * pr->J1 * 4;
        sz[1] = (size_t)pr->I2 * pr->J2 * 4;
        sz[2] = (size_t)pr->I3 * pr->J3 * 4;
        sz[3] = (size_t)pr->J1 * pr->J2 * pr->J3 * 4;
        float** d[4] = {&f.A, &f.B, &f.C, &f.G};
        for (int t = 0; t < 4; ++t)
            if (hipMalloc(reinterpret_cast<void**>(d[t]), std::max<size_t>(sz[t], 16)) != hipSuccess) {
                (void)hipGetLastError();
                return hipErrorOutOfMemory;
            }
        return hipSuccess;
    }
    hipError_t load(const snect_factors* src, hipStream_t st)
    {
        const float* s_[4] = {src->A, src->B, src->C, src->G};
        float* d_[4] = {f.A, f.B, f.C, f.G};
        for (int t = 0; t < 4; ++t) {
            const hipError_t e = hipMemcpyAsync(d_[t], s_[t], sz[t], hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
};

int snect_autotune(snect_problem* pr, const snect_factors* f, int32_t trials, snect_exec* best, double* best_ms)
{
    if (!pr) return SNECT_E_ARG;
    snect_ctx* ctx = pr->ctx;
    ctx->err.clear();
    int rc = check_factors(ctx, f);
    if (rc) return rc;
    if (trials < 1) return set_err(ctx, SNECT_E_ARG, "trials must be >= 1");
    HIP_TRY(hipSetDevice(ctx->device));
    FactorCopy fc;
    if (fc.alloc(pr) != hipSuccess) return set_err(ctx, SNECT_E_OOM, "autotune scratch factors");
    const int keep_path = pr->path, keep_nw = pr->nw, keep_rc = pr->rec_cap;
    const bool keep_pl = pr->per_launch;
    pr->per_launch = false;
    snect_exec b{0, keep_path, keep_nw, keep_rc, pr->wait_limit};
    double bt = -1.0;
    for (int path : {SNECT_PATH_PERSISTENT, SNECT_PATH_MULTI})
        for (int nw : {kDefaultWaves})
            for (int rcap = pr->rec_cap_max; rcap >= std::min(256, pr->rec_cap_max); rcap /= 2) {
                if (configure_exec(pr, nw, rcap) != hipSuccess) continue;
                pr->path = path;
                if (path == SNECT_PATH_PERSISTENT && !pr->persistent_ok()) continue;
                double t = -1.0;
                for (int k = 0; k < trials; ++k) {
                    HIP_TRY(fc.load(f, ctx->stream));
                    rc = snect_train(pr, &fc.f, 0, 1, nullptr, nullptr);
                    if (rc) break;
                    const double ms = pr->t_ms[0] + pr->t_ms[1] + pr->t_ms[2];
                    t = t < 0 ? ms : std::min(t, ms);
                }
                if (rc) {
                    (void)configure_exec(pr, keep_nw, keep_rc);
                    pr->path = keep_path;
                    pr->per_launch = keep_pl;
                    return rc;
                }
                if (bt < 0 || t < bt) {
                    bt = t;
                    b = snect_exec{0, path, nw, rcap, pr->wait_limit};
                }
            }
    pr->per_launch = keep_pl;
    if (bt < 0) {
        (void)configure_exec(pr, keep_nw, keep_rc);
        pr->path = keep_path;
        return set_err(ctx, SNECT_E_UNSUPPORTED, "no execution choice could run");
    }
    HIP_TRY(configure_exec(pr, b.waves, b.rec_cap));
    pr->path = b.path;
    b.per_launch_timing = keep_pl ? 1 : 0;
    if (best) *best = b;
    if (best_ms) *best_ms = bt;
    return SNECT_OK;
}

int snect_sweep_autotune(snect_ctx* ctx, int32_t n, snect_problem* const* probs, const snect_factors* fs,
                         int32_t trials, double* best_ms)
{
    if (!ctx) return SNECT_E_ARG;
    ctx->err.clear();
    if (n < 1 || !probs || !fs || trials < 1) return set_err(ctx, SNECT_E_ARG, "bad sweep autotune arguments");
    for (int i = 0; i < n; ++i)
        if (!probs[i] || probs[i]->ctx != ctx) return set_err(ctx, SNECT_E_ARG, "problem not on ctx");
    HIP_TRY(hipSetDevice(ctx->device));
    std::vector<std::unique_ptr<FactorCopy>> fc(n);
    std::vector<snect_factors> sf(n);
    std::vector<int> keep(n);
    for (int i = 0; i < n; ++i) {
        fc[i].reset(new (std::nothrow) FactorCopy());
        if (!fc[i] || fc[i]->alloc(probs[i]) != hipSuccess) return set_err(ctx, SNECT_E_OOM, "autotune scratch");
        sf[i] = fc[i]->f;
        keep[i] = probs[i]->sweep_rec_cap;
    }
    // candidates: every problem's record chunk scaled by 1, 1/2, 1/4 (>= 256)
    double bt = -1.0;
    int bshift = 0;
    int rc = SNECT_OK;
    for (int shift = 0; shift <= 2; ++shift) {
        for (int i = 0; i < n; ++i)
            probs[i]->sweep_rec_cap = std::max(std::min(256, probs[i]->rec_cap_max), probs[i]->rec_cap_max >> shift);
        double t = -1.0;
        for (int k = 0; k < trials && !rc; ++k) {
            for (int i = 0; i < n; ++i) HIP_TRY(fc[i]->load(&fs[i], ctx->stream));
            const auto t0 = std::chrono::steady_clock::now();
            rc = snect_sweep_train(ctx, n, probs, sf.data(), 0, 1, nullptr, nullptr);
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            t = t < 0 ? ms : std::min(t, ms);
        }
        if (rc) break;
        if (bt < 0 || t < bt) {
            bt = t;
            bshift = shift;
        }
    }
    for (int i = 0; i < n; ++i)
        probs[i]->sweep_rec_cap =
            rc ? keep[i] : std::max(std::min(256, probs[i]->rec_cap_max), probs[i]->rec_cap_max >> bshift);
    if (rc) return rc;
    if (best_ms) *best_ms = bt;
    return SNECT_OK;
}

// Algorithm 1's random start: A, B, C, G (in that order, row-major) i.i.d.
// N(0, sigma^2), sigma = (mean x^2 / (J1 J2 J3))^(1/8) (1 without data), by
// the Box-Muller transform of uniforms from the seed's initialisation
// stream, in double, rounded once to float.
static std::vector<float> random_start(const snect_tensor* X, const snect_params* pa)
{
    double ss = 0.0;
    for (int64_t t = 0; t < X->nnz; ++t) ss += (double)X->x[t] * (double)X->x[t];
    const double ms = X->nnz > 0 ? ss / (double)X->nnz : 0.0;
    const double sigma = ms > 0.0 ? std::pow(ms / ((double)pa->J1 * pa->J2 * pa->J3), 0.125) : 1.0;
    const size_t n = (size_t)X->I1 * pa->J1 + (size_t)X->I2 * pa->J2 + (size_t)X->I3 * pa->J3 +
                     (size_t)pa->J1 * pa->J2 * pa->J3;
    std::vector<float> v(n);
    uint64_t s = stream_start(pa->seed, kInitStream);
    const double two_pi = 6.283185307179586476925286766559;
    auto uniform = [&]() { return ((double)(sm64_next(s) >> 11) + 0.5) * 0x1.0p-53; };
    for (size_t t = 0; t < n; t += 2) {
        const double u1 = uniform(), u2 = uniform();
        const double r = std::sqrt(-2.0 * std::log(u1));
        v[t] = (float)(sigma * (r * std::cos(two_pi * u2)));
        if (t + 1 < n) v[t + 1] = (float)(sigma * (r * std::sin(two_pi * u2)));
    }
    return v;
}

int snect_decompose(snect_ctx* ctx, const snect_tensor* X, const snect_graph* Y, const snect_params* params,
                    const snect_factors* init, snect_factors* out, int32_t start_epoch, int32_t epochs, double* loss,
                    double* rmse)
{
    if (!ctx) return SNECT_E_ARG;
    ctx->err.clear();
    int rc = init ? check_factors(ctx, init) : SNECT_OK;
    if (rc) return rc;
    rc = check_factors(ctx, out);
    if (rc) return rc;
    snect_problem* pr = nullptr;
    rc = snect_problem_create(ctx, X, Y, params, &pr);
    if (rc) return rc;
    const size_t szA = (size_t)X->I1 * params->J1 * 4, szB = (size_t)X->I2 * params->J2 * 4,
                 szC = (size_t)X->I3 * params->J3 * 4, szG = (size_t)params->J1 * params->J2 * params->J3 * 4;
    hipStream_t st = ctx->stream;
    hipError_t e = hipSuccess;
    if (init) {
        if (init->A != out->A) e = e ? e : hipMemcpyAsync(out->A, init->A, szA, hipMemcpyDeviceToDevice, st);
        if (init->B != out->B) e = e ? e : hipMemcpyAsync(out->B, init->B, szB, hipMemcpyDeviceToDevice, st);
        if (init->C != out->C) e = e ? e : hipMemcpyAsync(out->C, init->C, szC, hipMemcpyDeviceToDevice, st);
        if (init->G != out->G) e = e ? e : hipMemcpyAsync(out->G, init->G, szG, hipMemcpyDeviceToDevice, st);
    } else {
        std::vector<float> v;
        try {
            v = random_start(X, params);
        } catch (const std::bad_alloc&) {
            snect_problem_destroy(pr);
            return set_err(ctx, SNECT_E_OOM, "host allocation for the random start");
        }
        const char* h = reinterpret_cast<const char*>(v.data());
        // synchronous copies: the host vector is released on return
        e = e ? e : hipMemcpy(out->A, h, szA, hipMemcpyHostToDevice);
        e = e ? e : hipMemcpy(out->B, h + szA, szB, hipMemcpyHostToDevice);
        e = e ? e : hipMemcpy(out->C, h + szA + szB, szC, hipMemcpyHostToDevice);
        e = e ? e : hipMemcpy(out->G, h + szA + szB + szC, szG, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        snect_problem_destroy(pr);
        return set_err(ctx, SNECT_E_HIP, std::string("copy init: ") + hipGetErrorString(e));
    }
    rc = snect_train(pr, out, start_epoch, epochs, loss, rmse);
    std::string msg = ctx->err;
    snect_problem_destroy(pr);
    ctx->err = msg;
    return rc;
}

int snect_plan_export(const snect_problem* pr, int32_t epoch, int32_t* perm1, int32_t* perm2, int32_t* strata)
{
    if (!pr || epoch < 0) return SNECT_E_ARG;
    if (perm1) std::memcpy(perm1, pr->perm1.data(), pr->perm1.size() * 4);
    if (perm2) std::memcpy(perm2, pr->perm2.data(), pr->perm2.size() * 4);
    if (strata) {
        const std::vector<int32_t> o = stratum_order(pr->P, pr->seed, epoch);
        std::memcpy(strata, o.data(), o.size() * 4);
    }
    return SNECT_OK;
}

int snect_plan_layout(const snect_problem* pr, uint32_t* word, float* x, int32_t* tile_off, int32_t* tile_k,
                      int32_t* blk_tile)
{
    if (!pr) return SNECT_E_ARG;
    snect_ctx* ctx = pr->ctx;
    ctx->err.clear();
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (word || x) {
        std::vector<uint2> rec((size_t)pr->nnz);
        if (pr->nnz > 0) HIP_TRY(hipMemcpy(rec.data(), pr->d_nz, (size_t)pr->nnz * sizeof(uint2), hipMemcpyDeviceToHost));
        for (int64_t t = 0; t < pr->nnz; ++t) {
            if (word) word[t] = rec[t].x;
            if (x) std::memcpy(&x[t], &rec[t].y, 4);
        }
    }
    if (tile_off) HIP_TRY(hipMemcpy(tile_off, pr->d_tile_off, (size_t)(pr->ntiles + 1) * 4, hipMemcpyDeviceToHost));
    if (tile_k && pr->ntiles > 0)
        HIP_TRY(hipMemcpy(tile_k, pr->d_tile_k, (size_t)pr->ntiles * 4, hipMemcpyDeviceToHost));
    if (blk_tile)
        HIP_TRY(hipMemcpy(blk_tile, pr->d_blk_tile, ((size_t)pr->P * pr->P + 1) * 4, hipMemcpyDeviceToHost));
    return SNECT_OK;
}

int snect_last_timing(const snect_problem* pr, double* ms5)
{
    if (!pr || !ms5) return SNECT_E_ARG;
    for (int t = 0; t < 5; ++t) ms5[t] = pr->t_ms[t];
    return SNECT_OK;
}

int snect_set_exec(snect_problem* pr, const snect_exec* ex)
{
    if (!pr || !ex) return SNECT_E_ARG;
    if (ex->path < SNECT_PATH_AUTO || ex->path > SNECT_PATH_MULTI)
        return set_err(pr->ctx, SNECT_E_ARG, "unknown path");
    const int nw = ex->waves == 0 ? kDefaultWaves : ex->waves;
    if (nw != kDefaultWaves) return set_err(pr->ctx, SNECT_E_ARG, "waves must be 0 or 8");
    if (ex->wait_limit < 0) return set_err(pr->ctx, SNECT_E_ARG, "wait_limit must be 0 or positive");
    const int rc = ex->rec_cap == 0 ? pr->rec_cap_max : ex->rec_cap;
    if (rc < kTileMax || rc > pr->rec_cap_max || (rc & (rc - 1)) != 0)
        return set_err(pr->ctx, SNECT_E_ARG,
                       "rec_cap must be 0 or a power of two in [64, " + std::to_string(pr->rec_cap_max) + "]");
    snect_ctx* ctx = pr->ctx;
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(configure_exec(pr, nw, rc));
    pr->per_launch = ex->per_launch_timing != 0;
    pr->path = ex->path;
    pr->wait_limit = ex->wait_limit;
    return SNECT_OK;
}

static int check_qr_args(snect_ctx* ctx, int32_t I1, int32_t I2, int32_t I3, int32_t J1, int32_t J2, int32_t J3,
                         const snect_factors* f)
{
    int rc = check_factors(ctx, f);
    if (rc) return rc;
    if (I1 < 1 || I2 < 1 || I3 < 1 || J1 < 1 || J2 < 1 || J3 < 1)
        return set_err(ctx, SNECT_E_ARG, "sizes must be positive");
    if (J1 > SNECT_MAX_RANK || J2 > SNECT_MAX_RANK || J3 > SNECT_MAX_RANK || J1 > I1 || J2 > I2 || J3 > I3)
        return set_err(ctx, SNECT_E_RANK, "orthonormalisation needs J_n <= I_n and J_n <= 32");
    return SNECT_OK;
}

// The three modes in turn on `scratch` (qr_scratch_bytes(), FP64) with six
// status words at `status`; waits for the stream and reports a
// rank-deficient factor.
static int run_qr(snect_ctx* ctx, int32_t I1, int32_t I2, int32_t I3, int32_t J1, int32_t J2, int32_t J3,
                  snect_factors* f, void* scratch, int* status)
{
    const int Is[3] = {I1, I2, I3}, Js[3] = {J1, J2, J3};
    float* Us[3] = {f->A, f->B, f->C};
    hipError_t e = launch_qr_clear(status, 6, ctx->stream);
    for (int n = 0; n < 3 && e == hipSuccess; ++n)
        e = launch_qr_mode(Us[n], Is[n], Js[n], f->G, J1, J2, J3, n, scratch, status + 2 * n, ctx->stream);
    int hs[6] = {0, 0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return set_err(ctx, SNECT_E_HIP, std::string("orthonormalize: ") + hipGetErrorString(e));
    for (int n = 0; n < 3; ++n)
        if (hs[2 * n] || hs[2 * n + 1])
            return set_err(ctx, SNECT_E_ARG, "factor " + std::to_string(n + 1) + " is rank-deficient");
    return SNECT_OK;
}

int snect_orthonormalize(snect_ctx* ctx, int32_t I1, int32_t I2, int32_t I3, int32_t J1, int32_t J2, int32_t J3,
                         snect_factors* f)
{
    if (!ctx) return SNECT_E_ARG;
    ctx->err.clear();
    int rc = check_qr_args(ctx, I1, I2, I3, J1, J2, J3, f);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    const size_t bytes = qr_scratch_bytes();
    void* scratch = nullptr;
    int* status = nullptr;
    if (hipMalloc(&scratch, bytes) != hipSuccess || hipMalloc((void**)&status, 6 * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        if (scratch) (void)hipFree(scratch);
        return set_err(ctx, SNECT_E_OOM, "QR scratch allocation failed");
    }
    rc = run_qr(ctx, I1, I2, I3, J1, J2, J3, f, scratch, status);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(scratch);
    (void)hipFree(status);
    return rc;
}

int snect_orthonormalize_noalloc(snect_ctx* ctx, int32_t I1, int32_t I2, int32_t I3, int32_t J1, int32_t J2,
                                 int32_t J3, snect_factors* f)
{
    if (!ctx) return SNECT_E_ARG;
    ctx->err.clear();
    int rc = check_qr_args(ctx, I1, I2, I3, J1, J2, J3, f);
    if (rc) return rc;
    if (qr_scratch_bytes() + 6 * sizeof(int) > qr_static_scratch_bytes())
        return set_err(ctx, SNECT_E_UNSUPPORTED, "the fixed QR scratch is smaller than one mode needs");
    if (!ctx->qr_static) return set_err(ctx, SNECT_E_HIP, "the fixed QR scratch has no device address");
    HIP_TRY(hipSetDevice(ctx->device));
    char* base = static_cast<char*>(ctx->qr_static);
    int* status = reinterpret_cast<int*>(base + qr_scratch_bytes());
    return run_qr(ctx, I1, I2, I3, J1, J2, J3, f, base, status);
}

int snect_exec_path(const snect_problem* pr)
{
    if (!pr) return SNECT_E_ARG;
    return pr->chosen_path();
}

}  // extern "C"
