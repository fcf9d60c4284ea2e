// Fold-in / top-k server with continuous batching (host side).
//
// Requests are admitted while a slot (a HIP stream of default priority) and
// room in the device request pool are free; each admitted request is copied
// to the device, folded in and searched on its own stream, so requests that
// arrive while others run overlap on the device.  Completion is observed
// with one HIP event per slot.  A request that does not fit now gets
// SNECT_E_BUSY and may be submitted again later; a request larger than the
// whole pool gets SNECT_E_UNSUPPORTED; a malformed request fails alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include <emmintrin.h>

#include "../../include/snect.h"
#include "snect_internal.h"

namespace snect {
hipError_t launch_serve_setup(const float* A, const float* B, const float* C, const float* G, int I1, int I2, int I3,
                              int J1, int J2, int J3, float* W, float* anrm, float* At, hipStream_t st);
hipError_t launch_serve_request(const int32_t* jj, const int32_t* kk, const float* xx, int n, const float* W, int I2,
                                int J1, double lam, int pg_iters, const float* At, const float* anrm, int I1,
                                int topk, float* part, float* scores, double* out, int* status, hipStream_t st);
int serve_parts(int n);
}  // namespace snect

using namespace snect;

namespace {

constexpr size_t kAlign = 256;
// Pinned request staging of a slot, allocated when the server is created
// (requests of up to about 87,000 cells fit; larger ones grow it).
constexpr size_t kStagingStart = size_t(1) << 20;

size_t align_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, size) with coalescing frees.
struct PoolAlloc {
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t s)
    {
        size = s;
        free_.clear();
        free_[0] = s;
    }
    bool take(size_t n, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n;
                const size_t noff = it->first + n;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                return true;
            }
        return false;
    }
    void give(size_t off, size_t n)
    {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    // timing events around the request's kernels (recorded only by a replay
    // that measures device-busy time)
    hipEvent_t k0 = nullptr, k1 = nullptr;
    bool busy = false;
    int64_t ticket = -1;
    size_t off = 0, bytes = 0;
    // pinned host staging of the request upload
    char* h_in = nullptr;
    size_t h_in_cap = 0;
    // results: out_len() doubles, then the status word in one more double,
    // on the device and in pinned host memory (one download per request)
    double* h_out = nullptr;
    // per-slot device scratch
    float* d_part = nullptr;
    float* d_scores = nullptr;
    double* d_out = nullptr;
};

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct snect_server {
    int device = 0;
    snect_ctx* ctx = nullptr;
    std::string* err = nullptr;  // the owning context's message
    int32_t I1 = 0, I2 = 0, I3 = 0, J1 = 0;
    snect_server_config cfg{};
    float* d_W = nullptr;       // [I3][I2][J1]
    float* d_anrm = nullptr;    // [I1]
    float* d_At = nullptr;      // [J1][I1], A transposed
    char* d_pool = nullptr;
    PoolAlloc pool;
    std::vector<Slot> slots;
    int64_t next_ticket = 0;
    std::map<int64_t, int> where;  // ticket -> slot
    bool counted = false;          // included in the context's live count
    int out_len() const { return J1 + 2 * cfg.topk; }
};

static int srv_err(snect_server* s, int code, const std::string& m)
{
    if (s && s->err) *s->err = m;
    return code;
}

extern "C" {

int snect_server_create(snect_ctx* ctx, int32_t I1, int32_t I2, int32_t I3, int32_t J1, int32_t J2, int32_t J3,
                        const snect_factors* f, const snect_server_config* cfg, snect_server** out)
{
    if (!ctx) return SNECT_E_ARG;
    const int device = ctx->device;
    void* stream = ctx->stream;
    std::string* err = &ctx->err;
    err->clear();
    if (!f || !f->A || !f->B || !f->C || !f->G || !cfg || !out) {
        *err = "null argument";
        return SNECT_E_ARG;
    }
    *out = nullptr;
    if (I1 < 1 || I2 < 1 || I3 < 1 || J1 < 1 || J2 < 1 || J3 < 1 || J1 > SNECT_MAX_RANK || J2 > SNECT_MAX_RANK ||
        J3 > SNECT_MAX_RANK) {
        *err = "bad sizes";
        return SNECT_E_RANK;
    }
    if (cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->pool_bytes < 4096 || cfg->pg_iters < 0 || cfg->topk < 1 ||
        cfg->topk > 64 || cfg->topk > I1 || !(cfg->lambda >= 0) || !std::isfinite(cfg->lambda)) {
        *err = "bad server configuration";
        return SNECT_E_ARG;
    }
    if (hipSetDevice(device) != hipSuccess) return SNECT_E_HIP;
    snect_server* s = new (std::nothrow) snect_server();
    if (!s) return SNECT_E_OOM;
    s->device = device;
    s->ctx = ctx;
    s->err = err;
    s->I1 = I1; s->I2 = I2; s->I3 = I3; s->J1 = J1;
    s->cfg = *cfg;
    auto fail = [&](int code, const std::string& m) {
        snect_server_destroy(s);
        *err = m;
        return code;
    };
    if (hipMalloc((void**)&s->d_W, sizeof(float) * (size_t)I3 * I2 * J1) != hipSuccess ||
        hipMalloc((void**)&s->d_anrm, sizeof(float) * (size_t)I1) != hipSuccess ||
        hipMalloc((void**)&s->d_At, sizeof(float) * (size_t)J1 * I1) != hipSuccess ||
        hipMalloc((void**)&s->d_pool, (size_t)cfg->pool_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SNECT_E_OOM, "server device allocation failed");
    }
    s->pool.init((size_t)cfg->pool_bytes);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (launch_serve_setup(f->A, f->B, f->C, f->G, I1, I2, I3, J1, J2, J3, s->d_W, s->d_anrm, s->d_At, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(SNECT_E_HIP, "server setup kernels failed");
    s->slots.resize(cfg->max_slots);
    const int ne = J1 * (J1 + 1) / 2 + J1;
    for (auto& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreate(&sl.k0) != hipSuccess || hipEventCreate(&sl.k1) != hipSuccess ||
            hipMalloc((void**)&sl.d_part, sizeof(float) * kServeMaxParts * ne) != hipSuccess ||
            hipMalloc((void**)&sl.d_scores, sizeof(float) * (size_t)I1) != hipSuccess ||
            hipMalloc((void**)&sl.d_out, sizeof(double) * (s->out_len() + 1)) != hipSuccess ||
            hipHostMalloc((void**)&sl.h_out, sizeof(double) * (s->out_len() + 1), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&sl.h_in, kStagingStart, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(SNECT_E_OOM, "server slot allocation failed");
        }
        sl.h_in_cap = kStagingStart;
    }
    // the first command on a stream binds it to a hardware queue, which is
    // slow: done here for every slot rather than on a request's path
    for (auto& sl : s->slots) {
        std::memset(sl.h_out, 0, sizeof(double) * (s->out_len() + 1));
        if (hipMemcpyAsync(sl.d_out, sl.h_out, sizeof(double) * (s->out_len() + 1), hipMemcpyHostToDevice,
                           sl.stream) != hipSuccess)
            return fail(SNECT_E_HIP, "server slot set-up failed");
    }
    for (auto& sl : s->slots)
        if (hipStreamSynchronize(sl.stream) != hipSuccess) return fail(SNECT_E_HIP, "server slot set-up failed");
    ctx->live_problems++;
    s->counted = true;
    *out = s;
    return SNECT_OK;
}

int snect_server_destroy(snect_server* s)
{
    if (!s) return SNECT_E_ARG;
    if (s->counted && s->ctx) s->ctx->live_problems--;
    (void)hipSetDevice(s->device);
    for (auto& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.k0) (void)hipEventDestroy(sl.k0);
        if (sl.k1) (void)hipEventDestroy(sl.k1);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.d_part) (void)hipFree(sl.d_part);
        if (sl.d_scores) (void)hipFree(sl.d_scores);
        if (sl.d_out) (void)hipFree(sl.d_out);
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
    }
    if (s->d_W) (void)hipFree(s->d_W);
    if (s->d_anrm) (void)hipFree(s->d_anrm);
    if (s->d_At) (void)hipFree(s->d_At);
    if (s->d_pool) (void)hipFree(s->d_pool);
    delete s;
    return SNECT_OK;
}

}  // extern "C"

// Admission of one request; `timed` brackets its kernels with the slot's
// timing events.
static int submit_request(snect_server* s, int64_t nnz, const int32_t* j, const int32_t* k, const float* x,
                          int64_t* ticket, bool timed)
{
    if (!s || !ticket || nnz < 0 || nnz >= (int64_t(1) << 31) || (nnz > 0 && (!j || !k || !x)))
        return srv_err(s, SNECT_E_ARG, "bad request arguments");
    int free_slot = -1;
    for (size_t i = 0; i < s->slots.size(); ++i)
        if (!s->slots[i].busy) {
            free_slot = (int)i;
            break;
        }
    const size_t bj = align_up((size_t)nnz * 4), bytes = std::max<size_t>(3 * bj, kAlign);
    if (bytes > s->pool.size) return srv_err(s, SNECT_E_UNSUPPORTED, "request larger than the request pool");
    if (free_slot < 0) return srv_err(s, SNECT_E_BUSY, "no free slot");
    Slot& sl = s->slots[free_slot];
    (void)hipSetDevice(s->device);
    if (sl.h_in_cap < bytes) {
        // grows to the next power of two (pinned allocations and frees are
        // slow and can wait for the device, so they are kept rare)
        size_t cap = kStagingStart;
        while (cap < bytes) cap *= 2;
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        sl.h_in = nullptr;
        sl.h_in_cap = 0;
        if (hipHostMalloc((void**)&sl.h_in, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return srv_err(s, SNECT_E_OOM, "pinned staging allocation failed");
        }
        sl.h_in_cap = cap;
    }
    // copy the cells to the slot's pinned staging and check them in the same
    // branch-free pass, four cells per step.  The staging is written with
    // non-temporal stores (no read of the destination lines, nothing of it
    // left in the caches; its three arrays start 256-byte aligned); the store
    // fence after the pass orders them before the upload is queued.
    {
        int32_t* hj = reinterpret_cast<int32_t*>(sl.h_in);
        int32_t* hk = reinterpret_cast<int32_t*>(sl.h_in + bj);
        float* hx = reinterpret_cast<float*>(sl.h_in + 2 * bj);
        const uint32_t I2 = (uint32_t)s->I2, I3 = (uint32_t)s->I3;
        // unsigned v < I: (v ^ 2^31) < (I ^ 2^31) as signed 32-bit integers
        const __m128i bias = _mm_set1_epi32(INT32_MIN), expo = _mm_set1_epi32(0x7f800000);
        const __m128i lim2 = _mm_set1_epi32((int32_t)(I2 ^ 0x80000000u)), lim3 = _mm_set1_epi32((int32_t)(I3 ^ 0x80000000u));
        __m128i ok = _mm_set1_epi32(-1), inf = _mm_setzero_si128();
        int64_t t = 0;
        for (; t + 4 <= nnz; t += 4) {
            const __m128i vj = _mm_loadu_si128(reinterpret_cast<const __m128i*>(j + t));
            const __m128i vk = _mm_loadu_si128(reinterpret_cast<const __m128i*>(k + t));
            const __m128i vx = _mm_loadu_si128(reinterpret_cast<const __m128i*>(x + t));
            ok = _mm_and_si128(ok, _mm_and_si128(_mm_cmpgt_epi32(lim2, _mm_xor_si128(vj, bias)),
                                                 _mm_cmpgt_epi32(lim3, _mm_xor_si128(vk, bias))));
            inf = _mm_or_si128(inf, _mm_cmpeq_epi32(_mm_and_si128(vx, expo), expo));  // Inf or NaN
            _mm_stream_si128(reinterpret_cast<__m128i*>(hj + t), vj);
            _mm_stream_si128(reinterpret_cast<__m128i*>(hk + t), vk);
            _mm_stream_si128(reinterpret_cast<__m128i*>(hx + t), vx);
        }
        uint32_t bad_index = _mm_movemask_epi8(ok) != 0xffff, bad_value = _mm_movemask_epi8(inf) != 0;
        for (; t < nnz; ++t) {
            const int32_t jt = j[t], kt = k[t];
            const float xt = x[t];
            uint32_t xb;
            std::memcpy(&xb, &xt, 4);
            bad_index |= (uint32_t)((uint32_t)jt >= I2) | (uint32_t)((uint32_t)kt >= I3);
            bad_value |= (uint32_t)((xb & 0x7f800000u) == 0x7f800000u);
            hj[t] = jt;
            hk[t] = kt;
            hx[t] = xt;
        }
        _mm_sfence();
        if (bad_index) return srv_err(s, SNECT_E_INDEX, "request cell out of range");
        if (bad_value) return srv_err(s, SNECT_E_ARG, "non-finite request value");
    }
    size_t off = 0;
    if (!s->pool.take(bytes, &off)) return srv_err(s, SNECT_E_BUSY, "request pool full");
    char* dbase = s->d_pool + off;
    hipError_t e = hipSuccess;
    if (nnz > 0) e = hipMemcpyAsync(dbase, sl.h_in, 3 * bj, hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess && timed) e = hipEventRecord(sl.k0, sl.stream);
    if (e == hipSuccess)
        e = launch_serve_request(reinterpret_cast<const int32_t*>(dbase), reinterpret_cast<const int32_t*>(dbase + bj),
                                 reinterpret_cast<const float*>(dbase + 2 * bj), (int)nnz, s->d_W, s->I2, s->J1,
                                 s->cfg.lambda, s->cfg.pg_iters, s->d_At, s->d_anrm, s->I1, s->cfg.topk, sl.d_part,
                                 sl.d_scores, sl.d_out, reinterpret_cast<int*>(sl.d_out + s->out_len()), sl.stream);
    if (e == hipSuccess && timed) e = hipEventRecord(sl.k1, sl.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.h_out, sl.d_out, sizeof(double) * (s->out_len() + 1), hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(sl.stream);
        s->pool.give(off, bytes);
        return srv_err(s, SNECT_E_HIP, std::string("request launch: ") + hipGetErrorString(e));
    }
    sl.busy = true;
    sl.off = off;
    sl.bytes = bytes;
    sl.ticket = s->next_ticket++;
    s->where[sl.ticket] = free_slot;
    *ticket = sl.ticket;
    return SNECT_OK;
}

extern "C" {

int snect_server_submit(snect_server* s, int64_t nnz, const int32_t* j, const int32_t* k, const float* x,
                        int64_t* ticket)
{
    return submit_request(s, nnz, j, k, x, ticket, false);
}

int snect_server_poll(snect_server* s, int64_t ticket, double* u, int32_t* idx, double* score)
{
    if (!s) return SNECT_E_ARG;
    auto it = s->where.find(ticket);
    if (it == s->where.end()) return srv_err(s, SNECT_E_ARG, "unknown ticket");
    Slot& sl = s->slots[it->second];
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) return srv_err(s, SNECT_E_HIP, std::string("request: ") + hipGetErrorString(q));
    const int J1 = s->J1, K = s->cfg.topk;
    if (u) std::memcpy(u, sl.h_out, sizeof(double) * J1);
    if (score) std::memcpy(score, sl.h_out + J1, sizeof(double) * K);
    if (idx)
        for (int t = 0; t < K; ++t) idx[t] = (int32_t)sl.h_out[J1 + K + t];
    const int bad = *reinterpret_cast<const int*>(sl.h_out + s->out_len());
    s->pool.give(sl.off, sl.bytes);
    sl.busy = false;
    s->where.erase(it);
    if (bad) return srv_err(s, SNECT_E_ARG, "fold-in system not positive definite (add lambda > 0)");
    return 1;
}

int snect_server_replay(snect_server* s, int64_t nreq, const double* arrival_s, const int64_t* offsets,
                        const int32_t* j, const int32_t* k, const float* x, double* latency_s, double* u,
                        int32_t* idx, double* score, int32_t* status, double* wall_s, double* gpu_busy_s)
{
    if (!s || nreq < 0 || !arrival_s || !offsets || !latency_s) return SNECT_E_ARG;
    const int J1 = s->J1, K = s->cfg.topk;
    std::vector<int64_t> tick(nreq, -1);
    std::vector<int64_t> inflight;
    int64_t next = 0, done = 0;
    // device-busy time: the union of the requests' kernel windows, each read
    // from its slot's timing events relative to a reference event recorded
    // (and completed) before the first admission
    const bool timed = gpu_busy_s != nullptr;
    hipEvent_t ref = nullptr;
    std::vector<std::pair<float, float>> win;
    if (timed) {
        (void)hipSetDevice(s->device);
        if (hipEventCreate(&ref) != hipSuccess || hipEventRecord(ref, s->slots[0].stream) != hipSuccess ||
            hipEventSynchronize(ref) != hipSuccess) {
            if (ref) (void)hipEventDestroy(ref);
            return srv_err(s, SNECT_E_HIP, "replay timing event");
        }
        win.reserve((size_t)nreq);
    }
    const double t0 = now_s();
    while (done < nreq) {
        // completions first, so that a finished request is timed before the
        // host prepares the next ones
        for (size_t t = 0; t < inflight.size();) {
            const int64_t r = inflight[t];
            const int si = s->where.count(tick[r]) ? s->where[tick[r]] : -1;
            const int rc = snect_server_poll(s, tick[r], u ? u + r * J1 : nullptr, idx ? idx + r * K : nullptr,
                                             score ? score + r * K : nullptr);
            if (rc == 0) {
                ++t;
                continue;
            }
            latency_s[r] = (now_s() - t0) - arrival_s[r];
            if (status) status[r] = rc == 1 ? SNECT_OK : rc;
            float a = 0.f, b = 0.f;
            if (timed && si >= 0 && hipEventElapsedTime(&a, ref, s->slots[si].k0) == hipSuccess &&
                hipEventElapsedTime(&b, ref, s->slots[si].k1) == hipSuccess)
                win.emplace_back(a, b);
            ++done;
            inflight[t] = inflight.back();
            inflight.pop_back();
        }
        // admit every arrived request that fits, in arrival order
        const double now = now_s() - t0;
        while (next < nreq && arrival_s[next] <= now) {
            const int64_t a = offsets[next], n = offsets[next + 1] - a;
            int64_t tk = -1;
            const int rc = submit_request(s, n, j + a, k + a, x + a, &tk, timed);
            if (rc == SNECT_E_BUSY) break;  // retry after completions
            if (rc != SNECT_OK) {           // a malformed request fails alone
                latency_s[next] = (now_s() - t0) - arrival_s[next];
                if (status) status[next] = rc;
                ++next;
                ++done;
                continue;
            }
            tick[next] = tk;
            inflight.push_back(next);
            ++next;
        }
    }
    if (wall_s) *wall_s = now_s() - t0;
    if (timed) {
        (void)hipGetLastError();
        (void)hipEventDestroy(ref);
        std::sort(win.begin(), win.end());
        double busy_ms = 0.0, lo = 0.0, hi = -1.0;
        for (const auto& w : win) {
            if (w.first > hi) {
                if (hi > lo) busy_ms += hi - lo;
                lo = w.first;
                hi = w.second;
            } else {
                hi = std::max<double>(hi, w.second);
            }
        }
        if (hi > lo) busy_ms += hi - lo;
        *gpu_busy_s = 1e-3 * busy_ms;
    }
    return SNECT_OK;
}

}  // extern "C"
