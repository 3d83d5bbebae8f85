// C ABI of the Radic library: argument validation, workspace layout, launch-shape
// selection and dispatch to the HIP kernels.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "radic_internal.h"
#include "split.h"

namespace radic {

hipError_t launch_float(int m, int prec, bool export_terms, const FloatJob& J, int grid, int block, hipStream_t s);
hipError_t launch_finalize_float(const Partial* parts, int G, const Partial* fb_parts, int G2, const DetHeader* h,
                                 radic_f64_result* out, unsigned long long count, int use_scale, hipStream_t s);
int refactor_grid(int grid, int block);
hipError_t launch_refactor(int m, const FloatJob& J, int grid, int block, hipStream_t s);
hipError_t launch_zero_result(radic_f64_result* out, hipStream_t s);
hipError_t upload_binomials_float(const unsigned long long* host_table);
hipError_t upload_binomials_int(const unsigned long long* host_table);
hipError_t upload_primes(const unsigned* primes, int count);
hipError_t launch_int_bound(const int* A, int m, int n, long long lda, void* ws, int prime_count, hipStream_t s);
hipError_t launch_int_main(const int* A, int m, int n, long long lda, unsigned long long count, int spl,
                           int grid_x, int n_primes, int block, void* ws, hipStream_t s);
hipError_t launch_int_finalize(int grid_x, int launched, void* ws, void* out, hipStream_t s);
int int_shared_lds(int m, int n, int waves, int cap);
size_t run_bytes();
hipError_t launch_2xn(const double* A, long long lda, long long n, int G, void* runs, void* flag,
                      radic_f64_result* out, hipStream_t s);
hipError_t upload_binomials_wide(const unsigned long long* host_table);
hipError_t launch_wide(const FloatJob& J, int spl, int grid, hipStream_t s);
hipError_t launch_int_shared(const int* A, int m, int n, long long lda, unsigned long long total,
                             unsigned long long n_prefix, unsigned colex_pairs, unsigned long long colex_blocks,
                             int cap, int grid_x, int n_primes, int block, void* ws, hipStream_t s);
size_t int_workspace_bytes();
hipError_t upload_binomials_batched(const unsigned long long* t);
hipError_t upload_primes_batched(const unsigned* primes, int count);
size_t batched_workspace_bytes(int batch);
void host_batch_chunking(int kind, unsigned long long total, int spl, unsigned long long* chunk,
                         unsigned long long* nchunks);
hipError_t launch_batched(const radic_matrix_desc* desc, int batch, const double* f64, const int* i32, int prec,
                          double tau, int spl_float, int spl_int, int prime_count, radic_batch_result* out,
                          void* ws, hipStream_t s);
size_t int_result_size();
int int_lds(int m, int n);
int float_lds_bytes(int m, int n, int prec, int waves);
hipError_t upload_binomials_shared(const unsigned long long* host_table);
int shared_lds(int m, int n, int prec, int waves, int cap);
hipError_t launch_shared(int m, int prec, const FloatJob& J, int grid, int block, hipStream_t s);
hipError_t upload_binomials_shared3(const unsigned long long* host_table);
int shared3_lds(int m, int n, int prec, int waves, int cap);
int shared3_slot_bytes(int prec);
hipError_t launch_shared3(int m, int prec, const FloatJob& J, int grid, int block, hipStream_t s);

constexpr int kBinomRows = RADIC_MAX_N + 1;
constexpr int kBinomCols = 33;
constexpr size_t kHeaderBytes = 256;
constexpr int kMaxLds = 64 * 1024;
constexpr int kSharedLds = 50 * 1024;   // dynamic LDS per prefix-shared workgroup (three per 160 KiB compute unit)
constexpr unsigned long long kRankLimit = 1ull << 63;

// ---------------------------------------------------------------- binomials
int host_binomial(int a, int b, unsigned long long* out) {
    *out = 0;
    if (a < 0 || b < 0 || b > a) return RADIC_OK;
    if (b > a - b) b = a - b;
    unsigned __int128 v = 1;
    for (int i = 1; i <= b; ++i) {
        v = v * (unsigned __int128)(a - b + i) / (unsigned __int128)i;   // exact at every step
        if (v > (unsigned __int128)~0ull) return RADIC_EOVERFLOW;
    }
    *out = (unsigned long long)v;
    return RADIC_OK;
}

// ---------------------------------------------------------------- error reporting
static thread_local char g_last_error[256] = "";

static int device_error(const char* what, hipError_t e) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
    if (std::getenv("RADIC_LOG")) std::fprintf(stderr, "[radic] %s\n", g_last_error);
    return RADIC_EDEVICE;
}

static int host_error(int status, const char* what) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s", what);
    if (std::getenv("RADIC_LOG")) std::fprintf(stderr, "[radic] %s\n", g_last_error);
    return status;
}

// ---------------------------------------------------------------- static scratch
// The workspace of radic_det_batched_noalloc: a file-scope device array, so
// that the call allocates nothing.  Every device the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address is taken once per device at
// set-up (ensure_device, with that device current) and only that address is
// used.  Sized for kScratchBatch matrices of the batched layout (checked at
// set-up).
constexpr int kScratchBatch = 4096;
constexpr size_t kScratchBytes = (size_t)36 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void* g_scratch[64];   // per device: the address of that device's scratch

// ---------------------------------------------------------------- primes of the exact path
// Deterministic Miller-Rabin: bases 2, 3, 5, 7 decide every n < 3,215,031,751.
static bool is_prime_u32(unsigned n) {
    if (n < 2) return false;
    for (unsigned d : {2u, 3u, 5u, 7u}) {
        if (n == d) return true;
        if (n % d == 0) return false;
    }
    unsigned long long d = n - 1;
    int r = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++r;
    }
    for (unsigned long long a : {2ull, 3ull, 5ull, 7ull}) {
        unsigned long long x = 1, b = a % n, e = d;
        while (e) {
            if (e & 1) x = x * b % n;
            b = b * b % n;
            e >>= 1;
        }
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int i = 1; i < r; ++i) {
            x = x * x % n;
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

static std::vector<unsigned> default_primes() {
    std::vector<unsigned> v;
    for (unsigned c = 0x7FFFFFFFu; v.size() < (size_t)RADIC_MAX_PRIMES; c -= 2)
        if (is_prime_u32(c)) v.push_back(c);
    return v;
}

static std::vector<unsigned> g_primes = default_primes();
static int g_prime_version = 1;

// ---------------------------------------------------------------- per-device state
static std::mutex g_mu;
static bool g_dev_ready[64];
static int g_dev_prime_version[64];

static int g_dev_lds[64];   // dynamic LDS a workgroup may use, per device

static int ensure_device(int* lds_limit = nullptr) {
    int dev = 0;
    hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return device_error("hipGetDevice", ge);
    if (dev < 0 || dev >= 64) return RADIC_ENOTSUP;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_dev_prime_version[dev] != g_prime_version) {
        hipError_t pe = upload_primes(g_primes.data(), (int)g_primes.size());
        if (pe == hipSuccess) pe = upload_primes_batched(g_primes.data(), (int)g_primes.size());
        if (pe != hipSuccess) return device_error("upload of the prime set", pe);
        g_dev_prime_version[dev] = g_prime_version;
    }
    if (g_dev_ready[dev]) {
        if (lds_limit) *lds_limit = g_dev_lds[dev];
        return RADIC_OK;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds < kMaxLds)
        lds = kMaxLds;
    g_dev_lds[dev] = lds;
    if (lds_limit) *lds_limit = lds;
    std::vector<unsigned long long> t((size_t)kBinomRows * kBinomCols, 0);
    for (int x = 0; x < kBinomRows; ++x)
        for (int y = 0; y < kBinomCols; ++y) {
            unsigned long long v = 0;
            if (host_binomial(x, y, &v) != RADIC_OK) v = ~0ull;   // saturate; never used
            t[(size_t)x * kBinomCols + y] = v;
        }
    hipError_t ue = upload_binomials_float(t.data());
    if (ue == hipSuccess) ue = upload_binomials_int(t.data());
    if (ue == hipSuccess) ue = upload_binomials_batched(t.data());
    if (ue == hipSuccess) ue = upload_binomials_shared(t.data());
    if (ue == hipSuccess) ue = upload_binomials_shared3(t.data());
    if (ue == hipSuccess) ue = upload_binomials_wide(t.data());
    if (ue != hipSuccess) return device_error("upload of the binomial table", ue);
    if (batched_workspace_bytes(kScratchBatch) > kScratchBytes)
        return host_error(RADIC_ENOTSUP, "static scratch smaller than the batched layout needs");
    void* sp = nullptr;
    const hipError_t se = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
    if (se != hipSuccess) return device_error("hipGetSymbolAddress of the static scratch", se);
    if (sp == nullptr || (reinterpret_cast<uintptr_t>(sp) & 255u))
        return host_error(RADIC_EDEVICE, "static scratch address missing or misaligned");
    g_scratch[dev] = sp;
    g_dev_ready[dev] = true;
    return RADIC_OK;
}

// ---------------------------------------------------------------- launch shapes
struct Shape {
    int spl;
    int block;
    bool spl_set = false;   // spl tuned or forced (not the default)
};
// Prefix-shared paths: about 64 * spl minors per block of a whole rank space
// (subsets per lane per block); their default spl.
constexpr int kSharedSplFloat = 64;
constexpr int kSharedSplInt = 32;
// Tuned launch shapes, (kind, prec, m, column bucket) -> shape.  A shape is
// tuned on one n and serves the n of its bucket: every n up to 16, then runs of
// 8 up to 64, then of 32.
// tuned launch shapes keyed by (kind, precision, m, n bucket, enumeration)
static std::map<std::tuple<int, int, int, int, int>, Shape> g_tuned;
static int n_bucket(int n) { return n <= 16 ? n : (n <= 64 ? (n + 7) / 8 * 8 : (n + 31) / 32 * 32); }
static int g_force_spl = 0, g_force_block = 0;
static int g_enumeration = RADIC_ENUM_AUTO;
static double g_tau = 1.0 / 1024.0;

static Shape default_shape(int kind, int prec, int m, int n) {
    (void)n;
    Shape s{8, 256};
    if (kind == RADIC_WS_BATCHED) {
        // chunks of at least 64 * 32 ranks: measured on the 4096-matrix batch
        // (62.0 / 51.2 / 47.5 / 46.6 / 49.1 / 55.1 ms at spl 4 / 8 / 16 / 32 / 64 / 128)
        s.spl = 32;
        return s;
    }
    if (m <= 3) s.spl = 32;
    return s;
}

static Shape pick_shape(int kind, int prec, int m, int n) {
    Shape s = default_shape(kind, prec, m, n);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        const int mode = kind == RADIC_WS_BATCHED ? 0 : g_enumeration;
        auto it = g_tuned.find(std::make_tuple(kind, prec, m, n_bucket(n), mode));
        if (it != g_tuned.end()) {
            s = it->second;
            s.spl_set = true;
        }
        if (g_force_spl > 0) {
            s.spl = g_force_spl;
            s.spl_set = true;
        }
        if (g_force_block > 0) s.block = g_force_block;
    }
    return s;
}

// ---------------------------------------------------------------- profiling hook
static bool g_prof = false;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_events;
static std::vector<hipEvent_t> g_event_pool;

static hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    // timing only: without the system-scope fence at the event the kernel
    // that follows is not held back by a cache write-back
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit ProfScope(hipStream_t st) : s(st) {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_prof) return;
        a = take_event();
        b = take_event();
        if (a && b && hipEventRecord(a, s) == hipSuccess) return;
        release();   // an unrecorded pair is not timed
    }
    ~ProfScope() {
        if (!a || !b) return;
        const bool ok = hipEventRecord(b, s) == hipSuccess;
        std::lock_guard<std::mutex> lk(g_mu);
        if (ok) g_prof_events.emplace_back(a, b);
        else release();
    }
    void release() {   // caller holds g_mu
        if (a) g_event_pool.push_back(a);
        if (b) g_event_pool.push_back(b);
        a = b = nullptr;
    }
};

TimedLaunch& timed_launch() {
    static thread_local TimedLaunch t;
    return t;
}

// Times the one main kernel that launch_timed dispatches during its lifetime:
// the events are bound to that dispatch instead of being recorded around it.
struct KernelTimer {
    hipEvent_t a = nullptr, b = nullptr;
    KernelTimer() {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_prof) return;
        a = take_event();
        b = take_event();
        if (a && b) timed_launch() = TimedLaunch{a, b, false};
        else release();
    }
    ~KernelTimer() {
        const bool used = timed_launch().used;
        timed_launch() = TimedLaunch{};
        if (!a || !b) return;
        std::lock_guard<std::mutex> lk(g_mu);
        if (used) g_prof_events.emplace_back(a, b);
        else release();
    }
    void release() {   // caller holds g_mu
        if (a) g_event_pool.push_back(a);
        if (b) g_event_pool.push_back(b);
        a = b = nullptr;
    }
};

// ---------------------------------------------------------------- two-sided blocks
// Number of two-sided blocks (the kernels' split_block): per last column v and
// side s, split_count prefixes in runs of colex_run(n-1-v, K).
static unsigned long long split_block_count(int m, int n, unsigned K) {
    const int P = m - 2;
    unsigned long long total = 0;
    for (int v = P - 1; v <= n - 3; ++v) {
        const unsigned long long k = (unsigned long long)colex_run(n - 1 - v, K);
        for (int side = 0; side < 2; ++side) {
            int a, b, imin;
            bool on;
            split_shape(P, n, side, v, a, b, imin, on);
            if (!on) continue;
            unsigned long long cnt = 0;
            for (int i = imin; i <= P - 1; ++i) {
                unsigned long long x = 0, y = 0;
                host_binomial(a, i, &x);
                host_binomial(b, P - 1 - i, &y);
                cnt += x * y;
            }
            total += (cnt + k - 1) / k;
        }
    }
    return total;
}

// ---------------------------------------------------------------- validation helpers
static int check_workspace(void* ws, size_t bytes, size_t need) {
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) || bytes < need) return RADIC_EWORKSPACE;
    return RADIC_OK;
}

// Single-matrix workspace: header | partials[kMaxGrid] | refactor partials[kMaxGrid] |
// per-wave segment counts [kMaxGrid*4] | deferral entries [kDeferEntries] (16 B each), split
// evenly over the launch's waves
static size_t ws_partials() { return kHeaderBytes; }
static size_t ws_fb_partials() { return ws_partials() + sizeof(Partial) * (size_t)kMaxGrid; }
static size_t ws_fb_count() { return ws_fb_partials() + sizeof(Partial) * (size_t)kMaxGrid; }
static size_t ws_fb_entries() { return ws_fb_count() + sizeof(unsigned) * (size_t)kMaxGrid * 4; }
// FP32-bulk deferral entries for an m x n matrix: one per 64 minors (several
// times the flagged share of random minors, a few per mille), at least
// kDeferEntries and at most kDeferEntriesMax.  A wave whose share overflows
// redoes its blocks in double, which is correct but slow.
constexpr unsigned long long kDeferEntriesMax = 1ull << 25;
static unsigned long long defer_entries_for(int m, int n) {
    unsigned long long total = 0;
    if (m >= 1 && n >= m && host_binomial(n, m, &total) != RADIC_OK) total = ~0ull;
    unsigned long long e = total / 64;
    if (e < (unsigned long long)kDeferEntries) e = kDeferEntries;
    if (e > kDeferEntriesMax) e = kDeferEntriesMax;
    return e;
}
static size_t det_workspace_bytes(int m, int n) { return ws_fb_entries() + 16 * (size_t)defer_entries_for(m, n); }

// Deferral entries per wave for a launch of `grid` workgroups of `block` threads.
static int defer_cap_for(int grid, int block, unsigned long long entries) {
    const long long waves = (long long)grid * (block / kWave);
    long long c = (long long)entries / (waves > 0 ? waves : 1);
    if (c > 4096) c = 4096;
    return (int)c;
}

static int float_common_checks(const double* dA, int m, int n, long long lda, int prec, int max_m = RADIC_MAX_M) {
    if (!dA || m < 1 || n < 1 || lda < n) return RADIC_EINVAL;
    if (prec != RADIC_FP64 && prec != RADIC_FP32_BULK) return RADIC_EINVAL;
    if (m > n) return RADIC_OK;
    if (m > max_m || n > RADIC_MAX_N) return RADIC_ENOTSUP;
    return RADIC_OK;
}

static int zero_result(radic_f64_result* out, hipStream_t s) {
    hipError_t e = launch_zero_result(out, s);
    return e == hipSuccess ? RADIC_OK : device_error("launch of the zero-result kernel", e);
}

// Each wave keeps its own copy of A in LDS; for wide matrices use fewer waves
// per workgroup so that the workgroup's LDS stays within kMaxLds.
static bool fit_lds(int m, int n, int prec, Shape& sh) {
    while (float_lds_bytes(m, n, prec, sh.block / kWave) > kMaxLds) {
        if (sh.block <= kWave) return false;
        sh.block -= kWave;
    }
    return true;
}

static int grid_for(unsigned long long chunks, int block) {
    const unsigned long long wave_chunks = (chunks + kWave - 1) / kWave;
    const unsigned long long wpb = (unsigned long long)(block / kWave);
    unsigned long long g = (wave_chunks + wpb - 1) / wpb;
    if (g > (unsigned long long)kMaxGrid) g = kMaxGrid;
    if (g < 1) g = 1;
    return (int)g;
}

// Host unranking (Section 4) into 0-based columns.
static void host_unrank0(int m, int n, unsigned long long q, int* cols) {
    int c = 0;
    for (int k = 0; k < m; ++k) {
        for (;;) {
            unsigned long long w = 0;
            host_binomial(n - 1 - c, m - 1 - k, &w);
            if (q < w) break;
            q -= w;
            ++c;
        }
        cols[k] = c++;
    }
}

// Number of the prefix (first m-kt columns) of the sequence of rank q, in the
// dictionary order of the (m-kt)-subsets of the first n-kt columns.
static unsigned long long host_prefix_index(int m, int n, unsigned long long q, int kt) {
    int cols[RADIC_MAX_M];
    host_unrank0(m, n, q, cols);
    const int P = m - kt;
    unsigned long long r = 0;
    int prev = -1;
    for (int k = 0; k < P; ++k) {
        for (int v = prev + 1; v < cols[k]; ++v) {
            unsigned long long w = 0;
            host_binomial(n - kt - 1 - v, P - 1 - k, &w);
            r += w;
        }
        prev = cols[k];
    }
    return r;
}

// The float enumeration of a call: 0 per-minor, 2 prefix-shared (minors with
// equal first m-2 columns share those LU steps), 3 group-shared (equal first
// m-3 columns).  The shared kernels cover 3 <= m <= 12 in both precisions
// (group-shared from m = 4).  The automatic choice is prefix-shared (measured
// at least as fast as group-shared on the 8 x 32 workload, and faster than the
// per-minor kernel at every m it covers).
static int float_enumeration(int m, int n, int prec) {
    int mode;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        mode = g_enumeration;
    }
    if (mode == RADIC_ENUM_PER_MINOR) return 0;
    const bool ok2 = m >= 3 && m <= 12;
    const bool ok3 = ok2 && m >= 4;
    if (mode == RADIC_ENUM_GROUP_SHARED) return ok3 ? 3 : (ok2 ? 2 : 0);
    return ok2 ? 2 : 0;
}

// Projected-column slots per wave: what the workgroup LDS budget leaves after
// the per-wave records, at least one prefix of the widest kind (n - m + kt
// columns) and at most what a block of prefixes can fill.
static int shared_cap(int kt, int m, int n, int prec, int waves, int lds_limit) {
    const int need = n - m + kt;
    const int slot = kt == 2 ? 16 : shared3_slot_bytes(prec);   // bytes per projected-column slot
    const int fixed = kt == 2 ? shared_lds(m, n, prec, waves, 0) : shared3_lds(m, n, prec, waves, 0);
    const int budget = kSharedLds < lds_limit ? kSharedLds : lds_limit;
    int cap = (budget - fixed) / (waves * slot);
    const int most = (kt == 2 ? kPrefixBlock : kGroupBlock) * need;
    if (cap > most) cap = most;
    return cap > need ? cap : need;
}

static int det_range_impl(const double* dA, int m, int n, long long lda, int prec, unsigned long long q_begin,
                          unsigned long long count, bool whole, radic_f64_result* dOut, void* dWork,
                          size_t work_bytes, hipStream_t stream) {
    if (!dOut) return RADIC_EINVAL;
    int rc = float_common_checks(dA, m, n, lda, prec, RADIC_MAX_M_WIDE);
    if (rc != RADIC_OK) return rc;
    int lds_limit = kMaxLds;
    if ((rc = ensure_device(&lds_limit)) != RADIC_OK) return rc;
    if (m > n) return zero_result(dOut, stream);
    unsigned long long total = 0;
    if (host_binomial(n, m, &total) != RADIC_OK || total >= kRankLimit) return RADIC_EOVERFLOW;
    if ((rc = check_workspace(dWork, work_bytes, det_workspace_bytes(m, n))) != RADIC_OK) return rc;
    if (whole) {
        q_begin = 0;
        count = total;
    } else {
        if (q_begin >= total) count = 0;
        else if (count > total - q_begin) count = total - q_begin;
    }
    if (count == 0) return zero_result(dOut, stream);
    if (m > RADIC_MAX_M) {
        // wide minors: a group of 32 lanes per minor, in double
        FloatJob J{};
        J.A = dA;
        J.lda = lda;
        J.m = m;
        J.n = n;
        J.q_begin = q_begin;
        J.count = count;
        unsigned char* ws = static_cast<unsigned char*>(dWork);
        J.header = reinterpret_cast<DetHeader*>(ws);
        J.partials = reinterpret_cast<Partial*>(ws + ws_partials());
        const int spl = 16;
        const unsigned long long chunks = (count + spl - 1) / spl;
        unsigned long long g = (chunks + 3) / 4;   // 4 groups per workgroup
        const int grid = (int)(g > (unsigned long long)kMaxGrid ? kMaxGrid : (g < 1 ? 1 : g));
        hipError_t e;
        {
            KernelTimer timer;
            e = launch_wide(J, spl, grid, stream);
        }
        if (e != hipSuccess) return device_error("launch of the wide-minor kernel", e);
        e = launch_finalize_float(J.partials, grid, nullptr, 0, J.header, dOut, count, 0, stream);
        return e == hipSuccess ? RADIC_OK : device_error("launch of the finalize kernel", e);
    }
    // FP32-bulk over fewer minors than a float sum can absorb: the double
    // kernel, with every minor reported as done in double
    const bool all_double = prec == RADIC_FP32_BULK && count < kF32MinMinors;
    if (all_double) prec = RADIC_FP64;
    Shape sh = pick_shape(RADIC_WS_DET, prec, m, n);
    if (!fit_lds(m, n, prec, sh)) return RADIC_ENOTSUP;

    unsigned char* ws = static_cast<unsigned char*>(dWork);
    FloatJob J{};
    J.A = dA;
    J.lda = lda;
    J.m = m;
    J.n = n;
    J.q_begin = q_begin;
    J.count = count;
    J.spl = sh.spl;
    J.chunks = (count + sh.spl - 1) / sh.spl;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        J.tau = effective_tau(g_tau, count);
    }
    J.header = reinterpret_cast<DetHeader*>(ws);
    J.partials = reinterpret_cast<Partial*>(ws + ws_partials());
    J.fb_partials = reinterpret_cast<Partial*>(ws + ws_fb_partials());
    J.fb_count = reinterpret_cast<unsigned*>(ws + ws_fb_count());
    J.fb_entries = reinterpret_cast<unsigned*>(ws + ws_fb_entries());
    J.total = total;
    int grid = grid_for(J.chunks, sh.block);
    const int kt = float_enumeration(m, n, prec);
    bool shared = kt != 0;
    if (shared) {
        auto lds = [&](int waves, int cap) {
            return kt == 2 ? shared_lds(m, n, prec, waves, cap) : shared3_lds(m, n, prec, waves, cap);
        };
        J.mapping = kt - 1;
        host_binomial(n - kt, m - kt, &J.n_prefix);
        J.p_begin = host_prefix_index(m, n, q_begin, kt);
        J.p_end = host_prefix_index(m, n, q_begin + count - 1, kt) + 1;
        int block = sh.block;
        J.cap = shared_cap(kt, m, n, prec, block / kWave, lds_limit);
        while (block > kWave && lds(block / kWave, J.cap) > lds_limit) {
            block -= kWave;
            J.cap = shared_cap(kt, m, n, prec, block / kWave, lds_limit);
        }
        if (lds(block / kWave, J.cap) > lds_limit) {
            shared = false;
            J.mapping = 0;
        } else {
            sh.block = block;
            // a whole rank space takes its prefixes in two-sided blocks
            // (heaviest first)
            J.colex = (kt == 2 && J.p_begin == 0 && J.p_end == J.n_prefix) ? 1 : 0;
            J.colex_pairs = 64u * (unsigned)(sh.spl_set ? sh.spl : kSharedSplFloat);
            J.colex_blocks = J.colex ? split_block_count(m, n, J.colex_pairs) : 0;
            const unsigned long long per_block = kt == 2 ? kPrefixBlock : kGroupBlock;
            const unsigned long long blocks =
                J.colex ? J.colex_blocks : (J.p_end - J.p_begin + per_block - 1) / per_block;
            const unsigned long long wpb = (unsigned long long)(block / kWave);
            unsigned long long g = (blocks + wpb - 1) / wpb;
            grid = (int)(g > (unsigned long long)kMaxGrid ? kMaxGrid : (g < 1 ? 1 : g));
        }
    }
    const bool defer = prec == RADIC_FP32_BULK;
    J.defer_cap = defer_cap_for(grid, sh.block, (work_bytes - ws_fb_entries()) / 16);
    hipError_t e;
    {
        KernelTimer timer;
        e = !shared ? launch_float(m, prec, false, J, grid, sh.block, stream)
                    : (kt == 2 ? launch_shared(m, prec, J, grid, sh.block, stream)
                               : launch_shared3(m, prec, J, grid, sh.block, stream));
    }
    if (e != hipSuccess) return device_error("launch of the enumeration kernel", e);
    // the shared kernels refactor their flagged minors at the end of each
    // workgroup up to m = 8; otherwise the refactorisation kernel does
    const bool refactor = defer && !(shared && shared_tail_refactor(m));
    if (refactor) {
        e = launch_refactor(m, J, grid, sh.block, stream);
        if (e != hipSuccess) return device_error("launch of the refactorisation kernel", e);
    }
    e = launch_finalize_float(J.partials, grid, refactor ? J.fb_partials : nullptr, refactor_grid(grid, sh.block),
                              J.header, dOut, count, (defer ? 1 : 0) | (all_double ? 2 : 0), stream);
    return e == hipSuccess ? RADIC_OK : device_error("launch of the finalize kernel", e);
}

}  // namespace radic

using namespace radic;

// ---------------------------------------------------------------- autotuning
namespace {

// Deterministic synthetic inputs for tuning (xorshift64*, Box-Muller free: uniform in [-1, 1)).
struct TuneRng {
    unsigned long long s;
    explicit TuneRng(unsigned long long seed) : s(seed ? seed : 0x9E3779B97F4A7C15ull) {}
    unsigned long long next() {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        return s * 0x2545F4914F6CDD1Dull;
    }
    double uniform() { return (double)(next() >> 11) * (2.0 / 9007199254740992.0) - 1.0; }
};

struct DeviceBuffers {
    std::vector<void*> ptrs;
    ~DeviceBuffers() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    void* alloc(size_t bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
};

// Median over `reps` samples of the time per call of fn() on `stream` (after
// one warm-up), in ms.
template <typename F>
static float time_runs(F fn, hipStream_t stream, int reps, int* rc_out, int calls = 1) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        *rc_out = RADIC_EDEVICE;
        return 0.f;
    }
    std::vector<float> t;
    int rc = fn();
    (void)hipStreamSynchronize(stream);
    for (int r = 0; r < reps && rc == RADIC_OK; ++r) {
        // `calls` calls back to back per sample: after the first, the stream
        // holds queued work, so the host's launch latency drops out
        (void)hipEventRecord(a, stream);
        for (int c = 0; c < calls && rc == RADIC_OK; ++c) rc = fn();
        (void)hipEventRecord(b, stream);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        t.push_back(ms / (float)calls);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *rc_out = rc;
    if (t.empty()) return 0.f;
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace

// Two-sided blocks on the host: the kernels' own enumeration (split.h) over a
// host binomial table C(x, y), x <= n, y <= m (0 where it does not fit 64 bits,
// never read then: the space is below kRankLimit).
static std::vector<unsigned long long> host_binom_table(int n, int m) {
    std::vector<unsigned long long> t((size_t)(n + 1) * (m + 1), 0ull);
    for (int x = 0; x <= n; ++x)
        for (int y = 0; y <= m; ++y) {
            unsigned long long v = 0;
            if (host_binomial(x, y, &v) == RADIC_OK) t[(size_t)x * (m + 1) + y] = v;
        }
    return t;
}

static int split_args(int m, int n, int side, int v) {
    if (m < 3 || m > RADIC_MAX_M || n < m || n > RADIC_MAX_N || side < 0 || side > 1 || v < m - 3 || v > n - 3)
        return RADIC_EINVAL;
    unsigned long long total = 0;
    if (host_binomial(n, m, &total) != RADIC_OK || total >= kRankLimit) return RADIC_EOVERFLOW;
    return RADIC_OK;
}

template <int P>
static void host_split_p(int n, int side, int v, unsigned long long j, const unsigned long long* bt, int stride,
                         unsigned long long* count, int* cols) {
    if (count) *count = split_count<P>(n, side, v, bt, stride);
    if (cols) {
        int c[P];
        split_unrank<P>(j, n, side, v, bt, stride, c);
        for (int k = 0; k < P; ++k) cols[k] = c[k];
    }
}

static void host_split(int m, int n, int side, int v, unsigned long long j, unsigned long long* count, int* cols) {
    const std::vector<unsigned long long> bt = host_binom_table(n, m);
    const unsigned long long* b = bt.data();
    const int st = m + 1;
    switch (m - 2) {
#define RADIC_CASE(PP) \
    case PP: host_split_p<PP>(n, side, v, j, b, st, count, cols); break;
        RADIC_CASE(1) RADIC_CASE(2) RADIC_CASE(3) RADIC_CASE(4) RADIC_CASE(5) RADIC_CASE(6)
        RADIC_CASE(7) RADIC_CASE(8) RADIC_CASE(9) RADIC_CASE(10)
#undef RADIC_CASE
        default: break;
    }
}

// Primes the exact path's modular kernel is launched for, enough for any int32
// matrix of the shape.  The bound kernel asks for the fewest primes whose
// product exceeds 2 (e_m + 1), e_m the m-th elementary symmetric function of
// the column norms (at least sum |det(A_J)| by Hadamard's inequality).  Entries
// below 2^31 in magnitude give column norms below sqrt(m) 2^31, so
// e_m < C(n, m) (sqrt(m) 2^31)^m; the same rule on that bound, with a bit of
// margin, plus one prime, never asks for fewer.
static int int_prime_upper_bound(int m, int n, const std::vector<unsigned>& primes) {
    unsigned long long c = 0;
    host_binomial(n, m, &c);
    const double need = std::log2((double)c) + m * (31.0 + 0.5 * std::log2((double)m)) + 2.01;
    double have = 0.0;
    int k = 0;
    while (k < (int)primes.size() && have <= need) have += std::log2((double)primes[k++]);
    return std::min((int)primes.size(), k + 1);
}

// Pinned host buffers for the exact result: the CRT kernel writes the result
// straight into one, so reading it back needs no copy command, only the wait
// for the stream.  A pool holds one buffer per call in flight; buffers live as
// long as the process.
static std::mutex g_pin_mu;
static std::vector<void*> g_pin_free;

struct PinnedResult {
    void* p = nullptr;
    PinnedResult() {
        {
            std::lock_guard<std::mutex> lk(g_pin_mu);
            if (!g_pin_free.empty()) {
                p = g_pin_free.back();
                g_pin_free.pop_back();
                return;
            }
        }
        if (hipHostMalloc(&p, int_result_size(), hipHostMallocDefault) != hipSuccess) p = nullptr;
    }
    ~PinnedResult() {
        if (!p) return;
        std::lock_guard<std::mutex> lk(g_pin_mu);
        g_pin_free.push_back(p);
    }
    PinnedResult(const PinnedResult&) = delete;
    PinnedResult& operator=(const PinnedResult&) = delete;
};

extern "C" {

const char* radic_status_string(int status) {
    switch (status) {
        case RADIC_OK: return "RADIC_OK";
        case RADIC_EINVAL: return "RADIC_EINVAL: invalid argument";
        case RADIC_ENOTSUP: return "RADIC_ENOTSUP: shape not supported";
        case RADIC_EOVERFLOW: return "RADIC_EOVERFLOW: count or result does not fit";
        case RADIC_ENOMEM: return "RADIC_ENOMEM: host allocation failed";
        case RADIC_EDEVICE: return "RADIC_EDEVICE: HIP call failed";
        case RADIC_EWORKSPACE: return "RADIC_EWORKSPACE: workspace missing, misaligned or too small";
        case RADIC_ENONFINITE: return "RADIC_ENONFINITE: non-finite input";
        default: return "unknown radic status";
    }
}

int radic_version(void) { return 101; }

const char* radic_last_error(void) { return g_last_error; }

size_t radic_workspace_bytes(int kind, int m, int n, int batch) {
    switch (kind) {
        case RADIC_WS_DET:
            if (m < 1 || n < 1) return 0;
            return det_workspace_bytes(m, n);
        case RADIC_WS_INT:
            if (m < 1 || n < 1) return 0;
            return int_workspace_bytes();
        case RADIC_WS_BATCHED:
            if (batch < 1) return 0;
            return batched_workspace_bytes(batch);
        default:
            (void)batch;
            return 0;
    }
}

int radic_det(const double* dA, int m, int n, int64_t lda, int prec, radic_f64_result* dOut, void* dWork,
              size_t work_bytes, hipStream_t stream) {
    return det_range_impl(dA, m, n, lda, prec, 0, 0, true, dOut, dWork, work_bytes, stream);
}

int radic_det_range(const double* dA, int m, int n, int64_t lda, int prec, uint64_t q_begin, uint64_t count,
                    radic_f64_result* dOut, void* dWork, size_t work_bytes, hipStream_t stream) {
    return det_range_impl(dA, m, n, lda, prec, q_begin, count, false, dOut, dWork, work_bytes, stream);
}

int radic_det_subsets(const double* dA, int m, int n, int64_t lda, int prec, uint64_t q_begin, uint64_t count,
                      double* dTerms, uint8_t* dCols, hipStream_t stream) {
    if (!dTerms) return RADIC_EINVAL;
    int rc = float_common_checks(dA, m, n, lda, prec);
    if (rc != RADIC_OK) return rc;
    if (m > n) return RADIC_EINVAL;   // no terms exist
    if (dCols && n > 255) return RADIC_ENOTSUP;
    if ((rc = ensure_device()) != RADIC_OK) return rc;
    unsigned long long total = 0;
    if (host_binomial(n, m, &total) != RADIC_OK || total >= kRankLimit) return RADIC_EOVERFLOW;
    if (q_begin >= total || count == 0) return RADIC_OK;
    if (count > total - q_begin) count = total - q_begin;
    if (count > (1ull << 31)) return RADIC_EOVERFLOW;
    Shape sh = pick_shape(RADIC_WS_DET, prec, m, n);
    if (!fit_lds(m, n, prec, sh)) return RADIC_ENOTSUP;
    FloatJob J{};
    J.A = dA;
    J.lda = lda;
    J.m = m;
    J.n = n;
    J.q_begin = q_begin;
    J.count = count;
    J.spl = sh.spl;
    J.chunks = (count + sh.spl - 1) / sh.spl;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        J.tau = g_tau;
    }
    J.terms = dTerms;
    J.cols = dCols;
    const int grid = grid_for(J.chunks, sh.block);
    hipError_t e = launch_float(m, prec, true, J, grid, sh.block, stream);
    return e == hipSuccess ? RADIC_OK : device_error("launch of the export kernel", e);
}

int radic_det_2xn(const double* dA, int64_t n, int64_t lda, radic_f64_result* dOut, void* dWork, size_t work_bytes,
                  hipStream_t stream) {
    if (!dA || !dOut || n < 1 || lda < n) return RADIC_EINVAL;
    int rc = check_workspace(dWork, work_bytes, det_workspace_bytes(2, 2));
    if (rc != RADIC_OK) return rc;
    if ((rc = ensure_device()) != RADIC_OK) return rc;
    if (n < 2) return zero_result(dOut, stream);   // m = 2 > n: zero (Definition 3)
    long long G = (n + 4095) / 4096;
    if (G > kMaxGrid) G = kMaxGrid;
    if ((size_t)G * run_bytes() > 16 * (size_t)kDeferEntries) return RADIC_ENOTSUP;
    unsigned char* ws = static_cast<unsigned char*>(dWork);
    hipError_t e;
    {
        ProfScope ps(stream);
        e = launch_2xn(dA, (long long)lda, (long long)n, (int)G, ws + ws_fb_entries(), ws, dOut, stream);
    }
    return e == hipSuccess ? RADIC_OK : device_error("launch of the two-row kernels", e);
}

int radic_det_int_exact(const int32_t* dA, int m, int n, int64_t lda, uint32_t* hMag, int mag_capacity,
                        int* hMagLen, int* hSign, void* dWork, size_t work_bytes, hipStream_t stream) {
    if (!dA || !hMag || !hMagLen || !hSign || mag_capacity < 0 || m < 1 || n < 1 || lda < n) return RADIC_EINVAL;
    *hMagLen = 0;
    *hSign = 0;
    if (m > n) return RADIC_OK;   // Definition 3: zero
    if (m > RADIC_MAX_M || n > RADIC_MAX_N) return RADIC_ENOTSUP;
    unsigned long long total = 0;
    if (host_binomial(n, m, &total) != RADIC_OK || total >= kRankLimit) return RADIC_EOVERFLOW;
    int rc = check_workspace(dWork, work_bytes, int_workspace_bytes());
    if (rc != RADIC_OK) return rc;
    if ((rc = ensure_device()) != RADIC_OK) return rc;
    std::vector<unsigned> primes;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        primes = g_primes;
    }
    const int prime_count = (int)primes.size();
    Shape sh = pick_shape(RADIC_WS_INT, 0, m, n);
    if (int_lds(m, n) > kMaxLds) return RADIC_ENOTSUP;
    PinnedResult pinned;
    if (!pinned.p) return host_error(RADIC_ENOMEM, "pinned buffer for the exact result");
    // 1. bound -> number of primes, on the device; the modular kernel is
    // launched for an upper bound on it that needs no look at A (entries below
    // 2^31 in magnitude), and the primes it does not need exit at once, so the
    // only host synchronisation is the final read-back
    hipError_t e = launch_int_bound(dA, m, n, lda, dWork, prime_count, stream);
    if (e != hipSuccess) return device_error("launch of the bound kernel", e);
    const int k = int_prime_upper_bound(m, n, primes);
    // 2. residue sums per (workgroup, prime), 3. CRT
    int mode;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        mode = g_enumeration;
    }
    const int cap = std::max(256, n - m + 2);
    bool shared = mode != RADIC_ENUM_PER_MINOR && m >= 3 && m <= 10;
    int block = sh.block;
    if (shared) {
        while (block > kWave && int_shared_lds(m, n, block / kWave, cap) > kMaxLds) block -= kWave;
        shared = int_shared_lds(m, n, block / kWave, cap) <= kMaxLds;
    }
    int grid;
    if (shared) {
        unsigned long long n_prefix = 0;
        host_binomial(n - 2, m - 2, &n_prefix);
        const unsigned K = 64u * (unsigned)(sh.spl_set ? sh.spl : kSharedSplInt);
        const unsigned long long blocks = split_block_count(m, n, K);
        const unsigned long long wpb = (unsigned long long)(block / kWave);
        unsigned long long g = (blocks + wpb - 1) / wpb;
        grid = (int)(g > (unsigned long long)kMaxGrid ? kMaxGrid : (g < 1 ? 1 : g));
        KernelTimer timer;
        e = launch_int_shared(dA, m, n, lda, total, n_prefix, K, blocks, cap, grid, k, block, dWork, stream);
    } else {
        const unsigned long long chunks = (total + sh.spl - 1) / sh.spl;
        grid = grid_for(chunks, sh.block);
        KernelTimer timer;
        e = launch_int_main(dA, m, n, lda, total, sh.spl, grid, k, sh.block, dWork, stream);
    }
    if (e != hipSuccess) return device_error("launch of the modular kernel", e);
    e = launch_int_finalize(grid, k, dWork, pinned.p, stream);
    if (e != hipSuccess) return device_error("launch of the CRT kernel", e);
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return device_error("wait for the exact result", e);
    const unsigned char* res = static_cast<const unsigned char*>(pinned.p);
    int fields[4];
    std::memcpy(fields, res, sizeof(fields));   // status, sign, mag_len, n_primes
    if (fields[0] != RADIC_OK) return fields[0];
    *hMagLen = fields[2];
    if (fields[2] > mag_capacity) return RADIC_EOVERFLOW;
    std::memcpy(hMag, res + sizeof(fields), sizeof(uint32_t) * (size_t)fields[2]);
    *hSign = fields[1];
    return RADIC_OK;
}

// The batched launch sequence on a workspace that has been checked; shared by
// radic_det_batched (caller's workspace) and radic_det_batched_noalloc (the
// device's static scratch).
static int batched_launch(const radic_matrix_desc* dDesc, int batch, const double* dF64, const int32_t* dI32,
                          int prec, radic_batch_result* dOut, void* dWork, hipStream_t stream, bool timed) {
    const Shape sf = pick_shape(RADIC_WS_BATCHED, prec, 0, 0);
    const Shape si = pick_shape(RADIC_WS_BATCHED, 2, 0, 0);
    double tau;
    int prime_count;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        tau = g_tau;
        prime_count = (int)g_primes.size();
    }
    hipError_t e;
    if (timed) {
        ProfScope ps(stream);
        e = launch_batched(dDesc, batch, dF64, reinterpret_cast<const int*>(dI32), prec, tau, sf.spl, si.spl,
                           prime_count, dOut, dWork, stream);
    } else {
        e = launch_batched(dDesc, batch, dF64, reinterpret_cast<const int*>(dI32), prec, tau, sf.spl, si.spl,
                           prime_count, dOut, dWork, stream);
    }
    return e == hipSuccess ? RADIC_OK : device_error("launch of the batched kernels", e);
}

int radic_det_batched(const radic_matrix_desc* dDesc, int batch, const double* dF64, const int32_t* dI32, int prec,
                      radic_batch_result* dOut, void* dWork, size_t work_bytes, hipStream_t stream) {
    if (!dDesc || !dOut || batch < 0) return RADIC_EINVAL;
    if (prec != RADIC_FP64 && prec != RADIC_FP32_BULK) return RADIC_EINVAL;
    if (batch == 0) return RADIC_OK;
    if (batch > (1 << 24)) return RADIC_ENOTSUP;
    int rc = check_workspace(dWork, work_bytes, batched_workspace_bytes(batch));
    if (rc != RADIC_OK) return rc;
    if ((rc = ensure_device()) != RADIC_OK) return rc;
    return batched_launch(dDesc, batch, dF64, dI32, prec, dOut, dWork, stream, true);
}

int radic_det_batched_noalloc(const radic_matrix_desc* dDesc, int batch, const double* dF64, const int32_t* dI32,
                              int prec, radic_batch_result* dOut, hipStream_t stream) {
    if (!dDesc || !dOut || batch < 0) return RADIC_EINVAL;
    if (prec != RADIC_FP64 && prec != RADIC_FP32_BULK) return RADIC_EINVAL;
    if (batch == 0) return RADIC_OK;
    if (batch > kScratchBatch)
        return host_error(RADIC_ENOTSUP, "radic_det_batched_noalloc: more matrices than the static scratch holds "
                                         "(at most 4096)");
    int rc = ensure_device();
    if (rc != RADIC_OK) return rc;
    int dev = 0;
    const hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return device_error("hipGetDevice", ge);
    void* ws = g_scratch[dev];   // set by ensure_device for this device
    if (!ws) return host_error(RADIC_EDEVICE, "static scratch not set up on this device");
    // the timing hook is not used here: it may create HIP events
    return batched_launch(dDesc, batch, dF64, dI32, prec, dOut, ws, stream, false);
}

struct GraphHandle {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int radic_batched_graph_create(const radic_matrix_desc* dDesc, int batch, const double* dF64, const int32_t* dI32,
                               int prec, radic_batch_result* dOut, void* dWork, size_t work_bytes, void** hGraph) {
    if (!hGraph) return RADIC_EINVAL;
    *hGraph = nullptr;
    if (!dDesc || !dOut || batch < 1) return RADIC_EINVAL;
    if (prec != RADIC_FP64 && prec != RADIC_FP32_BULK) return RADIC_EINVAL;
    int rc = check_workspace(dWork, work_bytes, batched_workspace_bytes(batch));
    if (rc != RADIC_OK) return rc;
    if ((rc = ensure_device()) != RADIC_OK) return rc;   // table uploads happen outside the capture
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return device_error("hipStreamCreateWithFlags", e);
    GraphHandle* h = new (std::nothrow) GraphHandle();
    if (!h) {
        (void)hipStreamDestroy(cs);
        return RADIC_ENOMEM;
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        int lrc = radic_det_batched(dDesc, batch, dF64, dI32, prec, dOut, dWork, work_bytes, cs);
        hipError_t ee = hipStreamEndCapture(cs, &h->graph);
        if (lrc != RADIC_OK) rc = lrc;
        else if (ee != hipSuccess) rc = device_error("hipStreamEndCapture", ee);
        else {
            ee = hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0);
            if (ee != hipSuccess) rc = device_error("hipGraphInstantiate", ee);
        }
    } else {
        rc = device_error("hipStreamBeginCapture", e);
    }
    (void)hipStreamDestroy(cs);
    if (rc != RADIC_OK) {
        if (h->exec) (void)hipGraphExecDestroy(h->exec);
        if (h->graph) (void)hipGraphDestroy(h->graph);
        delete h;
        return rc;
    }
    *hGraph = h;
    return RADIC_OK;
}

int radic_graph_launch(void* hGraph, hipStream_t stream) {
    if (!hGraph) return RADIC_EINVAL;
    GraphHandle* h = static_cast<GraphHandle*>(hGraph);
    hipError_t e;
    {
        ProfScope ps(stream);
        e = hipGraphLaunch(h->exec, stream);
    }
    return e == hipSuccess ? RADIC_OK : device_error("hipGraphLaunch", e);
}

int radic_graph_destroy(void* hGraph) {
    if (!hGraph) return RADIC_EINVAL;
    GraphHandle* h = static_cast<GraphHandle*>(hGraph);
    hipError_t e1 = h->exec ? hipGraphExecDestroy(h->exec) : hipSuccess;
    hipError_t e2 = h->graph ? hipGraphDestroy(h->graph) : hipSuccess;
    delete h;
    if (e1 != hipSuccess) return device_error("hipGraphExecDestroy", e1);
    if (e2 != hipSuccess) return device_error("hipGraphDestroy", e2);
    return RADIC_OK;
}


int radic_autotune(int kind, int m, int n, int prec, int* hBest, hipStream_t stream) {
    if (kind != RADIC_WS_DET && kind != RADIC_WS_INT && kind != RADIC_WS_BATCHED) return RADIC_EINVAL;
    if (kind == RADIC_WS_DET && prec != RADIC_FP64 && prec != RADIC_FP32_BULK) return RADIC_EINVAL;
    if (kind == RADIC_WS_BATCHED && prec != RADIC_FP64 && prec != RADIC_FP32_BULK && prec != 2) return RADIC_EINVAL;
    if (kind != RADIC_WS_BATCHED && (m < 1 || n < m || m > RADIC_MAX_M || n > RADIC_MAX_N)) return RADIC_EINVAL;
    int rc = ensure_device();
    if (rc != RADIC_OK) return rc;
    unsigned long long total = 0;
    if (kind != RADIC_WS_BATCHED && (host_binomial(n, m, &total) != RADIC_OK || total >= kRankLimit))
        return RADIC_EOVERFLOW;
    int saved_spl, saved_block;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        saved_spl = g_force_spl;
        saved_block = g_force_block;
    }
    DeviceBuffers buf;
    TuneRng rng(0x5eed0000ull + (unsigned long long)(kind * 1000003 + m * 1009 + n));
    std::function<int()> run;
    std::vector<int> spls = {1, 2, 4, 8, 16, 32, 64};
    std::vector<int> blocks = {64, 128, 256};
    int reps = 3, calls = 1;
    std::vector<double> hf;
    std::vector<int> hi;
    radic_matrix_desc* dDesc = nullptr;
    int batch = 0;
    if (kind == RADIC_WS_DET) {
        hf.resize((size_t)m * n);
        for (double& x : hf) x = rng.uniform();
        double* dA = static_cast<double*>(buf.alloc(hf.size() * 8));
        void* out = buf.alloc(sizeof(radic_f64_result));
        void* ws = buf.alloc(det_workspace_bytes(m, n));
        if (!dA || !out || !ws) return RADIC_ENOMEM;
        if (hipMemcpy(dA, hf.data(), hf.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return RADIC_EDEVICE;
        run = [=]() { return radic_det(dA, m, n, n, prec, static_cast<radic_f64_result*>(out), ws,
                                       det_workspace_bytes(m, n), stream); };
        if (float_enumeration(m, n, prec) == 2) {
            // prefix-shared: spl sets the two-sided blocks (64 spl minors each),
            // and with them how the blocks fill the waves; the workgroup size
            // follows the LDS budget.  Neighbouring sizes differ by a few per
            // cent, hence the finer steps and more runs per candidate.
            spls = {16, 24, 32, 40, 48, 56, 64, 80, 96, 128};
            blocks = {256};
            reps = 15;
            calls = 4;
        }
    } else if (kind == RADIC_WS_INT) {
        hi.resize((size_t)m * n);
        for (int& x : hi) x = (int)(rng.next() % 19) - 9;
        int* dA = static_cast<int*>(buf.alloc(hi.size() * 4));
        void* ws = buf.alloc(int_workspace_bytes());
        if (!dA || !ws) return RADIC_ENOMEM;
        if (hipMemcpy(dA, hi.data(), hi.size() * 4, hipMemcpyHostToDevice) != hipSuccess) return RADIC_EDEVICE;
        run = [=]() {
            uint32_t mag[RADIC_MAX_PRIMES + 1];
            int len = 0, sg = 0;
            return radic_det_int_exact(dA, m, n, n, mag, RADIC_MAX_PRIMES + 1, &len, &sg, ws, int_workspace_bytes(),
                                       stream);
        };
        int mode;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            mode = g_enumeration;
        }
        if (mode != RADIC_ENUM_PER_MINOR && m >= 3 && m <= 10) {   // the prefix-shared exact kernel
            spls = {8, 16, 24, 32, 40, 48, 64};
            blocks = {256};
            reps = 15;
            calls = 4;
        }
    } else {
        // a synthetic mixed batch of the shapes the persistent kernels serve (m in [2, 10], n in [m, 24])
        batch = 512;
        std::vector<radic_matrix_desc> desc((size_t)batch);
        long long fo = 0, io = 0;
        for (int b = 0; b < batch; ++b) {
            const int mm = 2 + (int)(rng.next() % 9);
            const int nn = mm + (int)(rng.next() % (25 - mm));
            const int dt = prec == 2 ? 1 : 0;   // the exact or the float classes alone
            desc[(size_t)b] = radic_matrix_desc{mm, nn, dt, 0, dt ? io : fo, nn};
            for (int e = 0; e < mm * nn; ++e) {
                if (dt) hi.push_back((int)(rng.next() % 256));
                else hf.push_back(rng.uniform());
            }
            (dt ? io : fo) += (long long)mm * nn;
        }
        dDesc = static_cast<radic_matrix_desc*>(buf.alloc(sizeof(radic_matrix_desc) * batch));
        double* dF = static_cast<double*>(buf.alloc(std::max<size_t>(hf.size(), 1) * 8));
        int* dI = static_cast<int*>(buf.alloc(std::max<size_t>(hi.size(), 1) * 4));
        void* out = buf.alloc(sizeof(radic_batch_result) * batch);
        const size_t wsb = batched_workspace_bytes(batch);
        void* ws = buf.alloc(wsb);
        if (!dDesc || !dF || !dI || !out || !ws) return RADIC_ENOMEM;
        if (hipMemcpy(dDesc, desc.data(), sizeof(radic_matrix_desc) * batch, hipMemcpyHostToDevice) != hipSuccess ||
            (!hf.empty() && hipMemcpy(dF, hf.data(), hf.size() * 8, hipMemcpyHostToDevice) != hipSuccess) ||
            (!hi.empty() && hipMemcpy(dI, hi.data(), hi.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
            return RADIC_EDEVICE;
        const int p = prec == 2 ? RADIC_FP64 : prec;
        run = [=]() { return radic_det_batched(dDesc, batch, dF, dI, p, static_cast<radic_batch_result*>(out), ws,
                                               wsb, stream); };
        blocks = {256};   // the persistent kernels have a fixed workgroup
    }
    float best_ms = 0.f;
    Shape best{0, 0};
    for (int spl : spls) {
        for (int block : blocks) {
            {
                std::lock_guard<std::mutex> lk(g_mu);
                g_force_spl = spl;
                g_force_block = block;
            }
            int trc = RADIC_OK;
            const float ms = time_runs(run, stream, reps, &trc, calls);
            if (trc != RADIC_OK) continue;
            if (best.spl == 0 || ms < best_ms) {
                best_ms = ms;
                best = Shape{spl, block};
            }
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_force_spl = saved_spl;
    g_force_block = saved_block;
    if (best.spl == 0) return RADIC_EDEVICE;
    const int key_prec = kind == RADIC_WS_DET ? prec : (kind == RADIC_WS_INT ? 0 : prec);
    const int km = kind == RADIC_WS_BATCHED ? 0 : m, kn = kind == RADIC_WS_BATCHED ? 0 : n_bucket(n);
    g_tuned[std::make_tuple(kind, key_prec, km, kn, kind == RADIC_WS_BATCHED ? 0 : g_enumeration)] = best;
    if (hBest) {
        hBest[0] = best.spl;
        hBest[1] = best.block;
    }
    return RADIC_OK;
}

// The current device's architecture name without feature suffixes ("gfx950"),
// or "none" without a usable device.
static std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t pr;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "none";
    }
    std::string a = pr.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

constexpr int kBatchBlock = 256;   // the batched persistent kernels' workgroup size

int radic_autotune_batched(const radic_matrix_desc* dDesc, int batch, const double* dF64, const int32_t* dI32,
                           int prec, radic_batch_result* dOut, void* dWork, size_t work_bytes, int* hBest,
                           hipStream_t stream) {
    if (!dDesc || !dOut || batch <= 0) return RADIC_EINVAL;
    if (prec != RADIC_FP64 && prec != RADIC_FP32_BULK) return RADIC_EINVAL;
    if (batch > (1 << 24)) return RADIC_ENOTSUP;
    int rc = check_workspace(dWork, work_bytes, batched_workspace_bytes(batch));
    if (rc != RADIC_OK) return rc;
    if ((rc = ensure_device()) != RADIC_OK) return rc;
    int saved_spl, saved_block;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        saved_spl = g_force_spl;
        saved_block = g_force_block;
    }
    // one subsets-per-lane value for the float and the exact classes: the chunk
    // sizes of both grow with it, and the classes of one launch run in sequence
    const int spls[] = {8, 16, 32, 64, 128};
    float best_ms = 0.f;
    int best = 0;
    for (int spl : spls) {
        {
            std::lock_guard<std::mutex> lk(g_mu);
            g_force_spl = spl;
            g_force_block = 0;
        }
        int trc = RADIC_OK;
        const float ms = time_runs([&]() { return batched_launch(dDesc, batch, dF64, dI32, prec, dOut, dWork, stream,
                                                                 false); },
                                   stream, 3, &trc);
        if (trc != RADIC_OK) continue;
        if (best == 0 || ms < best_ms) {
            best_ms = ms;
            best = spl;
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_force_spl = saved_spl;
    g_force_block = saved_block;
    if (best == 0) return RADIC_EDEVICE;
    g_tuned[std::make_tuple((int)RADIC_WS_BATCHED, prec, 0, 0, 0)] = Shape{best, kBatchBlock};
    g_tuned[std::make_tuple((int)RADIC_WS_BATCHED, 2, 0, 0, 0)] = Shape{best, kBatchBlock};
    if (hBest) {
        hBest[0] = best;
        hBest[1] = kBatchBlock;
    }
    return RADIC_OK;
}

int radic_tune_save(const char* path) {
    if (!path) return RADIC_EINVAL;
    const std::string arch = device_arch();
    FILE* f = std::fopen(path, "w");
    if (!f) return RADIC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    std::fprintf(f, "# radic launch-shape table: kind prec m n_bucket enumeration subsets_per_lane block\n");
    std::fprintf(f, "arch %s version %d\n", arch.c_str(), radic_version());
    for (const auto& kv : g_tuned)
        std::fprintf(f, "%d %d %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                     std::get<3>(kv.first), std::get<4>(kv.first), kv.second.spl, kv.second.block);
    return std::fclose(f) == 0 ? RADIC_OK : RADIC_EINVAL;
}

int radic_tune_load(const char* path) {
    if (!path) return RADIC_EINVAL;
    FILE* f = std::fopen(path, "r");
    if (!f) return RADIC_EINVAL;
    std::map<std::tuple<int, int, int, int, int>, Shape> t;
    char line[256];
    int rc = RADIC_OK;
    bool header = false;
    const std::string arch = device_arch();
    while (std::fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        if (!header) {
            // the table's device and library: shapes tuned elsewhere are refused
            char a[64];
            int v = 0;
            if (std::sscanf(line, "arch %63s version %d", a, &v) != 2 || v != radic_version() ||
                (arch != "none" && arch != a)) {
                rc = RADIC_EINVAL;
                break;
            }
            header = true;
            continue;
        }
        int k, p, m, n, e, spl, block;
        if (std::sscanf(line, "%d %d %d %d %d %d %d", &k, &p, &m, &n, &e, &spl, &block) != 7 || e < 0 || e > 3 ||
            spl < 1 || spl > 4096 || block < kWave || block > kMaxBlock || block % kWave) {
            rc = RADIC_EINVAL;
            break;
        }
        t[std::make_tuple(k, p, m, n, e)] = Shape{spl, block};
    }
    std::fclose(f);
    if (rc == RADIC_OK && !header) rc = RADIC_EINVAL;
    if (rc != RADIC_OK) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto& kv : t) g_tuned[kv.first] = kv.second;
    return RADIC_OK;
}

int radic_set_launch(int subsets_per_lane, int block_size) {
    if (subsets_per_lane < 0 || subsets_per_lane > 4096) return RADIC_EINVAL;
    // kernels are compiled for at most kMaxBlock threads per workgroup
    if (block_size != 0 && (block_size < kWave || block_size > kMaxBlock || block_size % kWave)) return RADIC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_force_spl = subsets_per_lane;
    g_force_block = block_size;
    return RADIC_OK;
}

int radic_set_fallback_tau(double tau) {
    if (std::isnan(tau) || tau < 0) return RADIC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_tau = tau;
    return RADIC_OK;
}

double radic_fallback_tau_for(uint64_t minors) {
    std::lock_guard<std::mutex> lk(g_mu);
    return effective_tau(g_tau, minors);
}

int radic_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof = on != 0;
    return RADIC_OK;
}

static int profile_collect(std::vector<double>& ms_out) {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ev.swap(g_prof_events);
    }
    int rc = RADIC_OK;
    for (auto& p : ev) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second) != hipSuccess || hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess)
            rc = RADIC_EDEVICE;
        ms_out.push_back(ms);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& p : ev) {
        g_event_pool.push_back(p.first);
        g_event_pool.push_back(p.second);
    }
    return rc;
}

int radic_profile_read(double* hTotalMs, int* hLaunches) {
    if (!hTotalMs || !hLaunches) return RADIC_EINVAL;
    std::vector<double> ms;
    int rc = profile_collect(ms);
    double total = 0.0;
    for (double v : ms) total += v;
    *hTotalMs = total;
    *hLaunches = (int)ms.size();
    return rc;
}

int radic_profile_read_launches(double* hMs, int capacity, int* hCount) {
    if (!hCount || capacity < 0 || (capacity > 0 && !hMs)) return RADIC_EINVAL;
    std::vector<double> ms;
    int rc = profile_collect(ms);
    for (int i = 0; i < (int)ms.size() && i < capacity; ++i) hMs[i] = ms[i];
    *hCount = (int)ms.size();
    return rc;
}

int radic_host_binomial(int a, int b, uint64_t* hOut) {
    if (!hOut || a < 0 || b < 0) return RADIC_EINVAL;
    unsigned long long v = 0;
    int rc = host_binomial(a, b, &v);
    *hOut = v;
    return rc;
}

int radic_host_unrank(int m, int n, uint64_t q, int* hCols) {
    if (!hCols || m < 1 || n < m || m > 64) return RADIC_EINVAL;
    unsigned long long total = 0;
    if (host_binomial(n, m, &total) != RADIC_OK) return RADIC_EOVERFLOW;
    if (q >= total) return RADIC_EINVAL;
    int c = 0;
    for (int k = 0; k < m; ++k) {
        for (;;) {
            unsigned long long w = 0;
            host_binomial(n - 1 - c, m - 1 - k, &w);
            if (q < w) break;
            q -= w;
            ++c;
        }
        hCols[k] = c + 1;
        ++c;
    }
    return RADIC_OK;
}

int radic_host_batch_chunking(int dtype, int m, int n, int subsets_per_lane, uint64_t* hChunk, uint64_t* hChunks) {
    if (!hChunk || !hChunks || (dtype != 0 && dtype != 1) || m < 1 || n < m || subsets_per_lane < 1)
        return RADIC_EINVAL;
    unsigned long long total = 0;
    if (host_binomial(n, m, &total) != RADIC_OK || total >= kRankLimit) return RADIC_EOVERFLOW;
    unsigned long long c = 0, k = 0;
    if (batch_uses_blocks(dtype, m)) {
        const unsigned long long nb = split_block_count(m, n, 64u * (unsigned)subsets_per_lane);
        batch_block_chunking(nb, dtype == 0 ? (unsigned long long)kBatchChunksPerMatrix : (1ull << 16), c, k);
    } else {
        host_batch_chunking(dtype, total, subsets_per_lane, &c, &k);
    }
    *hChunk = c;
    *hChunks = k;
    return RADIC_OK;
}

int radic_host_split_count(int m, int n, int side, int v, uint64_t* hCount) {
    if (!hCount) return RADIC_EINVAL;
    const int rc = split_args(m, n, side, v);
    if (rc != RADIC_OK) return rc;
    unsigned long long c = 0;
    host_split(m, n, side, v, 0, &c, nullptr);
    *hCount = c;
    return RADIC_OK;
}

int radic_host_split_prefix(int m, int n, int side, int v, uint64_t j, int* hCols) {
    if (!hCols) return RADIC_EINVAL;
    const int rc = split_args(m, n, side, v);
    if (rc != RADIC_OK) return rc;
    unsigned long long c = 0;
    host_split(m, n, side, v, 0, &c, nullptr);
    if (j >= c) return RADIC_EINVAL;
    host_split(m, n, side, v, j, nullptr, hCols);
    return RADIC_OK;
}

int radic_host_split_blocks(int m, int n, int minors_per_block, uint64_t* hBlocks) {
    if (!hBlocks || minors_per_block < 1) return RADIC_EINVAL;
    const int rc = split_args(m, n, 0, m - 3);
    if (rc != RADIC_OK) return rc;
    *hBlocks = split_block_count(m, n, (unsigned)minors_per_block);
    return RADIC_OK;
}

int radic_set_enumeration(int mode) {
    if (mode != RADIC_ENUM_AUTO && mode != RADIC_ENUM_PER_MINOR && mode != RADIC_ENUM_PREFIX_SHARED &&
        mode != RADIC_ENUM_GROUP_SHARED)
        return RADIC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    g_enumeration = mode;
    return RADIC_OK;
}

int radic_host_prime(int i, uint32_t* hPrime) {
    if (!hPrime) return RADIC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || i >= (int)g_primes.size()) return RADIC_EINVAL;
    *hPrime = g_primes[(size_t)i];
    return RADIC_OK;
}

int radic_set_prime_set(const uint32_t* hPrimes, int count) {
    if (count < 0 || count > RADIC_MAX_PRIMES || (count > 0 && !hPrimes)) return RADIC_EINVAL;
    std::vector<unsigned> v;
    if (count == 0) {
        v = default_primes();
    } else {
        for (int i = 0; i < count; ++i) {
            const unsigned p = hPrimes[i];
            if (p < 3 || p >= 0x80000000u || !is_prime_u32(p)) return RADIC_EINVAL;
            for (unsigned q : v)
                if (q == p) return RADIC_EINVAL;
            v.push_back(p);
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_primes = v;
    ++g_prime_version;
    return RADIC_OK;
}

}  // extern "C"
