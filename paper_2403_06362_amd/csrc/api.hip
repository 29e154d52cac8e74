// Host side of the C ABI declared in include/mcrng.h: argument validation,
// slab geometry (merged cells), stride skip-ahead tables, work units, device
// buffers of a context, hipGraph capture, the launch-option autotuner and the
// generation loop of the pulse problem.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pulse.hpp"
#include "uniforms.hpp"
#include "mcrng.h"

using namespace mcrng;

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(e_ == hipErrorOutOfMemory ? MCRNG_ENOMEM : MCRNG_EDEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                      \
    } while (0)

extern "C" const char* mcrng_last_error(void) { return g_last_error.c_str(); }
extern "C" int mcrng_version(void) { return MCRNG_ABI_VERSION; }

// ------------------------------------------------------------------ LCG maths (host)

typedef unsigned __int128 u128;

static uint64_t mask_bits(uint32_t m) { return m >= 64 ? ~0ull : ((1ull << m) - 1ull); }

struct Affine {   // X -> G X + C (mod 2^m)
    uint64_t G, C;
};

// b after a: X -> bG (aG X + aC) + bC
static Affine compose(const Affine& a, const Affine& b, uint64_t mask) {
    return Affine{(b.G * a.G) & mask, (b.G * a.C + b.C) & mask};
}

// The map of k LCG steps, by binary doubling of the one-step map (eq. (2)).
static Affine affine_power(uint64_t g, uint64_t c, uint64_t k, uint64_t mask) {
    Affine acc{1ull & mask, 0}, sq{g & mask, c & mask};
    while (k) {
        if (k & 1) acc = compose(acc, sq, mask);
        sq = compose(sq, sq, mask);
        k >>= 1;
    }
    return acc;
}

static int validate_lcg(const mcrng_lcg* L, uint32_t min_m, LcgDev* out) {
    if (!L) return fail(MCRNG_EINVAL, "lcg is NULL");
    if (L->m < min_m || L->m > 64) return fail(MCRNG_EINVAL, "lcg.m = %u outside [%u, 64]", L->m, min_m);
    if (L->reserved != 0) return fail(MCRNG_EINVAL, "lcg.reserved must be 0");
    out->mask = mask_bits(L->m);
    out->g = L->g & out->mask;
    out->c = L->c & out->mask;
    out->m = L->m;
    out->shift53 = L->m >= 53 ? L->m - 53 : 0;
    return MCRNG_OK;
}

// ------------------------------------------------------------------ arena

// A bump allocator over a fixed device region (the static scratch of the
// allocation-free entry point).  Buffers carved from it are never freed;
// reset() hands the whole region out again.  Stride tables are computed on
// the host when carved and uploaded later, once the whole run is known to
// fit, so that a run that does not fit enqueues nothing.
struct Arena {
    char* base = nullptr;     // device address of the region on its device
    size_t cap = 0;
    size_t used = 0;
    struct Table {
        uint64_t g, c, Q;
        uint32_t m;
        size_t off;
        std::vector<uint64_t> host;
    };
    std::vector<Table> tables;   // carved this run; uploaded by flush_tables
    size_t uploaded = 0;         // tables[0 .. uploaded) are on the device
    static size_t round(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~static_cast<size_t>(255); }
    void reset() {
        used = 0;
        tables.clear();
        uploaded = 0;
    }
};

// ------------------------------------------------------------------ stride tables

// Process-wide cache of device skip tables, one per (device, g, c, m, Q).
// Tables are immutable once built, so concurrent users can share them.
struct TableKey {
    int dev;
    uint64_t g, c, Q;
    uint32_t m;
    bool operator<(const TableKey& o) const {
        if (dev != o.dev) return dev < o.dev;
        if (g != o.g) return g < o.g;
        if (c != o.c) return c < o.c;
        if (Q != o.Q) return Q < o.Q;
        return m < o.m;
    }
};
static std::mutex g_table_mu;
static std::map<TableKey, uint64_t*> g_tables;

// Host values of the skip table of stride Q (see TableKey).
static std::vector<uint64_t> stride_table_host(const LcgDev& L, uint64_t Q) {
    std::vector<uint64_t> h(2 * kStrideDigits * kStrideRadix);
    for (int d = 0; d < kStrideDigits; ++d) {
        // Q * 16^d steps, taken modulo 2^64 (the cycle length 2^m divides it)
        const uint64_t steps = Q << (kStrideRadixBits * d);
        const Affine step = affine_power(L.g, L.c, steps, L.mask);
        Affine cur{1ull & L.mask, 0};
        for (int v = 0; v < kStrideRadix; ++v) {
            h[2 * (d * kStrideRadix + v)] = cur.G;
            h[2 * (d * kStrideRadix + v) + 1] = cur.C;
            cur = compose(cur, step, L.mask);
        }
    }
    return h;
}

// The device skip table of stride Q: from the process-wide cache, or (with
// an arena) carved from the arena, its upload deferred to flush_tables.
static int get_stride_table(const LcgDev& L, uint64_t Q, const uint64_t** out, Arena* arena = nullptr) {
    if (arena) {
        for (const Arena::Table& t : arena->tables)
            if (t.g == L.g && t.c == L.c && t.Q == Q && t.m == L.m) {
                *out = reinterpret_cast<const uint64_t*>(arena->base + t.off);
                return MCRNG_OK;
            }
        const size_t bytes = 2 * kStrideDigits * kStrideRadix * sizeof(uint64_t);
        if (arena->used + Arena::round(bytes) > arena->cap)
            return fail(MCRNG_EINVAL, "stride tables exceed the %zu-byte static scratch", arena->cap);
        arena->tables.push_back(Arena::Table{L.g, L.c, Q, L.m, arena->used, stride_table_host(L, Q)});
        *out = reinterpret_cast<const uint64_t*>(arena->base + arena->used);
        arena->used += Arena::round(bytes);
        return MCRNG_OK;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    TableKey key{dev, L.g, L.c, Q, L.m};
    std::lock_guard<std::mutex> lk(g_table_mu);
    auto it = g_tables.find(key);
    if (it != g_tables.end()) {
        *out = it->second;
        return MCRNG_OK;
    }
    const std::vector<uint64_t> h = stride_table_host(L, Q);
    uint64_t* d_tab = nullptr;
    HIP_TRY(hipMalloc(&d_tab, h.size() * sizeof(uint64_t)));
    hipError_t e = hipMemcpy(d_tab, h.data(), h.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d_tab);
        return fail(MCRNG_EDEVICE, "stride table upload: %s", hipGetErrorString(e));
    }
    g_tables[key] = d_tab;
    *out = d_tab;
    return MCRNG_OK;
}

// Round-alignment tables of the draw kernel, one per (device, g, c, round
// length D), for m = 63 and 64 and odd g (AlignEntry in internal.hpp): the
// inverse step Y -> g^-1 (Y - c) modulo 2^64 applied h times, and minus the
// sum of the states it passes.
struct AlignKey {
    int dev;
    uint64_t g, c;
    int d;
    bool operator<(const AlignKey& o) const {
        if (dev != o.dev) return dev < o.dev;
        if (g != o.g) return g < o.g;
        if (c != o.c) return c < o.c;
        return d < o.d;
    }
};
static std::map<AlignKey, AlignEntry*> g_align;

static int get_align_table(const LcgDev& L, int D, const AlignEntry** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    AlignKey key{dev, L.g, L.c, D};
    std::lock_guard<std::mutex> lk(g_table_mu);
    auto it = g_align.find(key);
    if (it != g_align.end()) {
        *out = it->second;
        return MCRNG_OK;
    }
    uint64_t gi = L.g;   // g^-1 modulo 2^64 by Newton's iteration (3 correct bits, doubling)
    for (int k = 0; k < 5; ++k) gi *= 2ull - L.g * gi;
    std::vector<AlignEntry> h(kMaxRound + kSkipMaps);
    uint64_t a = 1, b = 0, sa = 0, sb = 0;   // rewind of h steps, and the sums of the first h of them
    for (int k = 0; k < kMaxRound; ++k) {
        h[k] = AlignEntry{a, b, 0ull - sa, 0ull - sb};
        sa += a;
        sb += b;
        a = gi * a;
        b = gi * b - gi * L.c;
    }
    // skip-ahead by 2^e rounds: one round (D steps), then doubling
    uint64_t G = 1, C = 0;
    for (int k = 0; k < D; ++k) {
        C = L.g * C + L.c;
        G = L.g * G;
    }
    for (int e = 0; e < kSkipMaps; ++e) {
        h[kMaxRound + e] = AlignEntry{G, C, 0ull, 0ull};
        C = G * C + C;
        G = G * G;
    }
    AlignEntry* d_tab = nullptr;
    HIP_TRY(hipMalloc(&d_tab, h.size() * sizeof(AlignEntry)));
    hipError_t e = hipMemcpy(d_tab, h.data(), h.size() * sizeof(AlignEntry), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d_tab);
        return fail(MCRNG_EDEVICE, "alignment table upload: %s", hipGetErrorString(e));
    }
    g_align[key] = d_tab;
    *out = d_tab;
    return MCRNG_OK;
}

static uint32_t hex_digits(uint64_t v) {
    uint32_t d = 0;
    while (v) {
        ++d;
        v >>= kStrideRadixBits;
    }
    return d;
}

// Fills *S for n streams; returns MCRNG_WSTRIDE_WRAP when a stride
// allocation passes 2^m states.
static int build_seed(const LcgDev& L, const mcrng_seeding* sd, uint64_t n, SeedDev* S, Arena* arena = nullptr) {
    if (!sd) return fail(MCRNG_EINVAL, "seeding is NULL");
    S->first_index = sd->first_index;
    S->table = nullptr;
    S->stride_digits = 0;
    if (sd->kind == MCRNG_SEED_HASH) {
        S->kind = SEED_HASH;
        const uint64_t parent = sd->hier ? murmur_hash(sd->group_key, sd->base) : sd->base;
        S->base = murmur_seed_part(parent);
        return MCRNG_OK;
    }
    if (sd->kind != MCRNG_SEED_STRIDE) return fail(MCRNG_EINVAL, "seeding.kind = %u unknown", sd->kind);
    if (sd->stride == 0) return fail(MCRNG_EINVAL, "stride seeding needs stride >= 1");
    S->kind = SEED_STRIDE;
    S->base = sd->base & L.mask;
    const uint64_t last = n ? sd->first_index + n - 1 : sd->first_index;
    if (n && last < sd->first_index) return fail(MCRNG_EINVAL, "stream index overflows 64 bits");
    S->stride_digits = hex_digits(last);
    int rc = get_stride_table(L, sd->stride, &S->table, arena);
    if (rc < 0) return rc;
    const u128 used = (static_cast<u128>(sd->first_index) + n) * static_cast<u128>(sd->stride);
    const u128 cycle = static_cast<u128>(1) << L.m;
    return used > cycle ? MCRNG_WSTRIDE_WRAP : MCRNG_OK;
}

// ------------------------------------------------------------------ streams

extern "C" int mcrng_init_streams(const mcrng_lcg* lcg, const mcrng_seeding* seeding, uint64_t n,
                                  uint64_t* d_state, void* stream) {
    LcgDev L;
    int rc = validate_lcg(lcg, 1, &L);
    if (rc < 0) return rc;
    if (n == 0) return MCRNG_OK;
    if (!d_state) return fail(MCRNG_EINVAL, "d_state is NULL");
    if (n >> 40) return fail(MCRNG_EINVAL, "n = %llu too large", (unsigned long long)n);
    SeedDev S;
    rc = build_seed(L, seeding, n, &S);
    if (rc < 0) return rc;
    HIP_TRY(launch_init_streams(L, S, n, d_state, static_cast<hipStream_t>(stream)));
    return rc;
}

extern "C" int mcrng_draw(const mcrng_lcg* lcg, const mcrng_seeding* seeding, uint64_t n,
                          const uint32_t* d_count, uint64_t* d_state, uint64_t* d_checksum, void* stream) {
    LcgDev L;
    int rc = validate_lcg(lcg, 1, &L);
    if (rc < 0) return rc;
    if (n == 0) return MCRNG_OK;
    if (!d_count || !d_checksum) return fail(MCRNG_EINVAL, "d_count and d_checksum are required");
    if (!seeding && !d_state) return fail(MCRNG_EINVAL, "d_state is required when seeding is NULL");
    if (n >> 40) return fail(MCRNG_EINVAL, "n = %llu too large", (unsigned long long)n);
    // (the kernel needs fewer than 2^28 streams per wave: the launcher uses at
    // least n / 2^30 + 1 blocks of 4 waves, at most 1025 for n < 2^40)
    DrawParams p;
    std::memset(&p, 0, sizeof p);
    p.lcg = L;
    p.n = n;
    p.count = d_count;
    p.state = d_state;
    p.checksum = d_checksum;
    int mode = SEED_LOAD;
    if (seeding) {
        rc = build_seed(L, seeding, n, &p.seed);
        if (rc < 0) return rc;
        mode = p.seed.kind;
    }
    int bpc = 32, round = 20, generic = 0;
    if (const char* env = getenv("MCRNG_DRAW_BLOCKS_PER_CU")) bpc = atoi(env);
    if (const char* env = getenv("MCRNG_DRAW_ROUND")) round = atoi(env);
    if (const char* env = getenv("MCRNG_DRAW_GENERIC")) generic = atoi(env);
    if (round != 8 && round != 16 && round != 24 && round != 32) round = 20;
    // m = 63 or 64 with an odd multiplier: the round-aligned kernel
    if (!generic && L.m >= 63 && (L.g & 1ull)) {
        int r2 = get_align_table(L, round, &p.align);
        if (r2 < 0) return r2;
    }
    HIP_TRY(launch_draw(p, mode, static_cast<hipStream_t>(stream), bpc, round));
    return rc;
}

// ------------------------------------------------------------------ context

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    Arena* arena = nullptr;   // set: carved from the arena, never hipMalloc'd or freed
};

struct mcrng_ctx {
    int device = 0;
    hipStream_t capture_stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timing_valid = false;
    const char* last_kernel = "";                        // transport kernel of the last run
    std::map<uint64_t, const char*> graph_kernel;        // ... of each cached graph

    DevBuf problems, edges64, sig64, scat64, cbin, edges32, sig32, tedges64, tedges32;
    DevBuf units, order, partial, unit_diag, counter, groups, dx, dt, pu_begin;
    DevBuf bank_a, bank_b, records, rec_begin;   // event schedule
    DevBuf pulse_tedges, pulse_misc, pulse_diag, pulse_bank[2], pulse_stack;   // pulse problem
    DevBuf pulse_census, pulse_copies, pulse_pop;                             // population control
    std::vector<double> h_pulse_tedges;
    uint64_t* h_pinned = nullptr;   // pinned host words for per-generation readbacks
    std::vector<uint64_t> h_rec_begin;
    std::vector<uint32_t> h_group_first;   // per unit: the first unit of its (problem, batch) (host only)

    // host copies of the current tables (kept alive while copies are staged)
    std::vector<DevProblem> h_problems;
    std::vector<double> h_edges64, h_sig64, h_scat64, h_tedges64, h_dx, h_dt;
    std::vector<float> h_edges32, h_sig32, h_tedges32;
    std::vector<int32_t> h_cbin;
    std::vector<WorkUnit> h_units;
    std::vector<uint32_t> h_order, h_pu_begin;
    std::vector<ReduceGroup> h_groups;

    uint64_t tables_sig = 0;      // signature of the uploaded tables
    bool have_run = false;
    uint32_t n_problems = 0;
    uint32_t max_cells = 0, max_tedges = 0, max_slice = 0;
    bool any_timed = false;
    uint64_t partial_words = 0;

    std::map<uint64_t, hipGraphExec_t> graphs;          // (tables, opts) -> executable
    std::map<uint64_t, mcrng_run_opts> tuned;           // shape -> options

    Arena* arena = nullptr;   // allocation-free runs: every buffer and table comes from here
};

static int ensure(DevBuf& b, size_t bytes, hipStream_t st, size_t growth_quarters = 5) {
    if (bytes <= b.cap) return MCRNG_OK;
    if (b.arena) {
        Arena& a = *b.arena;
        if (a.used + Arena::round(bytes) > a.cap)
            return fail(MCRNG_EINVAL, "the run needs more than the %zu-byte static scratch", a.cap);
        b.p = a.base + a.used;
        b.cap = bytes;
        a.used += Arena::round(bytes);
        return MCRNG_OK;
    }
    if (b.p) {
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = std::max<size_t>(bytes / 4 * growth_quarters + bytes % 4, 256);
    HIP_TRY(hipMalloc(&b.p, want));
    b.cap = want;
    return MCRNG_OK;
}

template <class T>
static int upload(DevBuf& b, const std::vector<T>& h, hipStream_t st) {
    const size_t bytes = h.size() * sizeof(T);
    int rc = ensure(b, bytes, st);
    if (rc < 0) return rc;
    if (bytes) HIP_TRY(hipMemcpyAsync(b.p, h.data(), bytes, hipMemcpyHostToDevice, st));
    return MCRNG_OK;
}

static void clear_graphs(mcrng_ctx* ctx) {
    for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
    ctx->graph_kernel.clear();
}

extern "C" int mcrng_ctx_create(int device, mcrng_ctx** out) {
    if (!out) return fail(MCRNG_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(MCRNG_EINVAL, "device %d not present (%d devices)", device, n);
    HIP_TRY(hipSetDevice(device));
    mcrng_ctx* c = new (std::nothrow) mcrng_ctx();
    if (!c) return fail(MCRNG_ENOMEM, "context allocation");
    c->device = device;
    hipError_t e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&c->ev0);
    if (e == hipSuccess) e = hipEventCreate(&c->ev1);
    if (e != hipSuccess) {
        delete c;
        return fail(MCRNG_EDEVICE, "context setup: %s", hipGetErrorString(e));
    }
    *out = c;
    return MCRNG_OK;
}

extern "C" int mcrng_ctx_destroy(mcrng_ctx* ctx) {
    if (!ctx) return MCRNG_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    clear_graphs(ctx);
    DevBuf* bufs[] = {&ctx->problems, &ctx->edges64, &ctx->sig64, &ctx->scat64, &ctx->cbin, &ctx->edges32,
                      &ctx->sig32, &ctx->tedges64, &ctx->tedges32, &ctx->units, &ctx->order, &ctx->partial,
                      &ctx->unit_diag, &ctx->counter, &ctx->groups, &ctx->dx, &ctx->dt, &ctx->pu_begin,
                      &ctx->bank_a, &ctx->bank_b, &ctx->records, &ctx->rec_begin, &ctx->pulse_tedges,
                      &ctx->pulse_misc, &ctx->pulse_diag, &ctx->pulse_bank[0], &ctx->pulse_bank[1],
                      &ctx->pulse_stack, &ctx->pulse_census, &ctx->pulse_copies, &ctx->pulse_pop};
    for (DevBuf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
    return MCRNG_OK;
}

// ------------------------------------------------------------------ problem tables

static uint64_t fnv(uint64_t h, const void* data, size_t n) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

static uint64_t tally_bins_of(const mcrng_problem& P) {
    return static_cast<uint64_t>(P.n_batches) * std::max<uint32_t>(P.n_time_bins, 1) * P.n_space_bins;
}

extern "C" uint64_t mcrng_tally_bins(const mcrng_problem* problems, uint32_t n) {
    if (!problems) return 0;
    uint64_t t = 0;
    for (uint32_t i = 0; i < n; ++i) t += tally_bins_of(problems[i]);
    return t;
}

static bool increasing(const double* a, uint32_t n) {
    for (uint32_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i]) || (i && !(a[i] > a[i - 1]))) return false;
    return true;
}

constexpr uint32_t kMaxCells = 4096;
constexpr uint32_t kMaxSlice = 8192;
constexpr double kTauMax = 36.75;   // above -ln(2^-53) = 36.7368...
constexpr double kMaxCoord = 0x1p40;
constexpr double kMinSigma = 0x1p-64, kMaxSigma = 0x1p64;

static int validate_problem(const mcrng_problem& P, uint32_t idx) {
    if (P.n_regions < 1 || P.n_space_bins < 1 || P.n_batches < 1)
        return fail(MCRNG_EINVAL, "problem %u: n_regions, n_space_bins and n_batches must be >= 1", idx);
    if (!P.region_edges || !P.sigma_t || !P.scatter || !P.bin_edges)
        return fail(MCRNG_EINVAL, "problem %u: NULL geometry array", idx);
    if ((P.n_time_bins > 0) != (P.time_edges != nullptr))
        return fail(MCRNG_EINVAL, "problem %u: time_edges must be given exactly when n_time_bins > 0", idx);
    if (!increasing(P.region_edges, P.n_regions + 1) || !increasing(P.bin_edges, P.n_space_bins + 1))
        return fail(MCRNG_EINVAL, "problem %u: edges must be finite and strictly increasing", idx);
    if (P.region_edges[0] != P.bin_edges[0] || P.region_edges[P.n_regions] != P.bin_edges[P.n_space_bins])
        return fail(MCRNG_EINVAL, "problem %u: region and bin edges must span the same interval", idx);
    if (P.n_time_bins > 0 && !increasing(P.time_edges, P.n_time_bins + 1))
        return fail(MCRNG_EINVAL, "problem %u: time edges must be finite and strictly increasing", idx);
    // the kernels divide by sigma_t and by direction cosines through refined
    // reciprocals, exact while operands stay well inside the exponent range
    if (!(std::fabs(P.region_edges[0]) <= kMaxCoord && std::fabs(P.region_edges[P.n_regions]) <= kMaxCoord))
        return fail(MCRNG_EINVAL, "problem %u: edges must lie within [-2^40, 2^40]", idx);
    double min_sig = INFINITY;
    for (uint32_t r = 0; r < P.n_regions; ++r) {
        if (!(P.sigma_t[r] >= kMinSigma && P.sigma_t[r] <= kMaxSigma))
            return fail(MCRNG_EINVAL, "problem %u: sigma_t[%u] must lie within [2^-64, 2^64]", idx, r);
        if (!(P.scatter[r] >= 0.0 && P.scatter[r] <= 1.0))
            return fail(MCRNG_EINVAL, "problem %u: scatter[%u] must be in [0, 1]", idx, r);
        min_sig = std::min(min_sig, P.sigma_t[r]);
    }
    double bound = kTauMax / min_sig;
    if (P.n_time_bins > 0) {
        double wmax = 0;
        for (uint32_t t = 0; t < P.n_time_bins; ++t) wmax = std::max(wmax, P.time_edges[t + 1] - P.time_edges[t]);
        bound = std::min(bound, wmax);
    }
    if (!(bound < 128.0))
        return fail(MCRNG_ERANGE, "problem %u: track lengths may reach 2^7 (bound %.3f)", idx, bound);
    if (P.n_time_bins > 0 && static_cast<uint64_t>(P.n_time_bins) * P.n_space_bins > kMaxSlice)
        return fail(MCRNG_EINVAL, "problem %u: more than %u tally bins per batch", idx, kMaxSlice);
    if (P.n_space_bins > kMaxSlice) return fail(MCRNG_EINVAL, "problem %u: too many space bins", idx);
    if (P.n_regions + P.n_space_bins > kMaxCells)
        return fail(MCRNG_EINVAL, "problem %u: more than %u cells", idx, kMaxCells);
    if (P.n_histories >> 40) return fail(MCRNG_EINVAL, "problem %u: n_histories too large", idx);
    return MCRNG_OK;
}

static uint64_t signature(const mcrng_lcg* lcg, const mcrng_problem* P, uint32_t n, uint32_t unit_hist) {
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, lcg, sizeof *lcg);
    h = fnv(h, &n, sizeof n);
    h = fnv(h, &unit_hist, sizeof unit_hist);
    for (uint32_t i = 0; i < n; ++i) {
        h = fnv(h, &P[i].n_regions, 4 * sizeof(uint32_t));
        h = fnv(h, &P[i].n_histories, sizeof(uint64_t));
        h = fnv(h, &P[i].seeding, sizeof(mcrng_seeding));
        h = fnv(h, P[i].region_edges, (P[i].n_regions + 1) * sizeof(double));
        h = fnv(h, P[i].sigma_t, P[i].n_regions * sizeof(double));
        h = fnv(h, P[i].scatter, P[i].n_regions * sizeof(double));
        h = fnv(h, P[i].bin_edges, (P[i].n_space_bins + 1) * sizeof(double));
        if (P[i].n_time_bins) h = fnv(h, P[i].time_edges, (P[i].n_time_bins + 1) * sizeof(double));
    }
    return h;
}

// Work units of a chained run by default (total histories / kChainUnits).
constexpr uint64_t kChainUnits = 10240;
// The chained kernel holds two units per block, so the block waits whenever
// a unit is handed out before the one before it has ended; on the long-chain
// slab (heavy-tailed history lengths) that costs little from about 20
// histories per lane per unit up (block 256: 34.5-35.2 ms at 5425-12207
// histories per unit, 44 ms at 3051, 67 ms at 1525; the per-unit kernel
// 38.1 ms).  Smaller units run on the per-unit kernel.
constexpr uint32_t kChainMinPerLane = 20;

// MCRNG_TRANSPORT_CHAIN: 0 keeps one-problem runs on the per-unit kernel;
// 2 takes the chained kernel for every run of one problem with one history
// per lane and one tally copy, whatever its units and even where it costs
// blocks per CU (other history-schedule runs fail); otherwise it is taken
// for units of at least kChainMinPerLane histories per lane where it costs
// no blocks per CU.
static int chain_mode() {
    const char* env = getenv("MCRNG_TRANSPORT_CHAIN");
    const int m = env ? atoi(env) : 1;
    return (m == 0 || m == 2) ? m : 1;
}
static bool chain_enabled() { return chain_mode() != 0; }

// Whether a run of these problems with these options will take the chained
// kernel (estimated from the problem's sizes: the merged cells are at most
// regions + bins; the launch decides on the exact tables).
static bool chain_planned(const mcrng_problem* P, uint32_t n, const mcrng_run_opts& o) {
    if (n != 1 || o.schedule != MCRNG_SCHED_HISTORY || o.hist_per_lane != 1 || o.tally_copies != 1 ||
        !chain_enabled())
        return false;
    const uint64_t unit = o.unit_histories ? o.unit_histories : P[0].n_histories / kChainUnits;
    if (chain_mode() != 2 && unit < static_cast<uint64_t>(kChainMinPerLane) * o.block) return false;
    TransportParams a{};
    a.max_slice = std::max<uint32_t>(P[0].n_time_bins, 1) * P[0].n_space_bins;
    a.max_cells = P[0].n_regions + P[0].n_space_bins;
    a.max_tedges = P[0].n_time_bins ? P[0].n_time_bins + 1 : 0;
    a.tally_copies = 1;
    TransportParams b = a;
    b.tally_copies = 2;
    LaunchShape s{};
    s.block = static_cast<int>(o.block);
    s.hist_per_lane = 1;
    s.f32 = o.precision == MCRNG_FP32;
    s.timed = P[0].n_time_bins > 0;
    bool fits = false;
    return transport_chain_fits(a, b, s, &fits) == hipSuccess && fits;
}

// Histories per work unit.  The per-unit kernel pays a pause at the end of
// each unit, so its units are few (a few per resident block); the chained
// kernel pauses only at the end of the launch, where small units even out
// the blocks' finishing times.
static uint32_t default_unit_histories(const mcrng_problem* P, uint32_t n, bool chained) {
    uint64_t total = 0;
    for (uint32_t i = 0; i < n; ++i) total += P[i].n_histories;
    uint64_t u = total / (chained ? kChainUnits : 4096);
    u = std::max<uint64_t>(u, 512);
    u = std::min<uint64_t>(u, 65536);
    return static_cast<uint32_t>(u);
}

// Builds every table of the problem set on the host and uploads them.
static int build_tables(mcrng_ctx* ctx, const LcgDev& L, const mcrng_problem* P, uint32_t n, uint32_t unit_hist,
                        hipStream_t st, int* warn) {
    ctx->h_problems.assign(n, DevProblem{});
    ctx->h_edges64.clear();
    ctx->h_sig64.clear();
    ctx->h_scat64.clear();
    ctx->h_cbin.clear();
    ctx->h_tedges64.clear();
    ctx->h_dx.clear();
    ctx->h_dt.clear();
    ctx->h_units.clear();
    ctx->h_groups.clear();
    ctx->h_pu_begin.assign(n + 1, 0);
    ctx->max_cells = ctx->max_tedges = ctx->max_slice = 0;
    ctx->any_timed = false;
    uint64_t slot = 0, out_off = 0;
    *warn = MCRNG_OK;
    for (uint32_t p = 0; p < n; ++p) {
        const mcrng_problem& Q = P[p];
        DevProblem& D = ctx->h_problems[p];
        // merged cell edges: union of region and bin edges (exact doubles)
        std::vector<double> E;
        E.reserve(Q.n_regions + Q.n_space_bins + 2);
        uint32_t a = 0, b = 0;
        while (a <= Q.n_regions || b <= Q.n_space_bins) {
            double v;
            if (b > Q.n_space_bins || (a <= Q.n_regions && Q.region_edges[a] < Q.bin_edges[b]))
                v = Q.region_edges[a++];
            else if (a > Q.n_regions || Q.bin_edges[b] < Q.region_edges[a])
                v = Q.bin_edges[b++];
            else {
                v = Q.region_edges[a];
                ++a;
                ++b;
            }
            E.push_back(v);
        }
        const uint32_t nc = static_cast<uint32_t>(E.size() - 1);
        D.cell_off = static_cast<uint32_t>(ctx->h_sig64.size());
        D.edge_off = static_cast<uint32_t>(ctx->h_edges64.size());
        D.n_cells = nc;
        uint32_t reg = 0, sb = 0;
        for (uint32_t c = 0; c < nc; ++c) {
            while (reg + 1 < Q.n_regions && Q.region_edges[reg + 1] <= E[c]) ++reg;
            while (sb + 1 < Q.n_space_bins && Q.bin_edges[sb + 1] <= E[c]) ++sb;
            ctx->h_sig64.push_back(Q.sigma_t[reg]);
            ctx->h_scat64.push_back(Q.scatter[reg]);
            ctx->h_cbin.push_back(static_cast<int32_t>(sb));
        }
        ctx->h_edges64.insert(ctx->h_edges64.end(), E.begin(), E.end());
        D.n_time_bins = Q.n_time_bins;
        D.n_space_bins = Q.n_space_bins;
        D.slice_bins = std::max<uint32_t>(Q.n_time_bins, 1) * Q.n_space_bins;
        D.tedge_off = static_cast<uint32_t>(ctx->h_tedges64.size());
        if (Q.n_time_bins) {
            ctx->h_tedges64.insert(ctx->h_tedges64.end(), Q.time_edges, Q.time_edges + Q.n_time_bins + 1);
            ctx->any_timed = true;
            ctx->max_tedges = std::max(ctx->max_tedges, Q.n_time_bins + 1);
        }
        ctx->max_cells = std::max(ctx->max_cells, nc);
        ctx->max_slice = std::max(ctx->max_slice, D.slice_bins);
        // seeding
        SeedDev S;
        int rc = build_seed(L, &Q.seeding, Q.n_histories, &S, ctx->arena);
        if (rc < 0) return rc;
        if (rc > 0) *warn = rc;
        D.seed_kind = static_cast<uint32_t>(S.kind);
        D.stride_digits = S.stride_digits;
        D.seed_base = S.base;
        D.first_index = S.first_index;
        D.stride_q = (S.kind == SEED_STRIDE) ? Q.seeding.stride : 0;
        D.table = S.table;
        // bin widths for the flux normalisation
        const uint32_t dx_off = static_cast<uint32_t>(ctx->h_dx.size());
        for (uint32_t i = 0; i < Q.n_space_bins; ++i) ctx->h_dx.push_back(Q.bin_edges[i + 1] - Q.bin_edges[i]);
        const uint32_t dt_off = static_cast<uint32_t>(ctx->h_dt.size());
        for (uint32_t i = 0; i < Q.n_time_bins; ++i) ctx->h_dt.push_back(Q.time_edges[i + 1] - Q.time_edges[i]);
        // work units: batches split into runs of unit_hist histories
        ctx->h_pu_begin[p] = static_cast<uint32_t>(ctx->h_units.size());
        const uint64_t nb = Q.n_batches;
        uint64_t bs = (Q.n_histories + nb - 1) / nb;
        if (bs == 0) bs = 1;
        for (uint64_t bt = 0; bt < nb; ++bt) {
            const uint64_t j0 = std::min<uint64_t>(bt * bs, Q.n_histories);
            const uint64_t j1 = std::min<uint64_t>((bt + 1) * bs, Q.n_histories);
            ReduceGroup G;
            G.problem = p;
            G.unit_begin = static_cast<uint32_t>(ctx->h_units.size());
            for (uint64_t j = j0; j < j1; j += unit_hist) {
                WorkUnit U;
                U.problem = p;
                U.batch = static_cast<uint32_t>(bt);
                U.j0 = j;
                U.count = static_cast<uint32_t>(std::min<uint64_t>(unit_hist, j1 - j));
                U.slice_bins = D.slice_bins;
                U.slot = slot;
                slot += 2ull * D.slice_bins;
                ctx->h_units.push_back(U);
            }
            G.unit_end = static_cast<uint32_t>(ctx->h_units.size());
            G.slice_bins = D.slice_bins;
            G.n_space_bins = Q.n_space_bins;
            G.n_time_bins = Q.n_time_bins;
            G.out_off = out_off;
            G.n_hist = j1 - j0;
            G.dx_off = dx_off;
            G.dt_off = dt_off;
            out_off += D.slice_bins;
            ctx->h_groups.push_back(G);
        }
    }
    ctx->h_pu_begin[n] = static_cast<uint32_t>(ctx->h_units.size());
    if (ctx->h_units.size() > 0xffffffffull) return fail(MCRNG_EINVAL, "too many work units");
    if (ctx->h_groups.size() > 65535)
        return fail(MCRNG_EINVAL, "more than 65535 (problem, batch) tally groups in one run");
    // schedule: largest units first (stable), so short units fill the tail
    ctx->h_order.resize(ctx->h_units.size());
    for (uint32_t i = 0; i < ctx->h_order.size(); ++i) ctx->h_order[i] = i;
    std::stable_sort(ctx->h_order.begin(), ctx->h_order.end(), [&](uint32_t x, uint32_t y) {
        return ctx->h_units[x].count > ctx->h_units[y].count;
    });
    // FP32 flight tables, each rounded once from a double: per problem the
    // cell widths (n_cells, then a 0 to keep the edge offsets) and the
    // time-bin durations (n_time_bins, then a 0)
    ctx->h_edges32.assign(ctx->h_edges64.size(), 0.0f);
    ctx->h_tedges32.assign(ctx->h_tedges64.size(), 0.0f);
    for (const DevProblem& D : ctx->h_problems) {
        for (uint32_t c = 0; c < D.n_cells; ++c)
            ctx->h_edges32[D.edge_off + c] =
                static_cast<float>(ctx->h_edges64[D.edge_off + c + 1] - ctx->h_edges64[D.edge_off + c]);
        for (uint32_t t = 0; t < D.n_time_bins; ++t)
            ctx->h_tedges32[D.tedge_off + t] =
                static_cast<float>(ctx->h_tedges64[D.tedge_off + t + 1] - ctx->h_tedges64[D.tedge_off + t]);
    }
    ctx->h_sig32.assign(ctx->h_sig64.begin(), ctx->h_sig64.end());
    if (ctx->h_tedges64.empty()) {
        ctx->h_tedges64.push_back(0.0);
        ctx->h_tedges32.assign(1, 0.0f);
    }
    if (ctx->h_dt.empty()) ctx->h_dt.push_back(0.0);
    ctx->partial_words = slot;
    ctx->h_rec_begin.assign(ctx->h_units.size() + 1, 0);
    for (size_t u = 0; u < ctx->h_units.size(); ++u)
        ctx->h_rec_begin[u + 1] = ctx->h_rec_begin[u] + ctx->h_units[u].count;
    ctx->h_group_first.assign(std::max<size_t>(ctx->h_units.size(), 1), 0);
    for (const ReduceGroup& G : ctx->h_groups)
        for (uint32_t u = G.unit_begin; u < G.unit_end; ++u) ctx->h_group_first[u] = G.unit_begin;
    if (ctx->arena) {
        // the device copies below, in the order they are carved: all must
        // fit before anything is enqueued
        Arena& a = *ctx->arena;
        const size_t sizes[] = {
            ctx->h_problems.size() * sizeof(DevProblem), ctx->h_edges64.size() * sizeof(double),
            ctx->h_sig64.size() * sizeof(double), ctx->h_scat64.size() * sizeof(double),
            ctx->h_cbin.size() * sizeof(int32_t), ctx->h_edges32.size() * sizeof(float),
            ctx->h_sig32.size() * sizeof(float), ctx->h_tedges64.size() * sizeof(double),
            ctx->h_tedges32.size() * sizeof(float), ctx->h_units.size() * sizeof(WorkUnit),
            ctx->h_order.size() * sizeof(uint32_t), ctx->h_groups.size() * sizeof(ReduceGroup),
            ctx->h_dx.size() * sizeof(double), ctx->h_dt.size() * sizeof(double),
            ctx->h_pu_begin.size() * sizeof(uint32_t), ctx->h_rec_begin.size() * sizeof(uint64_t),
            std::max<uint64_t>(slot, 2) * sizeof(uint64_t),
            std::max<size_t>(ctx->h_units.size(), 1) * kNDiag * sizeof(uint64_t), 64};
        size_t need = a.used;
        for (size_t b : sizes)
            if (b) need += Arena::round(b);
        if (need > a.cap)
            return fail(MCRNG_EINVAL, "the run needs %zu bytes of scratch, more than the %zu-byte static scratch", need,
                        a.cap);
        for (; a.uploaded < a.tables.size(); ++a.uploaded) {
            const Arena::Table& t = a.tables[a.uploaded];
            HIP_TRY(hipMemcpyAsync(a.base + t.off, t.host.data(), t.host.size() * sizeof(uint64_t),
                                   hipMemcpyHostToDevice, st));
        }
    }
    int rc;
    if ((rc = upload(ctx->problems, ctx->h_problems, st)) < 0) return rc;
    if ((rc = upload(ctx->edges64, ctx->h_edges64, st)) < 0) return rc;
    if ((rc = upload(ctx->sig64, ctx->h_sig64, st)) < 0) return rc;
    if ((rc = upload(ctx->scat64, ctx->h_scat64, st)) < 0) return rc;
    if ((rc = upload(ctx->cbin, ctx->h_cbin, st)) < 0) return rc;
    if ((rc = upload(ctx->edges32, ctx->h_edges32, st)) < 0) return rc;
    if ((rc = upload(ctx->sig32, ctx->h_sig32, st)) < 0) return rc;
    if ((rc = upload(ctx->tedges64, ctx->h_tedges64, st)) < 0) return rc;
    if ((rc = upload(ctx->tedges32, ctx->h_tedges32, st)) < 0) return rc;
    if ((rc = upload(ctx->units, ctx->h_units, st)) < 0) return rc;
    if ((rc = upload(ctx->order, ctx->h_order, st)) < 0) return rc;
    if ((rc = upload(ctx->groups, ctx->h_groups, st)) < 0) return rc;
    if ((rc = upload(ctx->dx, ctx->h_dx, st)) < 0) return rc;
    if ((rc = upload(ctx->dt, ctx->h_dt, st)) < 0) return rc;
    if ((rc = upload(ctx->pu_begin, ctx->h_pu_begin, st)) < 0) return rc;
    if ((rc = upload(ctx->rec_begin, ctx->h_rec_begin, st)) < 0) return rc;
    if ((rc = ensure(ctx->partial, std::max<uint64_t>(slot, 2) * sizeof(uint64_t), st)) < 0) return rc;
    if ((rc = ensure(ctx->unit_diag, std::max<size_t>(ctx->h_units.size(), 1) * kNDiag * sizeof(uint64_t), st)) < 0)
        return rc;
    if ((rc = ensure(ctx->counter, 64, st)) < 0) return rc;
    ctx->n_problems = n;
    return MCRNG_OK;
}

static TransportParams make_params(mcrng_ctx* ctx, const LcgDev& L, uint32_t copies) {
    TransportParams tp;
    std::memset(&tp, 0, sizeof tp);
    tp.lcg = L;
    tp.problems = static_cast<const DevProblem*>(ctx->problems.p);
    tp.units = static_cast<const WorkUnit*>(ctx->units.p);
    tp.order = static_cast<const uint32_t*>(ctx->order.p);
    tp.n_units = static_cast<uint32_t>(ctx->h_units.size());
    tp.max_cells = ctx->max_cells;
    tp.max_tedges = ctx->max_tedges;
    tp.max_slice = ctx->max_slice;
    tp.tally_copies = copies;
    tp.coll_batch = 1;
    tp.edges64 = static_cast<const double*>(ctx->edges64.p);
    tp.sig64 = static_cast<const double*>(ctx->sig64.p);
    tp.scat64 = static_cast<const double*>(ctx->scat64.p);
    tp.cbin = static_cast<const int32_t*>(ctx->cbin.p);
    tp.edges32 = static_cast<const float*>(ctx->edges32.p);
    tp.sig32 = static_cast<const float*>(ctx->sig32.p);
    tp.tedges64 = static_cast<const double*>(ctx->tedges64.p);
    tp.tedges32 = static_cast<const float*>(ctx->tedges32.p);
    tp.partial = static_cast<uint64_t*>(ctx->partial.p);
    tp.unit_diag = static_cast<uint64_t*>(ctx->unit_diag.p);
    tp.unit_counter = static_cast<uint32_t*>(ctx->counter.p);
    return tp;
}


static int normalise_opts(const mcrng_run_opts* in, mcrng_run_opts* o) {
    std::memset(o, 0, sizeof *o);
    if (in) *o = *in;
    for (uint32_t r : o->reserved)
        if (r) return fail(MCRNG_EINVAL, "opts.reserved must be 0");
    if (o->precision > MCRNG_FP32) return fail(MCRNG_EINVAL, "opts.precision unknown");
    if (o->schedule > MCRNG_SCHED_EVENT) return fail(MCRNG_EINVAL, "opts.schedule unknown");
    if (o->block == 0) o->block = 256;
    if (o->block != 64 && o->block != 128 && o->block != 256 && o->block != 512 && o->block != 1024)
        return fail(MCRNG_EINVAL, "opts.block = %u not in {64,128,256,512,1024}", o->block);
    if (o->hist_per_lane == 0) o->hist_per_lane = 1;
    if (o->hist_per_lane != 1 && o->hist_per_lane != 2 && o->hist_per_lane != 4)
        return fail(MCRNG_EINVAL, "opts.hist_per_lane = %u not in {1,2,4}", o->hist_per_lane);
    // a wave's collision pass once 36 of its 64 lanes wait: the best batch in
    // a model of the long-chain slab's lane occupancy (a geometry step ends at
    // a collision one time in three; a collision pass costs about twice a
    // geometry pass); the autotuner searches around it
    if (o->coll_batch == 0) o->coll_batch = 36;
    if (o->coll_batch > 64 * o->hist_per_lane) o->coll_batch = 64 * o->hist_per_lane;
    if (o->tally_copies == 0) o->tally_copies = 1;
    if (o->tally_copies > 2) return fail(MCRNG_EINVAL, "opts.tally_copies must be 1 or 2");
    // a unit's LDS tally words take plain 64-bit adds of 32-bit halves: exact
    // while fewer than 2^32 of its scores fall in one bin
    if (o->unit_histories > kMaxUnitHistories)
        return fail(MCRNG_EINVAL, "opts.unit_histories = %u exceeds %u", o->unit_histories, kMaxUnitHistories);
    return MCRNG_OK;
}

static int run_prepared(mcrng_ctx* ctx, const LcgDev& L, const mcrng_run_opts& o, hipStream_t st);

extern "C" int mcrng_run_histories(mcrng_ctx* ctx, const mcrng_lcg* lcg, const mcrng_problem* problems,
                                   uint32_t n_problems, const mcrng_run_opts* opts, void* stream) {
    if (!ctx) return fail(MCRNG_EINVAL, "ctx is NULL");
    if (!problems && n_problems) return fail(MCRNG_EINVAL, "problems is NULL");
    if (n_problems == 0) return fail(MCRNG_EINVAL, "n_problems must be >= 1");
    LcgDev L;
    int rc = validate_lcg(lcg, 53, &L);
    if (rc < 0) return rc;
    mcrng_run_opts o;
    if ((rc = normalise_opts(opts, &o)) < 0) return rc;
    for (uint32_t i = 0; i < n_problems; ++i)
        if ((rc = validate_problem(problems[i], i)) < 0) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t unit_hist =
        o.unit_histories ? o.unit_histories : default_unit_histories(problems, n_problems, chain_planned(problems, n_problems, o));
    o.unit_histories = unit_hist;
    const uint64_t sig = signature(lcg, problems, n_problems, unit_hist);
    int warn = MCRNG_OK;
    if (!ctx->have_run || sig != ctx->tables_sig) {
        clear_graphs(ctx);
        ctx->have_run = false;
        if ((rc = build_tables(ctx, L, problems, n_problems, unit_hist, st, &warn)) < 0) return rc;
        ctx->tables_sig = sig;
    } else {
        // seeding warnings do not depend on the upload
        for (uint32_t i = 0; i < n_problems; ++i) {
            SeedDev S;
            int r2 = build_seed(L, &problems[i].seeding, problems[i].n_histories, &S);
            if (r2 < 0) return r2;
            if (r2 > 0) warn = r2;
        }
    }
    if ((rc = run_prepared(ctx, L, o, st)) < 0) return rc;
    ctx->have_run = true;
    return warn;
}

static int enqueue_run(mcrng_ctx* ctx, const LcgDev& L, const mcrng_run_opts& o, hipStream_t st) {
    TransportParams tp = make_params(ctx, L, o.tally_copies == 2 ? std::max<uint32_t>(o.block / 64, 1) : 1);
    tp.coll_batch = o.coll_batch;
    LaunchShape sh;
    sh.block = static_cast<int>(o.block);
    sh.hist_per_lane = static_cast<int>(o.hist_per_lane);
    sh.grid = static_cast<int>(o.grid);
    sh.f32 = o.precision == MCRNG_FP32;
    sh.timed = ctx->any_timed;
    sh.chain = 0;
    // one problem, one history per lane, one tally copy, units of at least
    // kChainMinPerLane histories per lane: the chained kernel, if its second
    // tally slice costs no blocks per CU
    const bool big_units = o.unit_histories >= kChainMinPerLane * o.block;
    if (ctx->h_problems.size() == 1 && o.hist_per_lane == 1 && o.tally_copies == 1 &&
        (chain_mode() == 2 || (chain_mode() == 1 && big_units))) {
        TransportParams t2 = tp;
        t2.tally_copies = 2;
        bool fits = chain_mode() == 2;
        if (!fits) HIP_TRY(transport_chain_fits(tp, t2, sh, &fits));
        if (fits) {
            tp = t2;
            sh.chain = 1;
        }
    }
    if (!sh.chain && chain_mode() == 2)
        return fail(MCRNG_EINVAL, "MCRNG_TRANSPORT_CHAIN=2 and the chained kernel does not take this run");
    int dev_lds = 0;
    HIP_TRY(hipDeviceGetAttribute(&dev_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    const size_t lds_need = transport_lds_bytes(tp, sh.f32) + transport_static_lds_bytes(sh.block);
    if (lds_need > static_cast<size_t>(dev_lds))
        return fail(MCRNG_EINVAL, "LDS needed (%zu bytes) exceeds the device's %d", lds_need, dev_lds);
    ctx->last_kernel = sh.chain ? "k_transport_chain" : "k_transport";
    HIP_TRY(launch_fill_u32(tp.unit_counter, 16, 0u, st));
    // the chained kernel writes each block's diagnostics to one of its units
    if (sh.chain) HIP_TRY(launch_fill_u64(tp.unit_diag, static_cast<uint64_t>(tp.n_units) * kNDiag, 0ull, st));
    HIP_TRY(launch_transport(tp, sh, st, nullptr));
    return MCRNG_OK;
}

// Carves one particle bank of `cap` entries out of a device buffer.
static EventBank carve_bank(void* base, uint64_t cap) {
    char* p = static_cast<char*>(base);
    auto take = [&](size_t bytes) {
        char* r = p;
        p += (bytes + 255) & ~static_cast<size_t>(255);
        return r;
    };
    EventBank b;
    b.x64 = reinterpret_cast<double*>(take(cap * 8));
    b.mu64 = reinterpret_cast<double*>(take(cap * 8));
    b.t64 = reinterpret_cast<double*>(take(cap * 8));
    b.tau64 = reinterpret_cast<double*>(take(cap * 8));
    b.x32 = reinterpret_cast<float*>(take(cap * 4));
    b.mu32 = reinterpret_cast<float*>(take(cap * 4));
    b.t32 = reinterpret_cast<float*>(take(cap * 4));
    b.tau32 = reinterpret_cast<float*>(take(cap * 4));
    b.X = reinterpret_cast<uint64_t*>(take(cap * 8));
    b.cell = reinterpret_cast<int32_t*>(take(cap * 4));
    b.tb = reinterpret_cast<int32_t*>(take(cap * 4));
    b.hdraws = reinterpret_cast<uint32_t*>(take(cap * 4));
    b.events = reinterpret_cast<uint32_t*>(take(cap * 4));
    b.colls = reinterpret_cast<uint32_t*>(take(cap * 4));
    b.unit = reinterpret_cast<uint32_t*>(take(cap * 4));
    b.rec = reinterpret_cast<uint32_t*>(take(cap * 4));
    return b;
}
static size_t bank_bytes(uint64_t cap) { return 16 * (((cap * 8) + 255) & ~static_cast<uint64_t>(255)); }

// Event-sorted schedule: slices of whole work units fill a particle bank;
// each launch advances every live particle by one event and compacts the
// survivors into the other bank; the host reads the live count every few
// launches.  Partial slots are zeroed and accumulated with integer atomics.
namespace mcrng {
hipError_t launch_event_finish(const EventParams& p, int f32, int timed, hipStream_t st);   // events.hip
}


static int run_event_schedule(mcrng_ctx* ctx, const LcgDev& L, const mcrng_run_opts& o, hipStream_t st) {
    const uint64_t total = ctx->h_rec_begin.back();
    if (total >> 32) return fail(MCRNG_EINVAL, "event schedule: more than 2^32 histories in one run");
    uint64_t cap = o.bank_size ? o.bank_size : (1u << 22);
    for (const WorkUnit& U : ctx->h_units) cap = std::max<uint64_t>(cap, U.count);
    int rc;
    if ((rc = ensure(ctx->bank_a, bank_bytes(cap), st)) < 0) return rc;
    if ((rc = ensure(ctx->bank_b, bank_bytes(cap), st)) < 0) return rc;
    if ((rc = ensure(ctx->records, std::max<uint64_t>(total, 1) * sizeof(HistoryRecord), st)) < 0) return rc;
    EventParams ep;
    std::memset(&ep, 0, sizeof ep);
    ep.tp = make_params(ctx, L, 1);
    ep.records = static_cast<HistoryRecord*>(ctx->records.p);
    ep.rec_begin = static_cast<const uint64_t*>(ctx->rec_begin.p);
    // live counts rotate over three device words: launch s reads word s % 3,
    // appends to word (s + 1) % 3 and zeroes word (s + 2) % 3
    uint32_t* cnt = static_cast<uint32_t*>(ctx->counter.p) + 4;
    EventBank A = carve_bank(ctx->bank_a.p, cap), B = carve_bank(ctx->bank_b.p, cap);
    const int f32 = o.precision == MCRNG_FP32;
    const int timed = ctx->any_timed;
    HIP_TRY(launch_fill_u64(ep.tp.partial, ctx->partial_words, 0ull, st));
    if (!ctx->h_pinned) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&ctx->h_pinned), 64, hipHostMallocDefault));
    const uint32_t nu = static_cast<uint32_t>(ctx->h_units.size());
    uint32_t u0 = 0;
    while (u0 < nu) {
        uint32_t u1 = u0;
        while (u1 < nu && ctx->h_rec_begin[u1 + 1] - ctx->h_rec_begin[u0] <= cap) ++u1;
        ep.unit_begin = u0;
        ep.unit_end = u1;
        ep.one_group = ctx->h_group_first[u1 - 1] <= u0;   // units [u0, u1) of one (problem, batch)
        ep.in = A;
        ep.out = B;
        ep.n_in = static_cast<uint32_t>(ctx->h_rec_begin[u1] - ctx->h_rec_begin[u0]);
        HIP_TRY(launch_event_init(ep, f32, timed, st));
        HIP_TRY(launch_fill_u32(cnt, 1, ep.n_in, st));
        HIP_TRY(launch_fill_u32(cnt + 1, 1, 0u, st));
        // below 1/64 of the bank (64Ki live particles for the default bank) the
        // slice's remaining particles run to their ends in one launch; the host
        // reads the live count every few launches and sizes the grids from it
        const uint64_t finish_below = cap / 64;
        constexpr uint32_t kStepsPerRead = 4;
        uint32_t s = 0;
        while (ep.n_in > 0) {
            if (ep.n_in < finish_below) {
                ep.n_live = cnt + s % 3;
                HIP_TRY(launch_event_finish(ep, f32, timed, st));
                break;
            }
            for (uint32_t k = 0; k < kStepsPerRead; ++k, ++s) {
                ep.n_live = cnt + s % 3;
                ep.n_out = cnt + (s + 1) % 3;
                ep.n_clear = cnt + (s + 2) % 3;
                HIP_TRY(launch_event_step(ep, f32, timed, st));
                std::swap(ep.in, ep.out);
            }
            HIP_TRY(hipMemcpyAsync(ctx->h_pinned, cnt + s % 3, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            uint32_t live = 0;
            std::memcpy(&live, ctx->h_pinned, sizeof live);
            if (live > ep.n_in) return fail(MCRNG_EDEVICE, "event schedule: bank count grew");
            ep.n_in = live;
        }
        u0 = u1;
    }
    HIP_TRY(launch_event_unit_diag(ep, st));
    return MCRNG_OK;
}

static uint64_t opts_key(uint64_t tables_sig, const mcrng_run_opts& o) {
    return fnv(tables_sig, &o, sizeof o);
}

static int run_prepared(mcrng_ctx* ctx, const LcgDev& L, const mcrng_run_opts& o, hipStream_t st) {
    HIP_TRY(hipEventRecord(ctx->ev0, st));
    if (o.schedule == MCRNG_SCHED_EVENT) {
        ctx->last_kernel = "k_event_step";
        int rc = run_event_schedule(ctx, L, o, st);
        if (rc < 0) return rc;
    } else if (o.use_graph) {
        const uint64_t key = opts_key(ctx->tables_sig, o);
        auto it = ctx->graphs.find(key);
        if (it == ctx->graphs.end()) {
            // the tables were uploaded on `st`; the capture stream must see them
            HIP_TRY(hipStreamSynchronize(st));
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_run(ctx, L, o, ctx->capture_stream);
            hipError_t e = hipStreamEndCapture(ctx->capture_stream, &g);
            if (rc < 0) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(MCRNG_EDEVICE, "graph capture: %s", hipGetErrorString(e));
            hipGraphExec_t ex = nullptr;
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(MCRNG_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
            it = ctx->graphs.emplace(key, ex).first;
            ctx->graph_kernel[key] = ctx->last_kernel;
        }
        ctx->last_kernel = ctx->graph_kernel[key];
        HIP_TRY(hipGraphLaunch(it->second, st));
    } else {
        int rc = enqueue_run(ctx, L, o, st);
        if (rc < 0) return rc;
    }
    HIP_TRY(hipEventRecord(ctx->ev1, st));
    ctx->timing_valid = true;
    return MCRNG_OK;
}

extern "C" const char* mcrng_last_run_kernel(const mcrng_ctx* ctx) { return ctx ? ctx->last_kernel : ""; }

extern "C" float mcrng_last_run_ms(mcrng_ctx* ctx) {
    if (!ctx || !ctx->timing_valid) return -1.0f;
    if (hipEventSynchronize(ctx->ev1) != hipSuccess) return -1.0f;
    float ms = -1.0f;
    if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) != hipSuccess) return -1.0f;
    return ms;
}

static int enqueue_reduce(mcrng_ctx* ctx, uint64_t* d_raw, double* d_flux, uint64_t* d_diag, hipStream_t st) {
    ReduceParams rp;
    std::memset(&rp, 0, sizeof rp);
    rp.groups = static_cast<const ReduceGroup*>(ctx->groups.p);
    rp.n_groups = static_cast<uint32_t>(ctx->h_groups.size());
    rp.max_slice = ctx->max_slice;
    rp.units = static_cast<const WorkUnit*>(ctx->units.p);
    rp.partial = static_cast<const uint64_t*>(ctx->partial.p);
    rp.dx = static_cast<const double*>(ctx->dx.p);
    rp.dt = static_cast<const double*>(ctx->dt.p);
    rp.raw = d_raw;
    rp.flux = d_flux;
    rp.pu_begin = static_cast<const uint32_t*>(ctx->pu_begin.p);
    rp.n_problems = ctx->n_problems;
    rp.unit_diag = static_cast<const uint64_t*>(ctx->unit_diag.p);
    rp.diag = d_diag;
    HIP_TRY(launch_reduce(rp, st));
    return MCRNG_OK;
}

extern "C" int mcrng_reduce_tallies(mcrng_ctx* ctx, uint64_t* d_raw, double* d_flux, uint64_t* d_diag, void* stream) {
    if (!ctx) return fail(MCRNG_EINVAL, "ctx is NULL");
    if (!ctx->have_run) return fail(MCRNG_ESTATE, "reduce_tallies before any run_histories");
    if (!d_raw || !d_flux) return fail(MCRNG_EINVAL, "d_raw and d_flux are required");
    HIP_TRY(hipSetDevice(ctx->device));
    return enqueue_reduce(ctx, d_raw, d_flux, d_diag, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ allocation-free runs

// Device memory of mcrng_run_histories_noalloc: tables, work units, partial
// tallies, unit diagnostics and the scheduling counter of a run, carved in
// order by an Arena.  The array belongs to this file's code object, which
// the runtime loads on a device (and so allocates the array there) when its
// address is first taken on that device; it stays until the process ends.
// Host code must use the per-device address from hipGetSymbolAddress, never
// the array's name.
constexpr size_t kStaticScratchBytes = static_cast<size_t>(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct StaticDevice {
    std::mutex mu;      // one host thread at a time builds and enqueues a run
    Arena arena;
    mcrng_ctx ctx;      // host tables of the last run; every buffer is carved from `arena`
};
static std::mutex g_static_mu;
static std::map<int, StaticDevice*> g_static;   // per device, kept for the process (like the array)

// The device's static state; on the first call for a device (the current
// one) takes the array's address there.
static int static_device(int dev, StaticDevice** out) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    auto it = g_static.find(dev);
    if (it != g_static.end()) {
        *out = it->second;
        return MCRNG_OK;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        return fail(MCRNG_EDEVICE, "static scratch address on device %d: %s", dev, hipGetErrorString(e));
    StaticDevice* d = new (std::nothrow) StaticDevice();
    if (!d) return fail(MCRNG_ENOMEM, "static state");
    d->arena.base = static_cast<char*>(ptr);
    d->arena.cap = kStaticScratchBytes;
    d->ctx.device = dev;
    d->ctx.arena = &d->arena;
    DevBuf* bufs[] = {&d->ctx.problems, &d->ctx.edges64, &d->ctx.sig64, &d->ctx.scat64, &d->ctx.cbin,
                      &d->ctx.edges32, &d->ctx.sig32, &d->ctx.tedges64, &d->ctx.tedges32, &d->ctx.units,
                      &d->ctx.order, &d->ctx.partial, &d->ctx.unit_diag, &d->ctx.counter, &d->ctx.groups,
                      &d->ctx.dx, &d->ctx.dt, &d->ctx.pu_begin, &d->ctx.rec_begin};
    for (DevBuf* b : bufs) b->arena = &d->arena;
    g_static[dev] = d;
    *out = d;
    return MCRNG_OK;
}

extern "C" int mcrng_run_histories_noalloc(const mcrng_lcg* lcg, const mcrng_problem* problems, uint32_t n_problems,
                                           const mcrng_run_opts* opts, uint64_t* d_raw, double* d_flux,
                                           uint64_t* d_diag, void* stream) {
    if (!problems) return fail(MCRNG_EINVAL, "problems is NULL");
    if (n_problems == 0) return fail(MCRNG_EINVAL, "n_problems must be >= 1");
    if (!d_raw || !d_flux) return fail(MCRNG_EINVAL, "d_raw and d_flux are required");
    LcgDev L;
    int rc = validate_lcg(lcg, 53, &L);
    if (rc < 0) return rc;
    mcrng_run_opts o;
    if ((rc = normalise_opts(opts, &o)) < 0) return rc;
    if (o.schedule != MCRNG_SCHED_HISTORY) return fail(MCRNG_EINVAL, "the allocation-free run has the history schedule only");
    if (o.use_graph) return fail(MCRNG_EINVAL, "the allocation-free run does not capture graphs");
    for (uint32_t i = 0; i < n_problems; ++i)
        if ((rc = validate_problem(problems[i], i)) < 0) return rc;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    StaticDevice* sd = nullptr;
    if ((rc = static_device(dev, &sd)) < 0) return rc;
    std::lock_guard<std::mutex> lk(sd->mu);
    mcrng_ctx* ctx = &sd->ctx;
    sd->arena.reset();
    DevBuf* bufs[] = {&ctx->problems, &ctx->edges64, &ctx->sig64, &ctx->scat64, &ctx->cbin, &ctx->edges32,
                      &ctx->sig32, &ctx->tedges64, &ctx->tedges32, &ctx->units, &ctx->order, &ctx->partial,
                      &ctx->unit_diag, &ctx->counter, &ctx->groups, &ctx->dx, &ctx->dt, &ctx->pu_begin,
                      &ctx->rec_begin};
    for (DevBuf* b : bufs) {
        b->p = nullptr;
        b->cap = 0;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!o.unit_histories)
        o.unit_histories = default_unit_histories(problems, n_problems, chain_planned(problems, n_problems, o));
    int warn = MCRNG_OK;
    if ((rc = build_tables(ctx, L, problems, n_problems, o.unit_histories, st, &warn)) < 0) return rc;
    if ((rc = enqueue_run(ctx, L, o, st)) < 0) return rc;
    if ((rc = enqueue_reduce(ctx, d_raw, d_flux, d_diag, st)) < 0) return rc;
    return warn;
}

// ------------------------------------------------------------------ autotuner

// Cache key of a tuning: the problem set (generator, geometry, seeding,
// history counts) and every base option, normalised (the search overwrites
// block, hist_per_lane, tally_copies, coll_batch and unit_histories, but
// the other fields, e.g. grid and bank_size, change what is timed).
static uint64_t shape_key(const mcrng_lcg* lcg, const mcrng_problem* P, uint32_t n, const mcrng_run_opts& base) {
    uint64_t h = signature(lcg, P, n, 0);
    return fnv(h, &base, sizeof base);
}

extern "C" int mcrng_autotune(mcrng_ctx* ctx, const mcrng_lcg* lcg, const mcrng_problem* problems, uint32_t n_problems,
                              const mcrng_run_opts* base, mcrng_run_opts* best, float* best_ms, void* stream) {
    if (!ctx || !best) return fail(MCRNG_EINVAL, "ctx and best are required");
    if (!problems) return fail(MCRNG_EINVAL, "problems is NULL");
    if (n_problems == 0) return fail(MCRNG_EINVAL, "n_problems must be >= 1");
    LcgDev L;
    int rc = validate_lcg(lcg, 53, &L);
    if (rc < 0) return rc;
    mcrng_run_opts b0;
    if ((rc = normalise_opts(base, &b0)) < 0) return rc;
    for (uint32_t i = 0; i < n_problems; ++i)
        if ((rc = validate_problem(problems[i], i)) < 0) return rc;
    const uint64_t key = shape_key(lcg, problems, n_problems, b0);
    auto hit = ctx->tuned.find(key);
    if (hit != ctx->tuned.end()) {
        *best = hit->second;
        if (best_ms) *best_ms = -1.0f;
        return MCRNG_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto timed_run = [&](const mcrng_run_opts& o, float* ms) -> int {
        int r = mcrng_run_histories(ctx, lcg, problems, n_problems, &o, stream);
        if (r < 0) return r;
        r = mcrng_run_histories(ctx, lcg, problems, n_problems, &o, stream);
        if (r < 0) return r;
        *ms = mcrng_last_run_ms(ctx);
        return *ms < 0 ? fail(MCRNG_EDEVICE, "timing failed") : MCRNG_OK;
    };
    mcrng_run_opts cur = b0;
    cur.unit_histories = 0;
    cur.use_graph = 0;
    float cur_ms = 0;
    if ((rc = timed_run(cur, &cur_ms)) < 0) return rc;
    auto try_field = [&](uint32_t mcrng_run_opts::*field, std::initializer_list<uint32_t> vals) -> int {
        for (uint32_t v : vals) {
            if (cur.*field == v) continue;
            mcrng_run_opts cand = cur;
            cand.*field = v;
            float ms = 0;
            int r = timed_run(cand, &ms);
            if (r == MCRNG_EINVAL) continue;   // e.g. LDS does not fit this shape
            if (r < 0) return r;
            if (ms < cur_ms) {
                cur = cand;
                cur_ms = ms;
            }
        }
        return MCRNG_OK;
    };
    if ((rc = try_field(&mcrng_run_opts::block, {64, 128, 256, 512, 1024})) < 0) return rc;
    if ((rc = try_field(&mcrng_run_opts::hist_per_lane, {1, 2, 4})) < 0) return rc;
    if ((rc = try_field(&mcrng_run_opts::tally_copies, {1, 2})) < 0) return rc;
    if (cur.schedule == MCRNG_SCHED_HISTORY)
        if ((rc = try_field(&mcrng_run_opts::coll_batch, {1, 16, 24, 32, 36, 40, 48})) < 0) return rc;
    const uint32_t u0 = default_unit_histories(problems, n_problems, chain_planned(problems, n_problems, cur));
    if ((rc = try_field(&mcrng_run_opts::unit_histories, {u0 / 4 > 256 ? u0 / 4 : 256, u0, u0 * 4})) < 0) return rc;
    if (cur.unit_histories == 0) cur.unit_histories = u0;
    cur.use_graph = b0.use_graph;
    HIP_TRY(hipStreamSynchronize(st));
    ctx->tuned[key] = cur;
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return MCRNG_OK;
}

// ------------------------------------------------------------ uniforms

extern "C" int mcrng_uniforms(const mcrng_lcg* lcg, const mcrng_seeding* seeding, uint64_t n, uint32_t k,
                              uint64_t* d_state, double* d_u, void* stream) {
    LcgDev L;
    int rc = validate_lcg(lcg, 53, &L);
    if (rc < 0) return rc;
    if (n == 0 || k == 0) return MCRNG_OK;
    if (!d_u) return fail(MCRNG_EINVAL, "d_u is NULL");
    if (!seeding && !d_state) return fail(MCRNG_EINVAL, "d_state is required when seeding is NULL");
    if (n >> 40) return fail(MCRNG_EINVAL, "n = %llu too large", (unsigned long long)n);
    SeedDev S;
    std::memset(&S, 0, sizeof S);
    int mode = SEED_LOAD;
    if (seeding) {
        rc = build_seed(L, seeding, n, &S);
        if (rc < 0) return rc;
        mode = S.kind;
    }
    HIP_TRY(launch_uniforms(L, S, mode, n, k, d_state, d_u, static_cast<hipStream_t>(stream)));
    return rc;
}

// ------------------------------------------------------------ pulse problem

static int validate_pulse(const mcrng_pulse_problem* P) {
    if (!P) return fail(MCRNG_EINVAL, "problem is NULL");
    if (!(P->sigma_t >= kMinSigma && P->sigma_t <= kMaxSigma))
        return fail(MCRNG_EINVAL, "sigma_t must lie within [2^-64, 2^64]");
    if (!(P->scatter >= 0.0 && P->scatter <= 1.0)) return fail(MCRNG_EINVAL, "scatter must be in [0, 1]");
    if (!(P->multiplicity >= 0.0 && P->multiplicity <= 14.0))
        return fail(MCRNG_EINVAL, "multiplicity must be in [0, 14]");
    if (!std::isfinite(P->x_lo) || !std::isfinite(P->x_hi) || !(P->x_lo < P->x_hi))
        return fail(MCRNG_EINVAL, "the tally interval needs finite x_lo < x_hi");
    if (P->n_time_bins < 1 || P->n_time_bins > 4096) return fail(MCRNG_EINVAL, "n_time_bins must be in 1..4096");
    if (!P->time_edges) return fail(MCRNG_EINVAL, "time_edges is NULL");
    if (!(P->time_edges[0] >= 0.0) || !increasing(P->time_edges, P->n_time_bins + 1) ||
        !std::isfinite(P->time_edges[P->n_time_bins]))
        return fail(MCRNG_EINVAL, "time edges must be finite, >= 0 and strictly increasing");
    if (P->n_batches < 1 || P->per_batch < 1) return fail(MCRNG_EINVAL, "n_batches and per_batch must be >= 1");
    if ((static_cast<u128>(P->n_batches) * P->per_batch) >> 40) return fail(MCRNG_EINVAL, "more than 2^40 sources");
    if ((static_cast<u128>(P->first_batch) + P->n_batches) * P->per_batch >> 64)
        return fail(MCRNG_EINVAL, "source index overflows 64 bits");
    const mcrng_seeding& S = P->seeding;
    if (S.kind != MCRNG_SEED_HASH && S.kind != MCRNG_SEED_STRIDE) return fail(MCRNG_EINVAL, "seeding.kind unknown");
    if (S.hier || S.first_index || S.group_key)
        return fail(MCRNG_EINVAL, "pulse seeding uses first_batch; hier, first_index and group_key must be 0");
    if (S.kind == MCRNG_SEED_STRIDE && S.stride == 0) return fail(MCRNG_EINVAL, "stride seeding needs stride >= 1");
    return MCRNG_OK;
}

static PulseBankView carve_pulse_bank(void* base, uint64_t cap) {
    char* p = static_cast<char*>(base);
    PulseBankView v;
    v.x = reinterpret_cast<double*>(p);
    v.t = reinterpret_cast<double*>(p + cap * 8);
    v.X = reinterpret_cast<uint64_t*>(p + cap * 16);
    v.batch = reinterpret_cast<uint32_t*>(p + cap * 24);
    v.tb = reinterpret_cast<int32_t*>(p + cap * 28);
    return v;
}

// Reads n <= 8 device words (through a pinned host buffer) after the work
// queued on st.
// Input particles a wave of the bank kernel takes per atomic on the item
// counter: small launches keep many waves busy, large ones need few atomics
// on that one counter (its same-address atomics serialise across the GPU).
static uint32_t pulse_auto_chunk(uint64_t n) {
    uint32_t c = 256;
    while (c < 4096 && static_cast<uint64_t>(c) * 1024 * 2 <= n) c *= 2;
    return c;
}

static int read_words(mcrng_ctx* ctx, const uint64_t* d, uint32_t n, uint64_t* h, hipStream_t st) {
    if (!ctx->h_pinned) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&ctx->h_pinned), 64, hipHostMallocDefault));
    HIP_TRY(hipMemcpyAsync(ctx->h_pinned, d, n * sizeof *h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (uint32_t i = 0; i < n; ++i) h[i] = ctx->h_pinned[i];
    return MCRNG_OK;
}

static int read_u64(mcrng_ctx* ctx, const uint64_t* d, uint64_t* h, hipStream_t st) {
    return read_words(ctx, d, 1, h, st);
}

// Grows b to at least `bytes`, keeping its first `used` bytes.
static int ensure_keep(DevBuf& b, size_t used, size_t bytes, hipStream_t st) {
    if (bytes <= b.cap) return MCRNG_OK;
    const size_t want = std::max<size_t>(std::max<size_t>(bytes + bytes / 4, 2 * b.cap), 256);
    void* np = nullptr;
    HIP_TRY(hipMalloc(&np, want));
    if (used) HIP_TRY(hipMemcpyAsync(np, b.p, used, hipMemcpyDeviceToDevice, st));
    if (b.p) {
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipFree(b.p));
    }
    b.p = np;
    b.cap = want;
    return MCRNG_OK;
}

static int run_pulse(mcrng_ctx* ctx, const mcrng_lcg* lcg, const mcrng_pulse_problem* P, const mcrng_pulse_pc* pc,
                     const mcrng_pulse_opts* opts, uint64_t* d_counts, double* d_flux, uint64_t* d_diag,
                     uint64_t* d_pop, void* stream) {
    LcgDev L;
    int rc = validate_lcg(lcg, 53, &L);
    if (rc < 0) return rc;
    if ((rc = validate_pulse(P)) < 0) return rc;
    if (pc) {
        if (pc->census_every == 0) return fail(MCRNG_EINVAL, "pc.census_every must be >= 1");
        if (pc->target == 0 || pc->target > (1ull << 40)) return fail(MCRNG_EINVAL, "pc.target must be in 1..2^40");
        if (pc->reserved0 || pc->reserved[0] || pc->reserved[1]) return fail(MCRNG_EINVAL, "pc.reserved must be 0");
        if (P->seeding.kind != MCRNG_SEED_HASH)
            return fail(MCRNG_EINVAL, "population control needs hash seeding (census copies are seeded by eq. 5)");
    }
    mcrng_pulse_opts o;
    std::memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    for (uint32_t r : o.reserved)
        if (r) return fail(MCRNG_EINVAL, "opts.reserved must be 0");
    if (o.finish_div == 0) o.finish_div = 1;
    if (o.chunk != 0 && (o.chunk < 64 || o.chunk > (1u << 20)))
        return fail(MCRNG_EINVAL, "opts.chunk must be 0 or in 64..2^20");
    const bool hash = P->seeding.kind == MCRNG_SEED_HASH;
    const uint64_t n_src = static_cast<uint64_t>(P->n_batches) * P->per_batch;
    if (o.block == 0) o.block = 256;
    if (o.schedule != MCRNG_PULSE_AUTO && o.schedule != MCRNG_PULSE_BANK && o.schedule != MCRNG_PULSE_FAMILY &&
        o.schedule != MCRNG_PULSE_EVENT)
        return fail(MCRNG_EINVAL, "opts.schedule unknown");
    if ((o.schedule == MCRNG_PULSE_BANK || o.schedule == MCRNG_PULSE_EVENT) && !hash)
        return fail(MCRNG_EINVAL, "the bank and event schedules need hash seeding (stride families share one stream)");
    if (pc && o.schedule == MCRNG_PULSE_FAMILY)
        return fail(MCRNG_EINVAL, "population control runs on the bank schedule");
    if (o.block != 64 && o.block != 128 && o.block != 256 && o.block != 512 && o.block != 1024)
        return fail(MCRNG_EINVAL, "opts.block = %u not in {64,128,256,512,1024}", o.block);
    if (o.stack_depth == 0) o.stack_depth = 128;
    if (o.stack_depth > 65535) return fail(MCRNG_EINVAL, "opts.stack_depth must be <= 65535");
    if (!ctx) return fail(MCRNG_EINVAL, "ctx is NULL");
    if (!d_counts) return fail(MCRNG_EINVAL, "d_counts is NULL");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    // hash seeding lets every particle run anywhere: generation banks, or
    // depth-first families once there are enough of them to fill every lane
    // many times over (measured crossover on the 1000-source batches: about
    // 16 families per resident lane); stride families must run depth first
    // on one lane; population control needs the banks
    if (o.schedule == MCRNG_PULSE_AUTO) {
        const uint64_t lanes = static_cast<uint64_t>(pulse_family_grid(static_cast<int>(o.block))) * o.block;
        if (!hash)
            o.schedule = MCRNG_PULSE_FAMILY;
        else if (!pc && n_src >= 16 * lanes)
            o.schedule = MCRNG_PULSE_FAMILY;
        else
            o.schedule = MCRNG_PULSE_BANK;
    }

    PulseParams pp;
    std::memset(&pp, 0, sizeof pp);
    pp.lcg = L;
    pp.first_batch = P->first_batch;
    pp.per_batch = P->per_batch;
    pp.n_batches = P->n_batches;
    pp.n_time_bins = P->n_time_bins;
    pp.hash = hash ? 1u : 0u;
    const double nu_floor = std::floor(P->multiplicity);
    pp.n_floor = static_cast<uint32_t>(nu_floor);
    pp.nu_frac = P->multiplicity - nu_floor;
    pp.sigma_t = P->sigma_t;
    pp.scatter = P->scatter;
    pp.x_lo = P->x_lo;
    pp.x_hi = P->x_hi;
    pp.t_end = P->time_edges[P->n_time_bins];
    pp.tb0 = -1;
    while (pp.tb0 + 1 < static_cast<int32_t>(P->n_time_bins) && P->time_edges[pp.tb0 + 1] <= 0.0) pp.tb0++;
    pp.stack_depth = o.stack_depth;
    int warn = MCRNG_OK;
    if (hash) {
        pp.seed.kind = SEED_HASH;
        pp.seed.base = P->seeding.base;   // the global seed s; batch parents are hashed on the device
    } else {
        mcrng_seeding sd = P->seeding;
        sd.first_index = P->first_batch * P->per_batch;
        if ((rc = build_seed(L, &sd, n_src, &pp.seed)) < 0) return rc;
        warn = rc;
        pp.stride_q = P->seeding.stride;
    }
    const uint32_t n_max = pp.n_floor + (pp.nu_frac > 0.0 ? 1u : 0u);

    ctx->h_pulse_tedges.assign(P->time_edges, P->time_edges + P->n_time_bins + 1);
    if ((rc = upload(ctx->pulse_tedges, ctx->h_pulse_tedges, st)) < 0) return rc;
    if ((rc = ensure(ctx->pulse_misc, 64, st)) < 0) return rc;
    if ((rc = ensure(ctx->pulse_diag, kNDiag * sizeof(uint64_t), st)) < 0) return rc;
    pp.t_edges = static_cast<const double*>(ctx->pulse_tedges.p);
    pp.counts = d_counts;
    const uint64_t n_counters = static_cast<uint64_t>(P->n_batches) * P->n_time_bins;
    pp.n_counters = static_cast<uint32_t>(std::min<uint64_t>(n_counters, 0xffffffffu));
    pp.lds_tally = n_counters <= kPulseLdsCounters ? 1u : 0u;
    pp.diag = static_cast<uint64_t*>(ctx->pulse_diag.p);
    // misc words: out_count, item_counter (reset per bank launch), family_counter, overflow,
    // census arrivals, census copies
    uint64_t* misc = static_cast<uint64_t*>(ctx->pulse_misc.p);
    pp.out_count = misc;
    pp.item_counter = misc + 1;
    pp.family_counter = misc + 2;
    pp.overflow = reinterpret_cast<uint32_t*>(misc + 3);
    pp.cen_count = misc + 4;
    pp.copy_count = misc + 5;
    const uint32_t K = pc ? pc->census_every : 0;
    const uint32_t n_census = pc ? (P->n_time_bins - 1) / K : 0;
    const uint64_t n_pop = static_cast<uint64_t>(P->n_batches) * n_census * 2;
    if (pc) {
        pp.census_every = K;
        pp.n_census = n_census;
        pp.pc_target = pc->target;
        pp.pc_seed = pc->seed;
        if ((rc = ensure(ctx->pulse_pop, std::max<uint64_t>(n_pop, 1) * 8, st)) < 0) return rc;
        pp.pop = static_cast<uint64_t*>(ctx->pulse_pop.p);
        if (n_pop) HIP_TRY(launch_fill_u64(pp.pop, n_pop, 0ull, st));
    }
    HIP_TRY(launch_fill_u64(misc, 8, 0ull, st));
    HIP_TRY(launch_fill_u64(pp.diag, kNDiag, 0ull, st));
    HIP_TRY(launch_fill_u64(d_counts, static_cast<uint64_t>(P->n_batches) * P->n_time_bins, 0ull, st));
    HIP_TRY(hipEventRecord(ctx->ev0, st));
    ctx->timing_valid = false;

    // Generations: a launch runs the lines of descent of its input items
    // (their first emerging particles inline) and banks the siblings for
    // the next launch.  Capacity per launch: the continue budget (2 per
    // input item), n_max per input item, and one LDS stage plus one
    // iteration's appends per wave.  With `pcen` (a census of population
    // control ends the epoch) every line ends at most once at the census, so
    // the census bank grows by at most the launch's items.
    // The tail of a chain (a generation that shrank to at most 1/finish_div
    // of the largest, and to at most kFinishItems) is finished by one launch
    // that runs each particle's descendants depth first (up to kFinishBudget
    // particles each; the rest, if any, is the next generation).
    constexpr uint64_t kFinishItems = 65536;
    constexpr uint32_t kFinishBudget = 64, kFinishDepth = 32;
    auto generations = [&](int kind, uint64_t n, bool pcen, uint64_t* cen_used) -> int {
        int cur = 0, nxt = 1;
        uint64_t in_cap = 0, peak = 0, prev = ~0ull;
        while (n > 0) {
            pp.chunk = o.chunk ? o.chunk : pulse_auto_chunk(n);
            peak = std::max(peak, n);
            const bool fin = kind == PULSE_ITEMS_BANK && o.finish_div != 0xffffffffu && n <= kFinishItems &&
                             n < prev && n * o.finish_div <= peak;
            prev = n;
            if (fin) {
                const uint32_t grid = pulse_finish_grid(n);
                const uint64_t lanes = static_cast<uint64_t>(grid) * 256;
                int r = ensure(ctx->pulse_stack, lanes * kFinishDepth * sizeof(PulseStackEntry), st);
                if (r < 0) return r;
                const uint64_t ocap = n * (kFinishBudget + kFinishDepth + 1) * static_cast<uint64_t>(n_max) + 64;
                if ((r = ensure(ctx->pulse_bank[nxt], ocap * 32, st, 8)) < 0) return r;
                if (pcen) {
                    r = ensure_keep(ctx->pulse_census, *cen_used * sizeof(PulseCensusEntry),
                                    (*cen_used + n * kFinishBudget) * sizeof(PulseCensusEntry), st);
                    if (r < 0) return r;
                    pp.cen = static_cast<PulseCensusEntry*>(ctx->pulse_census.p);
                    pp.cen_cap = ctx->pulse_census.cap / sizeof(PulseCensusEntry);
                }
                pp.in = carve_pulse_bank(ctx->pulse_bank[cur].p, in_cap);
                pp.n_in = n;
                pp.out = carve_pulse_bank(ctx->pulse_bank[nxt].p, ocap);
                pp.out_cap = ocap;
                pp.stack = static_cast<PulseStackEntry*>(ctx->pulse_stack.p);
                pp.stack_depth = kFinishDepth;
                pp.lane_budget = kFinishBudget;
                HIP_TRY(launch_fill_u64(misc, 3, 0ull, st));
                HIP_TRY(launch_pulse_finish(pp, pcen, grid, st));
                uint64_t w[5];
                if ((r = read_words(ctx, misc, 5, w, st)) < 0) return r;
                if (w[3] & 0xffffffffull) return fail(MCRNG_ERANGE, "a particle bank ran out of room");
                n = w[0];
                if (pcen) *cen_used = w[4];
                std::swap(cur, nxt);
                in_cap = ocap;
                continue;
            }
            const uint32_t grid = pulse_bank_grid(pp, kind, pcen, static_cast<int>(o.block), n);
            const uint64_t waves = static_cast<uint64_t>(grid) * o.block / 64;
            // event schedule: no line runs on within a launch (one flight
            // and collision per particle and launch)
            const uint64_t budget = o.schedule == MCRNG_PULSE_EVENT ? 0 : 2 * n;
            const uint64_t slack =
                (waves + 1) * (pulse_bank_stage(static_cast<int>(o.block)) + 64 * static_cast<uint64_t>(n_max));
            const uint64_t ocap = budget + static_cast<uint64_t>(n_max) * n + slack;
            int r = ensure(ctx->pulse_bank[nxt], ocap * 32, st, 8);
            if (r < 0) return r;
            if (pcen) {
                r = ensure_keep(ctx->pulse_census, *cen_used * sizeof(PulseCensusEntry),
                                (*cen_used + n) * sizeof(PulseCensusEntry), st);
                if (r < 0) return r;
                pp.cen = static_cast<PulseCensusEntry*>(ctx->pulse_census.p);
                pp.cen_cap = ctx->pulse_census.cap / sizeof(PulseCensusEntry);
            }
            if (kind == PULSE_ITEMS_BANK) pp.in = carve_pulse_bank(ctx->pulse_bank[cur].p, in_cap);
            pp.n_in = kind == PULSE_ITEMS_SOURCES ? 0 : n;
            pp.out = carve_pulse_bank(ctx->pulse_bank[nxt].p, ocap);
            pp.out_cap = ocap;
            pp.cont_budget = budget;
            HIP_TRY(launch_fill_u64(misc, 2, 0ull, st));
            HIP_TRY(launch_pulse_bank(pp, kind, pcen, static_cast<int>(o.block), grid, st));
            uint64_t w[5];
            if ((r = read_words(ctx, misc, 5, w, st)) < 0) return r;
            // a bank that ran out of room (never, by the capacities above)
            // ends the run before any launch reads past it
            if (w[3] & 0xffffffffull) return fail(MCRNG_ERANGE, "a particle bank ran out of room");
            n = w[0];
            if (pcen) *cen_used = w[4];
            std::swap(cur, nxt);
            in_cap = ocap;
            kind = PULSE_ITEMS_BANK;
        }
        return MCRNG_OK;
    };

    if (pc) {
        // Epochs between census times, chunk by chunk of whole batches
        // (population control is per batch).  After each census: arrivals
        // per batch, then the copies, which start the next epoch.
        const uint64_t chunk_b = std::max<uint64_t>(
            1, std::min<uint64_t>(kPulsePcChunkBatches, (1ull << 23) / P->per_batch));
        for (uint64_t b0 = 0; b0 < P->n_batches; b0 += chunk_b) {
            const uint64_t b1 = std::min<uint64_t>(P->n_batches, b0 + chunk_b);
            pp.src_begin = b0 * P->per_batch;
            pp.src_end = b1 * P->per_batch;
            pp.batch_lo = static_cast<uint32_t>(b0);
            pp.n_chunk_batches = static_cast<uint32_t>(b1 - b0);
            uint64_t n_copies = 0;
            for (uint32_t e = 0; e <= n_census; ++e) {
                const bool pcen = e < n_census;
                pp.t_end = pcen ? P->time_edges[static_cast<size_t>(e + 1) * K] : P->time_edges[P->n_time_bins];
                uint64_t cen_used = 0;
                HIP_TRY(launch_fill_u64(pp.cen_count, 1, 0ull, st));
                if (e == 0) {
                    rc = generations(PULSE_ITEMS_SOURCES, pp.src_end - pp.src_begin, pcen, &cen_used);
                } else {
                    pp.copies = static_cast<const PulseCensusEntry*>(ctx->pulse_copies.p);
                    pp.t_start = P->time_edges[static_cast<size_t>(e) * K];
                    pp.tb_start = static_cast<int32_t>(e * K);
                    rc = generations(PULSE_ITEMS_COPIES, n_copies, pcen, &cen_used);
                }
                if (rc < 0) return rc;
                if (!pcen) break;
                pp.census = e;
                HIP_TRY(launch_pulse_census_count(pp, cen_used, st));
                // copies: at most M + N per batch
                const uint64_t ccap = (b1 - b0) * pc->target + cen_used;
                if ((rc = ensure(ctx->pulse_copies, std::max<uint64_t>(ccap, 1) * sizeof(PulseCensusEntry), st)) < 0)
                    return rc;
                pp.copies_out = static_cast<PulseCensusEntry*>(ctx->pulse_copies.p);
                pp.copy_cap = ccap;
                HIP_TRY(launch_fill_u64(pp.copy_count, 1, 0ull, st));
                HIP_TRY(launch_pulse_split(pp, cen_used, st));
                uint64_t w[6];
                if ((rc = read_words(ctx, misc, 6, w, st)) < 0) return rc;
                if (w[3] & 0xffffffffull) return fail(MCRNG_ERANGE, "the census copies ran out of room");
                n_copies = w[5];
            }
        }
    } else if (o.schedule == MCRNG_PULSE_BANK || o.schedule == MCRNG_PULSE_EVENT) {
        // Sources go in chunks so that the banks stay within tens of GB.
        const uint64_t chunk = 1ull << 23;
        for (uint64_t c0 = 0; c0 < n_src; c0 += chunk) {
            pp.src_begin = c0;
            pp.src_end = std::min(n_src, c0 + chunk);
            if ((rc = generations(PULSE_ITEMS_SOURCES, pp.src_end - pp.src_begin, false, nullptr)) < 0) return rc;
        }
    } else {
        const uint32_t grid = pulse_family_grid(static_cast<int>(o.block));
        const uint64_t lanes = static_cast<uint64_t>(grid) * o.block;
        if ((rc = ensure(ctx->pulse_stack, lanes * o.stack_depth * sizeof(PulseStackEntry), st)) < 0) return rc;
        pp.stack = static_cast<PulseStackEntry*>(ctx->pulse_stack.p);
        pp.src_begin = 0;
        pp.src_end = n_src;
        HIP_TRY(launch_pulse_family(pp, static_cast<int>(o.block), grid, st));
    }
    HIP_TRY(hipEventRecord(ctx->ev1, st));
    ctx->timing_valid = true;
    if (d_flux) HIP_TRY(launch_pulse_flux(pp, d_flux, st));
    if (d_diag)
        HIP_TRY(hipMemcpyAsync(d_diag, pp.diag, kNDiag * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    if (d_pop && n_pop)
        HIP_TRY(hipMemcpyAsync(d_pop, pp.pop, n_pop * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    uint64_t flags = 0;
    if ((rc = read_u64(ctx, misc + 3, &flags, st)) < 0) return rc;
    if (flags & 0xffffffffull)
        return fail(MCRNG_ERANGE, "a family stack (opts.stack_depth = %u) or a bank ran out of room", o.stack_depth);
    return warn;
}

extern "C" int mcrng_run_pulse(mcrng_ctx* ctx, const mcrng_lcg* lcg, const mcrng_pulse_problem* P,
                               const mcrng_pulse_opts* opts, uint64_t* d_counts, double* d_flux, uint64_t* d_diag,
                               void* stream) {
    return run_pulse(ctx, lcg, P, nullptr, opts, d_counts, d_flux, d_diag, nullptr, stream);
}

extern "C" int mcrng_run_pulse_pc(mcrng_ctx* ctx, const mcrng_lcg* lcg, const mcrng_pulse_problem* P,
                                  const mcrng_pulse_pc* pc, const mcrng_pulse_opts* opts, uint64_t* d_counts,
                                  double* d_flux, uint64_t* d_diag, uint64_t* d_pop, void* stream) {
    if (!pc) return fail(MCRNG_EINVAL, "pc is NULL");
    return run_pulse(ctx, lcg, P, pc, opts, d_counts, d_flux, d_diag, d_pop, stream);
}
