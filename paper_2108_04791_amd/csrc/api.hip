// api.hip -- the C ABI: device initialisation, the plain and batched entry
// points, configuration and diagnostics.  Host code only enqueues work; every
// step of the path runs in the kernels of sieve.hip, classify.hip and mr.hip.
//
// Plain call (isprime_u64), all on the caller's stream:
//   classify_kernel -> mr_phase1_kernel -> mr_phase2_kernel
// Each kernel writes one count per workgroup and the next scans them, so no
// counter needs clearing and no kernel uses a global atomic.
// Batched call: the same three kernels over the virtual concatenation of the
// arrays, recorded once into a HIP graph per (device, stream) together with
// the host-to-device copy of the descriptor table, then replayed per call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.h"

using namespace isp;

namespace {

constexpr int MAX_DEVICES = 64;
// A plain call is split into pieces of at most this many elements, so the
// 32-bit device counters never overflow and a workspace stays below 8 GiB.
constexpr size_t PLAIN_PIECE = (size_t)1 << 28;
// Interval pieces of fewer full segments (RANGE_SEG_SMALL numbers) than this, where
// the sieve cannot be complete, sieve by the primes below
// 2^PARTIAL_SHORT_LOG2, in up to this many segments of at least
// RANGE_MIN_CHUNK numbers.
constexpr unsigned PARTIAL_FULL_GRID = 256;
constexpr int PARTIAL_SHORT_LOG2 = 18;
constexpr uint64_t RANGE_MIN_CHUNK = 4096;
// Elements per batched call (its survivors share one 32-bit counter).
constexpr uint64_t BATCH_MAX_ELEMS = (uint64_t)1 << 30;
// A plain call over len elements uses at most ceil(len / this) Miller-Rabin
// workgroups.
constexpr size_t SMALL_CALL_PER_BLOCK = 1024;

// The allocation-free entry point (isprime_u64_noalloc) takes its workspace
// from one static device array instead of hipMalloc: calls of up to
// NOALLOC_MAX elements, laid out as the allocated workspace (survivor
// regions, base-2 passer regions, their Montgomery constants, the per-block
// counts).  Each device holds its own copy for the life of the process.
constexpr size_t NOALLOC_MAX = (size_t)1 << 20;
constexpr size_t NOALLOC_SURV_OFF = 0;
constexpr size_t NOALLOC_CAND_OFF =
    NOALLOC_SURV_OFF + (NOALLOC_MAX + 64 * (size_t)MAX_GRID) * sizeof(Survivor);
constexpr size_t NOALLOC_PREP_OFF =
    NOALLOC_CAND_OFF + (NOALLOC_MAX + (size_t)MAX_GRID) * sizeof(Survivor);
constexpr size_t NOALLOC_COUNTS_OFF =
    NOALLOC_PREP_OFF + (NOALLOC_MAX + (size_t)MAX_GRID) * sizeof(MontPrep);
constexpr size_t NOALLOC_BYTES = NOALLOC_COUNTS_OFF + 2 * (size_t)MAX_GRID * sizeof(uint32_t);
static_assert(NOALLOC_CAND_OFF % 256 == 0 && NOALLOC_PREP_OFF % 256 == 0 &&
                  NOALLOC_COUNTS_OFF % 256 == 0,
              "every part of the scratch array starts 256-byte aligned");

// Host code never names this array directly (on the host the name is only a
// stand-in for the symbol): isp_init looks up each device's address of it
// once, and the entry point passes that address to the kernels.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_init_mu;
DeviceState g_dev[MAX_DEVICES];
std::atomic<int> g_last_err{0};

std::mutex g_cfg_mu;
// The autotuner's choice for 2^26 values of mixed magnitude; other classes
// are in the tuning database that paper_2108_04791_amd/tune.py writes.
constexpr isp_config DEFAULT_CONFIG = {512, 8, 8, 8, 1, 1024, 2, 3, -1, -1};
isp_config g_cfg = DEFAULT_CONFIG;

int fail(hipError_t e)
{
    g_last_err.store((int)e);
    return e == hipErrorOutOfMemory ? ISP_ENOMEM : ISP_EDEVICE;
}

bool valid_config(const isp_config &c)
{
    auto blk = [](int b, int mx) { return b >= 64 && b <= mx && b % 64 == 0; };
    return blk(c.classify_block, 1024) &&
           (c.classify_ept == 1 || c.classify_ept == 2 || c.classify_ept == 4 ||
            c.classify_ept == 8) &&
           c.classify_blocks_per_cu >= 1 && c.classify_blocks_per_cu <= 16 &&
           (c.filter_primes == -1 || c.filter_primes == 8 || c.filter_primes == 16 ||
            c.filter_primes == 24 || c.filter_primes == 32 || c.filter_primes == 48 ||
            c.filter_primes == 64) &&
           (c.sort_survivors == -1 || c.sort_survivors == 1) && blk(c.mr_block, MR_MAX_BLOCK) &&
           c.mr_blocks_per_cu >= 1 && c.mr_blocks_per_cu <= 16 && c.mr_window >= 1 &&
           c.mr_window <= 4 && (c.rest_test == -1 || c.rest_test == 1) &&
           (c.wheel_log2 == -1 ||
            (c.wheel_log2 >= WHEEL_MIN_LOG2 && c.wheel_log2 <= WHEEL_MAX_LOG2));
}

Tuning tuning_snapshot()
{
    std::lock_guard<std::mutex> g(g_cfg_mu);
    Tuning t;
    t.classify_block = g_cfg.classify_block;
    t.classify_ept = g_cfg.classify_ept;
    t.classify_blocks_per_cu = g_cfg.classify_blocks_per_cu;
    t.filter_primes = g_cfg.filter_primes < 0 ? 0 : g_cfg.filter_primes;
    t.sort_survivors = g_cfg.sort_survivors > 0;
    t.mr_block = g_cfg.mr_block;
    t.mr_blocks_per_cu = g_cfg.mr_blocks_per_cu;
    t.mr_window = g_cfg.mr_window;
    t.rest_test = g_cfg.rest_test > 0;
    t.wheel_log2 = g_cfg.wheel_log2 > 0 ? g_cfg.wheel_log2 : 0;
    return t;
}

unsigned grid_of(int cus, int per_cu) { return (unsigned)std::min(MAX_GRID, std::max(1, cus * per_cu)); }

bool same_tuning(const Tuning &a, const Tuning &b) { return std::memcmp(&a, &b, sizeof(Tuning)) == 0; }

// ------------------------------------------------------------ workspaces

struct StreamWs {
    std::mutex mu;  // held while a call enqueues work that uses the buffers
    int device = -1;
    Workspace ws;
    RangeWs rws;    // interval buckets
};

// The bucket buffers only (the residues stay).
void free_bucket_ws(RangeWs &rw)
{
    if (rw.counts)
        (void)hipFree(rw.counts);
    if (rw.hits)
        (void)hipFree(rw.hits);
    if (rw.stream)
        (void)hipFree(rw.stream);
    rw.counts = rw.hits = rw.stream = nullptr;
    rw.count_cap = rw.hit_cap = 0;
}

void free_range_ws(RangeWs &rw)
{
    free_bucket_ws(rw);
    if (rw.res)
        (void)hipFree(rw.res);
    rw = RangeWs();
}

// The residue buffer of `rw` (RANGE_MAX_PRIMES entries, allocated once).
int ensure_range_res(RangeWs &rw)
{
    if (rw.res)
        return ISP_OK;
    const hipError_t e = hipMalloc(&rw.res, (size_t)RANGE_MAX_PRIMES * sizeof(SievePrime));
    if (e != hipSuccess) {
        rw.res = nullptr;
        return fail(e);
    }
    return ISP_OK;
}

// Grows `rw` to the given capacities (words); `stream` is synchronised
// before old buffers are freed.
int ensure_range_ws(RangeWs &rw, uint64_t count_cap, uint64_t hit_cap, hipStream_t stream)
{
    if (rw.counts && rw.count_cap >= count_cap && rw.hit_cap >= hit_cap)
        return ISP_OK;
    count_cap = std::max(count_cap, rw.count_cap);
    hit_cap = std::max(hit_cap, rw.hit_cap);
    if (rw.counts) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess)
            return fail(e);
    }
    free_bucket_ws(rw);
    hipError_t e = hipMalloc(&rw.counts, count_cap * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc(&rw.hits, hit_cap * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc(&rw.stream, hit_cap * sizeof(uint32_t));
    if (e != hipSuccess) {
        free_bucket_ws(rw);
        return fail(e);
    }
    rw.count_cap = count_cap;
    rw.hit_cap = hit_cap;
    return ISP_OK;
}


// An upper bound on the bucket hits of one piece of `len` numbers: each odd
// prime p in (BUCKET_SMALL, root] has at most floor(len / 2p) + 1 odd
// multiples in it.  Rosser and Schoenfeld (Illinois J. Math. 6, 1962) give
// sum_{p <= x} 1/p < ln ln x + B + 1/ln^2 x and > ln ln x + B - 1/(2 ln^2 x),
// and pi(x) < 1.25506 x / ln x, for x > 1.
uint64_t bucket_hit_bound(uint64_t len, uint64_t root)
{
    const double x = (double)root, y = (double)BUCKET_SMALL;
    const double lx = std::log(x), ly = std::log(y);
    const double recip = std::log(lx / ly) + 1.0 / (lx * lx) + 1.0 / (2.0 * ly * ly);
    const double pi_x = 1.25506 * x / lx;
    return (uint64_t)(0.5 * (double)len * recip * 1.02 + pi_x * 1.02) + 4096;
}

std::mutex g_ws_mu;
std::map<std::pair<int, void *>, std::unique_ptr<StreamWs>> g_ws;
// The counts of the last call per (device, stream): classify and base-2
// grids and the workspace that holds them.
struct LastCounts {
    const uint32_t *counts = nullptr;
    unsigned grid_c = 0, grid1 = 0;
};
std::map<std::pair<int, void *>, LastCounts> g_last;

void free_ws(Workspace &ws)
{
    if (ws.surv)
        (void)hipFree(ws.surv);
    if (ws.cand)
        (void)hipFree(ws.cand);
    if (ws.prep)
        (void)hipFree(ws.prep);
    if (ws.counts)
        (void)hipFree(ws.counts);
    ws = Workspace();
}

// Grows `ws` to serve calls of up to `cap` elements.  Caller holds the
// workspace mutex; `stream` is synchronised before old buffers are freed.
int ensure_ws(Workspace &ws, size_t cap, hipStream_t stream)
{
    if (ws.surv && ws.cap >= cap)
        return ISP_OK;
    size_t newcap = 1 << 16;
    while (newcap < cap)
        newcap <<= 1;
    if (ws.surv) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess)
            return fail(e);
    }
    free_ws(ws);
    // classify regions are rounded up to 64 elements each; passer regions
    // to one element each
    hipError_t e = hipMalloc(&ws.surv, (newcap + 64 * (size_t)MAX_GRID) * sizeof(Survivor));
    if (e == hipSuccess)
        e = hipMalloc(&ws.cand, (newcap + (size_t)MAX_GRID) * sizeof(Survivor));
    if (e == hipSuccess)
        e = hipMalloc(&ws.prep, (newcap + (size_t)MAX_GRID) * sizeof(MontPrep));
    if (e == hipSuccess)
        e = hipMalloc(&ws.counts, 2 * (size_t)MAX_GRID * sizeof(uint32_t));
    if (e != hipSuccess) {
        free_ws(ws);
        return fail(e);
    }
    ws.cap = newcap;
    return ISP_OK;
}

StreamWs *stream_ws(int dev, void *stream)
{
    std::lock_guard<std::mutex> g(g_ws_mu);
    auto &p = g_ws[{dev, stream}];
    if (!p) {
        p.reset(new StreamWs());
        p->device = dev;
    }
    return p.get();
}

void note_counts(int dev, void *stream, const Workspace &ws, unsigned grid_c, unsigned grid1)
{
    std::lock_guard<std::mutex> g(g_ws_mu);
    g_last[{dev, stream}] = LastCounts{ws.counts, grid_c, grid1};
}

// Arguments of the three kernels for one call.  `len` (0: unknown, as for a
// recorded graph) trims the grids for small inputs, so a short call does not
// pay for thousands of idle workgroups.
void make_args(const DeviceState &ds, const Workspace &ws, const Tuning &t, size_t len,
               ClassifyArgs &ca, MrArgs &ma, unsigned &grid_c, unsigned &grid1)
{
    grid_c = grid_of(ds.cus, t.classify_blocks_per_cu);
    grid1 = grid_of(ds.cus, t.mr_blocks_per_cu);
    if (len) {
        const size_t per_pass = (size_t)t.classify_block * t.classify_ept;
        grid_c = (unsigned)std::min<size_t>(grid_c, (len + per_pass - 1) / per_pass);
        grid1 = (unsigned)std::min<size_t>(grid1, (len + SMALL_CALL_PER_BLOCK - 1) / SMALL_CALL_PER_BLOCK);
    }
    ca = ClassifyArgs();
    ca.wtable = ds.wtable;
    ca.nfilter = t.filter_primes;
    ca.surv = ws.surv;
    ca.counts = ws.counts;
    ma = MrArgs();
    ma.grid_c = grid_c;
    ma.surv = ws.surv;
    ma.counts_c = ws.counts;
    ma.grid1 = grid1;
    ma.cand = ws.cand;
    ma.prep = t.rest_test > 0 ? nullptr : ws.prep;
    ma.counts1 = ws.counts + MAX_GRID;
    // phase 2's list of the candidates that pass base 325: the survivor
    // regions, free once phase 1 has read them (at least 4 words per element)
    ma.keep = reinterpret_cast<uint32_t *>(ws.surv);
}

// Per-stage event timing (isp_profile).  Used by one measuring thread.
std::mutex g_prof_mu;
bool g_prof_on = false;
hipEvent_t g_prof_ev[ISP_NUM_STAGES + 1];
int g_prof_dev = -1;
double g_prof_ms[ISP_NUM_STAGES];
uint64_t g_prof_calls = 0;

// A plain call small enough for the fused kernel (which runs the seven
// Miller-Rabin bases; the Baillie-PSW alternative and the wheel stage keep
// the separate kernels).
bool small_call(size_t len, const Tuning &t)
{
    return len <= SMALL_MAX && t.rest_test <= 0 && t.wheel_log2 == 0;
}

// Enqueues the whole plain path.
int run_plain(const uint64_t *n, uint8_t *out, size_t len, const DeviceState &ds,
              const Workspace &ws, const Tuning &t, hipStream_t s)
{
    std::unique_lock<std::mutex> pg(g_prof_mu);
    const bool prof = g_prof_on && g_prof_dev == ds.device;
    if (!prof)
        pg.unlock();
    ClassifyArgs ca;
    MrArgs ma;
    unsigned grid_c, grid1;
    make_args(ds, ws, t, len, ca, ma, grid_c, grid1);
    ca.n = n;
    ca.out = out;
    ca.total = len;
    ma.total = len;
    hipError_t e = hipSuccess;
    auto mark = [&](int k) {
        if (prof && e == hipSuccess)
            e = hipEventRecord(g_prof_ev[k], s);
    };
    mark(ISP_STAGE_CLASSIFY);
    if (small_call(len, t)) {
        // one fused launch; its time counts as the classify stage
        if (e == hipSuccess)
            e = launch_small(n, out, len, ds.table, t.filter_primes, s);
        for (int k = ISP_STAGE_CLASSIFY + 1; k <= ISP_NUM_STAGES; ++k)
            mark(k);
    } else {
        if (e == hipSuccess)
            e = launch_classify(ca, grid_c, t.classify_block, t.classify_ept, s);
        mark(ISP_STAGE_FILTER2);
        if (e == hipSuccess)
            e = launch_filter2(ws.surv, ws.counts, grid_c, len, nullptr, t.filter_primes,
                               t.sort_survivors, s);
        if (e == hipSuccess && t.wheel_log2)
            e = launch_wheel(ws.surv, ws.counts, grid_c, len, nullptr, t.wheel_log2, s);
        mark(ISP_STAGE_MR_BASE2);
        if (e == hipSuccess)
            e = launch_mr1(ma, t.mr_block, s);
        mark(ISP_STAGE_MR_REST);
        if (e == hipSuccess)
            e = t.rest_test ? launch_lucas(ma, ds.cus, t.mr_blocks_per_cu, grid1, t.mr_block, s)
                            : launch_mr2(ma, ds.cus, t.mr_blocks_per_cu, grid1, t.mr_block,
                                         t.mr_window, s);
        mark(ISP_NUM_STAGES);
    }
    if (prof && e == hipSuccess) {
        e = hipEventSynchronize(g_prof_ev[ISP_NUM_STAGES]);
        for (int k = 0; k < ISP_NUM_STAGES && e == hipSuccess; ++k) {
            float ms = 0;
            e = hipEventElapsedTime(&ms, g_prof_ev[k], g_prof_ev[k + 1]);
            g_prof_ms[k] += ms;
        }
        ++g_prof_calls;
    }
    return e == hipSuccess ? ISP_OK : fail(e);
}

int current_device(int *dev)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess)
        return fail(e);
    if (*dev < 0 || *dev >= MAX_DEVICES)
        return ISP_EINVAL;
    return isp_init(*dev);
}

// -------------------------------------------------------------- batched

// Two pinned descriptor buffers, each with its own recorded graph (whose
// first node copies that buffer to the device): a call writes the buffer
// the call before last used, so it waits only for that replay (normally
// long finished), and back-to-back calls keep the device busy.
struct BatchCtx {
    std::mutex mu;
    int device = -1;
    Workspace ws;
    size_t arr_cap = 0;
    size_t desc_bytes = 0;
    void *d_desc = nullptr;
    void *h_desc[2] = {nullptr, nullptr};  // pinned
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};  // done[k] recorded after the last replay of exec[k]
    unsigned next = 0;                 // buffer of the next call
    Tuning tuned{};
    unsigned grid_c = 0, grid1 = 0;
};

std::mutex g_batch_mu;
std::map<std::pair<int, void *>, std::unique_ptr<BatchCtx>> g_batch;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Descriptor layout: BatchDesc header, then n_ptrs, out_ptrs (num_arrays
// each) and elem_prefix (num_arrays + 1).
size_t desc_size(size_t arrays)
{
    size_t b = align_up(sizeof(BatchDesc), 64);
    b += 3 * arrays * 8 + 8;
    return align_up(b, 64);
}

void free_batch(BatchCtx &c)
{
    for (int k = 0; k < 2; ++k) {
        if (c.exec[k])
            (void)hipGraphExecDestroy(c.exec[k]);
        if (c.h_desc[k])
            (void)hipHostFree(c.h_desc[k]);
        if (c.done[k])
            (void)hipEventDestroy(c.done[k]);
        c.exec[k] = nullptr;
        c.h_desc[k] = nullptr;
        c.done[k] = nullptr;
        c.pending[k] = false;
    }
    if (c.d_desc)
        (void)hipFree(c.d_desc);
    if (c.cap_stream)
        (void)hipStreamDestroy(c.cap_stream);
    free_ws(c.ws);
    c.d_desc = nullptr;
    c.cap_stream = nullptr;
    c.arr_cap = 0;
    c.desc_bytes = 0;
    c.next = 0;
}

// Wait for both buffers' last replays (before anything they use is replaced).
hipError_t drain_batch(BatchCtx &c)
{
    for (int k = 0; k < 2; ++k) {
        if (c.pending[k]) {
            const hipError_t e = hipEventSynchronize(c.done[k]);
            if (e != hipSuccess)
                return e;
            c.pending[k] = false;
        }
    }
    return hipSuccess;
}

// Records exec[k]: the copy of h_desc[k] to the device descriptor, then the
// three kernels over the virtual concatenation of the arrays.
int build_graph_one(BatchCtx &c, const DeviceState &ds, const Tuning &t, int k)
{
    if (c.exec[k]) {
        (void)hipGraphExecDestroy(c.exec[k]);
        c.exec[k] = nullptr;
    }
    ClassifyArgs ca;
    MrArgs ma;
    unsigned grid_c, grid1;
    make_args(ds, c.ws, t, 0, ca, ma, grid_c, grid1);
    const BatchDesc *d = reinterpret_cast<const BatchDesc *>(c.d_desc);
    ca.desc = d;
    ma.total_dev = &d->total;
    hipError_t e = hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return fail(e);
    hipError_t ee = hipMemcpyAsync(c.d_desc, c.h_desc[k], c.desc_bytes, hipMemcpyHostToDevice,
                                   c.cap_stream);
    if (ee == hipSuccess)
        ee = launch_classify(ca, grid_c, t.classify_block, t.classify_ept, c.cap_stream);
    if (ee == hipSuccess)
        ee = launch_filter2(c.ws.surv, c.ws.counts, grid_c, 0, &d->total, t.filter_primes,
                            t.sort_survivors, c.cap_stream);
    if (ee == hipSuccess && t.wheel_log2)
        ee = launch_wheel(c.ws.surv, c.ws.counts, grid_c, 0, &d->total, t.wheel_log2,
                          c.cap_stream);
    if (ee == hipSuccess)
        ee = launch_mr1(ma, t.mr_block, c.cap_stream);
    if (ee == hipSuccess)
        ee = t.rest_test ? launch_lucas(ma, ds.cus, t.mr_blocks_per_cu, MAX_GRID, t.mr_block,
                                        c.cap_stream)
                         : launch_mr2(ma, ds.cus, t.mr_blocks_per_cu, MAX_GRID, t.mr_block,
                                      t.mr_window, c.cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c.cap_stream, &g);
    if (ee != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        return fail(ee);
    }
    if (e != hipSuccess)
        return fail(e);
    e = hipGraphInstantiate(&c.exec[k], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c.exec[k] = nullptr;
        return fail(e);
    }
    c.tuned = t;
    c.grid_c = grid_c;
    c.grid1 = grid1;
    return ISP_OK;
}

int build_graph(BatchCtx &c, const DeviceState &ds, const Tuning &t)
{
    int st = build_graph_one(c, ds, t, 0);
    if (st == ISP_OK)
        st = build_graph_one(c, ds, t, 1);
    return st;
}

}  // namespace

namespace {

// How one piece of an interval call runs (isprime_range_u64), from its
// first number and length.
struct RangePlan {
    uint64_t root;           // floor(sqrt(last number of the piece))
    bool bucket;             // bucket mode: every segment complete, no Miller-Rabin
    unsigned grid;           // sieve workgroups (segments)
    unsigned groups;         // bucket mode: groups of the bucket passes
    uint64_t count_words;    // bucket mode: bucket counts and scan sums
    uint64_t hit_words;      // bucket mode: bound on the bucket hits
    bool complete;           // the sieve decides every number (no Miller-Rabin)
    int partial_log2;        // otherwise the primes below 2^this, then Miller-Rabin
    int complete_log2;       // segments whose root is below 2^this are complete
};

RangePlan plan_range_piece(uint64_t first, uint64_t piece)
{
    RangePlan p{};
    p.root = isqrt_u64(first + (piece - 1));
    // Bucket mode (every segment complete, no Miller-Rabin) once the
    // per-segment loop over the primes up to the root costs more than the
    // bucket passes (measured: roots above 2^23), and while the passes'
    // cost is below Miller-Rabin's on the piece's survivors.  Measured on
    // 2^28-number pieces: the bucket mode takes about 2.5 ps per number
    // plus 11 ps per prime up to the root, Miller-Rabin about 12 ps per
    // number, so buckets win while pi(root) < 0.85 len (pi(root) is taken
    // as root / ln root, a few percent low; a choice of mode only, which
    // changes no output bit).
    const double pi_root = (double)p.root / std::log((double)p.root + 2.0);
    p.bucket = p.root > ((uint64_t)1 << BUCKET_FROM_LOG2) && pi_root < 0.8 * (double)piece;
    const unsigned full = (unsigned)((piece + RANGE_SEG - 1) / RANGE_SEG);
    if (p.bucket) {
        p.grid = full;
        const uint64_t words = (p.root >> 6) + 1 - ((BUCKET_SMALL + 1) >> 6);
        // groups of 1024 threads, two per CU (their LDS allows it): one per
        // 1024 table words, at most MAX_BUCKET_GROUPS, and half of that for
        // roots below 2^26 (fewer words per group do not pay for the longer
        // count array and scans) and for pieces of more than 512 segments
        // (whose count array grows with groups x segments); measured on 2^28
        // and 2^30 numbers at 2^48 .. 2^64
        const uint64_t gmax = p.grid > 512 || words < ((uint64_t)1 << 20) ? MAX_BUCKET_GROUPS / 2
                                                                          : MAX_BUCKET_GROUPS;
        p.groups = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(gmax, words / 1024));
        p.hit_words = bucket_hit_bound(piece, p.root);
        p.count_words = bucket_layout(p.grid, p.groups, p.hit_words, piece, p.root).count_words;
        p.complete = true;
        return p;
    }
    // every segment of a piece whose square root is below 2^25 is decided
    // by the sieve alone (no survivors, no Miller-Rabin), unless the piece
    // is short and the primes up to its root many: then its few segments
    // would each wait on a pass over all of them, and the primes below 2^18
    // with Miller-Rabin on the 4.5% that survive cost less.  Measured: a
    // segment pass costs about 0.45 ns per prime, Miller-Rabin on the
    // survivors about 0.011 ns per number of the piece, over 0.03 ms more
    // of fixed cost.
    const unsigned full_small = (unsigned)((piece + RANGE_SEG_SMALL - 1) / RANGE_SEG_SMALL);
    const bool short_piece = full_small < PARTIAL_FULL_GRID;
    const bool force_partial = short_piece && p.root >= ((uint64_t)1 << PARTIAL_SHORT_LOG2) &&
                               pi_root > (double)piece / 40.0 + 65536.0;
    p.complete_log2 = force_partial ? PARTIAL_SHORT_LOG2 : RANGE_PRIME_LOG2;
    p.complete = p.root < ((uint64_t)1 << p.complete_log2);
    // a short piece has few segments, each visiting all the primes below
    // the bound one after another: a lower bound there costs more
    // Miller-Rabin on the extra survivors but far less sieve latency
    p.partial_log2 = short_piece ? PARTIAL_SHORT_LOG2 : RANGE_PARTIAL_LOG2;
    // segments of RANGE_SEG numbers where every segment visits primes past
    // 2^20 and the piece fills at least PARTIAL_FULL_GRID of them (each
    // prime's first multiple is then found once per 2^20 numbers; measured
    // on 2^28 numbers at 2^44, complete up to 2^22: 0.360 -> 0.273 ms), else
    // of RANGE_SEG_SMALL (twice the workgroups: at 2^34, primes up to 2^17,
    // 0.099 ms against 0.118 ms).  A short piece in Miller-Rabin mode is cut
    // into up to PARTIAL_FULL_GRID shorter segments (at least RANGE_MIN_CHUNK
    // numbers each): its workgroups then share the crossings, while each
    // still visits the few primes below the short-piece bound (in complete
    // mode each segment visits every prime up to the root, so more segments
    // would only repeat that work)
    const uint64_t sieve_bound = p.complete ? p.root : ((uint64_t)1 << p.partial_log2);
    if (sieve_bound > ((uint64_t)1 << 20) && full >= PARTIAL_FULL_GRID)
        p.grid = full;
    else
        p.grid = p.complete || !short_piece
                     ? full_small
                     : (unsigned)std::max<uint64_t>(
                           full_small, std::min<uint64_t>(PARTIAL_FULL_GRID, piece / RANGE_MIN_CHUNK));
    return p;
}

}  // namespace

namespace isp {

// The workspace of `stream` on `dev`, grown now to serve plain calls of up
// to `len` elements (the request server reserves its slots' workspaces at
// creation, so serving allocates nothing).  Returns its size in bytes.
int reserve_stream_ws(int dev, void *stream, size_t len, uint64_t *bytes)
{
    StreamWs *sw = stream_ws(dev, stream);
    std::lock_guard<std::mutex> g(sw->mu);
    const int st = ensure_ws(sw->ws, std::min(len, PLAIN_PIECE), (hipStream_t)stream);
    if (st == ISP_OK && bytes)
        *bytes = isp_workspace_bytes(sw->ws.cap);
    return st;
}

// Frees the workspaces kept for `stream` on `dev` (the stream is about to be
// destroyed; nothing may be in flight on it).
void release_stream_ws(int dev, void *stream)
{
    std::unique_ptr<StreamWs> sw;
    {
        std::lock_guard<std::mutex> g(g_ws_mu);
        auto it = g_ws.find({dev, stream});
        if (it != g_ws.end()) {
            sw = std::move(it->second);
            g_ws.erase(it);
        }
        g_last.erase({dev, stream});
    }
    if (sw) {
        std::lock_guard<std::mutex> g(sw->mu);
        free_ws(sw->ws);
        free_range_ws(sw->rws);
    }
}

}  // namespace isp

// =================================================================== C ABI

extern "C" {

int isp_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES)
        return ISP_EINVAL;
    std::lock_guard<std::mutex> g(g_init_mu);
    DeviceState &ds = g_dev[device];
    if (ds.table)
        return ISP_OK;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess)
        return fail(e);
    if (device >= ndev)
        return ISP_EINVAL;
    int prev = 0;
    e = hipGetDevice(&prev);
    if (e != hipSuccess)
        return fail(e);
    e = hipSetDevice(device);
    if (e != hipSuccess)
        return fail(e);
    hipDeviceProp_t prop;
    hipStream_t s = nullptr;
    e = hipGetDeviceProperties(&prop, device);
    DeviceState st;
    st.device = device;
    st.cus = prop.multiProcessorCount;
    if (e == hipSuccess)
        e = hipMalloc(&st.table, TABLE_WORDS * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc(&st.wtable, WHEEL_WORDS * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc(&st.base_primes, MAX_BASE_PRIMES * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc(&st.base_count, sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = launch_base_primes(st, s);
    if (e == hipSuccess)
        e = launch_sieve(st, s);
    if (e == hipSuccess)
        e = launch_wheel_table(st, s);
    uint32_t count = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&count, st.base_count, sizeof(count), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (s)
        (void)hipStreamDestroy(s);
    if (e == hipSuccess && count != 6541)
        e = hipErrorUnknown;  // the base-prime sieve must find all 6541 odd primes < 2^16
    if (e != hipSuccess) {
        (void)hipFree(st.table);
        (void)hipFree(st.wtable);
        (void)hipFree(st.base_primes);
        (void)hipFree(st.base_count);
        (void)hipSetDevice(prev);
        return fail(e);
    }
    st.num_base_primes = (int)count;
    // this device's copy of the allocation-free entry point's scratch array
    // (the device is current here)
    void *sp = nullptr;
    e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !sp) {
        (void)hipFree(st.table);
        (void)hipFree(st.wtable);
        (void)hipFree(st.base_primes);
        (void)hipFree(st.base_count);
        (void)hipSetDevice(prev);
        return fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
    }
    st.scratch = static_cast<unsigned char *>(sp);
    ds = st;
    (void)hipSetDevice(prev);
    return ISP_OK;
}

void isp_shutdown(void)
{
    {
        std::lock_guard<std::mutex> g(g_batch_mu);
        for (auto &kv : g_batch) {
            std::lock_guard<std::mutex> gg(kv.second->mu);
            (void)drain_batch(*kv.second);
            free_batch(*kv.second);
        }
        g_batch.clear();
    }
    {
        std::lock_guard<std::mutex> g(g_ws_mu);
        for (auto &kv : g_ws) {
            std::lock_guard<std::mutex> gg(kv.second->mu);
            free_ws(kv.second->ws);
            free_range_ws(kv.second->rws);
        }
        g_ws.clear();
        g_last.clear();
    }
    std::lock_guard<std::mutex> g(g_init_mu);
    for (auto &ds : g_dev) {
        if (!ds.table)
            continue;
        (void)hipFree(ds.table);
        (void)hipFree(ds.wtable);
        (void)hipFree(ds.base_primes);
        (void)hipFree(ds.base_count);
        if (ds.range_primes)
            (void)hipFree(ds.range_primes);
        if (ds.range_inv)
            (void)hipFree(ds.range_inv);
        if (ds.range_count)
            (void)hipFree(ds.range_count);
        if (ds.chunk_primes)
            (void)hipFree(ds.chunk_primes);
        ds = DeviceState();
    }
}

int isprime_u64(const uint64_t *n, uint8_t *out, size_t len, void *stream)
{
    if (len == 0)
        return ISP_OK;
    if (!n || !out)
        return ISP_EINVAL;
    int dev = 0;
    int st = current_device(&dev);
    if (st != ISP_OK)
        return st;
    const Tuning t = tuning_snapshot();
    StreamWs *sw = stream_ws(dev, stream);
    std::lock_guard<std::mutex> g(sw->mu);
    hipStream_t s = (hipStream_t)stream;
    st = ensure_ws(sw->ws, std::min(len, PLAIN_PIECE), s);
    if (st != ISP_OK)
        return st;
    for (size_t off = 0; off < len && st == ISP_OK; off += PLAIN_PIECE)
        st = run_plain(n + off, out + off, std::min(PLAIN_PIECE, len - off), g_dev[dev], sw->ws,
                       t, s);
    {
        ClassifyArgs ca;
        MrArgs ma;
        unsigned gc, g1;
        make_args(g_dev[dev], sw->ws, t, std::min(len, PLAIN_PIECE), ca, ma, gc, g1);
        // (the fused kernel keeps no counters: both read as 0)
        if (small_call(len, t))
            gc = g1 = 0;
        note_counts(dev, stream, sw->ws, gc, g1);
    }
    return st;
}

int isprime_u64_noalloc(const uint64_t *n, uint8_t *out, size_t len, void *stream)
{
    if (len == 0)
        return ISP_OK;
    if (!n || !out)
        return ISP_EINVAL;
    if (len > NOALLOC_MAX)
        return ISP_ERANGE;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(e);
    if (dev < 0 || dev >= MAX_DEVICES)
        return ISP_EINVAL;
    DeviceState ds;
    {
        std::lock_guard<std::mutex> g(g_init_mu);
        ds = g_dev[dev];
    }
    if (!ds.table || !ds.scratch)
        return ISP_ENOINIT;  // isp_init allocates; this entry point must not
    Workspace ws;
    ws.surv = reinterpret_cast<Survivor *>(ds.scratch + NOALLOC_SURV_OFF);
    ws.cand = reinterpret_cast<Survivor *>(ds.scratch + NOALLOC_CAND_OFF);
    ws.prep = reinterpret_cast<MontPrep *>(ds.scratch + NOALLOC_PREP_OFF);
    ws.counts = reinterpret_cast<uint32_t *>(ds.scratch + NOALLOC_COUNTS_OFF);
    ws.cap = NOALLOC_MAX;
    // nothing in the workspace needs to start at zero: every count is
    // written by its producer kernel before its consumer reads it
    return run_plain(n, out, len, ds, ws, tuning_snapshot(), (hipStream_t)stream);
}

size_t isp_noalloc_max_len(void) { return NOALLOC_MAX; }


// Builds the interval sieve's prime list for `dev` on first use.
static int ensure_range_primes(int dev)
{
    std::lock_guard<std::mutex> g(g_init_mu);
    DeviceState &ds = g_dev[dev];
    if (ds.num_range_primes)
        return ISP_OK;
    hipStream_t s = nullptr;
    hipError_t e = hipMalloc(&ds.range_primes, RANGE_MAX_PRIMES * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc(&ds.range_inv, RANGE_MAX_PRIMES * sizeof(uint64_t));
    if (e == hipSuccess)
        e = hipMalloc(&ds.range_count, (RANGE_LIST_GROUPS + 1) * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMalloc(&ds.chunk_primes, chunk_primes_words() * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = launch_range_primes(ds, s);
    if (e == hipSuccess)
        e = launch_chunk_primes(ds, s);
    uint32_t count = 0, chunk_total = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&count, ds.range_count + RANGE_LIST_GROUPS, sizeof(count),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&chunk_total, ds.chunk_primes + TABLE_CHUNKS, sizeof(chunk_total),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (s)
        (void)hipStreamDestroy(s);
    // 2063688 odd primes below 2^25, 203280220 below 2^32
    if (e == hipSuccess && (count != RANGE_MAX_PRIMES - 1 || chunk_total != TABLE_ODD_PRIMES))
        e = hipErrorUnknown;
    if (e != hipSuccess) {
        (void)hipFree(ds.range_primes);
        (void)hipFree(ds.range_inv);
        (void)hipFree(ds.range_count);
        (void)hipFree(ds.chunk_primes);
        ds.range_primes = nullptr;
        ds.range_inv = nullptr;
        ds.range_count = nullptr;
        ds.chunk_primes = nullptr;
        return fail(e);
    }
    ds.num_range_primes = (int)count;
    return ISP_OK;
}

int isprime_range_u64(uint64_t lo, uint8_t *out, size_t len, void *stream)
{
    if (len == 0)
        return ISP_OK;
    if (!out || lo + (uint64_t)(len - 1) < lo)
        return ISP_EINVAL;  // NULL, or the interval passes 2^64 - 1
    int dev = 0;
    int st = current_device(&dev);
    if (st != ISP_OK)
        return st;
    st = ensure_range_primes(dev);
    if (st != ISP_OK)
        return st;
    const DeviceState &ds = g_dev[dev];
    const Tuning t = tuning_snapshot();
    hipStream_t s = (hipStream_t)stream;
    // below 2^32: the table
    const uint64_t below = lo < TABLE_BOUND ? std::min<uint64_t>(len, TABLE_BOUND - lo) : 0;
    if (below) {
        hipError_t e = launch_range_table(lo, out, below, ds, s);
        if (e != hipSuccess)
            return fail(e);
    }
    if (below == len)
        return ISP_OK;
    StreamWs *sw = stream_ws(dev, stream);
    std::lock_guard<std::mutex> g(sw->mu);
    // pieces decided by the sieve alone need no survivor workspace: it is
    // allocated (or grown) only for a piece that goes to Miller-Rabin
    const Workspace none;
    st = ensure_range_res(sw->rws);
    for (uint64_t off = below; off < len && st == ISP_OK; off += RANGE_PIECE) {
        const uint64_t piece = std::min<uint64_t>(RANGE_PIECE, len - off);
        const RangePlan pl = plan_range_piece(lo + off, piece);
        // the piece's residues modulo every prime its segments sieve by:
        // those up to the root, the primes up to BUCKET_SMALL in bucket mode,
        // and for Miller-Rabin pieces those below 2^partial_log2 or, in a
        // segment whose root is below 2^complete_log2, up to that root
        const uint64_t bound =
            pl.bucket ? std::min<uint64_t>(pl.root, BUCKET_SMALL)
                      : std::max<uint64_t>(std::min<uint64_t>(pl.root, ((uint64_t)1 << pl.complete_log2) - 1),
                                           ((uint64_t)1 << pl.partial_log2) - 1);
        hipError_t e = launch_range_residues(lo + off, bound, ds, sw->rws.res, s);
        if (e != hipSuccess) {
            st = fail(e);
            break;
        }
        if (pl.bucket) {
            st = ensure_range_ws(sw->rws, pl.count_words, pl.hit_words, s);
            if (st != ISP_OK)
                break;
            e = launch_range_buckets(lo + off, piece, pl.root, pl.groups, pl.hit_words, ds,
                                     sw->rws, s);
            if (e == hipSuccess)
                e = launch_range_sieve(lo + off, out + off, piece, pl.grid, RANGE_SEG, pl.groups,
                                       ds, none, sw->rws, s);
        } else {
            if (!pl.complete) {
                st = ensure_ws(sw->ws, piece, s);
                if (st != ISP_OK)
                    break;
            }
            const Workspace &ws = pl.complete ? none : sw->ws;
            ClassifyArgs ca;
            MrArgs ma;
            unsigned grid_c, grid1;
            make_args(ds, ws, t, piece, ca, ma, grid_c, grid1);
            ma.total = piece;
            ma.grid_c = pl.grid;
            e = launch_range_sieve(lo + off, out + off, piece, pl.grid,
                                   classify_chunk(piece, pl.grid), 0, ds, ws, sw->rws, s,
                                   pl.partial_log2, pl.complete_log2);
            if (e == hipSuccess && !pl.complete)
                e = launch_mr1(ma, t.mr_block, s);
            if (e == hipSuccess && !pl.complete)
                e = t.rest_test ? launch_lucas(ma, ds.cus, t.mr_blocks_per_cu, grid1, t.mr_block, s)
                                : launch_mr2(ma, ds.cus, t.mr_blocks_per_cu, grid1, t.mr_block,
                                             t.mr_window, s);
        }
        if (e != hipSuccess)
            st = fail(e);
    }
    return st;
}

int isprime_u64_batched(const uint64_t *const *n_ptrs, uint8_t *const *out_ptrs,
                        const uint64_t *lens, size_t num_arrays, void *stream)
{
    if (num_arrays == 0)
        return ISP_OK;
    if (!n_ptrs || !out_ptrs || !lens)
        return ISP_EINVAL;
    if (num_arrays > 0x7fffffffu)
        return ISP_EINVAL;
    const Tuning t = tuning_snapshot();
    uint64_t total = 0;
    for (size_t a = 0; a < num_arrays; ++a) {
        if (lens[a] && (!n_ptrs[a] || !out_ptrs[a]))
            return ISP_EINVAL;
        if (lens[a] > BATCH_MAX_ELEMS - total)  // also keeps the sum from wrapping
            return ISP_EINVAL;
        total += lens[a];
    }
    if (total == 0)
        return ISP_OK;
    int dev = 0;
    int st = current_device(&dev);
    if (st != ISP_OK)
        return st;
    const DeviceState &ds = g_dev[dev];
    hipStream_t s = (hipStream_t)stream;

    BatchCtx *c;
    {
        std::lock_guard<std::mutex> g(g_batch_mu);
        auto &p = g_batch[{dev, stream}];
        if (!p) {
            p.reset(new BatchCtx());
            p->device = dev;
        }
        c = p.get();
    }
    std::lock_guard<std::mutex> g(c->mu);
    hipError_t e;
    // The descriptor buffers and the workspace are baked into the graph, so
    // growing either re-records it.
    bool rebuild = !c->exec[0] || !c->exec[1] || !same_tuning(c->tuned, t);
    if (rebuild || num_arrays > c->arr_cap || !c->ws.surv || c->ws.cap < total) {
        // (re-recording or reallocating: nothing of the old replays may
        // still run)
        e = drain_batch(*c);
        if (e != hipSuccess)
            return fail(e);
    }
    if (num_arrays > c->arr_cap || !c->ws.surv || c->ws.cap < total) {
        if (num_arrays > c->arr_cap || !c->d_desc) {
            size_t arr_cap = std::max<size_t>(c->arr_cap, 1024);
            while (arr_cap < num_arrays)
                arr_cap <<= 1;
            if (c->d_desc)
                (void)hipFree(c->d_desc);
            for (int k = 0; k < 2; ++k) {
                if (c->h_desc[k])
                    (void)hipHostFree(c->h_desc[k]);
                c->h_desc[k] = nullptr;
            }
            c->d_desc = nullptr;
            c->desc_bytes = desc_size(arr_cap);
            e = hipMalloc(&c->d_desc, c->desc_bytes);
            for (int k = 0; k < 2 && e == hipSuccess; ++k)
                e = hipHostMalloc(&c->h_desc[k], c->desc_bytes, hipHostMallocDefault);
            if (e != hipSuccess) {
                free_batch(*c);
                return fail(e);
            }
            c->arr_cap = arr_cap;
        }
        st = ensure_ws(c->ws, total, s);
        if (st != ISP_OK) {
            free_batch(*c);
            return st;
        }
        rebuild = true;
    }
    if (!c->cap_stream) {
        e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
        for (int k = 0; k < 2 && e == hipSuccess; ++k)
            e = hipEventCreateWithFlags(&c->done[k], hipEventDisableTiming);
        if (e != hipSuccess)
            return fail(e);
    }
    // The replay that last used this buffer copies from it: wait for it
    // before rewriting (normally it finished long ago).
    const unsigned k = c->next;
    if (c->pending[k]) {
        e = hipEventSynchronize(c->done[k]);
        if (e != hipSuccess)
            return fail(e);
        c->pending[k] = false;
    }
    char *h = static_cast<char *>(c->h_desc[k]);
    char *d = static_cast<char *>(c->d_desc);
    const size_t off_n = align_up(sizeof(BatchDesc), 64);
    const size_t off_o = off_n + c->arr_cap * 8;
    const size_t off_p = off_o + c->arr_cap * 8;
    BatchDesc hd;
    std::memset(&hd, 0, sizeof(hd));
    hd.num_arrays = (uint32_t)num_arrays;
    hd.total = total;
    hd.n_ptrs = reinterpret_cast<const uint64_t *const *>(d + off_n);
    hd.out_ptrs = reinterpret_cast<uint8_t *const *>(d + off_o);
    hd.elem_prefix = reinterpret_cast<const uint64_t *>(d + off_p);
    std::memcpy(h, &hd, sizeof(hd));
    std::memcpy(h + off_n, n_ptrs, num_arrays * 8);
    std::memcpy(h + off_o, out_ptrs, num_arrays * 8);
    uint64_t *pre = reinterpret_cast<uint64_t *>(h + off_p);
    uint64_t acc = 0;
    for (size_t a = 0; a < num_arrays; ++a) {
        pre[a] = acc;
        acc += lens[a];
    }
    pre[num_arrays] = acc;
    if (rebuild) {
        st = build_graph(*c, ds, t);
        if (st != ISP_OK)
            return st;
    }
    e = hipGraphLaunch(c->exec[k], s);
    if (e == hipSuccess)
        e = hipEventRecord(c->done[k], s);
    if (e != hipSuccess)
        return fail(e);
    c->pending[k] = true;
    c->next = k ^ 1u;
    note_counts(dev, stream, c->ws, c->grid_c, c->grid1);
    return ISP_OK;
}

int isprime_u64_batched_offsets(const uint64_t *n, uint8_t *out, const uint64_t *offsets,
                                size_t num_arrays, void *stream)
{
    if (num_arrays == 0)
        return ISP_OK;
    if (!offsets || num_arrays > 0x7fffffffu)
        return ISP_EINVAL;
    int dev = 0;
    int st = current_device(&dev);
    if (st != ISP_OK)
        return st;
    // the offsets, wherever they live: device memory is read after the
    // stream's earlier work (which may have written them)
    std::vector<uint64_t> off(num_arrays + 1);
    hipPointerAttribute_t attr;
    const bool on_device = hipPointerGetAttributes(&attr, offsets) == hipSuccess &&
                           attr.type == hipMemoryTypeDevice;
    (void)hipGetLastError();  // a plain host pointer is not an error
    if (on_device) {
        hipError_t e = hipMemcpyAsync(off.data(), offsets, off.size() * sizeof(uint64_t),
                                      hipMemcpyDeviceToHost, (hipStream_t)stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess)
            return fail(e);
    } else {
        std::memcpy(off.data(), offsets, off.size() * sizeof(uint64_t));
    }
    for (size_t a = 0; a < num_arrays; ++a)
        if (off[a + 1] < off[a])
            return ISP_EINVAL;  // arrays must follow one another
    const uint64_t len = off[num_arrays] - off[0];
    if (len == 0)
        return ISP_OK;
    if (!n || !out)
        return ISP_EINVAL;
    // the arrays tile [off[0], off[num]) of the buffers and every element is
    // decided alone, so one launch sequence over that range decides them all
    return isprime_u64(n + off[0], out + off[0], len, stream);
}

size_t isp_workspace_bytes(size_t len)
{
    size_t cap = 1 << 16;
    while (cap < std::min(len, PLAIN_PIECE))
        cap <<= 1;
    return (2 * cap + 65 * (size_t)MAX_GRID) * sizeof(Survivor) +
           (cap + (size_t)MAX_GRID) * sizeof(MontPrep) + 2 * MAX_GRID * sizeof(uint32_t);
}

size_t isp_range_workspace_bytes(uint64_t lo, size_t len)
{
    if (len == 0 || lo + (uint64_t)(len - 1) < lo)
        return 0;
    const uint64_t below = lo < TABLE_BOUND ? std::min<uint64_t>(len, TABLE_BOUND - lo) : 0;
    size_t mr = 0, buckets = 0;
    for (uint64_t off = below; off < len; off += RANGE_PIECE) {
        const uint64_t piece = std::min<uint64_t>(RANGE_PIECE, len - off);
        const RangePlan p = plan_range_piece(lo + off, piece);
        if (p.bucket)
            buckets = std::max<size_t>(buckets, (p.count_words + 2 * p.hit_words) * sizeof(uint32_t));
        else if (!p.complete)
            mr = std::max(mr, isp_workspace_bytes(piece));
    }
    // and the sieving primes with their residues, for any piece above 2^32
    const size_t res = below < len ? (size_t)RANGE_MAX_PRIMES * sizeof(SievePrime) : 0;
    return mr + buckets + res;
}

int isp_last_device_error(void) { return g_last_err.load(); }

const char *isp_strerror(int status)
{
    switch (status) {
    case ISP_OK:
        return "ok";
    case ISP_EINVAL:
        return "invalid argument";
    case ISP_ENOMEM:
        return "out of memory";
    case ISP_EDEVICE:
        return "device error";
    case ISP_EBUSY:
        return "busy: request not admissible now";
    case ISP_ETIMEDOUT:
        return "timed out";
    case ISP_ENOENT:
        return "unknown ticket";
    case ISP_ERANGE:
        return "length above the allocation-free entry point's maximum (isp_noalloc_max_len)";
    case ISP_ENOINIT:
        return "device not initialised: call isp_init first";
    default:
        return "unknown status";
    }
}

int isp_get_config(isp_config *cfg)
{
    if (!cfg)
        return ISP_EINVAL;
    std::lock_guard<std::mutex> g(g_cfg_mu);
    *cfg = g_cfg;
    return ISP_OK;
}

int isp_set_config(const isp_config *cfg)
{
    if (!cfg)
        return ISP_EINVAL;
    isp_config c = *cfg;
    const isp_config &d = DEFAULT_CONFIG;
    if (!c.classify_block) c.classify_block = d.classify_block;
    if (!c.classify_ept) c.classify_ept = d.classify_ept;
    if (!c.classify_blocks_per_cu) c.classify_blocks_per_cu = d.classify_blocks_per_cu;
    if (!c.filter_primes) c.filter_primes = d.filter_primes;
    if (!c.sort_survivors) c.sort_survivors = d.sort_survivors;
    if (!c.mr_block) c.mr_block = d.mr_block;
    if (!c.mr_blocks_per_cu) c.mr_blocks_per_cu = d.mr_blocks_per_cu;
    if (!c.mr_window) c.mr_window = d.mr_window;
    if (!c.rest_test) c.rest_test = -1;
    if (!c.wheel_log2) c.wheel_log2 = -1;
    if (!valid_config(c))
        return ISP_EINVAL;
    std::lock_guard<std::mutex> g(g_cfg_mu);
    g_cfg = c;
    return ISP_OK;
}

int isp_montmul_u64(const uint64_t *a, const uint64_t *b, const uint64_t *n, uint64_t *out,
                    size_t len, void *stream)
{
    if (len == 0)
        return ISP_OK;
    if (!a || !b || !n || !out)
        return ISP_EINVAL;
    hipError_t e = launch_montmul_test(a, b, n, out, len, (hipStream_t)stream);
    return e == hipSuccess ? ISP_OK : fail(e);
}

int isp_profile(int enable)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(e);
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (enable && g_prof_dev != dev) {
        if (g_prof_dev >= 0)
            for (auto &ev : g_prof_ev)
                (void)hipEventDestroy(ev);
        g_prof_dev = -1;
        for (auto &ev : g_prof_ev) {
            e = hipEventCreate(&ev);
            if (e != hipSuccess)
                return fail(e);
        }
        g_prof_dev = dev;
    }
    g_prof_on = enable != 0;
    for (double &m : g_prof_ms)
        m = 0;
    g_prof_calls = 0;
    return ISP_OK;
}

int isp_profile_read(double *ms, uint64_t *calls)
{
    if (!ms || !calls)
        return ISP_EINVAL;
    std::lock_guard<std::mutex> g(g_prof_mu);
    for (int k = 0; k < ISP_NUM_STAGES; ++k)
        ms[k] = g_prof_ms[k];
    *calls = g_prof_calls;
    return ISP_OK;
}

int isp_table_rebuild(int device, double *ms, double *wheel_ms)
{
    if (!ms || !wheel_ms)
        return ISP_EINVAL;
    int st = isp_init(device);
    if (st != ISP_OK)
        return st;
    std::lock_guard<std::mutex> g(g_init_mu);
    DeviceState &ds = g_dev[device];
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess)
        return fail(e);
    e = hipSetDevice(device);
    if (e != hipSuccess)
        return fail(e);
    hipStream_t s = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
        e = hipEventCreate(&ev[k]);
    if (e == hipSuccess)
        e = hipEventRecord(ev[0], s);
    if (e == hipSuccess)
        e = launch_base_primes(ds, s);
    if (e == hipSuccess)
        e = launch_sieve(ds, s);
    if (e == hipSuccess)
        e = hipEventRecord(ev[1], s);
    if (e == hipSuccess)
        e = launch_wheel_table(ds, s);
    if (e == hipSuccess)
        e = hipEventRecord(ev[2], s);
    uint32_t count = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&count, ds.base_count, sizeof(count), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    float elapsed = 0, welapsed = 0;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&elapsed, ev[0], ev[1]);
    if (e == hipSuccess)
        e = hipEventElapsedTime(&welapsed, ev[1], ev[2]);
    if (e == hipSuccess && count != 6541)
        e = hipErrorUnknown;
    for (auto &x : ev)
        if (x)
            (void)hipEventDestroy(x);
    if (s)
        (void)hipStreamDestroy(s);
    (void)hipSetDevice(prev);
    if (e != hipSuccess)
        return fail(e);
    *ms = elapsed;
    *wheel_ms = welapsed;
    return ISP_OK;
}

int isp_wheel_table(int device, const uint32_t **table, size_t *words)
{
    if (!table || !words)
        return ISP_EINVAL;
    int st = isp_init(device);
    if (st != ISP_OK)
        return st;
    *table = g_dev[device].wtable;
    *words = WHEEL_WORDS;
    return ISP_OK;
}

int isp_table(int device, const uint32_t **table, size_t *words)
{
    if (!table || !words)
        return ISP_EINVAL;
    int st = isp_init(device);
    if (st != ISP_OK)
        return st;
    *table = g_dev[device].table;
    *words = TABLE_WORDS;
    return ISP_OK;
}

int isp_last_counts(void *stream, uint64_t *survivors, uint64_t *candidates)
{
    if (!survivors || !candidates)
        return ISP_EINVAL;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(e);
    LastCounts lc;
    {
        std::lock_guard<std::mutex> g(g_ws_mu);
        auto it = g_last.find({dev, stream});
        if (it != g_last.end())
            lc = it->second;
    }
    *survivors = *candidates = 0;
    if (!lc.counts)
        return ISP_OK;
    e = hipStreamSynchronize((hipStream_t)stream);
    std::vector<uint32_t> h(2 * (size_t)MAX_GRID);
    if (e == hipSuccess)
        e = hipMemcpy(h.data(), lc.counts, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail(e);
    for (unsigned k = 0; k < lc.grid_c; ++k)
        *survivors += h[k];
    for (unsigned k = 0; k < lc.grid1; ++k)
        *candidates += h[MAX_GRID + k];
    return ISP_OK;
}

}  // extern "C"
