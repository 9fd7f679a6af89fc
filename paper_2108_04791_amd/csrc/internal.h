// internal.h -- types and launchers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/isprime.h"

namespace isp {

// Values below TABLE_BOUND are answered by the sieve table; odd values at or
// above it go through the trial filter and Miller-Rabin.
constexpr uint64_t TABLE_BOUND = (uint64_t)1 << 32;
constexpr uint64_t TABLE_WORDS = (uint64_t)1 << 26;  // 2^31 odd numbers / 32
constexpr int MAX_BASE_PRIMES = 6542;                // odd primes below 2^16: 6541
// Prime counts of the table by chunks of 64 words (4096 numbers): entry c is
// the number of odd primes below 4096 c, c = 0 .. TABLE_CHUNKS.
constexpr uint64_t TABLE_CHUNKS = TABLE_WORDS / 64;
constexpr uint32_t TABLE_ODD_PRIMES = 203280220;  // odd primes below 2^32
// The lookup table for n < 2^32 on the 2*3*5*7 wheel: block q of 48 bits
// for the numbers 210 q + r with r coprime to 210 (48 residues in [1, 209]),
// bit 48 q + (index of r); the multiples of 3, 5 and 7 need no bit.
constexpr uint32_t WHEEL_MOD = 210;
constexpr uint32_t WHEEL_RES = 48;
constexpr uint64_t WHEEL_BLOCKS = (TABLE_BOUND + WHEEL_MOD - 1) / WHEEL_MOD;  // 20452226
constexpr uint64_t WHEEL_WORDS = (WHEEL_BLOCKS * WHEEL_RES + 31) / 32;          // 30678339
static_assert(WHEEL_WORDS == 30678339, "122.7 MB wheel table");

// The residues of the wheel: res[k], the k-th residue coprime to 210 in
// increasing order, and pos[r], the k with res[k] = r (0xff when r shares a
// factor with 210).
struct WheelResidues {
    uint8_t res[WHEEL_RES];
    uint8_t pos[WHEEL_MOD];
    constexpr WheelResidues() : res(), pos()
    {
        int k = 0;
        for (uint32_t r = 0; r < WHEEL_MOD; ++r) {
            const bool coprime = r % 2 != 0 && r % 3 != 0 && r % 5 != 0 && r % 7 != 0;
            pos[r] = coprime ? (uint8_t)k : (uint8_t)0xff;
            if (coprime)
                res[k++] = (uint8_t)r;
        }
    }
};
constexpr WheelResidues WHEEL{};
static_assert(WHEEL.res[0] == 1 && WHEEL.res[1] == 11 && WHEEL.res[WHEEL_RES - 1] == 209 &&
                  WHEEL.pos[209] == WHEEL_RES - 1 && WHEEL.pos[3] == 0xff,
              "48 residues coprime to 210");

// floor(sqrt(x)) for every x < 2^64 by the digit-by-digit method (one
// result bit per step, 32 steps at most): integer arithmetic only.
__host__ __device__ inline uint64_t isqrt_u64(uint64_t x)
{
    uint64_t r = 0, bit = (uint64_t)1 << 62;
    while (bit > x)
        bit >>= 2;
    while (bit != 0) {
        if (x >= r + bit) {
            x -= r + bit;
            r = (r >> 1) + bit;
        } else {
            r >>= 1;
        }
        bit >>= 2;
    }
    return r;
}

// floor(n / 210) for odd n < 2^32: floor((n >> 1) / 105), by the
// multiplier ceil(2^38 / 105) = 2617884829, exact for every value below
// 2^31 (its excess 2617884829 * 105 - 2^38 = 101 is below 2^7).
__host__ __device__ inline uint32_t div210_odd(uint32_t n)
{
    return (uint32_t)(((uint64_t)(n >> 1) * 2617884829u) >> 38);
}
constexpr int MAX_FILTER_PRIMES = 128;
constexpr int NUM_BINS = 32;                         // bit lengths 33..64
constexpr int MR_MAX_BLOCK = 1024;                   // launch bound of the Miller-Rabin kernels

// A survivor of the trial filter: the value and where its verdict goes.
struct Survivor {
    uint64_t n;
    uint8_t *out;
};

// Largest grid of the classify and Miller-Rabin kernels: their per-block
// counts are scanned in LDS by the consumer.
constexpr int MAX_GRID = 4096;
// Plain calls of at most SMALL_MAX elements run as one fused kernel (a team
// of SMALL_TEAM lanes per element, SMALL_BLOCK threads per workgroup).
constexpr size_t SMALL_MAX = 65536;
constexpr int SMALL_BLOCK = 256;
constexpr unsigned SMALL_TEAM = 8;

// Numbers per workgroup segment of the interval sieve (LDS holds the odd
// ones: 2^19 bits), and numbers per piece of an interval call.  Pieces
// whose sieving primes stay below 2^20, or that have fewer than 256 such
// segments, use segments of RANGE_SEG_SMALL numbers (more workgroups for
// less work each).
constexpr int RANGE_SEG_LOG2 = 20;
constexpr uint64_t RANGE_SEG = (uint64_t)1 << RANGE_SEG_LOG2;
constexpr uint64_t RANGE_SEG_SMALL = RANGE_SEG / 2;
constexpr uint64_t RANGE_PIECE = (uint64_t)1 << 30;
constexpr int RANGE_PRIME_LOG2 = 25;      // interval sieve primes: the odd primes below 2^25
constexpr int RANGE_PARTIAL_LOG2 = 22;    // primes used where the sieve cannot be complete
constexpr int RANGE_MAX_PRIMES = 2063689; // odd primes below 2^25: 2063688
constexpr int RANGE_LIST_GROUPS = 512;    // workgroups of the list build
// bucket mode (segments of RANGE_SEG numbers): primes above this come as
// precomputed hits (at most one per segment); the primes up to twice the
// segment length are cheaper for the segment kernel, which reads each with
// its constants in one load, than their scattered hits (measured on 2^28
// numbers against 2^20: 2^48 0.377 -> 0.328 ms, 2^50 0.400 -> 0.348, 2^63
// 0.876 -> 0.859; 2^22 was faster at 2^62 but slower at 2^63 and above)
constexpr uint32_t BUCKET_SMALL = (uint32_t)1 << 21;
constexpr int MAX_BUCKET_SEGS = (int)(RANGE_PIECE / RANGE_SEG);  // 1024
constexpr int MAX_BUCKET_GROUPS = 512;
constexpr int BUCKET_FROM_LOG2 = 23;  // bucket mode for pieces whose root exceeds 2^23

// Device-resident descriptor of a batched call.  The arrays follow the
// header in the same allocation; the pointers address them.
struct BatchDesc {
    uint32_t num_arrays;
    uint32_t pad;
    uint64_t total;                 // elements over all arrays
    const uint64_t *const *n_ptrs;  // num_arrays device pointers
    uint8_t *const *out_ptrs;       // num_arrays device pointers
    const uint64_t *elem_prefix;    // num_arrays + 1 exclusive element offsets
};

// Region size of classify block g: its element range, a multiple of 64.
__host__ __device__ inline uint64_t classify_chunk(uint64_t total, uint32_t grid)
{
    return ((total + grid - 1) / grid + 63) / 64 * 64;
}

// Region size of Miller-Rabin base-2 block g for its base-2 passers.
__host__ __device__ inline uint64_t cand_chunk(uint64_t total, uint32_t grid)
{
    return (total + grid - 1) / grid;
}

struct ClassifyArgs {
    const uint64_t *n;      // plain call: the input ...
    uint8_t *out;           // ... and its output
    const BatchDesc *desc;  // batched call (n, out unused); nullptr for plain
    uint64_t total;         // plain call: elements (batched: desc->total)
    const uint32_t *wtable; // the sieve table's bits on the 210-wheel
    int nfilter;            // odd primes in the trial filter: 0, 8, 16, 24, 32, 48 or 64
    Survivor *surv;         // grid regions of classify_chunk() entries
    uint32_t *counts;       // [grid] survivors per region
};

// Montgomery constants of one base-2 passer, computed once by the base-2
// kernel and read by every one of its later tasks.
struct MontPrep {
    uint64_t ninv;  // n^-1 mod 2^64
    uint64_t one;   // 2^64 mod n
    uint64_t r2;    // 2^128 mod n
};

struct MrArgs {
    uint64_t total;              // elements of the call ...
    const uint64_t *total_dev;   // ... or where to read them (batched)
    uint32_t grid_c;             // classify grid
    const Survivor *surv;        // classify regions
    const uint32_t *counts_c;    // [grid_c]
    uint32_t grid1;              // base-2 grid
    Survivor *cand;              // base-2 passer regions of cand_chunk() entries
    MontPrep *prep;              // the passers' constants, indexed like cand (or null:
                                 // not needed by the Lucas test)
    uint32_t *counts1;           // [grid1]
    uint32_t *keep;              // phase 2: one word per candidate (its list of the
                                 // candidates that pass base 325); the survivor regions
};

// Resolved launch parameters (the public isp_config after defaults).
struct Tuning {
    int classify_block;
    int classify_ept;
    int classify_blocks_per_cu;
    int filter_primes;
    int sort_survivors;
    int mr_block;
    int mr_blocks_per_cu;
    int mr_window;
    int rest_test;  // 0: the six remaining Miller-Rabin bases; 1: strong Lucas (Baillie-PSW)
    int wheel_log2; // 0: off; else survivors below 2^wheel_log2 go to the wheel stage
};

// Bounds of the optional wheel stage (wheel.hip): survivors below 2^b, with
// WHEEL_MIN_LOG2 <= b <= WHEEL_MAX_LOG2, are decided by trial division.
constexpr int WHEEL_MIN_LOG2 = 33;
constexpr int WHEEL_MAX_LOG2 = 40;

struct DeviceState {
    int device = -1;
    int cus = 0;
    uint32_t *table = nullptr;       // TABLE_WORDS words
    uint32_t *wtable = nullptr;      // WHEEL_WORDS words, derived from table
    uint32_t *base_primes = nullptr; // odd primes < 2^16
    uint32_t *base_count = nullptr;  // device word: how many
    int num_base_primes = 0;
    // interval sieve: odd primes below 2^25 and floor((2^64-1)/p), built on
    // first use of isprime_range_u64
    uint32_t *range_primes = nullptr;
    uint64_t *range_inv = nullptr;
    uint32_t *range_count = nullptr;  // RANGE_LIST_GROUPS + 1 words
    int num_range_primes = 0;
    // bucket mode: the table's prime counts by chunks (TABLE_CHUNKS + 1
    // words, then the build's scan sums), built with the list
    uint32_t *chunk_primes = nullptr;
    // device address of this device's copy of the allocation-free entry
    // point's static scratch array (hipGetSymbolAddress at isp_init)
    unsigned char *scratch = nullptr;
};

// Per-call workspace (one per stream, or per batched context).
// Interval buckets: per-(segment, group) counts turned offsets, and the hits.
// One sieving prime of an interval piece, with what a segment needs to find
// its first multiple: m = floor(2^32 / p) and the piece's residue
// (lo | 1) mod p, read by the segment kernel in one 12-byte load.
struct SievePrime {
    uint32_t p, m, res;
};

struct RangeWs {
    uint32_t *counts = nullptr;  // count_cap words
    uint32_t *hits = nullptr;    // hit_cap words
    uint32_t *stream = nullptr;  // hit_cap words: the fill pass's output, sorted into hits
    uint64_t count_cap = 0, hit_cap = 0;
    // each piece's sieving primes with their residues (RANGE_MAX_PRIMES entries)
    SievePrime *res = nullptr;
};

struct Workspace {
    Survivor *surv = nullptr;   // classify regions (cap + 64 * MAX_GRID entries)
    Survivor *cand = nullptr;   // base-2 passer regions (cap + MAX_GRID entries)
    MontPrep *prep = nullptr;   // constants of the passers, indexed like cand
    uint32_t *counts = nullptr; // 2 * MAX_GRID
    size_t cap = 0;             // elements per call this workspace serves
};

// ---- launchers (each enqueues on `stream` and returns hipError_t) ----
hipError_t launch_base_primes(DeviceState &ds, hipStream_t s);
hipError_t launch_sieve(DeviceState &ds, hipStream_t s);
hipError_t launch_wheel_table(DeviceState &ds, hipStream_t s);

hipError_t launch_classify(const ClassifyArgs &a, unsigned grid, int block, int ept,
                           hipStream_t s);
hipError_t launch_small(const uint64_t *n, uint8_t *out, size_t len, const uint32_t *table,
                        int nfilter, hipStream_t s);
// total_dev: where to read the element count (batched calls), else total.
// sorted: also order each window of the kept survivors by bit length.
hipError_t launch_filter2(Survivor *surv, uint32_t *counts, unsigned grid, uint64_t total,
                          const uint64_t *total_dev, int nf, int sorted, hipStream_t s);
// Decides the survivors below 2^log2_bound by wheel trial division and
// compacts the others in place (grid: the classify grid).
hipError_t launch_wheel(Survivor *surv, uint32_t *counts, unsigned grid, uint64_t total,
                        const uint64_t *total_dev, int log2_bound, hipStream_t s);
hipError_t launch_mr1(const MrArgs &a, int block, hipStream_t s);
hipError_t launch_mr2(const MrArgs &a, int cus, int per_cu, unsigned max_grid, int block,
                      int window, hipStream_t s);
hipError_t launch_lucas(const MrArgs &a, int cus, int per_cu, unsigned max_grid, int block,
                        hipStream_t s);

hipError_t launch_range_primes(DeviceState &ds, hipStream_t s);
// Builds ds.chunk_primes (chunk_primes_words() words) from the table.
size_t chunk_primes_words();
hipError_t launch_chunk_primes(DeviceState &ds, hipStream_t s);
hipError_t launch_range_table(uint64_t lo, uint8_t *out, uint64_t len, const DeviceState &ds,
                              hipStream_t s);
// Bucket mode's sort tile, per-tile launch size and count words for nseg
// segments, `groups` workgroups, room for hit_cap hits and a piece of len
// numbers up to root (ok false: no tile fits the scan).
struct BucketLayout {
    uint32_t tile = 0, max_tiles = 0;
    uint64_t count_words = 0;
    bool ok = false;
};
BucketLayout bucket_layout(uint32_t nseg, unsigned groups, uint64_t hit_cap, uint64_t len,
                           uint64_t root);
// hit_bound: an upper bound on the piece's hits (at most rw.hit_cap), from
// which the layout is sized.
hipError_t launch_range_buckets(uint64_t lo, uint64_t len, uint64_t root, unsigned groups,
                                uint64_t hit_bound, const DeviceState &ds, const RangeWs &rw,
                                hipStream_t s);
// res[k] = {p, floor(2^32 / p), (lo | 1) mod p} for the k-th interval prime p,
// every prime up to bound (rw.res of the piece's stream, before the sieve
// kernel reads it).
hipError_t launch_range_residues(uint64_t lo, uint64_t bound, const DeviceState &ds,
                                 SievePrime *res, hipStream_t s);
// Without buckets, a segment whose square root is below 2^complete_log2
// (partial_log2 .. RANGE_PRIME_LOG2) is decided by the sieve alone; the others
// are sieved by the primes below 2^partial_log2 (17 .. RANGE_PARTIAL_LOG2)
// and their survivors left to Miller-Rabin.
hipError_t launch_range_sieve(uint64_t lo, uint8_t *out, uint64_t len, unsigned grid,
                              uint64_t chunk, unsigned groups, const DeviceState &ds,
                              const Workspace &ws, const RangeWs &rw, hipStream_t s,
                              int partial_log2 = RANGE_PARTIAL_LOG2,
                              int complete_log2 = RANGE_PRIME_LOG2);

// (api.hip) Grows the workspace of `stream` on `dev` for plain calls of up
// to len elements; *bytes receives its size.  ISP_* status.
int reserve_stream_ws(int dev, void *stream, size_t len, uint64_t *bytes);
// (api.hip) Frees those workspaces (before the stream is destroyed).
void release_stream_ws(int dev, void *stream);

hipError_t launch_montmul_test(const uint64_t *a, const uint64_t *b, const uint64_t *n,
                               uint64_t *out, uint64_t len, hipStream_t s);

}  // namespace isp
