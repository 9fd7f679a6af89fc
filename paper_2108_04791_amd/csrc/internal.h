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
constexpr int MAX_FILTER_PRIMES = 256;
constexpr int NUM_BINS = 32;                         // bit lengths 33..64
constexpr int MR_MAX_BLOCK = 256;                    // launch bound of the Miller-Rabin kernels

// A survivor of the trial filter: the value and where its verdict goes.
struct Survivor {
    uint64_t n;
    uint8_t *out;
};

// Exact divisibility test by a small odd prime p without division
// (Granlund and Montgomery, PLDI 1994): p | n iff n * p^-1 mod 2^64 <= lim,
// with lim = floor((2^64 - 1) / p).
struct FilterPrime {
    uint64_t inv;
    uint64_t lim;
};

// Device-side counters of one call, cleared by a kernel at its start.
struct Counters {
    uint32_t survivors;           // appended by classify
    uint32_t candidates;          // base-2 passers appended by phase 1
    uint32_t work1, work2;        // chunk cursors of the persistent MR kernels
    uint32_t bin_count[NUM_BINS]; // survivors per bit-length bin
    uint32_t bin_cursor[NUM_BINS];
    uint32_t tile_cursor;         // batched classify tile cursor
    uint32_t pad[7];
};

// Device-resident descriptor of a batched call.  The arrays follow the
// header in the same allocation; the pointers address them.
struct BatchDesc {
    uint32_t num_arrays;
    uint32_t num_tiles;
    const uint64_t *const *n_ptrs;  // num_arrays device pointers
    uint8_t *const *out_ptrs;       // num_arrays device pointers
    const uint64_t *lens;           // num_arrays lengths
    const uint32_t *tile_prefix;    // num_arrays + 1 exclusive tile counts
};

// Resolved launch parameters (the public isp_config after defaults).
struct Tuning {
    int classify_block;
    int classify_ept;
    int filter_primes;
    int mr_block;
    int mr_bins;     // 0 or 1: no binning pass
    int mr_window;   // fixed window width of the phase-2 exponentiation
    int mr_blocks_per_cu;
    int batch_tile;  // elements per batched classify tile
};

struct DeviceState {
    int device = -1;
    int cus = 0;
    uint32_t *table = nullptr;       // TABLE_WORDS words
    uint32_t *base_primes = nullptr; // odd primes < 2^16
    uint32_t *base_count = nullptr;  // device word: how many
    FilterPrime *filter = nullptr;   // first MAX_FILTER_PRIMES odd primes
    int num_base_primes = 0;
};

// Per-call workspace (one per stream).
struct Workspace {
    Counters *ctr = nullptr;
    Survivor *surv = nullptr;    // classify output
    Survivor *sorted = nullptr;  // binning output; phase-2 list reuses `surv`
    size_t cap = 0;              // survivors each buffer holds
};

// ---- launchers (each enqueues on `stream` and returns hipError_t) ----
hipError_t launch_base_primes(DeviceState &ds, hipStream_t s);
hipError_t launch_sieve(DeviceState &ds, hipStream_t s);
hipError_t launch_filter_consts(DeviceState &ds, hipStream_t s);

hipError_t launch_reset(Counters *ctr, hipStream_t s);
hipError_t launch_classify(const uint64_t *n, uint8_t *out, uint64_t len, const DeviceState &ds,
                           const Workspace &ws, const Tuning &t, hipStream_t s);
hipError_t launch_classify_batched(const BatchDesc *desc, uint32_t grid, const DeviceState &ds,
                                   const Workspace &ws, const Tuning &t, hipStream_t s);
hipError_t launch_bin(const Workspace &ws, const Tuning &t, int cus, hipStream_t s);
hipError_t launch_mr1(const Workspace &ws, const Tuning &t, int cus, hipStream_t s);
hipError_t launch_mr2(const Workspace &ws, const Tuning &t, int cus, hipStream_t s);

hipError_t launch_montmul_test(const uint64_t *a, const uint64_t *b, const uint64_t *n,
                               uint64_t *out, uint64_t len, hipStream_t s);

}  // namespace isp
