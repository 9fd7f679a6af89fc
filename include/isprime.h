/*
 * isprime.h -- C ABI of the MI355X (gfx950) library for elementwise
 * primality of unsigned 64-bit integers.
 *
 * The operation is the one the paper's isprime_fast computes (section 1: an
 * array in, a logical array of the same size out; section 2: the domain is
 * every 64-bit unsigned integer): out[i] = 1 if n[i] is prime, else 0.
 *
 * How each element is decided (all exact integer arithmetic):
 *   n < 2, even n > 2      -> 0;  n == 2 -> 1
 *   odd n < 2^32           -> one bit of a device-resident sieve table
 *                             (sections 1 and 6.1.3: sieve once, then test
 *                             membership; here an O(1) bit lookup; arrays
 *                             above 65,536 elements read its copy on the
 *                             2*3*5*7 wheel of section 3, where a multiple
 *                             of 3, 5 or 7 needs no read)
 *   odd n >= 2^32          -> exact divisibility by small odd primes
 *                             (section 6.1.2: shrink the array first), then
 *                             the strong probable-prime test of section 2.1
 *                             (Eq. 1-3) over the seven bases of Eq. 4,
 *                             2, 325, 9375, 28178, 450775, 9780504,
 *                             1795265022, with Montgomery arithmetic.
 *
 * Conventions for every entry point:
 *   - Returns ISP_OK (0) or a negative ISP_E* status.  Argument errors are
 *     reported synchronously, before anything is enqueued.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it and is asynchronous: results are valid once the
 *     stream is synchronised.  A device fault behind an ISP_EDEVICE may be
 *     reported by this call, a later call, or the caller's synchronisation;
 *     isp_last_device_error() returns the hipError_t behind the last one.
 *   - Device pointers are owned by the caller; the library owns the sieve
 *     table (256 MiB per device, built once) and its workspaces.
 *   - There are no per-element errors: every uint64 value is in the domain.
 *   - Thread safety: all entry points may be called from several host
 *     threads.  Calls on different streams may overlap on the device (the
 *     table is read-only after isp_init; workspaces are per stream); calls on
 *     one stream are ordered by it.
 */
#ifndef ISPRIME_H
#define ISPRIME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ISP_OK = 0,
    ISP_EINVAL = -1,    /* bad argument (NULL pointer with len > 0, bad config) */
    ISP_ENOMEM = -2,    /* device or pinned host allocation failed */
    ISP_EDEVICE = -3,   /* a HIP call failed; see isp_last_device_error() */
    ISP_EBUSY = -4,     /* server: request not admissible now (non-blocking) */
    ISP_ETIMEDOUT = -5, /* server: wait timed out */
    ISP_ENOENT = -6,    /* server: unknown ticket */
    ISP_ERANGE = -7,    /* isprime_u64_noalloc: len above isp_noalloc_max_len() */
    ISP_ENOINIT = -8    /* isprime_u64_noalloc: isp_init has not run for the device */
};

/* Build the odd-only sieve table for n < 2^32 on `device` (bit i of the
 * table is 1 iff 2i+1 is prime; 2^31 bits = 256 MiB in HBM), together with
 * the base primes and the wheel table derived from it (isp_wheel_table,
 * 122.7 MB).  Blocking; idempotent; thread-safe.
 * Every other entry point calls it lazily for the current device.
 * Paper: section 1 (sieve of Eratosthenes), section 4 (odd numbers only). */
int isp_init(int device);

/* Free every device table, workspace and cached graph.  No call may be in
 * flight on any stream. */
void isp_shutdown(void);

/* out[i] = primality of n[i] for 0 <= i < len.
 *   n    device pointer to len uint64 values (read only; 8-byte aligned)
 *   out  device pointer to len bytes, each written 0 or 1
 *   len  0 returns ISP_OK without launching
 * n == NULL or out == NULL with len > 0 -> ISP_EINVAL.  n and out must not
 * overlap.  Uses the calling thread's current HIP device.  Calls of at most
 * 65,536 elements run as one fused kernel (a team of 8 lanes per element:
 * every lane runs base 2, six of them one other base each); larger calls,
 * and calls with the Baillie-PSW alternative or the wheel stage selected,
 * as the classify / second-filter / base-2 / remaining-bases kernels.  The
 * bytes are the same either way.
 * Paper: section 1 (inputs and outputs of isprime_fast), sections 2-6. */
int isprime_u64(const uint64_t *n, uint8_t *out, size_t len, void *stream);

/* isprime_u64 without any allocation on the call path, for callers that
 * cannot allocate device memory while they call (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, kernels and bytes as isprime_u64; the workspace is one static
 * device array per device, sized for isp_noalloc_max_len() = 1,048,576
 * elements (about 60 MiB, held by each device the library runs on until the
 * process ends).  It calls no hipMalloc, hipFree or other allocating
 * routine:
 *   - isp_init(device) must have run for the current device beforehand
 *     (it builds the table and looks up the array's device address):
 *     otherwise ISP_ENOINIT, with nothing enqueued;
 *   - len > isp_noalloc_max_len() -> ISP_ERANGE, with nothing enqueued;
 *   - len == 0 returns ISP_OK; NULL pointers with len > 0 -> ISP_EINVAL.
 * Every call on a device shares that device's array and no part of it needs
 * clearing between calls (each count is written before it is read).  Calls
 * that overlap on one device -- on different streams, or from several host
 * threads without ordering -- race on the array and may return wrong bytes:
 * order them on one stream.  isp_last_counts does not report these calls. */
int isprime_u64_noalloc(const uint64_t *n, uint8_t *out, size_t len, void *stream);

/* The largest len isprime_u64_noalloc accepts. */
size_t isp_noalloc_max_len(void);

/* Many independent arrays in one call: for each a < num_arrays and
 * i < lens[a], out_ptrs[a][i] = primality of n_ptrs[a][i].
 *   n_ptrs, out_ptrs, lens  HOST arrays of num_arrays entries; the pointers
 *                           they hold are device pointers owned by the caller
 * All arrays are classified by one persistent launch sequence that the
 * library records once as a HIP graph and replays; results are identical to
 * num_arrays separate isprime_u64 calls.  Empty arrays are allowed.  NULL
 * data pointers with a nonzero length -> ISP_EINVAL.  The host arrays may be
 * reused as soon as the call returns.  At most 2^30 elements in total per
 * call (ISP_EINVAL beyond); the workspace kept for the stream grows to the
 * largest call seen. */
int isprime_u64_batched(const uint64_t *const *n_ptrs, uint8_t *const *out_ptrs,
                        const uint64_t *lens, size_t num_arrays, void *stream);

/* Many arrays laid end to end in one buffer: array a is n[offsets[a] ..
 * offsets[a + 1]) with its verdicts at the same places of out.
 *   n, out     device pointers to the concatenated values and verdicts
 *   offsets    num_arrays + 1 non-decreasing element offsets, in device or
 *              host memory (device offsets are read after the stream's
 *              earlier work: the call waits for the stream)
 * Every element of [offsets[0], offsets[num_arrays]) is decided, and nothing
 * else is written.  Decreasing offsets -> ISP_EINVAL; NULL n or out with a
 * nonempty range -> ISP_EINVAL.  Since every element is decided alone, the
 * arrays of one buffer run as a single isprime_u64 launch sequence over the
 * covered range (for arrays in separate buffers, isprime_u64_batched).
 * Results are identical to one isprime_u64 call per array. */
int isprime_u64_batched_offsets(const uint64_t *n, uint8_t *out, const uint64_t *offsets,
                                size_t num_arrays, void *stream);

/* out[i] = primality of lo + i for 0 <= i < len: a contiguous interval,
 * with no input array.  lo + len - 1 must not exceed 2^64 - 1 (ISP_EINVAL).
 *   out  device pointer to len bytes, each written 0 or 1
 * The part below 2^32 is read from the sieve table.  Above it, each
 * workgroup sieves a segment of 2^20 or 2^19 numbers in LDS, in pieces of
 * at most 2^30 numbers.  A piece ending below 2^50 is sieved by every odd prime up
 * to the square root of its end, which decides it.  Above, a piece long
 * enough for the primes up to its square root (pi(sqrt) below 0.8 times its
 * length) also gets every such prime: those above 2^21 are sorted once into
 * per-segment buckets (bucket sieve), and the segments are again complete.
 * Otherwise it is sieved by the odd primes below 2^22 (below 2^18 for a
 * piece of fewer than 256 segments of 2^19, which is then cut into up to 256
 * shorter segments) and the survivors go through the same Miller-Rabin
 * kernels as isprime_u64.  The workspace kept
 * for the stream grows to the largest call seen.  Asynchronous on `stream`.
 * Paper: section 6.1.3 (sieve up to the maximum, then test membership),
 * section 1 (the sieve of Eratosthenes). */
int isprime_range_u64(uint64_t lo, uint8_t *out, size_t len, void *stream);

/* Bytes of device workspace a call over `len` elements may use. */
size_t isp_workspace_bytes(size_t len);

/* Bytes of device workspace isprime_range_u64(lo, ..., len) holds: the
 * survivor workspace of its largest piece that goes to Miller-Rabin and the
 * bucket workspace of its largest bucket-mode piece (pieces decided by the
 * sieve alone need neither), and, when any part lies above 2^32, the
 * piece's table of interval primes with their residues (12 bytes per
 * prime, 24.8 MB); 0 for an empty or
 * invalid interval.  The interval sieve's prime list and chunk prime counts
 * (28.9 MB per device, built on the first interval call) are not counted. */
size_t isp_range_workspace_bytes(uint64_t lo, size_t len);

/* The hipError_t (as int) behind the most recent ISP_EDEVICE. */
int isp_last_device_error(void);

/* A static string for a status code. */
const char *isp_strerror(int status);

/* Launch and algorithm parameters.  None of them changes any output bit;
 * the autotuner picks the launch shapes per workload class.  A zero field
 * means "library default". */
typedef struct {
    int32_t classify_block;         /* threads per classify block: 64..1024, multiple of 64 */
    int32_t classify_ept;           /* elements per classify thread and pass: 1, 2, 4 or 8 */
    int32_t classify_blocks_per_cu; /* classify grid = CUs x this (at most 4096): 1..16 */
    int32_t filter_primes;          /* odd primes in the trial filter: -1 (none), 8, 16, 24, 32, 48 or 64 */
    int32_t sort_survivors;         /* 1: order survivors by bit length; -1: keep input order */
    int32_t mr_block;               /* threads per Miller-Rabin block: 64..1024, multiple of 64 */
    int32_t mr_blocks_per_cu;       /* Miller-Rabin grids = CUs x this (at most 4096): 1..16 */
    int32_t mr_window;              /* fixed window width for bases other than 2: 1..4 */
    int32_t rest_test;              /* after base 2: -1 the six remaining Miller-Rabin bases of
                                       the paper (default); 1 the strong Lucas test with
                                       Selfridge's parameters (Baillie-PSW, the paper's future
                                       work, section 10.1) -- the same verdicts below 2^64 */
    int32_t wheel_log2;             /* -1 (default): off.  33..40: every filter survivor below
                                       2^wheel_log2 is decided by trial division on the
                                       2/3/5/7 wheel up to its square root (the paper's method
                                       for medium integers, section 3, Eq. 5-6) instead of
                                       Miller-Rabin; same verdicts, far more work (it exists to
                                       measure that crossover).  Calls then skip the fused
                                       small-array kernel. */
} isp_config;

/* Read / replace the process-wide configuration (ISP_EINVAL if out of range). */
int isp_get_config(isp_config *cfg);
int isp_set_config(const isp_config *cfg);

/* Diagnostics, used by the tests.
 * isp_montmul_u64: out[i] = a[i] * b[i] mod n[i] computed on the device by
 * converting to Montgomery form, one Montgomery product and converting back.
 * Requires odd n[i] >= 3 with a[i], b[i] < n[i] (otherwise out[i] is
 * unspecified).  Device pointers.  Paper: section 2.3 (ModMultiply). */
int isp_montmul_u64(const uint64_t *a, const uint64_t *b, const uint64_t *n, uint64_t *out,
                    size_t len, void *stream);

/* The device address and word count of the sieve table of `device` (built
 * on first use).  The table is read-only; the pointer stays valid until
 * isp_shutdown. */
int isp_table(int device, const uint32_t **table, size_t *words);

/* The same for the wheel table the array path reads: the bits of the sieve
 * table for the numbers below 2^32 coprime to 210, 48 per block of 210
 * numbers (bit 48 q + k stands for 210 q + r_k, r_k the k-th residue
 * coprime to 210 in increasing order: 1, 11, 13, ..., 209; 0 for numbers
 * at or above 2^32); 30,678,339 words, 122.7 MB.  Paper: section 3 (the
 * 2, 3, 5, 7 wheel, Eq. 5). */
int isp_wheel_table(int device, const uint32_t **table, size_t *words);

/* Counters of the last isprime_u64 / batched call on `stream`, read back
 * synchronously (the stream is synchronised): survivors of the trial filter
 * (both stages; with the wheel stage on, those it left to Miller-Rabin) and
 * base-2 passers sent to the remaining six bases.  A call that ran as
 * the fused kernel keeps no counters: both read 0. */
int isp_last_counts(void *stream, uint64_t *survivors, uint64_t *candidates);

/* Per-stage timing with HIP events, for measurement.  While enabled, every
 * plain isprime_u64 call on the current device records an event before and
 * after each of its kernels on the call's own stream, waits for the last
 * one, and adds the elapsed times to per-stage totals (so calls become
 * synchronous).  isp_profile(1) also resets the totals; isp_profile(0)
 * stops recording.  Meant for one measuring thread.
 * isp_profile_read: ms[ISP_NUM_STAGES] totals and the number of calls. */
enum {
    ISP_STAGE_CLASSIFY = 0, /* classify_kernel: dispatch + table lookup + first trial-filter
                               stage + compaction (a call that runs as the fused
                               small-array kernel: all of its time) */
    ISP_STAGE_FILTER2 = 1,  /* second trial-filter stage (+ the wheel stage when selected) */
    ISP_STAGE_MR_BASE2 = 2, /* Miller-Rabin base 2 over all survivors */
    ISP_STAGE_MR_REST = 3,  /* Miller-Rabin bases 325 .. 1795265022 over base-2 passers */
    ISP_NUM_STAGES = 4
};
int isp_profile(int enable);
int isp_profile_read(double *ms, uint64_t *calls);

/* Rebuild the tables of `device` in place and time the build kernels with
 * HIP events on a private stream: *ms receives the milliseconds of the
 * sieve (base primes, then the segment sieve), *wheel_ms those of the wheel
 * table derived from it.  Synchronises the device first; no call may be in
 * flight on it (the tables are rewritten with the same bits).  For
 * measurement only. */
int isp_table_rebuild(int device, double *ms, double *wheel_ms);

/* ---------------------------------------------------------------- serving
 * A request loop with continuous batching.  Requests carry HOST buffers
 * that the caller owns until isp_wait/isp_poll reports completion.  The
 * server admits a request while the bytes of admitted, unfinished requests
 * (9 per element) stay within `mem_budget_bytes`; the memory it works in
 * (max_inflight slots, each with a device workspace and pinned staging for
 * max_batch_elems elements) is a fixed footprint reserved at creation
 * (isp_server_footprint), so admission never allocates.  Requests that
 * arrive while others run are packed into the next batch as soon as a slot
 * frees up, each slot has its own stream and worker thread, and batches
 * overlap on the device.  Every result equals the plain isprime_u64 result
 * for the same input.  Paper: no section (the paper has no serving loop;
 * the arithmetic is that of isprime_u64, sections 1-6). */
typedef struct isp_server isp_server;

typedef struct {
    int32_t device;            /* HIP device ordinal */
    int32_t max_inflight;      /* batches on the device at once: 1..8 (0 = 8) */
    uint64_t mem_budget_bytes; /* bytes of admitted, unfinished requests, 9 per element
                                  (0 = 1 GiB); the slots' footprint is on top of it */
    uint64_t max_batch_elems;  /* elements per batch, at most 2^28 (0 = 262,144) */
    int32_t max_batch_reqs;    /* request pieces per batch (0 = 1024) */
    int32_t block_on_full;     /* 1: isp_submit waits for budget; 0: ISP_EBUSY */
    int32_t test_mode;         /* 0: the device; 1: a host stand-in that writes n & 1, for
                                  testing the queueing without a GPU (no HIP call at all) */
    int32_t test_fail_every;   /* test mode: every k-th batch fails with ISP_EDEVICE (0: never) */
    int32_t test_delay_us;     /* test mode: time each batch takes */
    int32_t reserved;
} isp_server_config;

int isp_server_create(const isp_server_config *cfg, isp_server **srv);
/* Queue one request; `ticket` receives its id.  len may be 0.  The request
 * holds 9 * len bytes of the budget until it completes; one larger than the
 * whole budget is admitted when nothing else holds any.  Requests are split
 * into pieces of at most max_batch_elems.  A len above (2^64 - 1) / 9 (no
 * such host array) is ISP_EINVAL. */
int isp_submit(isp_server *srv, const uint64_t *host_n, uint8_t *host_out, size_t len,
               uint64_t *ticket);
/* 1 done, 0 pending, <0 error (ISP_ENOENT for an unknown or consumed ticket). */
int isp_poll(isp_server *srv, uint64_t ticket);
/* Block until the request is done (timeout_us < 0: no limit).  Consumes the
 * ticket on success. */
int isp_wait(isp_server *srv, uint64_t ticket, int64_t timeout_us);
/* The memory the server holds for its lifetime, reserved at creation so
 * that serving allocates nothing: *device_bytes, the slots' device
 * workspaces (max_inflight x isp_workspace_bytes(max_batch_elems)), and
 * *pinned_bytes, the slots' pinned, mapped staging buffers (9 bytes per
 * element of max_batch_elems each, which the kernels read and write
 * directly).  Admitted requests count against mem_budget_bytes on top of
 * this fixed footprint. */
int isp_server_footprint(const isp_server *srv, uint64_t *device_bytes, uint64_t *pinned_bytes);

/* Finish every queued request, stop the worker threads, free the server.
 * No other call on this server may be in progress or follow. */
int isp_server_destroy(isp_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* ISPRIME_H */
