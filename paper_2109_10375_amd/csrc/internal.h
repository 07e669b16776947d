// Internal declarations shared by the host API and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/amber.h"

// Optional per-kernel timing: a pool of HIP event pairs recorded around each
// launch on the launch's own stream (amber_profile_begin / amber_profile_end).
struct Profiler {
    int capacity = 0;
    int used = 0;
    int dropped = 0;
    hipEvent_t* ev = nullptr;     // 2 * capacity events
    const char** names = nullptr;  // kernel name per slot
};

struct amber_plan_s {
    int n = 0;             // grid size per axis
    double box_len = 0.0;  // box side
    int device = -1;
    float2* d_tw = nullptr;  // tw[j] = exp(-2 pi i j / n), j < n, FP64-rounded to FP32
    unsigned* d_sticky = nullptr;  // device status bits accumulated until amber_status (same allocation)
    void* d_scratch = nullptr;     // this device's copy of the static scratch of amber_zre_noalloc
    int col_sched = 0;       // FFT column-pass candidate (0: default)
    int z_sched = 0;         // FFT z-pass candidate (0: default)
    Profiler* prof = nullptr;
};

// Lanes of a concurrent batch: the side streams and their events.
struct amber_executor_s {
    int n_lanes = 1;
    int device = -1;
    hipStream_t side[16] = {};     // lanes 1..n_lanes-1
    hipEvent_t fork = nullptr;     // recorded on the caller's stream
    hipEvent_t join[16] = {};      // recorded on each side lane
};

inline int prof_start(const amber_plan_s* p, const char* name, hipStream_t s) {
    Profiler* f = p->prof;
    if (!f) return -1;
    if (f->used >= f->capacity) {
        ++f->dropped;
        return -1;
    }
    const int slot = f->used++;
    f->names[slot] = name;
    (void)hipEventRecord(f->ev[2 * slot], s);
    return slot;
}

inline void prof_stop(const amber_plan_s* p, int slot, hipStream_t s) {
    if (slot >= 0) (void)hipEventRecord(p->prof->ev[2 * slot + 1], s);
}

// Launch with optional timing.  KERNEL may be a parenthesised template-id.
#define AMBER_LAUNCH(plan, name, KERNEL, grid, block, stream, ...)                  \
    do {                                                                          \
        const int slot_ = prof_start((plan), (name), (stream));                   \
        hipLaunchKernelGGL(KERNEL, grid, block, 0, stream, __VA_ARGS__);          \
        prof_stop((plan), slot_, (stream));                                       \
    } while (0)

// Byte layout of the caller's workspace for one plan.
struct WsLayout {
    size_t ctrl;        // control block (status, counters, histograms, totals)
    size_t spec_a;      // N x N x N/2 complex spectrum
    size_t nyq_a;       // N x N complex Nyquist plane (kz = N/2)
    size_t spec_b;      // second spectrum (several l_mfp)
    size_t nyq_b;
    size_t mesh[2];     // halo deposit meshes, N^3 FP32 each (halo sources only)
    size_t bins;        // halo tile bins: mass bound, counts, cursors, starts (+1), gate, scale (halo sources only)
    size_t halo_tab;    // per-axis window and phase factors, N double4 (halo sources only)
    size_t keys[2];     // sort keys (ping-pong), N^3 uint32
    size_t vals[2];     // cell indices, N^3 uint32
    size_t wts[2];      // weights carried with the keys, N^3 float
    size_t part2[2];    // second-level (cell, z) partition, N^3 uint32 + float
    size_t lookback;    // decoupled look-back tiles: 3 regions of lb_words() words
    size_t total;
};

WsLayout ws_layout(int n, int n_lmfp, bool halo_meshes = false);

// Device address of the static scratch array of amber_zre_noalloc on `device`
// (noalloc.hip), looked up once per device with that device current.
int noalloc_scratch_address(int device, void** out);

// Words in each look-back region: 256 per 4096-cell tile, plus 256 tiles of
// slack for partitions whose tiles do not straddle buckets.
inline long long lb_words(long long n3) { return ((n3 + 4095) / 4096 + 256) * 256; }

// Control block (lives at offset 0 of the workspace; zeroed by a kernel at the
// start of every ranking or matching call).
struct Ctrl {
    unsigned status;            // AMBER_STATUS_* bits of this call
    unsigned pad0;
    unsigned* sticky;           // the plan's accumulated status word (amber_status clears it)
    unsigned hist[4][256];      // digit histograms of the descending keys
    unsigned digit_off[4][256]; // exclusive prefix of hist
    unsigned long long msum[256];  // per-FP32-exponent sums of significands of w
    int qmin;                   // exponent of the smallest weight ulp (w = m 2^q)
    int wide;                   // 1 when the total needs more than 64 bits
    unsigned long long total_lo, total_hi;  // exact sum of w 2^-qmin
    // Radix passes 0-2 split their input into 8 segments (rank.hip): counts
    // of the pass's digit per segment, turned by the offsets kernel into
    // where the run of digit d from segment s starts in the output.
    unsigned segcnt[3][8][256];
    unsigned seg_start[4][9];   // pass k: first element of segment s (s = 8: n)
    unsigned seg_tile0[4][9];   // pass k: look-back id of segment s's first tile (s = 8: the pass's tiles)
    unsigned seg_ticket[4][8];  // pass k: next tile of segment s
};

// Decoupled look-back over 30-bit counts with a 2-bit flag (aggregate or
// inclusive prefix), one word per (tile, entry), 256 entries per tile.  The
// walk reads 8 predecessors per step, which keeps its latency from growing with
// the number of tiles in flight; it stops at the first prefix, and every tile
// at or after first_tile publishes its aggregate before walking, so it ends.
// A data error: the call's own status word and the plan's accumulated one.
__device__ __forceinline__ void report_status(Ctrl* ctrl, unsigned bit) {
    atomicOr(&ctrl->status, bit);
    atomicOr(ctrl->sticky, bit);
}

constexpr unsigned kLbAgg = 1u << 30, kLbPre = 2u << 30, kLbMask = (1u << 30) - 1;
constexpr int kLbBatch = 8;

__device__ __forceinline__ unsigned lb_walk(const unsigned* lb, long long tile, int d, long long first_tile) {
    unsigned excl = 0;
    long long t = tile - 1;
    while (true) {
        unsigned v[kLbBatch];
#pragma unroll
        for (int k = 0; k < kLbBatch; ++k)
            v[k] = (t - k >= first_tile)
                       ? __hip_atomic_load(lb + (t - k) * 256 + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       : kLbPre;
        int used = 0;
        bool done = false, stall = false;
#pragma unroll
        for (int k = 0; k < kLbBatch; ++k) {
            if (done || stall) continue;
            const unsigned f = v[k] & ~kLbMask;
            if (f == 0u) {
                stall = true;
                continue;
            }
            excl += v[k] & kLbMask;
            ++used;
            if (f == kLbPre) done = true;
        }
        if (done) break;
        t -= used;
        if (stall) __builtin_amdgcn_s_sleep(1);
    }
    return excl;
}

// FFT launches (fft.hip).
int fft_radiation(const amber_plan_s* p, const float* d_src, const double* l_mfp, int n_lmfp,
                  float* const* d_J, unsigned char* ws, const WsLayout& L, hipStream_t s);

// Forward transform only, into the given spectrum and Nyquist plane (fft.hip).
int fft_forward(const amber_plan_s* p, const float* d_src, float2* spec, float2* nyq, hipStream_t s);

// J_l = IDFT[spec Khat_l] / N^3 from a transformed spectrum (fft.hip); the
// spectrum is kept when n_lmfp > 1 (the products go through spec_tmp).
int fft_from_spectrum(const amber_plan_s* p, float2* spec, float2* nyq, const double* l_mfp, int n_lmfp,
                      float* const* d_J, float2* spec_tmp, float2* nyq_tmp, hipStream_t s);

// FFT launch candidates compiled for grid size n (fft.hip): how many for the
// column and z passes, and the split of candidate idx (kind 0: N1 threads per
// column and C columns per tile; kind 1: M1 threads per line and ZL lines).
int fft_schedule_count(int n, int* n_col, int* n_z);
int fft_schedule_info(int n, int kind, int idx, int* a, int* b);

// Edge of the cubic mesh tiles the halo deposit bins by; grids it does not
// divide use the direct (atomic) deposit.
constexpr int kHaloTile = 16;
inline size_t halo_tiles(int n) {
    const size_t t = (n % kHaloTile == 0) ? (size_t)(n / kHaloTile) : 0;
    return t * t * t;
}
// The binning's first level: up to this many superbins of up to this many
// tiles each, and up to this many blocks (one count per superbin and block).
constexpr int kHaloSuperMax = 512;
constexpr int kHaloSuperBlocks = 2048;
inline size_t halo_bin_words(int n) {
    return 2 * halo_tiles(n) + 8 + (size_t)kHaloSuperMax * (2 * kHaloSuperBlocks + 1) + 2 * kHaloSuperMax + 1;
}

// Halo catalogue -> interlaced, deconvolved source spectrum in spec_a (halos.hip).
int halo_source_spectrum(const amber_plan_s* p, const float* d_pos, const float* d_mass, long long n_halo,
                         int scheme, int interlace, unsigned char* ws, const WsLayout& L, hipStream_t s);

// Shell-binned spectra of two forward transforms (spectra.hip).
int spectra_bins(const amber_plan_s* p, const float2* spec_a, const float2* nyq_a, int kind_a,
                 const float2* spec_b, const float2* nyq_b, int kind_b, int n_bins, double* d_out, hipStream_t s);

// Ranking and matching launches (rank.hip, match.hip).
int rank_sort(const amber_plan_s* p, const float* d_J, const float* d_w, unsigned char* ws,
              const WsLayout& L, hipStream_t s, int carry_weights, uint32_t* d_perm_out);
int match_scan(const amber_plan_s* p, const amber_weibull* hist, int n_hist, float* const* d_zre,
               unsigned char* ws, const WsLayout& L, hipStream_t s);
// dst[0] = 0 (first) or dst[0] |= the status word of the workspace's control block.
int status_collect(const amber_plan_s* p, unsigned char* ws, const WsLayout& L, unsigned* dst, bool first,
                   hipStream_t s);

#define AMBER_HIP_CHECK(expr)                        \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return AMBER_E_HIP;    \
    } while (0)
