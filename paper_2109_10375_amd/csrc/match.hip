// Abundance matching on gfx950 (Sec. 3.4.2): for the cells in rank order, the
// cumulative gas mass C_n (inclusive: the cells ranked at or before n are
// ionized), the ionized mass fraction F_n = C_n / C_N, and the redshift z_n at
// which the history x_i(z) of Eq. (weibull) equals F_n, scattered back to the
// cells: z_re[perm[n]] = z_n.
//
// The cumulative mass is exact.  Each FP32 weight is the integer m 2^(q - qmin)
// in units of the smallest weight ulp 2^qmin, summed in 128-bit integers, so the
// prefix is the same for any summation order and any tiling.  F_n is the
// quotient of the two sums rounded to FP64 (round to nearest even), and the
// inversion interpolates the caller's FP64 table of x_i at z_j = a_w + j h with
// a fixed operation order and no fused multiply-add, so z_re is a pure function
// of (J, w, table).
//
// One block scans 4096 consecutive ranks: per-thread serial prefix of 16,
// wave and block scans in registers/LDS, then a decoupled look-back over the
// preceding tiles for the tile's starting sum (tiles take tickets in launch
// order, so every wait is on a tile that is already running).
#include <algorithm>

#include "internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kPer = 16;
constexpr int kTile = kThreads * kPer;
constexpr int kMaxHist = 3;
constexpr unsigned kAgg = 1u, kPre = 2u;
constexpr unsigned kPartAgg = kLbAgg, kPartPre = kLbPre, kPartMask = kLbMask;
constexpr int kGroup = 3;  // histories per scan launch

struct u128 {
    unsigned long long lo, hi;
};

__device__ __forceinline__ u128 add128(u128 a, u128 b) {
    u128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1ull : 0ull);
    return r;
}

// Unsigned 64-bit integer to the nearest FP64 (ties to even): both 32-bit
// halves convert exactly and the single addition rounds once.
__device__ __forceinline__ double u64_to_f64(unsigned long long v) {
    const double hi = (double)(unsigned)(v >> 32);
    const double lo = (double)(unsigned)(v & 0xffffffffull);
    return __dadd_rn(__dmul_rn(hi, 4294967296.0), lo);
}

// Unsigned 128-bit integer to the nearest FP64: take the leading 64 bits, fold
// every bit below them into a sticky bit 0 (below the rounding position), round
// that once, scale by the exact power of two.
__device__ __forceinline__ double u128_to_f64(u128 v) {
    if (v.hi == 0ull) return u64_to_f64(v.lo);
    const int lz = __clzll(v.hi);
    unsigned long long top = lz ? ((v.hi << lz) | (v.lo >> (64 - lz))) : v.hi;
    const unsigned long long rest = lz ? (v.lo << lz) : v.lo;
    if (rest) top |= 1ull;
    return ldexp(u64_to_f64(top), 64 - lz);
}

__device__ __forceinline__ u128 scaled_weight(float w, int qmin) {
    const unsigned b = __float_as_uint(w);
    const unsigned e = (b >> 23) & 255u;
    const unsigned long long m = (b & 0x7fffffu) | (e ? 0x800000u : 0u);
    const int q = (e == 0u ? 1 : (int)e) - 150;
    const int sh = q - qmin;
    u128 r;
    if (sh < 0 || sh >= 128) {  // invalid input, reported through the status word
        r.lo = 0; r.hi = 0;
    } else if (sh == 0) {
        r.lo = m; r.hi = 0;
    } else if (sh < 64) {
        r.lo = m << sh; r.hi = m >> (64 - sh);
    } else {
        r.lo = 0; r.hi = m << (sh - 64);
    }
    return r;
}

struct HistArg {
    double a, b, inv_c, h, z_top;
    long long T;
    const double* X;
    float* out;
};

struct HistArgs {
    HistArg h[kMaxHist];
    int n;
};

// Starting node for the bracket search: the closed-form inverse in FP32,
// (z - a)/h = b (-ln F)^(1/c) / h, with -ln F taken as -log1p(-(1 - F)) near 1.
// Its error is a small fraction of a node; the exact comparisons decide.
__device__ __forceinline__ long long guess_node(double F, const HistArg& H) {
    const double u = 1.0 - F;
    const float L = (u < 0.25) ? -log1pf(-(float)u) : -logf((float)F);
    const double r = (double)((float)H.b * powf(L, (float)H.inv_c)) / H.h;
    double gg = floor(r);
    if (!(gg >= 0.0)) gg = 0.0;  // also NaN
    if (gg > (double)(H.T - 1)) gg = (double)(H.T - 1);
    return (long long)gg;
}

struct HistArg;
__device__ __forceinline__ long long guess_node(double F, const HistArg& H);

// Exact bracket j = max{ j in [0, T] : X_j >= F } (X non-increasing, X_0 = 1),
// walking from a starting node: the comparisons with the table decide, so the
// result does not depend on where the walk starts.
__device__ __forceinline__ long long bracket_from(const double* __restrict__ X, double F, long long j, long long T) {
    while (j < T && X[j + 1] >= F) ++j;
    while (j > 0 && X[j] < F) --j;
    return j;
}

__device__ __forceinline__ double interpolate(const double* __restrict__ X, double F, long long j, double a, double h,
                                              long long T, double z_top) {
#pragma clang fp contract(off)
    if (j > T - 1) j = T - 1;
    const double zj = a + (double)j * h;
    const double zj1 = a + (double)(j + 1) * h;
    const double xj = X[j], xj1 = X[j + 1];
    const double den = xj - xj1;
    const double t = (den != 0.0) ? (xj - F) / den : 0.0;
    const double dz = zj1 - zj;
    const double z = zj + t * dz;
    return (z < z_top) ? z : z_top;
}

__device__ __forceinline__ u128 ld128(const unsigned long long* p) {
    u128 r;
    r.lo = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    r.hi = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return r;
}
__device__ __forceinline__ void st128(unsigned long long* p, u128 v) {
    __hip_atomic_store(p, v.lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, v.hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ u128 shfl_up128(u128 v, int d) {
    u128 o;
    o.lo = __shfl_up(v.lo, d, 64);
    o.hi = __shfl_up(v.hi, d, 64);
    return o;
}

// Exclusive scan of one value per thread over the 256 threads.
__device__ __forceinline__ unsigned block_excl_scan(unsigned v, unsigned* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned u = __shfl_up(x, o, 64);
        if (lane >= o) x += u;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    unsigned add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
        if (w < wave) add += sh[w];
    __syncthreads();
    return add + x - v;
}

// Exact unsigned division x / d for x < 2^30: FP64 reciprocal estimate, then
// an integer correction of at most one step.
__device__ __forceinline__ unsigned div_exact(unsigned x, unsigned d, double rinv) {
    unsigned q = (unsigned)((double)x * rinv);
    if (q * d > x) --q;
    else if ((q + 1u) * d <= x) ++q;
    return q;
}

// Fixed-point accumulator: 64-bit when the exact total fits (the usual case),
// 128-bit otherwise.  Both give the same integers, hence the same F.
template <bool WIDE>
struct Acc;

template <>
struct Acc<false> {
    unsigned long long v;
    __device__ static Acc zero() { return Acc{0ull}; }
    __device__ static Acc of(float w, int qmin) { return Acc{scaled_weight(w, qmin).lo}; }
    __device__ static Acc of128(u128 x) { return Acc{x.lo}; }
    __device__ Acc operator+(Acc o) const { return Acc{v + o.v}; }
    __device__ Acc shfl_up(int d) const { return Acc{__shfl_up(v, d, 64)}; }
    __device__ Acc shfl(int l) const { return Acc{__shfl(v, l, 64)}; }
    __device__ double to_f64() const { return u64_to_f64(v); }
    __device__ u128 wide() const { return u128{v, 0ull}; }
};

template <>
struct Acc<true> {
    u128 v;
    __device__ static Acc zero() { return Acc{u128{0ull, 0ull}}; }
    __device__ static Acc of(float w, int qmin) { return Acc{scaled_weight(w, qmin)}; }
    __device__ static Acc of128(u128 x) { return Acc{x}; }
    __device__ Acc operator+(Acc o) const { return Acc{add128(v, o.v)}; }
    __device__ Acc shfl_up(int d) const { return Acc{shfl_up128(v, d)}; }
    __device__ Acc shfl(int l) const {
        u128 r;
        r.lo = __shfl(v.lo, l, 64);
        r.hi = __shfl(v.hi, l, 64);
        return Acc{r};
    }
    __device__ double to_f64() const { return u128_to_f64(v); }
    __device__ u128 wide() const { return v; }
};

// Exact mass of every 4096-rank tile, before any rank is matched: block g sums
// tiles 64 g .. 64 g + 63 of the sorted weights in order and keeps, per tile,
// the exclusive prefix within the block (local[tile]) and the block's total.
// Every weight is also checked: its scaled value m 2^(q - qmin) must fit in
// 127 bits, and so must every partial sum.
constexpr int kTilesPerBlock = 64;

__global__ __launch_bounds__(kThreads) void k_tile_sums(const float* __restrict__ w_sorted, long long n, Ctrl* ctrl,
                                                        u128* __restrict__ local, u128* __restrict__ block_tot,
                                                        long long n_tiles) {
    __shared__ u128 s_wave[kWaves];
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_bad = 0;
    const int qmin = ctrl->qmin;
    u128 running = {0ull, 0ull};
    bool bad = false;
    for (int k = 0; k < kTilesPerBlock; ++k) {
        const long long tile = (long long)blockIdx.x * kTilesPerBlock + k;
        if (tile >= n_tiles) break;
        const long long p0 = tile * kTile + (long long)tid * kPer;
        u128 sum = {0ull, 0ull};
        if (p0 < n) {
            const float4* pw = reinterpret_cast<const float4*>(w_sorted + p0);
#pragma unroll
            for (int q = 0; q < kPer / 4; ++q) {
                const float4 b4 = pw[q];
                const float e[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const unsigned b = __float_as_uint(e[c]);
                    const unsigned ex = (b >> 23) & 255u;
                    const unsigned m = (b & 0x7fffffu) | (ex ? 0x800000u : 0u);
                    const int sh = (ex == 0u ? 1 : (int)ex) - 150 - qmin;
                    bad |= sh < 0 || sh + (m ? 32 - __clz(m) : 0) > 127;
                    const u128 v = scaled_weight(e[c], qmin);
                    const u128 t = add128(sum, v);
                    bad |= t.hi < sum.hi;
                    sum = t;
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            u128 w;
            w.lo = __shfl_xor(sum.lo, o, 64);
            w.hi = __shfl_xor(sum.hi, o, 64);
            const u128 t = add128(sum, w);
            bad |= t.hi < sum.hi;
            sum = t;
        }
        if (lane == 0) s_wave[wave] = sum;
        __syncthreads();
        if (tid == 0) {
            u128 t = {0ull, 0ull};
            for (int w = 0; w < kWaves; ++w) {
                const u128 u = add128(t, s_wave[w]);
                bad |= u.hi < t.hi;
                t = u;
            }
            local[tile] = running;
            const u128 r = add128(running, t);
            bad |= r.hi < running.hi;
            running = r;
        }
        __syncthreads();
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == 0) {
        block_tot[blockIdx.x] = running;
        if (s_bad) atomicOr(&ctrl->status, AMBER_STATUS_RANGE);
    }
}

// Exclusive prefix of the block totals (one block of 1024 threads), the exact
// grand total C_N, and whether it needs more than 64 bits.
constexpr int kPrefixThreads = 1024;
__global__ __launch_bounds__(kPrefixThreads) void k_block_prefix(u128* __restrict__ block_tot, long long nb,
                                                                 Ctrl* ctrl) {
    __shared__ u128 s_part[kPrefixThreads];
    const int tid = threadIdx.x;
    const long long per = (nb + kPrefixThreads - 1) / kPrefixThreads;
    const long long b0 = (long long)tid * per;
    u128 sum = {0ull, 0ull};
    bool bad = false;
    for (long long b = b0; b < b0 + per && b < nb; ++b) {
        const u128 t = add128(sum, block_tot[b]);
        bad |= t.hi < sum.hi;
        sum = t;
    }
    s_part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        u128 run = {0ull, 0ull};
        for (int i = 0; i < kPrefixThreads; ++i) {
            const u128 v = s_part[i];
            s_part[i] = run;
            const u128 t = add128(run, v);
            bad |= t.hi < run.hi;
            run = t;
        }
        ctrl->total_lo = run.lo;
        ctrl->total_hi = run.hi;
        ctrl->wide = run.hi != 0ull;
        if (bad || (run.hi >> 63)) atomicOr(&ctrl->status, AMBER_STATUS_RANGE);
    }
    __syncthreads();
    u128 run = s_part[tid];
    for (long long b = b0; b < b0 + per && b < nb; ++b) {
        const u128 v = block_tot[b];
        block_tot[b] = run;
        run = add128(run, v);
    }
    if (bad) atomicOr(&ctrl->status, AMBER_STATUS_RANGE);
}

// Tile of 4096 consecutive ranks; thread t owns ranks 16 t .. 16 t + 15.
//  1. load cell indices and weights (16-byte vector loads); count the tile's
//     members of each index-range bucket (bucket b = cells [b S, (b+1) S),
//     S = n / 256) and scan the thread totals of the exact weights;
//  2. take its slots in each bucket with one atomic add per bucket; its
//     starting mass comes from the tile prefix computed beforehand, so no
//     tile waits on another;
//  3. four ranks at a time: the exact prefix, F_n = RN(C_n)/RN(C_N), the
//     bracket for each history from the closed-form guess with all table reads
//     of the four ranks in flight together, z_n, and the (cell, z) pairs staged
//     in LDS bucket by bucket and written in coalesced runs.
// The launch runs the 64-bit variant when the exact total fits in 64 bits and
// the 128-bit one otherwise (the other variant's blocks return at once).
// fill[b] (cleared before the launch) counts the slots of bucket b handed out.
template <int NH, bool WIDE>
__global__ __launch_bounds__(kThreads) void k_scan_partition(
    const unsigned* __restrict__ perm, const float* __restrict__ w_sorted, long long n, Ctrl* ctrl,
    const u128* __restrict__ local, const u128* __restrict__ block_excl, unsigned* __restrict__ fill,
    unsigned bucket_size, double bucket_rinv, HistArgs hs, unsigned* __restrict__ part_idx,
    float* __restrict__ part_z0, float* __restrict__ part_z1, float* __restrict__ part_z2) {
    using A = Acc<WIDE>;
    if ((ctrl->wide != 0) != WIDE) return;
    __shared__ A s_wave[kWaves];
    __shared__ unsigned lcnt[256];
    __shared__ unsigned loff[256];
    __shared__ unsigned gbase[256];
    __shared__ unsigned scan_sh[kWaves];
    __shared__ unsigned st_idx[kTile];
    __shared__ float st_z[NH][kTile];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    lcnt[tid] = 0u;
    __syncthreads();
    const long long tile = blockIdx.x;
    const long long p0 = tile * kTile + (long long)tid * kPer;
    const bool ok = p0 < n;  // n is a multiple of 512: a thread's 16 ranks are all valid or all not
    const int qmin = ctrl->qmin;

    unsigned idx[kPer], rk[kPer];
    float wf[kPer];
    if (ok) {
        const uint4* pi = reinterpret_cast<const uint4*>(perm + p0);
        const float4* pw = reinterpret_cast<const float4*>(w_sorted + p0);
#pragma unroll
        for (int q = 0; q < kPer / 4; ++q) {
            const uint4 a = pi[q];
            const float4 b = pw[q];
            idx[4 * q] = a.x; idx[4 * q + 1] = a.y; idx[4 * q + 2] = a.z; idx[4 * q + 3] = a.w;
            wf[4 * q] = b.x; wf[4 * q + 1] = b.y; wf[4 * q + 2] = b.z; wf[4 * q + 3] = b.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            idx[j] = 0xffffffffu;
            wf[j] = 0.0f;
        }
    }
    A tsum = A::zero();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const bool live = ok && idx[j] < (unsigned long long)n;
        if (live) tsum = tsum + A::of(wf[j], qmin);
        rk[j] = live ? atomicAdd(&lcnt[div_exact(idx[j], bucket_size, bucket_rinv)], 1u) : 0xffffffffu;
    }
    // exclusive scan of the thread totals over the wave, then over the waves
    A inc = tsum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const A o = inc.shfl_up(d);
        if (lane >= d) inc = inc + o;
    }
    if (lane == 63) s_wave[wave] = inc;
    A thread_excl = inc.shfl_up(1);
    if (lane == 0) thread_excl = A::zero();
    __syncthreads();
    A wave_excl = A::zero();
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
        if (w < wave) wave_excl = wave_excl + s_wave[w];

    // this tile's slots in every bucket (any order within a bucket will do);
    // the atomic's result is only needed when the pairs are written
    const unsigned cnt = lcnt[tid];
    const unsigned slot0 = cnt ? atomicAdd(&fill[tid], cnt) : 0u;
    loff[tid] = block_excl_scan(cnt, scan_sh);
    __syncthreads();  // every bucket's loff is read below

    const u128 tile_excl = add128(block_excl[tile / kTilesPerBlock], local[tile]);
    A run = A::of128(tile_excl) + wave_excl + thread_excl;
    const u128 total = {ctrl->total_lo, ctrl->total_hi};
    const double tot = u128_to_f64(total);
    constexpr int kChunk = 4;
#pragma unroll
    for (int c0 = 0; c0 < kPer; c0 += kChunk) {
        double F[kChunk];
        unsigned pos[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            const int j = c0 + q;
            const bool live = rk[j] != 0xffffffffu;
            if (live) run = run + A::of(wf[j], qmin);
            F[q] = __ddiv_rn(run.to_f64(), tot);
            pos[q] = live ? loff[div_exact(idx[j], bucket_size, bucket_rinv)] + rk[j] : 0xffffffffu;
            if (pos[q] >= (unsigned)kTile) pos[q] = 0xffffffffu;  // unreachable for consistent counts
            if (pos[q] != 0xffffffffu) st_idx[pos[q]] = idx[j];
        }
#pragma unroll
        for (int hh = 0; hh < NH; ++hh) {
            const HistArg& H = hs.h[hh];
            long long g[kChunk];
            double x0[kChunk], x1[kChunk];
#pragma unroll
            for (int q = 0; q < kChunk; ++q) g[q] = guess_node(F[q], H);
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                x0[q] = H.X[g[q]];
                x1[q] = H.X[g[q] + 1];
            }
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                if (pos[q] == 0xffffffffu) continue;
                long long jj = g[q];
                if (!(x0[q] >= F[q] && x1[q] < F[q])) jj = bracket_from(H.X, F[q], jj, H.T);
                st_z[hh][pos[q]] = (float)interpolate(H.X, F[q], jj, H.a, H.h, H.T, H.z_top);
            }
        }
    }
    gbase[tid] = (unsigned)tid * bucket_size + slot0;
    __syncthreads();
    const long long valid_ll = n - tile * kTile;
    const int valid = valid_ll < kTile ? (int)valid_ll : kTile;
    for (int i = tid; i < valid; i += kThreads) {
        const unsigned c = st_idx[i];
        if (c >= (unsigned long long)n) continue;
        const unsigned b = div_exact(c, bucket_size, bucket_rinv);
        const long long dst = (long long)gbase[b] + (i - (int)loff[b]);
        if (dst < 0 || dst >= n) continue;  // unreachable for consistent counts
        part_idx[dst] = c;
        part_z0[dst] = st_z[0][i];
        if (NH > 1) part_z1[dst] = st_z[NH > 1 ? 1 : 0][i];
        if (NH > 2) part_z2[dst] = st_z[NH > 2 ? 2 : 0][i];
    }
}

// Second partition level, inside each first-level bucket: the pairs of bucket
// b (positions [b S1, (b+1) S1), cells of the same range) are split into 256
// sub-buckets of S2 = S1 / 256 cells.  Tiles never straddle buckets; each tile
// takes its slots in a sub-bucket with one atomic add on that sub-bucket's
// fill counter (order inside a sub-bucket does not matter).
__global__ __launch_bounds__(kThreads) void k_partition2(const unsigned* __restrict__ in_idx,
                                                         const float* __restrict__ in_z, long long n,
                                                         unsigned* __restrict__ fill, unsigned S1, unsigned S2,
                                                         unsigned tiles_per_bucket,
                                                         unsigned* __restrict__ out_idx,
                                                         float* __restrict__ out_z) {
    __shared__ unsigned lcnt[256];
    __shared__ unsigned loff[256];
    __shared__ unsigned gbase[256];
    __shared__ unsigned scan_sh[kWaves];
    __shared__ unsigned st_idx[kTile];
    __shared__ float st_z[kTile];
    const int tid = threadIdx.x;
    lcnt[tid] = 0u;
    __syncthreads();
    const unsigned tile = blockIdx.x;  // no waits on other tiles
    const unsigned b = tile / tiles_per_bucket, k = tile % tiles_per_bucket;
    const long long bstart = (long long)b * S1;
    const long long t0 = bstart + (long long)k * kTile;
    const long long t1 = t0 + kTile < bstart + S1 ? t0 + kTile : bstart + S1;
    const int valid = (int)(t1 - t0);
    unsigned idx[kPer], sb[kPer], rk[kPer];
    float z[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kThreads + tid;
        const bool ok = i < valid;
        idx[j] = ok ? in_idx[t0 + i] : 0u;
        z[j] = ok ? in_z[t0 + i] : 0.0f;
        const long long rel = (long long)idx[j] - bstart;
        const bool live = ok && rel >= 0 && rel < (long long)S1;
        sb[j] = live ? (unsigned)rel / S2 : 0u;
        rk[j] = live ? atomicAdd(&lcnt[sb[j]], 1u) : 0xffffffffu;
    }
    __syncthreads();
    const unsigned cnt = lcnt[tid];
    const unsigned slot0 = cnt ? atomicAdd(&fill[(long long)b * 256 + tid], cnt) : 0u;
    gbase[tid] = (unsigned)(bstart + (long long)tid * S2 + slot0);
    loff[tid] = block_excl_scan(cnt, scan_sh);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        if (rk[j] == 0xffffffffu) continue;
        const unsigned pos = loff[sb[j]] + rk[j];
        if (pos >= (unsigned)kTile) continue;
        st_idx[pos] = idx[j];
        st_z[pos] = z[j];
    }
    __syncthreads();
    for (int i = tid; i < valid; i += kThreads) {
        const unsigned c = st_idx[i];
        const long long rel = (long long)c - bstart;
        if (rel < 0 || rel >= (long long)S1) continue;
        const unsigned s2 = (unsigned)rel / S2;
        const long long dst = (long long)gbase[s2] + (i - (int)loff[s2]);
        if (dst < 0 || dst >= n) continue;
        out_idx[dst] = c;
        out_z[dst] = st_z[i];
    }
}

// Last level: block L owns cells [L S, (L+1) S) (S <= 16384) and exactly the
// pairs at positions [L S, (L+1) S); it places z by cell in LDS and writes the
// run of z_re contiguously.
constexpr int kLeafMax = 16384;
constexpr int kLeafThreads = 1024;
__global__ __launch_bounds__(kLeafThreads) void k_leaf_scatter(const unsigned* __restrict__ in_idx,
                                                               const float* __restrict__ in_z, long long n, unsigned S,
                                                               float* __restrict__ out) {
    __shared__ float zl[kLeafMax];
    const long long start = (long long)blockIdx.x * S;
#pragma unroll 4
    for (unsigned i = threadIdx.x; i < S; i += kLeafThreads) {
        const unsigned c = in_idx[start + i];
        const long long rel = (long long)c - start;
        if (rel >= 0 && rel < (long long)S) zl[rel] = in_z[start + i];
    }
    __syncthreads();
#pragma unroll 4
    for (unsigned i = threadIdx.x; i < S; i += kLeafThreads) out[start + i] = zl[i];
}

__global__ __launch_bounds__(kThreads) void k_clear(unsigned* __restrict__ p, long long words) {
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < words; i += (long long)gridDim.x * kThreads)
        p[i] = 0u;
}

}  // namespace

int match_scan(const amber_plan_s* p, const amber_weibull* hist, int n_hist, float* const* d_zre, unsigned char* ws,
               const WsLayout& L, hipStream_t s) {
    const long long n = (long long)p->n * p->n * p->n;
    const long long n_tiles = (n + kTile - 1) / kTile;
    const long long n_blocks = (n_tiles + kTilesPerBlock - 1) / kTilesPerBlock;
    const long long lbw = lb_words(n);  // words per look-back region
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
    const unsigned* perm = reinterpret_cast<const unsigned*>(ws + L.vals[0]);
    const float* w_sorted = reinterpret_cast<const float*>(ws + L.wts[0]);
    // region [0]: tile prefixes; [2]: first-level fill counters (cleared by the
    // last radix pass); [1]: second-level fill counters (cleared here)
    u128* local = reinterpret_cast<u128*>(ws + L.lookback);
    u128* block_excl = local + n_tiles;
    unsigned* base_words = reinterpret_cast<unsigned*>(ws + L.lookback);
    unsigned* fill2 = base_words + lbw;
    unsigned* fill1 = base_words + 2 * lbw;
    // first level: pairs in the sort buffers freed by the last radix pass
    unsigned* p1_idx = reinterpret_cast<unsigned*>(ws + L.keys[0]);
    float* p1_z[kGroup] = {reinterpret_cast<float*>(ws + L.keys[1]), reinterpret_cast<float*>(ws + L.vals[1]),
                           reinterpret_cast<float*>(ws + L.wts[1])};
    // second level: its own buffers, so the rank order survives for later groups
    unsigned* p2_idx = reinterpret_cast<unsigned*>(ws + L.part2[0]);
    float* p2_z = reinterpret_cast<float*>(ws + L.part2[1]);
    const unsigned S1 = (unsigned)(n / 256);  // n is a multiple of 512
    const bool two_level = S1 > (unsigned)kLeafMax;
    const unsigned S2 = two_level ? S1 / 256 : S1;  // divides exactly for the supported sizes
    const unsigned tpb = (S1 + kTile - 1) / kTile;
    const dim3 grid((unsigned)n_tiles), blk(kThreads);

    AMBER_LAUNCH(p, "match_tile_sums", k_tile_sums, dim3((unsigned)n_blocks), blk, s, w_sorted, n, ctrl, local,
                 block_excl, n_tiles);
    AMBER_LAUNCH(p, "match_block_prefix", k_block_prefix, dim3(1), dim3(kPrefixThreads), s, block_excl, n_blocks, ctrl);
    const double rinv = 1.0 / (double)S1;
    for (int g = 0; g * kGroup < n_hist; ++g) {
        const int h0 = g * kGroup;
        HistArgs hs{};
        hs.n = std::min(kGroup, n_hist - h0);
        for (int i = 0; i < hs.n; ++i) {
            const amber_weibull& w = hist[h0 + i];
            hs.h[i] = HistArg{w.a_w, w.b_w, 1.0 / w.c_w, w.h, w.z_top, (long long)(w.table_n - 1), w.d_table,
                              d_zre[h0 + i]};
        }
        if (g > 0) AMBER_LAUNCH(p, "match_clear", k_clear, dim3(1), blk, s, fill1, 256);
#define AMBER_SCAN(NHV)                                                                                      \
    AMBER_LAUNCH(p, "match_scan_partition", (k_scan_partition<NHV, false>), grid, blk, s, perm, w_sorted, n, \
                 ctrl, local, block_excl, fill1, S1, rinv, hs, p1_idx, p1_z[0], p1_z[1], p1_z[2]);           \
    AMBER_LAUNCH(p, "match_scan_partition_wide", (k_scan_partition<NHV, true>), grid, blk, s, perm, w_sorted, \
                 n, ctrl, local, block_excl, fill1, S1, rinv, hs, p1_idx, p1_z[0], p1_z[1], p1_z[2]);
        switch (hs.n) {
            case 1: AMBER_SCAN(1) break;
            case 2: AMBER_SCAN(2) break;
            default: AMBER_SCAN(3) break;
        }
#undef AMBER_SCAN
        for (int i = 0; i < hs.n; ++i) {
            if (two_level) {
                AMBER_LAUNCH(p, "match_clear", k_clear, dim3(256), blk, s, fill2, 65536);
                AMBER_LAUNCH(p, "match_partition2", k_partition2, dim3(256 * tpb), blk, s, p1_idx, p1_z[i], n, fill2,
                             S1, S2, tpb, p2_idx, p2_z);
                AMBER_LAUNCH(p, "match_leaf_scatter", k_leaf_scatter, dim3((unsigned)(n / S2)), dim3(kLeafThreads), s,
                             p2_idx, p2_z, n, S2, d_zre[h0 + i]);
            } else {
                AMBER_LAUNCH(p, "match_leaf_scatter", k_leaf_scatter, dim3(256), dim3(kLeafThreads), s, p1_idx,
                             p1_z[i], n, S1, d_zre[h0 + i]);
            }
        }
    }
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}
