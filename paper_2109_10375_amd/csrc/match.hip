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
constexpr int kMaxHist = 8;
constexpr unsigned kAgg = 1u, kPre = 2u;

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
    double a, h, z_top;
    long long T;
    const double* X;
    float* out;
};

struct HistArgs {
    HistArg h[kMaxHist];
    int n;
};

// j = max{ j in [lo, hi] : X_j >= F }, given X_lo >= F.
__device__ __forceinline__ long long bracket(const double* __restrict__ X, double F, long long lo, long long hi) {
    while (lo < hi) {
        const long long mid = lo + (hi - lo + 1) / 2;
        if (X[mid] >= F) lo = mid; else hi = mid - 1;
    }
    return lo;
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

// Look-back record of a tile (256 words, cleared by the last radix pass):
// word 0 = flag; words 2-5 = the tile's own sum (128 bits); words 6-9 = the
// inclusive prefix, written before the flag announces it.
__global__ __launch_bounds__(kThreads) void k_scan_invert(const unsigned* __restrict__ perm,
                                                          const float* __restrict__ w_sorted, long long n,
                                                          Ctrl* ctrl, unsigned* __restrict__ lb, HistArgs hs) {
    __shared__ unsigned s_tile;
    __shared__ u128 s_wave[kWaves];
    __shared__ u128 s_excl;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(&ctrl->tickets[4], 1u);
    __syncthreads();
    const unsigned tile = s_tile;
    const long long p0 = (long long)tile * kTile + (long long)tid * kPer;
    const int qmin = ctrl->qmin;

    unsigned idx[kPer];
    u128 pre[kPer];
    u128 run = {0ull, 0ull};
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const long long p = p0 + j;
        const bool ok = p < n;
        idx[j] = ok ? perm[p] : 0u;
        const u128 v = ok ? scaled_weight(w_sorted[p], qmin) : u128{0ull, 0ull};
        run = add128(run, v);
        pre[j] = run;
    }
    // wave-inclusive scan of the thread totals
    u128 inc = run;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        u128 o;
        o.lo = __shfl_up(inc.lo, d, 64);
        o.hi = __shfl_up(inc.hi, d, 64);
        if (lane >= d) inc = add128(inc, o);
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    u128 thread_excl = {0ull, 0ull};
    u128 tile_total = {0ull, 0ull};
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        if (w < wave) thread_excl = add128(thread_excl, s_wave[w]);
        tile_total = add128(tile_total, s_wave[w]);
    }
    {
        u128 o;
        o.lo = __shfl_up(inc.lo, 1, 64);
        o.hi = __shfl_up(inc.hi, 1, 64);
        if (lane > 0) thread_excl = add128(thread_excl, o);
    }

    if (tid == 0) {
        unsigned* me = lb + (long long)tile * 256;
        unsigned long long* me64 = reinterpret_cast<unsigned long long*>(me + 2);
        u128 excl = {0ull, 0ull};
        if (tile == 0) {
            st128(me64 + 2, tile_total);
            __atomic_thread_fence(__ATOMIC_RELEASE);
            __hip_atomic_store(me, kPre, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            st128(me64, tile_total);
            __atomic_thread_fence(__ATOMIC_RELEASE);
            __hip_atomic_store(me, kAgg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            long long t = (long long)tile - 1;
            while (true) {
                const unsigned* other = lb + t * 256;
                const unsigned f = __hip_atomic_load(other, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (f == 0u) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                const unsigned long long* o64 = reinterpret_cast<const unsigned long long*>(other + 2);
                if (f == kPre) {
                    excl = add128(excl, ld128(o64 + 2));
                    break;
                }
                excl = add128(excl, ld128(o64));
                --t;
            }
            st128(me64 + 2, add128(excl, tile_total));
            __atomic_thread_fence(__ATOMIC_RELEASE);
            __hip_atomic_store(me, kPre, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_excl = excl;
    }
    __syncthreads();
    const u128 base = add128(s_excl, thread_excl);
    const u128 total = {ctrl->total_lo, ctrl->total_hi};
    const double tot = u128_to_f64(total);

    double F[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) F[j] = __ddiv_rn(u128_to_f64(add128(base, pre[j])), tot);

    // Per history: bracket the wave's F range once, then each cell inside it.
    const long long p_first = (long long)tile * kTile + (long long)(tid - lane) * kPer;
    const long long wave_last = p_first + 64 * kPer - 1;
    const bool last_ok = wave_last < n;
    for (int hh = 0; hh < hs.n; ++hh) {
        const HistArg H = hs.h[hh];
        long long jA = 0, jB = 0;
        if (lane == 0) jA = bracket(H.X, F[0], 0, H.T);
        if (lane == 63) jB = last_ok ? bracket(H.X, F[kPer - 1], 0, H.T) : 0;
        jA = __shfl(jA, 0, 64);
        jB = __shfl(jB, 63, 64);
#pragma unroll 4
        for (int j = 0; j < kPer; ++j) {
            const long long p = p0 + j;
            if (p >= n) continue;
            const long long jj = bracket(H.X, F[j], jB, jA);
            const double z = interpolate(H.X, F[j], jj, H.a, H.h, H.T, H.z_top);
            if (idx[j] < (unsigned long long)n) H.out[idx[j]] = (float)z;
        }
    }
}

}  // namespace

int match_scan(const amber_plan_s* p, const amber_weibull* hist, int n_hist, float* const* d_zre, unsigned char* ws,
               const WsLayout& L, hipStream_t s) {
    const long long n = (long long)p->n * p->n * p->n;
    const long long n_tiles = (n + kTile - 1) / kTile;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
    const unsigned* perm = reinterpret_cast<const unsigned*>(ws + L.vals[0]);
    const float* w_sorted = reinterpret_cast<const float*>(ws + L.wts[0]);
    unsigned* lb = reinterpret_cast<unsigned*>(ws + L.lookback);  // cleared by the last radix pass
    for (int h0 = 0; h0 < n_hist; h0 += kMaxHist) {
        HistArgs hs{};
        hs.n = std::min(kMaxHist, n_hist - h0);
        for (int i = 0; i < hs.n; ++i) {
            const amber_weibull& w = hist[h0 + i];
            hs.h[i] = HistArg{w.a_w, w.h, w.z_top, (long long)(w.table_n - 1), w.d_table, d_zre[h0 + i]};
        }
        AMBER_LAUNCH(p, "match_scan_invert", k_scan_invert, dim3((unsigned)n_tiles), dim3(kThreads), s, perm, w_sorted,
                     n, ctrl, lb, hs);
    }
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}
