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
// Launches: exact sums of every tile of ranks (a streaming reduction that
// also checks the 127-bit range), their prefix, then one block per tile that
// matches its ranks and partitions the (cell, z) pairs by cell range; a second
// partition level and an LDS pass per 16K-cell range put z_re in cell order.
// No tile waits on another.
#include <algorithm>

#include "internal.h"

namespace {

constexpr int kPer = 16;                            // ranks (or pairs) per thread
constexpr int kScanThreads = 256;                   // tile sums and matching: one tile per block
constexpr int kScanWaves = kScanThreads / 64;
constexpr int kScanTile = kScanThreads * kPer;
constexpr int kPartThreads = 1024;                  // second partition level: 16384 pairs per block
constexpr int kPartTile = kPartThreads * kPer;
constexpr int kL1 = 128;          // first-level cell-range buckets
constexpr int kL2 = 65536 / kL1;  // second-level sub-buckets of each bucket
static_assert(kScanThreads >= 256 && kScanTile <= 65536, "tile geometry");
static_assert(kL1 >= 64 && kL1 % 64 == 0 && kL1 <= kScanThreads && kL2 <= kPartThreads, "bucket geometry");
constexpr int kMaxHist = 3;
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
    const double2* XG;  // (X_j, D(z_j)/D(z_mid)) at the nodes, or null
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

// The same interpolation with X_j and X_{j+1} already loaded (j <= T - 1).
__device__ __forceinline__ double interpolate_xy(double F, long long j, double xj, double xj1, double a, double h,
                                                 double z_top) {
#pragma clang fp contract(off)
    const double zj = a + (double)j * h;
    const double zj1 = a + (double)(j + 1) * h;
    const double den = xj - xj1;
    const double t = (den != 0.0) ? (xj - F) / den : 0.0;
    const double dz = zj1 - zj;
    const double z = zj + t * dz;
    return (z < z_top) ? z : z_top;
}

// Growth-rescaled matching (Sec. 3.4.2 with delta(z) = D(z)/D(z_mid) delta):
// rank with k cells ionized, ks = k s and ns = N s its count and the total in
// the units s of the exact sums, cn = RN(C_k), cN = RN(C_N):
//   h_j = (ks (1 - G_j) + G_j cn) / (ns (1 - G_j) + G_j cN) - X_j,
// z = a if h_0 > 0, z_top if h_T <= 0, else bisection on the node index keeping
// h_lo <= 0 < h_hi, then linear interpolation of h between the two nodes.
__device__ __forceinline__ double growth_gap(double ks, double ns, double cn, double cN, double G, double X) {
#pragma clang fp contract(off)
    const double one_m = 1.0 - G;
    const double m = ks * one_m + G * cn;
    const double M = ns * one_m + G * cN;
    return m / M - X;
}

// Sign of the gap RN(m/M) - X at one node: 1 when it is > 0, 0 when <= 0,
// -1 when unordered, the same as evaluating growth_gap and comparing.  With
// M > 0 and X >= 0 it is decided without the division where it can be: one
// fused multiply-add rounds m - X M once, so its sign is that of the exact
// value; m <= X M gives RN(m/M) <= X, and m >= X' M, X' the next double above
// X, gives RN(m/M) >= X' > X.  Only a quotient strictly between X and X'
// (where the rounding of m/M decides) takes the division.
__device__ __forceinline__ int growth_gap_sign(double ks, double ns, double cn, double cN, double G, double X) {
#pragma clang fp contract(off)
    const double one_m = 1.0 - G;
    const double m = ks * one_m + G * cn;
    const double M = ns * one_m + G * cN;
    if (M > 0.0 && X >= 0.0) {
        if (__builtin_fma(-X, M, m) <= 0.0) return 0;
        const double Xs = __longlong_as_double(__double_as_longlong(X) + 1);
        if (__builtin_fma(-Xs, M, m) >= 0.0) return 1;
    }
    const double g = m / M - X;
    return g > 0.0 ? 1 : (g <= 0.0 ? 0 : -1);
}

// The bracket of one rank: -1 when h_0 > 0 (z = a), T when h_T <= 0 (z =
// z_top), otherwise lo with h_lo <= 0 < h_{lo+1}.  Where the gap changes sign
// once over the nodes this answer is unique, so any search that finds a sign
// change finds it.  The search starts from hint (a bracket of the same kind
// found for a nearby rank), checks it, and otherwise gallops away from it in
// the direction of the sign change and bisects the last step.
__device__ long long growth_bracket(double ks, double ns, double cn, double cN, long long T,
                                    const double2* __restrict__ XG, long long hint) {
    auto sgn = [&](long long j) {
        const double2 nd = XG[j];  // X and G of the node in one read
        return growth_gap_sign(ks, ns, cn, cN, nd.y, nd.x);
    };
    long long lo, hi;  // sgn(lo) == 0 (h <= 0), sgn(hi) != 0 (h > 0 or unordered)
    if (hint < 0) {
        if (sgn(0) != 0) return -1;
        hint = 0;
    } else if (hint >= T) {
        if (sgn(T) == 0) return T;
        hint = T - 1;
    }
    if (sgn(hint) == 0) {
        if (sgn(hint + 1) != 0) return hint;  // the hint's bracket
        // the crossing lies above: gallop up
        long long step = 2, a = hint + 1;
        for (;;) {
            const long long b = a + step < T ? a + step : T;
            if (sgn(b) != 0) {
                lo = a;
                hi = b;
                break;
            }
            if (b == T) return T;
            a = b;
            step *= 2;
        }
    } else {
        // the crossing lies below: gallop down
        long long step = 1, b = hint;
        for (;;) {
            const long long a = b - step > 0 ? b - step : 0;
            if (sgn(a) == 0) {
                lo = a;
                hi = b;
                break;
            }
            if (a == 0) return -1;
            b = a;
            step *= 2;
        }
    }
    while (hi - lo > 1) {
        const long long mid = lo + (hi - lo) / 2;
        if (sgn(mid) == 0) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The same kind of bracket for one rank, searched by the 64 lanes of a wave
// together (every lane calls it with the same arguments): each round the lanes
// test 64 evenly spaced nodes of the current interval and keep the one
// between the last non-positive and the first positive gap, so 2^22 nodes take
// four rounds of reads in flight together.
__device__ long long wave_growth_bracket(double ks, double ns, double cn, double cN, long long T,
                                         const double2* __restrict__ XG) {
    const int lane = threadIdx.x & 63;
    auto sgn = [&](long long j) {
        const double2 nd = XG[j];
        return growth_gap_sign(ks, ns, cn, cN, nd.y, nd.x);
    };
    const int sp = sgn(lane == 0 ? 0 : T);
    const int s0 = __shfl(sp, 0, 64), sT = __shfl(sp, 1, 64);
    if (s0 == 1) return -1;
    if (sT != 1) return T;
    long long lo = 0, hi = T;
    while (hi - lo > 1) {
        const long long step = (hi - lo + 63) / 64;
        const long long node = lo + (long long)(lane + 1) * step;  // lane 63's node is at or past hi
        const bool pos = node >= hi ? true : (sgn(node) != 0);
        const unsigned long long m = __ballot(pos);
        const int first = __ffsll((long long)m) - 1;
        const long long nh = lo + (long long)(first + 1) * step;
        lo = lo + (long long)first * step;
        hi = nh < hi ? nh : hi;
    }
    return lo;
}

// z from a bracket whose two nodes' (X, G) pairs are at hand (nl for lo, nh
// for lo + 1): z = z_lo + t (z_hi - z_lo), t = -h_lo / (h_hi - h_lo), min
// z_top (FP64, this operation order, no fused multiply-add); a for lo < 0,
// z_top for lo >= T.
__device__ __forceinline__ double growth_z(long long lo, double ks, double ns, double cn, double cN, double a,
                                           double h, long long T, double z_top, double2 nl, double2 nh) {
#pragma clang fp contract(off)
    if (lo < 0) return a;
    if (lo >= T) return z_top;
    const double hlo = growth_gap(ks, ns, cn, cN, nl.y, nl.x);
    const double hhi = growth_gap(ks, ns, cn, cN, nh.y, nh.x);
    const double zl = a + (double)lo * h;
    const double zh = a + (double)(lo + 1) * h;
    const double t = -hlo / (hhi - hlo);
    const double z = zl + t * (zh - zl);
    return (z < z_top) ? z : z_top;
}

__device__ __forceinline__ u128 shfl_up128(u128 v, int d) {
    u128 o;
    o.lo = __shfl_up(v.lo, d, 64);
    o.hi = __shfl_up(v.hi, d, 64);
    return o;
}

// Exclusive scan over NB values held by threads 0..NB-1 (NB a multiple of 64);
// every thread of the block calls it (it contains a barrier), the result is
// defined for threads 0..NB-1.
template <int NB>
__device__ __forceinline__ unsigned bucket_excl_scan(unsigned v, unsigned* sh /* NB / 64 */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned u = __shfl_up(x, o, 64);
        if (lane >= o) x += u;
    }
    if (wave < NB / 64 && lane == 63) sh[wave] = x;
    __syncthreads();
    unsigned add = 0;
#pragma unroll
    for (int w = 0; w < NB / 64; ++w)
        if (w < wave) add += sh[w];
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
    // the 64-bit path runs only when the exact total is below 2^64, so every
    // scaled weight is too (sh < 64 for any weight m > 0)
    __device__ static Acc of(float w, int qmin) {
        const unsigned b = __float_as_uint(w);
        const unsigned e = (b >> 23) & 255u;
        const unsigned long long m = (b & 0x7fffffu) | (e ? 0x800000u : 0u);
        const int sh = (e == 0u ? 1 : (int)e) - 150 - qmin;
        return Acc{((unsigned)sh < 64u) ? m << sh : 0ull};
    }
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

// Exact mass of every tile, before any rank is matched: block g sums tiles
// tpb g .. tpb (g + 1) - 1 of the sorted weights (tpb <= kTilesPerBlock) and
// keeps, per tile, the exclusive prefix within the block (local[tile]) and the
// block's total.  Every weight is also checked: its scaled value m 2^(q - qmin)
// must fit in 127 bits, and so must every partial sum.
constexpr int kTilesPerBlock = 16;

__device__ __forceinline__ u128 add128_checked(u128 a, u128 b, bool& bad) {
    const u128 t = add128(a, b);
    bad |= t.hi < a.hi;
    return t;
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const float* __restrict__ w_sorted, long long n, Ctrl* ctrl,
                                                        u128* __restrict__ local, u128* __restrict__ block_tot,
                                                        long long n_tiles, int tpb) {
    __shared__ u128 s_wave[kTilesPerBlock][kScanWaves];
    __shared__ u128 s_tile[kTilesPerBlock];
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_bad = 0;
    const int qmin = ctrl->qmin;
    bool bad = false;
    // no barrier inside the loop: each wave keeps its sum per tile
#pragma unroll 2
    for (int k = 0; k < tpb; ++k) {
        const long long tile = (long long)blockIdx.x * tpb + k;
        const long long p0 = tile * kScanTile + (long long)tid * kPer;
        u128 sum = {0ull, 0ull};
        if (tile < n_tiles && p0 < n) {
            const float4* pw = reinterpret_cast<const float4*>(w_sorted + p0);
            float4 b4[kPer / 4];
#pragma unroll
            for (int q = 0; q < kPer / 4; ++q) b4[q] = pw[q];
#pragma unroll
            for (int q = 0; q < kPer / 4; ++q) {
                const float e[4] = {b4[q].x, b4[q].y, b4[q].z, b4[q].w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const unsigned b = __float_as_uint(e[c]);
                    const unsigned ex = (b >> 23) & 255u;
                    const unsigned m = (b & 0x7fffffu) | (ex ? 0x800000u : 0u);
                    const int sh = (ex == 0u ? 1 : (int)ex) - 150 - qmin;
                    bad |= sh < 0 || sh + (m ? 32 - __clz(m) : 0) > 127;
                    sum = add128_checked(sum, scaled_weight(e[c], qmin), bad);
                }
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            u128 w;
            w.lo = __shfl_xor(sum.lo, o, 64);
            w.hi = __shfl_xor(sum.hi, o, 64);
            sum = add128_checked(sum, w, bad);
        }
        if (lane == 0) s_wave[k][wave] = sum;
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid < tpb) {
        u128 t = {0ull, 0ull};
        bool b2 = false;
        for (int w = 0; w < kScanWaves; ++w) t = add128_checked(t, s_wave[tid][w], b2);
        s_tile[tid] = t;
        if (b2) s_bad = 1;
    }
    __syncthreads();
    if (tid == 0) {
        u128 running = {0ull, 0ull};
        bool b3 = false;
        for (int k = 0; k < tpb; ++k) {
            const long long tile = (long long)blockIdx.x * tpb + k;
            if (tile < n_tiles) local[tile] = running;
            running = add128_checked(running, s_tile[k], b3);
        }
        block_tot[blockIdx.x] = running;
        if (s_bad || b3) report_status(ctrl, AMBER_STATUS_RANGE);
    }
}

// Exclusive prefix of the block totals (one block of 1024 threads: a serial
// sum over each thread's chunk, a block-wide scan of the chunk sums, a serial
// pass writing the prefixes), the exact grand total C_N, and whether it needs
// more than 64 bits.
constexpr int kPrefixThreads = 1024;
__global__ __launch_bounds__(kPrefixThreads) void k_block_prefix(u128* __restrict__ block_tot, long long nb,
                                                                 Ctrl* ctrl) {
    __shared__ u128 s_wave[kPrefixThreads / 64];
    __shared__ int s_bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_bad = 0;
    const long long per = (nb + kPrefixThreads - 1) / kPrefixThreads;
    const long long b0 = (long long)tid * per;
    u128 sum = {0ull, 0ull};
    bool bad = false;
    for (long long b = b0; b < b0 + per && b < nb; ++b) sum = add128_checked(sum, block_tot[b], bad);
    // inclusive scan over the wave, then over the waves
    u128 inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const u128 o = shfl_up128(inc, d);
        if (lane >= d) inc = add128_checked(inc, o, bad);
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    u128 wave_excl = {0ull, 0ull};
    for (int w = 0; w < wave; ++w) wave_excl = add128_checked(wave_excl, s_wave[w], bad);
    u128 total = {0ull, 0ull};
    if (tid == kPrefixThreads - 1) total = add128_checked(wave_excl, inc, bad);
    u128 run = add128(wave_excl, inc);
    run = u128{run.lo - sum.lo, run.hi - sum.hi - (run.lo < sum.lo ? 1ull : 0ull)};  // exclusive
    for (long long b = b0; b < b0 + per && b < nb; ++b) {
        const u128 v = block_tot[b];
        block_tot[b] = run;
        run = add128(run, v);
    }
    if (bad) s_bad = 1;
    __syncthreads();
    if (tid == kPrefixThreads - 1) {
        ctrl->total_lo = total.lo;
        ctrl->total_hi = total.hi;
        ctrl->wide = total.hi != 0ull;
        if (s_bad || (total.hi >> 63)) report_status(ctrl, AMBER_STATUS_RANGE);
    }
}

// One block per tile of kScanTile consecutive ranks; thread t owns ranks
// 16 t .. 16 t + 15.
//  1. load cell indices and weights (16-byte vector loads); count the tile's
//     members of each cell-range bucket (bucket b = cells [b S, (b+1) S),
//     S = n / kL1) and scan the thread totals of the exact weights;
//  2. take the tile's slots in each bucket with one atomic add per bucket
//     (order inside a bucket does not matter); the tile's starting mass comes
//     from the tile prefixes computed beforehand;
//  3. F_n for the 16 ranks; the cell indices staged in LDS bucket by bucket,
//     each thread then takes slots tid + k kScanThreads, keeps their destinations
//     and writes the cells in runs;
//  4. per history: z_n (bracket from the closed-form guess, four ranks' table
//     reads in flight together), staged in the same LDS buffer and written to
//     the kept destinations.
// The launch runs the 64-bit variant when the exact total fits in 64 bits and
// the 128-bit one otherwise (the other variant's blocks return at once).
// fill[b] (cleared before the launch) counts the slots of bucket b handed out.
// With several histories the plain kernel is held to three waves per SIMD
// (168 registers, a few spilled): faster than two waves at 178 (at 1024^3
// with three histories 13.3 vs 16.7 ms) and than four at 128 (17.7 ms).  The
// growth kernel for one history runs at five (96 registers: 27.5 vs 28.3 ms
// at four; six was slower).
template <int NH, bool WIDE, bool GROWTH>
__global__ __launch_bounds__(kScanThreads, (NH > 1 && !GROWTH) ? 3 : ((NH == 1 && GROWTH) ? 5 : 1))
void k_scan_partition(
    const unsigned* __restrict__ perm, const float* __restrict__ w_sorted, long long n, Ctrl* ctrl,
    const u128* __restrict__ local, const u128* __restrict__ block_excl, unsigned* __restrict__ fill,
    int tpb, unsigned bucket_size, double bucket_rinv, HistArgs hs, unsigned* __restrict__ part_idx,
    float* __restrict__ part_z0, float* __restrict__ part_z1, float* __restrict__ part_z2) {
    using A = Acc<WIDE>;
    if ((ctrl->wide != 0) != WIDE) return;
    __shared__ A s_wave[kScanWaves];
    __shared__ unsigned lcnt[kL1];
    __shared__ unsigned loff[kL1];
    __shared__ unsigned gbase[kL1];
    __shared__ unsigned scan_sh[kL1 / 64];
    __shared__ unsigned stage[kScanTile];  // cells, then z of each history, in bucket order
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < kL1) lcnt[tid] = 0u;
    __syncthreads();
    const long long tile = blockIdx.x;
    const long long p0 = tile * kScanTile + (long long)tid * kPer;
    const bool ok = p0 < n;  // n is a multiple of 512: a thread's 16 ranks are all valid or all not
    const int qmin = ctrl->qmin;

    unsigned idx[kPer], rb[kPer];  // rb: bucket << 16 | rank inside the bucket, or ~0
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
        const unsigned b = live ? div_exact(idx[j], bucket_size, bucket_rinv) : 0u;
        rb[j] = live ? (b << 16) | atomicAdd(&lcnt[b], 1u) : 0xffffffffu;
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
    for (int w = 0; w < kScanWaves; ++w)
        if (w < wave) wave_excl = wave_excl + s_wave[w];

    // this tile's slots in every bucket
    unsigned cnt = 0, slot0 = 0;
    if (tid < kL1) {
        cnt = lcnt[tid];
        slot0 = cnt ? atomicAdd(&fill[tid], cnt) : 0u;
    }
    const unsigned lo = bucket_excl_scan<kL1>(cnt, scan_sh);
    if (tid < kL1) {
        loff[tid] = lo;
        gbase[tid] = (unsigned)tid * bucket_size + slot0;
    }
    __syncthreads();  // every bucket's loff and gbase are read below

    const u128 tile_excl = add128(block_excl[tile / tpb], local[tile]);
    A run = A::of128(tile_excl) + wave_excl + thread_excl;
    const u128 total = {ctrl->total_lo, ctrl->total_hi};
    const double tot = u128_to_f64(total);
    double cn[kPer];  // RN of the exact inclusive prefix of each rank
    unsigned pos[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const bool live = rb[j] != 0xffffffffu;
        if (live) run = run + A::of(wf[j], qmin);
        cn[j] = run.to_f64();
        pos[j] = live ? loff[rb[j] >> 16] + (rb[j] & 0xffffu) : 0xffffffffu;
        if (pos[j] >= (unsigned)kScanTile) pos[j] = 0xffffffffu;  // unreachable for consistent counts
        if (pos[j] != 0xffffffffu) stage[pos[j]] = idx[j];
    }
    __syncthreads();
    const long long valid_ll = n - tile * kScanTile;
    const int valid = valid_ll < kScanTile ? (int)valid_ll : kScanTile;
    // A thread's 16 ranks have nearly the same F, so one closed-form guess (at
    // the middle rank) and one read of the eight table nodes gl .. gl + 7
    // around it settle the bracket j = max{ j : X_j >= F } of every rank with
    // X_gl >= F > X_{gl+7}: j = gl + #{e in 1..6 : X_{gl+e} >= F}.  Other ranks
    // (the first ranks, where F grows fast relative to itself) walk exactly
    // from their own guess.  T >= 2^21.
    auto window = [&](const HistArg& H, long long& gl, double* x) {
        gl = guess_node(__ddiv_rn(cn[kPer / 2], tot), H) - 3;
        gl = gl < 0 ? 0 : (gl > H.T - 7 ? H.T - 7 : gl);
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = H.X[gl + e];
    };
    // z of the thread's ranks for one history
    const double unit = ldexp(1.0, -qmin);  // one cell in the units of the exact sums
    const double ns = (double)n * unit;
    auto z_of = [&](const HistArg& H, long long gl, const double* x, float* zf) {
#pragma clang fp contract(off)
        if constexpr (GROWTH) {
            if (H.XG) {
                // consecutive ranks nearly always share a bracket: the wave
                // brackets its first rank together, each rank first checks the
                // previous rank's bracket with the two nodes kept in registers
                // and searches (from that bracket) only when it has moved
                long long lo = wave_growth_bracket(__shfl((double)(p0 + 1) * unit, 0, 64), ns,
                                                   __shfl(cn[0], 0, 64), tot, H.T, H.XG);
                double2 nl, nh;  // (X, G) of nodes lo and lo + 1, clamped to [0, T]
                auto load_pair = [&](long long l) {
                    nl = H.XG[l < 0 ? 0 : (l > H.T ? H.T : l)];
                    nh = H.XG[l + 1 > H.T ? H.T : (l + 1 < 0 ? 0 : l + 1)];
                };
                load_pair(lo);
#pragma unroll
                for (int j = 0; j < kPer; ++j) {
                    zf[j] = 0.0f;
                    if (pos[j] == 0xffffffffu) continue;
                    const double ks = (double)(p0 + j + 1) * unit;
                    bool same;
                    if (lo < 0) {
                        same = growth_gap_sign(ks, ns, cn[j], tot, nl.y, nl.x) != 0;   // node 0: h_0 > 0
                    } else if (lo >= H.T) {
                        same = growth_gap_sign(ks, ns, cn[j], tot, nl.y, nl.x) == 0;   // node T: h_T <= 0
                    } else {
                        same = growth_gap_sign(ks, ns, cn[j], tot, nl.y, nl.x) == 0 &&
                               growth_gap_sign(ks, ns, cn[j], tot, nh.y, nh.x) != 0;
                    }
                    if (!same) {
                        lo = growth_bracket(ks, ns, cn[j], tot, H.T, H.XG, lo);
                        load_pair(lo);
                    }
                    zf[j] = (float)growth_z(lo, ks, ns, cn[j], tot, H.a, H.h, H.T, H.z_top, nl, nh);
                }
                return;
            }
        }
        // The middle rank's bracket and interpolation constants, once per
        // thread: a rank with X_jm >= F > X_jm+1 has exactly this bracket
        // (X is non-increasing), so only its own t needs computing.
        double xm0 = 0.0, xm1 = 0.0, zm = 0.0, denm = 0.0, dzm = 0.0;
        if (!H.XG) {
            const double fm = __ddiv_rn(cn[kPer / 2], tot);
            int km = 0;
#pragma unroll
            for (int e = 1; e < 7; ++e) km += (x[e] >= fm) ? 1 : 0;
            xm0 = x[0];
            xm1 = x[1];
#pragma unroll
            for (int e = 1; e < 7; ++e)
                if (km == e) {
                    xm0 = x[e];
                    xm1 = x[e + 1];
                }
            const long long jm = gl + km;
            zm = H.a + (double)jm * H.h;
            const double zm1 = H.a + (double)(jm + 1) * H.h;
            denm = xm0 - xm1;
            dzm = zm1 - zm;
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const double f = __ddiv_rn(cn[j], tot);  // F_n = RN(C_n) / RN(C_N)
            double z = 0.0;
            if (pos[j] != 0xffffffffu) {
                if (xm0 >= f && xm1 < f) {  // the same operations as interpolate_xy
                    const double t = (denm != 0.0) ? (xm0 - f) / denm : 0.0;
                    z = zm + t * dzm;
                    z = (z < H.z_top) ? z : H.z_top;
                } else if (x[0] >= f && x[7] < f) {
                    int kk = 0;
#pragma unroll
                    for (int e = 1; e < 7; ++e) kk += (x[e] >= f) ? 1 : 0;  // X non-increasing
                    double xj = x[0], xj1 = x[1];
#pragma unroll
                    for (int e = 1; e < 7; ++e)
                        if (kk == e) {
                            xj = x[e];
                            xj1 = x[e + 1];
                        }
                    z = interpolate_xy(f, gl + kk, xj, xj1, H.a, H.h, H.z_top);
                } else {
                    const long long jj = bracket_from(H.X, f, guess_node(f, H), H.T);
                    z = interpolate(H.X, f, jj, H.a, H.h, H.T, H.z_top);
                }
            }
            zf[j] = (float)z;
        }
    };
    // With one history its z is computed before any store is issued: a wait
    // for a load issued before stores that may or may not execute would also
    // wait for those stores.  (Several histories share one code path below,
    // which keeps the kernel's registers in check.)
    float zf0[kPer];
    if constexpr (NH == 1) {
        long long gl0 = 0;
        double x0[8] = {};
        if (!hs.h[0].XG) window(hs.h[0], gl0, x0);
        z_of(hs.h[0], gl0, x0, zf0);
    }

    unsigned dst[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int i = tid + k * kScanThreads;
        dst[k] = 0xffffffffu;
        if (i < valid) {
            const unsigned c = stage[i];
            if (c < (unsigned)n) {  // indices fit in 32 bits (n <= 2^30)
                const unsigned b = div_exact(c, bucket_size, bucket_rinv);
                const unsigned t = gbase[b] + ((unsigned)i - loff[b]);
                if (t < (unsigned)n) {  // always, for consistent counts
                    dst[k] = t;
                    part_idx[t] = c;
                }
            }
        }
    }
#pragma unroll 1
    for (int hh = 0; hh < NH; ++hh) {
        const HistArg& H = hs.h[hh];
        float* __restrict__ out = hh == 0 ? part_z0 : (hh == 1 ? part_z1 : part_z2);
        __syncthreads();  // the previous contents of the staging buffer are consumed
        if (NH == 1) {
#pragma unroll
            for (int j = 0; j < kPer; ++j)
                if (pos[j] != 0xffffffffu) stage[pos[j]] = __float_as_uint(zf0[j]);
        } else {
            long long gl = 0;
            double x[8] = {};
            float zf[kPer];
            if (!H.XG) window(H, gl, x);
            z_of(H, gl, x, zf);
#pragma unroll
            for (int j = 0; j < kPer; ++j)
                if (pos[j] != 0xffffffffu) stage[pos[j]] = __float_as_uint(zf[j]);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (dst[k] != 0xffffffffu) out[dst[k]] = __uint_as_float(stage[tid + k * kScanThreads]);
    }
}

// Second partition level, inside each first-level bucket: the pairs of bucket
// b (positions [b S1, (b+1) S1), cells of the same range) are split into kL2
// sub-buckets of S2 = S1 / kL2 cells.  Tiles never straddle buckets; each tile
// takes its slots in a sub-bucket with one atomic add on that sub-bucket's
// fill counter (order inside a sub-bucket does not matter).  A pair leaves
// with its cell's 16-bit offset inside the sub-bucket (S2 <= 16384): the
// sub-buckets tile the positions exactly as their cells tile the grid, so
// the position gives back the rest of the cell index.
// The z fields of up to kGroup histories that share one ranking.
struct ZSet {
    const float* in[kGroup];
    float* out[kGroup];
};

template <int NZ>
__global__ __launch_bounds__(kPartThreads) void k_partition2(const unsigned* __restrict__ in_idx, ZSet zs,
                                                         long long n, unsigned* __restrict__ fill, unsigned S1,
                                                         unsigned S2, double s2_rinv, unsigned tiles_per_bucket,
                                                         unsigned short* __restrict__ out_off) {
    __shared__ unsigned lcnt[kL2];
    __shared__ unsigned loff[kL2];
    __shared__ unsigned gbase[kL2];
    __shared__ unsigned scan_sh[kL2 / 64];
    __shared__ unsigned stage[kPartTile];  // cells, then z, in sub-bucket order
    const int tid = threadIdx.x;
    if (tid < kL2) lcnt[tid] = 0u;
    __syncthreads();
    // Blocks are dealt to the 8 XCDs round robin; block 8 j + x takes tile j
    // of XCD x's share, the tiles of buckets x, x + 8, ... in order, so each
    // bucket's runs (which meet inside cache lines in every sub-bucket) are
    // written from one L2.  No tile waits on another.
    const unsigned n_buckets = gridDim.x / tiles_per_bucket;
    unsigned b, k;
    if ((n_buckets & 7u) == 0u) {
        const unsigned x = blockIdx.x & 7u, j = blockIdx.x >> 3;
        b = x + 8u * (j / tiles_per_bucket);
        k = j % tiles_per_bucket;
    } else {
        b = blockIdx.x / tiles_per_bucket;
        k = blockIdx.x % tiles_per_bucket;
    }
    // cell and pair indices fit in 32 bits (n <= 2^30)
    const unsigned bstart = b * S1;
    const unsigned t0 = bstart + k * (unsigned)kPartTile;
    const unsigned t1 = t0 + kPartTile < bstart + S1 ? t0 + kPartTile : bstart + S1;
    const int valid = (int)(t1 - t0);
    unsigned idx[kPer], rb[kPer];
    // every load in flight before any is used: no branch around a load (the
    // last tile of a bucket clamps its positions instead)
    const unsigned lastv = (unsigned)valid - 1u;
    auto at_of = [&](int j) -> unsigned {
        const unsigned i = (unsigned)(j * kPartThreads + tid);
        return t0 + (valid == kPartTile ? i : (i < lastv ? i : lastv));
    };
    float z[kPer];  // the first history's z, loaded with the cells
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const unsigned at = at_of(j);
        idx[j] = in_idx[at];
        z[j] = zs.in[0][at];
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = j * kPartThreads + tid;
        const unsigned rel = idx[j] - bstart;  // wraps above S1 when idx < bstart
        const bool live = i < valid && rel < S1;
        const unsigned sb = live ? div_exact(rel, S2, s2_rinv) : 0u;
        rb[j] = live ? (sb << 16) | atomicAdd(&lcnt[sb], 1u) : 0xffffffffu;
    }
    __syncthreads();
    unsigned cnt = 0, slot0 = 0;
    if (tid < kL2) {
        cnt = lcnt[tid];
        slot0 = cnt ? atomicAdd(&fill[(long long)b * kL2 + tid], cnt) : 0u;
    }
    const unsigned lo = bucket_excl_scan<kL2>(cnt, scan_sh);
    if (tid < kL2) {
        loff[tid] = lo;
        gbase[tid] = bstart + (unsigned)tid * S2 + slot0;
    }
    __syncthreads();
    unsigned pos[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        pos[j] = rb[j] != 0xffffffffu ? loff[rb[j] >> 16] + (rb[j] & 0xffffu) : 0xffffffffu;
        if (pos[j] >= (unsigned)kPartTile) pos[j] = 0xffffffffu;  // unreachable for consistent counts
        if (pos[j] != 0xffffffffu) stage[pos[j]] = idx[j];
    }
    __syncthreads();
    unsigned dst[kPer];
#pragma unroll
    for (int kk = 0; kk < kPer; ++kk) {
        const int i = tid + kk * kPartThreads;
        dst[kk] = 0xffffffffu;
        if (i < valid) {
            const unsigned c = stage[i];
            const unsigned rel = c - bstart;
            if (rel < S1) {
                const unsigned s2 = div_exact(rel, S2, s2_rinv);
                const unsigned t = gbase[s2] + ((unsigned)i - loff[s2]);
                if (t < (unsigned)n) {
                    dst[kk] = t;
                    out_off[t] = (unsigned short)(rel - s2 * S2);  // < S2 <= 16384
                }
            }
        }
    }
#pragma unroll 1
    for (int h = 0; h < NZ; ++h) {
        if (h > 0) {  // the next history's z, all loads in flight together
#pragma unroll
            for (int j = 0; j < kPer; ++j) z[j] = zs.in[h][at_of(j)];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (pos[j] != 0xffffffffu) stage[pos[j]] = __float_as_uint(z[j]);
        __syncthreads();
        float* __restrict__ oz = zs.out[h];
#pragma unroll
        for (int kk = 0; kk < kPer; ++kk)
            if (dst[kk] != 0xffffffffu) oz[dst[kk]] = __uint_as_float(stage[tid + kk * kPartThreads]);
    }
}

// Last level: block L owns cells [L S, (L+1) S) (S <= 16384, a whole number of
// the previous level's ranges, whose pairs sit at exactly the positions of
// their cells) and the pairs at positions [L S, (L+1) S); it places z by cell
// in LDS and writes the run of z_re contiguously, for each of NZ histories
// whose pairs share the same cells and positions.  OFF16: the pairs carry
// their cell's offset inside its range of R cells (the second level's
// sub-buckets), so pair i of the block belongs to cell floor(i/R) R + offset;
// otherwise they carry the cell index.
constexpr int kLeafMax = 16384;
constexpr int kLeafThreads = 1024;
template <bool OFF16, int NZ>
__global__ __launch_bounds__(kLeafThreads) void k_leaf_scatter(const void* __restrict__ in_cell, ZSet zs, long long n,
                                                               unsigned S, unsigned R, double r_rinv) {
    constexpr int kR = kLeafMax / kLeafThreads;
    __shared__ float zl[kLeafMax];
    const long long start = (long long)blockIdx.x * S;
    const long long left = n - start;
    const unsigned valid = left < (long long)S ? (unsigned)left : S;
    unsigned rel[kR];  // the pair's cell relative to start, or ~0 (none)
    float z[kR];
    // every load in flight before any is used (clamped positions, no branch)
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const unsigned i = threadIdx.x + r * kLeafThreads;
        const long long at = start + (i < valid ? i : 0u);
        long long c;
        if (OFF16) {
            c = (long long)div_exact(i, R, r_rinv) * R + reinterpret_cast<const unsigned short*>(in_cell)[at];
        } else {
            c = (long long)reinterpret_cast<const unsigned*>(in_cell)[at] - start;
        }
        rel[r] = (i < valid && c >= 0 && c < (long long)valid) ? (unsigned)c : 0xffffffffu;
        z[r] = zs.in[0][at];
    }
#pragma unroll 1
    for (int h = 0; h < NZ; ++h) {
        if (h > 0) {
            __syncthreads();  // the previous history's run is written out
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const unsigned i = threadIdx.x + r * kLeafThreads;
                z[r] = zs.in[h][start + (i < valid ? i : 0u)];
            }
        }
#pragma unroll
        for (int r = 0; r < kR; ++r)
            if (rel[r] != 0xffffffffu) zl[rel[r]] = z[r];
        __syncthreads();
        float* __restrict__ out = zs.out[h];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const unsigned i = threadIdx.x + r * kLeafThreads;
            if (i < valid) out[start + i] = zl[i];
        }
    }
}

__global__ __launch_bounds__(256) void k_clear(unsigned* __restrict__ p, long long words) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < words; i += (long long)gridDim.x * 256)
        p[i] = 0u;
}

}  // namespace

int match_scan(const amber_plan_s* p, const amber_weibull* hist, int n_hist, float* const* d_zre, unsigned char* ws,
               const WsLayout& L, hipStream_t s) {
    const long long n = (long long)p->n * p->n * p->n;
    const long long n_tiles = (n + kScanTile - 1) / kScanTile;
    // tiles per tile-sum block: up to kTilesPerBlock, fewer when that would
    // leave the device short of blocks
    const int sum_tpb = (int)std::max(1LL, std::min((long long)kTilesPerBlock, n_tiles / 1024));
    const long long n_blocks = (n_tiles + sum_tpb - 1) / sum_tpb;
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
    unsigned short* p2_off = reinterpret_cast<unsigned short*>(ws + L.part2[0]);
    float* p2_z = reinterpret_cast<float*>(ws + L.part2[1]);
    const unsigned S1 = (unsigned)(n / kL1);  // n is a multiple of 512
    const bool two_level = S1 > (unsigned)kLeafMax;
    const unsigned S2 = two_level ? S1 / kL2 : S1;  // divides exactly for the supported sizes
    const unsigned tpb = (S1 + kPartTile - 1) / kPartTile;
    const double s2_rinv = 1.0 / (double)S2;
    // leaf blocks take whole ranges of the last level, up to kLeafMax cells
    const unsigned leaf = S2 * (unsigned)(kLeafMax / S2);
    const unsigned leaf_blocks = (unsigned)((n + leaf - 1) / leaf);
    const dim3 grid((unsigned)n_tiles), blk(kScanThreads);

    AMBER_LAUNCH(p, "match_tile_sums", k_tile_sums, dim3((unsigned)n_blocks), blk, s, w_sorted, n, ctrl, local,
                 block_excl, n_tiles, sum_tpb);
    AMBER_LAUNCH(p, "match_block_prefix", k_block_prefix, dim3(1), dim3(kPrefixThreads), s, block_excl, n_blocks, ctrl);
    const double rinv = 1.0 / (double)S1;
    // Groups of up to kGroup histories, the short one first: after the last
    // group's scan the rank order and sorted weights are no longer needed, so
    // their buffers hold that group's second-level z fields and its histories
    // share one second-level pass and one leaf pass.
    const int first = (n_hist % kGroup) ? n_hist % kGroup : kGroup;
    for (int g = 0, h0 = 0; h0 < n_hist; h0 += (g == 0 ? first : kGroup), ++g) {
        HistArgs hs{};
        hs.n = g == 0 ? first : kGroup;
        const bool last = h0 + hs.n == n_hist;
        for (int i = 0; i < hs.n; ++i) {
            const amber_weibull& w = hist[h0 + i];
            hs.h[i] = HistArg{w.a_w, w.b_w, 1.0 / w.c_w, w.h, w.z_top, (long long)(w.table_n - 1), w.d_table,
                              reinterpret_cast<const double2*>(w.d_growth), d_zre[h0 + i]};
        }
        if (g > 0) AMBER_LAUNCH(p, "match_clear", k_clear, dim3(1), dim3(256), s, fill1, kL1);
        bool growth = false;  // the growth inversion lives in its own kernels (it needs more registers)
        for (int i = 0; i < hs.n; ++i) growth |= hs.h[i].XG != nullptr;
#define AMBER_SCAN(NHV, GR)                                                                                       \
    AMBER_LAUNCH(p, "match_scan_partition", (k_scan_partition<NHV, false, GR>), grid, blk, s, perm, w_sorted, n,  \
                 ctrl, local, block_excl, fill1, sum_tpb, S1, rinv, hs, p1_idx, p1_z[0], p1_z[1], p1_z[2]);       \
    AMBER_LAUNCH(p, "match_scan_partition_wide", (k_scan_partition<NHV, true, GR>), grid, blk, s, perm, w_sorted, \
                 n, ctrl, local, block_excl, fill1, sum_tpb, S1, rinv, hs, p1_idx, p1_z[0], p1_z[1], p1_z[2]);
        switch (hs.n + (growth ? 3 : 0)) {
            case 1: AMBER_SCAN(1, false) break;
            case 2: AMBER_SCAN(2, false) break;
            case 3: AMBER_SCAN(3, false) break;
            case 4: AMBER_SCAN(1, true) break;
            case 5: AMBER_SCAN(2, true) break;
            default: AMBER_SCAN(3, true) break;
        }
#undef AMBER_SCAN
        // the group's z fields in (first level) and out (second level / z_re)
        auto zset = [&](int i0, int cnt, float* const* mid) {
            ZSet z{};
            for (int i = 0; i < cnt; ++i) {
                z.in[i] = mid ? mid[i] : p1_z[i0 + i];
                z.out[i] = mid ? mid[i] : d_zre[h0 + i0 + i];
            }
            return z;
        };
        auto second_level = [&](int nz, const ZSet& z) {
            AMBER_LAUNCH(p, "match_clear", k_clear, dim3(256), dim3(256), s, fill2, 65536);
            switch (nz) {
                case 1: AMBER_LAUNCH(p, "match_partition2", k_partition2<1>, dim3(kL1 * tpb), dim3(kPartThreads), s,
                                     p1_idx, z, n, fill2, S1, S2, s2_rinv, tpb, p2_off); break;
                case 2: AMBER_LAUNCH(p, "match_partition2", k_partition2<2>, dim3(kL1 * tpb), dim3(kPartThreads), s,
                                     p1_idx, z, n, fill2, S1, S2, s2_rinv, tpb, p2_off); break;
                default: AMBER_LAUNCH(p, "match_partition2", k_partition2<3>, dim3(kL1 * tpb), dim3(kPartThreads), s,
                                      p1_idx, z, n, fill2, S1, S2, s2_rinv, tpb, p2_off); break;
            }
        };
        auto leaf_pass = [&](bool off16, const void* cells, int nz, const ZSet& z) {
#define AMBER_LEAF(O, NZV)                                                                                             AMBER_LAUNCH(p, "match_leaf_scatter", (k_leaf_scatter<O, NZV>), dim3(leaf_blocks), dim3(kLeafThreads), s, cells,                  z, n, leaf, S2, s2_rinv)
            if (off16) {
                if (nz == 1) AMBER_LEAF(true, 1); else if (nz == 2) AMBER_LEAF(true, 2); else AMBER_LEAF(true, 3);
            } else {
                if (nz == 1) AMBER_LEAF(false, 1); else if (nz == 2) AMBER_LEAF(false, 2); else AMBER_LEAF(false, 3);
            }
#undef AMBER_LEAF
        };
        if (!two_level) {
            leaf_pass(false, p1_idx, hs.n, zset(0, hs.n, nullptr));
        } else if (last && hs.n > 1) {
            float* mid[kGroup] = {p2_z, reinterpret_cast<float*>(ws + L.vals[0]), reinterpret_cast<float*>(ws + L.wts[0])};
            ZSet z2 = zset(0, hs.n, nullptr);  // first level in, second level out
            ZSet zl = zset(0, hs.n, nullptr);  // second level in, z_re out
            for (int i = 0; i < hs.n; ++i) {
                z2.out[i] = mid[i];
                zl.in[i] = mid[i];
            }
            second_level(hs.n, z2);
            leaf_pass(true, p2_off, hs.n, zl);
        } else {
            for (int i = 0; i < hs.n; ++i) {
                ZSet z2{}, zl{};
                z2.in[0] = p1_z[i];
                z2.out[0] = p2_z;
                zl.in[0] = p2_z;
                zl.out[0] = d_zre[h0 + i];
                second_level(1, z2);
                leaf_pass(true, p2_off, 1, zl);
            }
        }
    }
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}
