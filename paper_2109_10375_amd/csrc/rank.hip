// Rank order for abundance matching on gfx950 (Sec. 3.4.2: "ranked in
// descending order"): a stable least-significant-digit radix sort of
// (key, cell index[, weight]) with 8-bit digits, one streaming pass per digit.
//
// Keys: FP32 intensity -> uint32 whose ascending order is the descending order
// of the intensity (-0 folded onto +0).  The input is read in cell-index order
// and every pass is stable, so equal intensities keep ascending cell index.
//
// Each pass ("onesweep"): a block takes the next 4096-key tile from a ticket
// counter, ranks its keys by digit with 64-lane ballots (the lanes that share a
// digit find each other with 8 ballots; the lowest of them bumps the wave's LDS
// counter), publishes its per-digit counts for later tiles and looks back over
// earlier tiles' published counts (decoupled look-back) to find where its
// digits start globally, then writes its keys digit by digit through LDS so
// that each digit's run is stored contiguously.  Tiles only wait on tiles that
// took earlier tickets, which are already running, so every wait ends.
#include <algorithm>

#include "internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kKeysPerThread = 16;
constexpr int kTile = kThreads * kKeysPerThread;  // 4096
constexpr unsigned kFlagAgg = 1u << 30;
constexpr unsigned kFlagPre = 2u << 30;
constexpr unsigned kValMask = (1u << 30) - 1;

__device__ __forceinline__ unsigned desc_key(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) == 0u) u = 0u;  // -0 == +0
    const unsigned asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ~asc;
}

__device__ __forceinline__ bool is_nan_bits(unsigned u) { return (u & 0x7fffffffu) > 0x7f800000u; }

__device__ __forceinline__ unsigned ld_acquire(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive block-wide scan of one unsigned per thread (256 threads).
__device__ __forceinline__ unsigned block_incl_scan(unsigned v, unsigned* sh /* kWaves */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        unsigned o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    if (lane == 63) sh[wave] = v;
    __syncthreads();
    unsigned add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
        if (w < wave) add += sh[w];
    __syncthreads();
    return v + add;
}

// Clears the control block and the first look-back buffer, counts the four
// digit histograms of the keys (read once), and flags NaN intensities.
__global__ __launch_bounds__(kThreads) void k_hist(const float* __restrict__ J, long long n, Ctrl* ctrl,
                                                   unsigned* __restrict__ lb0, long long lb_words) {
    __shared__ unsigned h[kWaves][4][256];
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kWaves * 4 * 256; i += kThreads) (&h[0][0][0])[i] = 0;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < lb_words; i += (long long)gridDim.x * kThreads)
        lb0[i] = 0;
    __syncthreads();
    bool nan = false;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const float f = J[i];
        nan |= is_nan_bits(__float_as_uint(f));
        const unsigned k = desc_key(f);
        atomicAdd(&h[wave][0][k & 255u], 1u);
        atomicAdd(&h[wave][1][(k >> 8) & 255u], 1u);
        atomicAdd(&h[wave][2][(k >> 16) & 255u], 1u);
        atomicAdd(&h[wave][3][k >> 24], 1u);
    }
    if (__any(nan) && (threadIdx.x & 63) == 0) atomicOr(&ctrl->status, AMBER_STATUS_NAN_J);
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * 256; i += kThreads) {
        unsigned s = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) s += (&h[w][0][0])[i];
        if (s) atomicAdd(&ctrl->hist[0][0] + i, s);
    }
}

__global__ void k_ctrl_init(Ctrl* ctrl) {
    unsigned* p = reinterpret_cast<unsigned*>(ctrl);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 4); i += blockDim.x) p[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) ctrl->qmin = 0x7fffffff;
}

// Exclusive prefix of each digit histogram: where each digit's run starts.
__global__ __launch_bounds__(kThreads) void k_digit_offsets(Ctrl* ctrl) {
    __shared__ unsigned sh[kWaves];
    for (int d = 0; d < 4; ++d) {
        const unsigned v = ctrl->hist[d][threadIdx.x];
        const unsigned inc = block_incl_scan(v, sh);
        ctrl->digit_off[d][threadIdx.x] = inc - v;
    }
}

// Decomposition of a positive finite FP32 weight as m 2^q, q the exponent of
// its unit in the last place (q = -149 for subnormals).
__device__ __forceinline__ int weight_q(unsigned bits) {
    const int e = (int)((bits >> 23) & 255u);
    return (e == 0 ? 1 : e) - 150;
}

// One digit pass.  FIRST: keys come from J and the index is the position.
// LAST: only the values (and weights) are written.  CARRY: weights travel with
// the keys; pass 0 also checks them and finds the smallest ulp exponent, pass 1
// (when SUMW) writes each tile's exact weight sum for the matching total.
template <bool FIRST, bool LAST, bool CARRY>
__global__ __launch_bounds__(kThreads) void k_onesweep(
    const float* __restrict__ J, const unsigned* __restrict__ keys_in, const unsigned* __restrict__ vals_in,
    const float* __restrict__ w_in, unsigned* __restrict__ keys_out, unsigned* __restrict__ vals_out,
    float* __restrict__ w_out, unsigned* __restrict__ lb, unsigned* __restrict__ lb_next,
    unsigned long long* __restrict__ tile_sums, Ctrl* ctrl, int pass, long long n) {
    __shared__ unsigned s_tile;
    __shared__ unsigned wcnt[kWaves][256];
    __shared__ unsigned loff[256];
    __shared__ unsigned gbase[256];
    __shared__ unsigned scan_sh[kWaves];
    __shared__ unsigned st_key[kTile];
    __shared__ unsigned st_val[kTile];
    __shared__ float st_w[CARRY ? kTile : 1];
    __shared__ int s_qmin[kWaves];
    __shared__ unsigned long long s_sum[kWaves][2];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(&ctrl->tickets[pass], 1u);
    for (int i = tid; i < kWaves * 256; i += kThreads) (&wcnt[0][0])[i] = 0u;
    __syncthreads();
    const unsigned tile = s_tile;
    const long long tile_base = (long long)tile * kTile;
    const int shift = 8 * pass;

    // The next pass's look-back entry for this tile starts cleared.
    if (lb_next) lb_next[(long long)tile * 256 + tid] = 0u;

    unsigned key[kKeysPerThread], val[kKeysPerThread], lrank[kKeysPerThread];
    float wt[kKeysPerThread];
    bool bad_w = false;
    int qmin = 0x7fffffff;
    const long long wbase = tile_base + (long long)wave * (64 * kKeysPerThread);
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        const long long pos = wbase + 64 * j + lane;
        const bool ok = pos < n;
        if (FIRST) {
            key[j] = ok ? desc_key(J[pos]) : 0xffffffffu;
            val[j] = (unsigned)pos;
        } else {
            key[j] = ok ? keys_in[pos] : 0xffffffffu;
            val[j] = ok ? vals_in[pos] : 0u;
        }
        if (CARRY) {
            wt[j] = ok ? w_in[pos] : 1.0f;
            if (FIRST && ok) {
                const unsigned b = __float_as_uint(wt[j]);
                const bool good = (b - 1u) < 0x7f7fffffu;  // 0 < w < inf, not NaN
                bad_w |= !good;
                const int q = weight_q(b);
                qmin = q < qmin ? q : qmin;
            }
        }
    }

    // Rank each key among the wave's keys with the same digit, in input order.
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        const bool ok = (wbase + 64 * j + lane) < n;
        const unsigned d = (key[j] >> shift) & 255u;
        unsigned long long peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        unsigned r = 0;
        if (ok) {
            const unsigned before = (unsigned)__popcll(peers & lt);
            const unsigned cnt = (unsigned)__popcll(peers);
            const unsigned old = wcnt[wave][d];
            r = old + before;
            if (before == 0) wcnt[wave][d] = old + cnt;  // lowest peer updates
        }
        lrank[j] = r;
    }
    __syncthreads();

    // Per digit: wave offsets, tile count, look-back, tile-local start.
    const int d = tid;
    const unsigned c0 = wcnt[0][d], c1 = wcnt[1][d], c2 = wcnt[2][d], c3 = wcnt[3][d];
    const unsigned tcnt = c0 + c1 + c2 + c3;
    {
        unsigned* me = lb + (long long)tile * 256 + d;
        if (tile == 0) {
            st_release(me, kFlagPre | tcnt);
            gbase[d] = ctrl->digit_off[pass][d];
        } else {
            st_release(me, kFlagAgg | tcnt);
            unsigned excl = 0;
            long long t = (long long)tile - 1;
            while (true) {
                const unsigned v = ld_acquire(lb + t * 256 + d);
                const unsigned f = v & ~kValMask;
                if (f == 0u) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += v & kValMask;
                if (f == kFlagPre) break;
                --t;
            }
            st_release(me, kFlagPre | (excl + tcnt));
            gbase[d] = ctrl->digit_off[pass][d] + excl;
        }
    }
    const unsigned incl = block_incl_scan(tcnt, scan_sh);
    loff[d] = incl - tcnt;
    wcnt[0][d] = 0;
    wcnt[1][d] = c0;
    wcnt[2][d] = c0 + c1;
    wcnt[3][d] = c0 + c1 + c2;
    // block-level reductions of the weight checks (pass 0)
    if (CARRY && FIRST) {
        int q = qmin;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int oq = __shfl_xor(q, o, 64);
            q = oq < q ? oq : q;
        }
        if (lane == 0) s_qmin[wave] = q;
        if (__any(bad_w) && lane == 0) atomicOr(&ctrl->status, AMBER_STATUS_BAD_W);
    }
    __syncthreads();
    if (CARRY && FIRST && tid == 0) {
        int q = s_qmin[0];
        for (int w = 1; w < kWaves; ++w) q = s_qmin[w] < q ? s_qmin[w] : q;
        if (q < __hip_atomic_load(&ctrl->qmin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(&ctrl->qmin, q);
    }

    // Stage the tile in digit order in LDS.
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        const bool ok = (wbase + 64 * j + lane) < n;
        if (ok) {
            const unsigned dd = (key[j] >> shift) & 255u;
            const unsigned p = loff[dd] + wcnt[wave][dd] + lrank[j];
            if (p >= (unsigned)kTile) continue;  // unreachable for consistent counts
            st_key[p] = key[j];
            st_val[p] = val[j];
            if (CARRY) st_w[p] = wt[j];
        }
    }
    __syncthreads();

    // Write out: consecutive threads write consecutive slots of a digit run.
    const long long valid_ll = n - tile_base;
    const int valid = valid_ll < kTile ? (int)valid_ll : kTile;
#pragma unroll 4
    for (int i = tid; i < valid; i += kThreads) {
        const unsigned k = st_key[i];
        const unsigned dd = (k >> shift) & 255u;
        const long long dst = (long long)gbase[dd] + (i - (int)loff[dd]);
        if (dst < 0 || dst >= n) continue;  // unreachable for consistent counts
        if (!LAST) keys_out[dst] = k;
        vals_out[dst] = st_val[i];
        if (CARRY) w_out[dst] = st_w[i];
    }

    // Pass 1 of a matching sort: exact tile sum of the weights, w 2^-qmin
    // (qmin is final once pass 0 has completed).
    if (CARRY && tile_sums) {
        const int qm = ctrl->qmin;
        unsigned long long lo = 0, hi = 0;
        bool ovf = false;
#pragma unroll
        for (int j = 0; j < kKeysPerThread; ++j) {
            const bool ok = (wbase + 64 * j + lane) < n;
            if (!ok) continue;
            const unsigned b = __float_as_uint(wt[j]);
            const unsigned long long m = (unsigned long long)((b & 0x7fffffu) | ((b >> 23) & 255u ? 0x800000u : 0u));
            const int sh = weight_q(b) - qm;  // >= 0 for valid weights
            unsigned long long tlo, thi;
            if (sh >= 128 || sh < 0) {
                tlo = 0; thi = 0;  // out of range: reported by k_range
            } else if (sh >= 64) {
                tlo = 0; thi = m << (sh - 64);
            } else if (sh == 0) {
                tlo = m; thi = 0;
            } else {
                tlo = m << sh; thi = m >> (64 - sh);
            }
            const unsigned long long nlo = lo + tlo;
            const unsigned long long nhi = hi + thi + (nlo < lo ? 1ull : 0ull);
            ovf |= nhi < hi;
            lo = nlo;
            hi = nhi;
        }
        // wave reduce (128-bit)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long olo = __shfl_xor(lo, o, 64);
            const unsigned long long ohi = __shfl_xor(hi, o, 64);
            const unsigned long long nlo = lo + olo;
            const unsigned long long nhi = hi + ohi + (nlo < lo ? 1ull : 0ull);
            ovf |= nhi < hi;
            lo = nlo;
            hi = nhi;
        }
        if (__any(ovf) && lane == 0) atomicOr(&ctrl->status, AMBER_STATUS_RANGE);
        if (lane == 0) {
            s_sum[wave][0] = lo;
            s_sum[wave][1] = hi;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long a = 0, b = 0;
            bool ov = false;
            for (int w = 0; w < kWaves; ++w) {
                const unsigned long long nlo = a + s_sum[w][0];
                const unsigned long long nb = b + s_sum[w][1] + (nlo < a ? 1ull : 0ull);
                ov |= nb < b;
                a = nlo;
                b = nb;
            }
            if (ov) atomicOr(&ctrl->status, AMBER_STATUS_RANGE);
            tile_sums[2 * (long long)tile] = a;
            tile_sums[2 * (long long)tile + 1] = b;
        }
    }
}

// Sum of the tile sums -> exact total (must stay below 2^127) and width flag.
__global__ __launch_bounds__(kThreads) void k_total(const unsigned long long* __restrict__ tile_sums, long long n_tiles,
                                                    Ctrl* ctrl) {
    __shared__ unsigned long long s[kThreads][2];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    unsigned long long lo = 0, hi = 0;
    bool bad = false;
    for (long long t = threadIdx.x; t < n_tiles; t += kThreads) {
        const unsigned long long a = tile_sums[2 * t], b = tile_sums[2 * t + 1];
        const unsigned long long nlo = lo + a;
        const unsigned long long nhi = hi + b + (nlo < lo ? 1ull : 0ull);
        bad |= nhi < hi;
        lo = nlo;
        hi = nhi;
    }
    s[threadIdx.x][0] = lo;
    s[threadIdx.x][1] = hi;
    if (bad) s_bad = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0;
        bool ov = s_bad != 0;
        for (int i = 0; i < kThreads; ++i) {
            const unsigned long long nlo = a + s[i][0];
            const unsigned long long nb = b + s[i][1] + (nlo < a ? 1ull : 0ull);
            ov |= nb < b;
            a = nlo;
            b = nb;
        }
        ov |= (b >> 63) != 0ull;
        ctrl->total_lo = a;
        ctrl->total_hi = b;
        ctrl->wide = (b != 0ull);
        if (ov) atomicOr(&ctrl->status, AMBER_STATUS_RANGE);
    }
}

// Flags weights whose scaled value m 2^(q - qmin) would need 128 bits or more.
__global__ __launch_bounds__(kThreads) void k_range(const float* __restrict__ w, long long n, Ctrl* ctrl) {
    const int qm = ctrl->qmin;
    bool bad = false;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads) {
        const unsigned b = __float_as_uint(w[i]);
        const unsigned m = (b & 0x7fffffu) | (((b >> 23) & 255u) ? 0x800000u : 0u);
        const int bits = m ? 32 - __clz(m) : 0;
        bad |= (weight_q(b) - qm) + bits > 127;
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&ctrl->status, AMBER_STATUS_RANGE);
}

}  // namespace

int rank_sort(const amber_plan_s* p, const float* d_J, const float* d_w, unsigned char* ws, const WsLayout& L,
              hipStream_t s, int carry, uint32_t* d_perm_out) {
    const long long n = (long long)p->n * p->n * p->n;
    const long long n_tiles = (n + kTile - 1) / kTile;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
    unsigned* keys[2] = {reinterpret_cast<unsigned*>(ws + L.keys[0]), reinterpret_cast<unsigned*>(ws + L.keys[1])};
    unsigned* vals[2] = {reinterpret_cast<unsigned*>(ws + L.vals[0]), reinterpret_cast<unsigned*>(ws + L.vals[1])};
    float* wts[2] = {reinterpret_cast<float*>(ws + L.wts[0]), reinterpret_cast<float*>(ws + L.wts[1])};
    unsigned* lb[2] = {reinterpret_cast<unsigned*>(ws + L.lookback),
                       reinterpret_cast<unsigned*>(ws + L.lookback) + n_tiles * 256};
    unsigned long long* tile_sums =
        reinterpret_cast<unsigned long long*>(ws + L.lookback + (size_t)n_tiles * 256 * 4 * 2);

    AMBER_LAUNCH(p, "rank_init", k_ctrl_init, dim3(1), dim3(256), s, ctrl);
    const unsigned hist_blocks = (unsigned)std::min<long long>(2048, (n + kThreads * 16 - 1) / (kThreads * 16));
    AMBER_LAUNCH(p, "rank_hist", k_hist, dim3(hist_blocks), dim3(kThreads), s, d_J, n, ctrl, lb[0], n_tiles * 256);
    AMBER_LAUNCH(p, "rank_digit_offsets", k_digit_offsets, dim3(1), dim3(kThreads), s, ctrl);
    const dim3 grid((unsigned)n_tiles), blk(kThreads);
    // pass 0: J, w -> buffers 1; pass 1: 1 -> 0; pass 2: 0 -> 1; pass 3: 1 -> 0 (values, weights)
    uint32_t* final_vals = d_perm_out ? d_perm_out : vals[0];
    if (carry) {
        AMBER_LAUNCH(p, "rank_pass0", (k_onesweep<true, false, true>), grid, blk, s, d_J, nullptr, nullptr, d_w, keys[1],
                           vals[1], wts[1], lb[0], lb[1], nullptr, ctrl, 0, n);
        AMBER_LAUNCH(p, "rank_pass1", (k_onesweep<false, false, true>), grid, blk, s, nullptr, keys[1], vals[1], wts[1],
                           keys[0], vals[0], wts[0], lb[1], lb[0], tile_sums, ctrl, 1, n);
        AMBER_LAUNCH(p, "rank_pass2", (k_onesweep<false, false, true>), grid, blk, s, nullptr, keys[0], vals[0], wts[0],
                           keys[1], vals[1], wts[1], lb[0], lb[1], nullptr, ctrl, 2, n);
        AMBER_LAUNCH(p, "rank_pass3", (k_onesweep<false, true, true>), grid, blk, s, nullptr, keys[1], vals[1], wts[1],
                           nullptr, final_vals, wts[0], lb[1], lb[0], nullptr, ctrl, 3, n);
        AMBER_LAUNCH(p, "match_total", k_total, dim3(1), dim3(kThreads), s, tile_sums, n_tiles, ctrl);
        const unsigned rb = (unsigned)std::min<long long>(1024, (n + kThreads * 16 - 1) / (kThreads * 16));
        AMBER_LAUNCH(p, "match_range", k_range, dim3(rb), dim3(kThreads), s, wts[0], n, ctrl);
    } else {
        AMBER_LAUNCH(p, "rank_pass0", (k_onesweep<true, false, false>), grid, blk, s, d_J, nullptr, nullptr, nullptr, keys[1],
                           vals[1], nullptr, lb[0], lb[1], nullptr, ctrl, 0, n);
        AMBER_LAUNCH(p, "rank_pass1", (k_onesweep<false, false, false>), grid, blk, s, nullptr, keys[1], vals[1], nullptr,
                           keys[0], vals[0], nullptr, lb[1], lb[0], nullptr, ctrl, 1, n);
        AMBER_LAUNCH(p, "rank_pass2", (k_onesweep<false, false, false>), grid, blk, s, nullptr, keys[0], vals[0], nullptr,
                           keys[1], vals[1], nullptr, lb[0], lb[1], nullptr, ctrl, 2, n);
        AMBER_LAUNCH(p, "rank_pass3", (k_onesweep<false, true, false>), grid, blk, s, nullptr, keys[1], vals[1], nullptr,
                           nullptr, final_vals, nullptr, lb[1], lb[0], nullptr, ctrl, 3, n);
    }
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}
