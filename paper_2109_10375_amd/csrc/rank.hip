// Rank order for abundance matching on gfx950 (Sec. 3.4.2: cells ordered by
// intensity, highest first): a stable least-significant-digit radix sort of
// (key, cell index[, weight]) with 8-bit digits, one streaming pass per digit.
// A pass writes only the key bits later passes still read: all 32 after the
// first digit, the top 16 after the second, the top 8 after the third.
//
// Keys: FP32 intensity -> uint32 whose ascending order is the descending order
// of the intensity (-0 folded onto +0).  The input is read in cell-index order
// and every pass is stable, so equal intensities keep ascending cell index.
//
// Each pass ("onesweep"): a block takes the next tile (16384 keys on large
// grids, 4096 on small ones) of one of the pass's input segments from that
// segment's ticket counter, ranks its keys by digit within each wave (the
// lanes that share a digit find each other through a per-digit LDS mask, or
// in the last pass with 8 ballots; the lowest of them bumps the wave's LDS
// counter), publishes its per-digit counts for the segment's later tiles and
// looks back over the segment's earlier tiles' published counts (decoupled
// look-back) to find where its digits start, then writes its keys digit by
// digit through LDS so that each digit's run is stored contiguously.  Tiles
// only wait on tiles that took earlier tickets, which are already running, so
// every wait ends.
#include <algorithm>

#include "internal.h"

namespace {

// 1024 threads: the histogram's 56 KB of LDS allow two blocks per CU, which
// at 256 threads left a streaming read of J with 8 waves per CU.
constexpr int kHistThreads = 1024;
constexpr int kHistWaves = kHistThreads / 64;
constexpr int kKeysPerThread = 16;
// One onesweep tile per block: 16384 keys (1024 threads) on large grids, where
// long digit runs keep the scattered writes close to whole cache lines; 4096
// keys (256 threads) below 2^24 keys, where more tiles keep more CUs busy.
constexpr int kBigThreads = 1024, kSmallThreads = 256;
constexpr long long kBigTileFrom = 1LL << 24;
constexpr unsigned kFlagAgg = 1u << 30;
constexpr unsigned kFlagPre = 2u << 30;

__device__ __forceinline__ unsigned desc_key(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) == 0u) u = 0u;  // -0 == +0
    const unsigned asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ~asc;
}

__device__ __forceinline__ bool is_nan_bits(unsigned u) { return (u & 0x7fffffffu) > 0x7f800000u; }

// p & ~(e ^ m) as one 3-input bit operation (gfx950 v_bitop3_b32; the truth
// table is indexed by (p, e, m) as bits 2, 1, 0: ones at 100 and 111).
__device__ __forceinline__ unsigned and_xnor(unsigned p, unsigned e, unsigned m) {
    return __builtin_amdgcn_bitop3_b32(p, e, m, 0x90);
}

__device__ __forceinline__ void st_release(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan over 256 values held by threads 0..255 (waves 0-3); every
// thread of the block calls it (it contains a barrier), the result is defined
// for threads 0..255.
__device__ __forceinline__ unsigned digit_excl_scan(unsigned v, unsigned* sh /* 4 */) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned o = __shfl_up(x, d, 64);
        if (lane >= d) x += o;
    }
    if (wave < 4 && lane == 63) sh[wave] = x;
    __syncthreads();
    unsigned add = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w)
        if (w < wave) add += sh[w];
    return x + add - v;
}

// Clears pass 0's look-back region, counts the digits of the keys per
// segment of each pass's input (keys read once, 16 per thread in flight) and
// flags NaN intensities.  n is a multiple of 4.  Segments: pass 0's are
// ranges of tps input tiles (tile / tps = (tile * seg_mul) >> 32); the input
// of pass k = 1, 2 is ordered by digit k-1, and its segment s holds the keys
// whose digit k-1 has top three bits s; the last pass has one segment.  The
// block's counts of passes 0-2 go to part[block] (or, when part is null,
// straight into the control block), the top digit's into the control block.
__global__ __launch_bounds__(kHistThreads) void k_hist(const float* __restrict__ J, long long n, Ctrl* ctrl,
                                                       unsigned* __restrict__ lb0, long long lb_words,
                                                       unsigned* __restrict__ part, int tile_shift,
                                                       unsigned long long seg_mul) {
    __shared__ unsigned h[3][8][256];
    // The top digit (sign and exponent) takes a handful of values, so one
    // LDS word per value would take the atomics of most lanes at once: it is
    // counted per lane instead, in 16-bit halves (lanes 2k and 2k+1 share a
    // word, the block's waves share the words: at most kHistWaves * 16 keys
    // per round per half, which the host keeps below 2^16).
    __shared__ unsigned top[256][32];
    const int lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < 3 * 8 * 256; i += kHistThreads) (&h[0][0][0])[i] = 0;
    for (int i = threadIdx.x; i < 256 * 32; i += kHistThreads) (&top[0][0])[i] = 0;
    for (long long i = (long long)blockIdx.x * kHistThreads + threadIdx.x; i < lb_words;
         i += (long long)gridDim.x * kHistThreads)
        lb0[i] = 0;
    __syncthreads();
    bool nan = false;
    const float4* J4 = reinterpret_cast<const float4*>(J);
    const long long n4 = n / 4;
    constexpr int kV = 4;  // float4 loads per thread per round
    for (long long base = (long long)blockIdx.x * kHistThreads * kV; base < n4;
         base += (long long)gridDim.x * kHistThreads * kV) {
        float4 v[kV];
#pragma unroll
        for (int k = 0; k < kV; ++k) {
            const long long i = base + k * kHistThreads + threadIdx.x;
            v[k] = i < n4 ? J4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < kV; ++k) {
            const long long i = base + k * kHistThreads + threadIdx.x;
            const bool live = i < n4;
            const unsigned tile = (unsigned)((4 * i) >> tile_shift);
            unsigned s0 = (unsigned)(((unsigned long long)tile * seg_mul) >> 32);  // tile < 2^17: no overflow
            s0 = s0 < 8u ? s0 : 7u;
            const float f[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const unsigned key = desc_key(f[e]);
                if (live) {
                    nan |= is_nan_bits(__float_as_uint(f[e]));
                    const unsigned d0 = key & 255u, d1 = (key >> 8) & 255u;
                    atomicAdd(&h[0][s0][d0], 1u);
                    atomicAdd(&h[1][d0 >> 5][d1], 1u);
                    atomicAdd(&h[2][d1 >> 5][(key >> 16) & 255u], 1u);
                    atomicAdd(&top[key >> 24][lane >> 1], (lane & 1) ? 65536u : 1u);
                }
            }
        }
    }
    if (__any(nan) && lane == 0) report_status(ctrl, AMBER_STATUS_NAN_J);
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += kHistThreads) {
        unsigned c = 0;
        for (int j = 0; j < 32; ++j) {
            const unsigned x = top[d][j];
            c += (x & 0xffffu) + (x >> 16);
        }
        if (c) atomicAdd(&ctrl->hist[3][d], c);
    }
    for (int i = threadIdx.x; i < 3 * 8 * 256; i += kHistThreads) {
        const unsigned c = (&h[0][0][0])[i];
        if (part) part[(long long)blockIdx.x * (3 * 8 * 256) + i] = c;
        else if (c) atomicAdd(&ctrl->segcnt[0][0][0] + i, c);
    }
}

// Sums the blocks' segment counts: block (x, y) adds rows y, y + gridDim.y, ...
// of columns 256 x .. 256 x + 255 into the control block.
__global__ __launch_bounds__(256) void k_seg_reduce(const unsigned* __restrict__ part, long long rows, Ctrl* ctrl) {
    const int col = blockIdx.x * 256 + threadIdx.x;  // < 3 * 8 * 256
    unsigned c = 0;
    for (long long r = blockIdx.y; r < rows; r += gridDim.y) c += part[r * (3 * 8 * 256) + col];
    if (c) atomicAdd(&ctrl->segcnt[0][0][0] + col, c);
}

__global__ void k_ctrl_init(Ctrl* ctrl, unsigned* sticky) {
    unsigned* p = reinterpret_cast<unsigned*>(ctrl);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 4); i += blockDim.x) p[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        ctrl->qmin = 0x7fffffff;
        ctrl->sticky = sticky;
    }
}

// Exclusive prefix of each digit histogram (where each digit's run starts),
// the start of each segment's runs (passes 0-2: the digit's start plus the
// counts of the earlier segments), and each pass's segments: where they start
// and the look-back id of their first tile (tiles of `tile` keys from the
// segment's start; pass 0's segments are ranges of tps tiles).
__global__ __launch_bounds__(256) void k_digit_offsets(Ctrl* ctrl, long long n, int tile, unsigned tps) {
    __shared__ unsigned sh[4];
    const int d = threadIdx.x;
    for (int k = 0; k < 3; ++k) {
        unsigned tot = 0;
        for (int s = 0; s < 8; ++s) tot += ctrl->segcnt[k][s][d];
        ctrl->hist[k][d] = tot;
        const unsigned ex = digit_excl_scan(tot, sh);
        ctrl->digit_off[k][d] = ex;
        unsigned run = ex;
        for (int s = 0; s < 8; ++s) {
            const unsigned c = ctrl->segcnt[k][s][d];
            ctrl->segcnt[k][s][d] = run;
            run += c;
        }
        __syncthreads();  // scan_sh is reused
    }
    ctrl->digit_off[3][d] = digit_excl_scan(ctrl->hist[3][d], sh);
    __syncthreads();  // the digit starts are read below by other threads
    if (d < 4) {
        const int k = d;
        unsigned st[9];
        for (int s = 0; s <= 8; ++s) {
            long long v;
            if (k == 0) v = std::min<long long>((long long)s * tps * tile, n);
            else if (k < 3) v = s == 8 ? n : ctrl->digit_off[k - 1][32 * s];
            else v = s == 0 ? 0 : n;
            st[s] = (unsigned)v;
        }
        unsigned t0 = 0;
        for (int s = 0; s <= 8; ++s) {
            ctrl->seg_start[k][s] = st[s];
            ctrl->seg_tile0[k][s] = t0;
            if (s < 8) t0 += (st[s + 1] - st[s] + (unsigned)tile - 1) / (unsigned)tile;
        }
    }
}

// Decomposition of a positive finite FP32 weight as m 2^q, q the exponent of
// its unit in the last place (q = -149 for subnormals).
__device__ __forceinline__ int weight_q(unsigned bits) {
    const int e = (int)((bits >> 23) & 255u);
    return (e == 0 ? 1 : e) - 150;
}

// Smallest ulp exponent over the tiles' values (one block).
__global__ __launch_bounds__(1024) void k_qmin(const int* __restrict__ qtile, long long n_tiles, Ctrl* ctrl) {
    __shared__ int sh[16];
    int q = 0x7fffffff;
    for (long long t = threadIdx.x; t < n_tiles; t += 1024) q = qtile[t] < q ? qtile[t] : q;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int oq = __shfl_xor(q, o, 64);
        q = oq < q ? oq : q;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 16; ++w) q = sh[w] < q ? sh[w] : q;
        q = sh[0] < q ? sh[0] : q;
        ctrl->qmin = q;
    }
}

// The last pass's stores: the indices (and weights) staged in digit order
// through LDS and written in runs, with no branch per element for a full tile
// (lanes past the end of the last tile stage into their lane's spare slot; a
// destination past the end, unreachable for consistent counts, is clamped into
// the array).  wrow is this wave's row of wave offsets.
template <int kThreads, bool CARRY, class Row>
__device__ __forceinline__ void last_pass_stores(const unsigned* key, const unsigned* val, const float* wt,
                                                 const unsigned* lrank, const Row& wrow, const unsigned* loff,
                                                 const unsigned* gbase, unsigned* stage, unsigned* __restrict__ vals_out,
                                                 float* __restrict__ w_out, unsigned tile_base, unsigned tend,
                                                 long long n, int shift) {
    constexpr int kTile = kThreads * kKeysPerThread;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned wbase = tile_base + (unsigned)wave * (64 * kKeysPerThread);
    const bool full = tile_base + kTile <= tend;
    unsigned lpos[kKeysPerThread];
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        const bool ok = (wbase + 64u * j + lane) < tend;
        const unsigned dd = (key[j] >> shift) & 255u;
        const unsigned p = loff[dd] + wrow[dd] + lrank[j];
        lpos[j] = (ok && p < (unsigned)kTile) ? p : (unsigned)kTile + lane;  // p < kTile for consistent counts
        stage[lpos[j]] = key[j];
    }
    __syncthreads();
    const int valid = (int)(tend - tile_base);  // <= kTile
    const unsigned last = (unsigned)(n - 1);
    unsigned dst[kKeysPerThread];
#pragma unroll
    for (int k = 0; k < kKeysPerThread; ++k) {
        const int i = tid + k * kThreads;
        const unsigned kk = stage[i];
        const unsigned dd = (kk >> shift) & 255u;
        const unsigned t = gbase[dd] + ((unsigned)i - loff[dd]);  // i >= loff[dd] inside the digit's run
        dst[k] = (full || i < valid) ? (t < last ? t : last) : 0xffffffffu;
    }
    auto pass_on = [&](const unsigned(&vals)[kKeysPerThread], unsigned* __restrict__ out) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kKeysPerThread; ++j) stage[lpos[j]] = vals[j];
        __syncthreads();
        if (full) {
#pragma unroll
            for (int k = 0; k < kKeysPerThread; ++k) out[dst[k]] = stage[tid + k * kThreads];
        } else {
#pragma unroll
            for (int k = 0; k < kKeysPerThread; ++k)
                if (dst[k] != 0xffffffffu) out[dst[k]] = stage[tid + k * kThreads];
        }
    };
    unsigned v[kKeysPerThread];
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) v[j] = val[j];
    pass_on(v, vals_out);
    if (CARRY) {
#pragma unroll
        for (int j = 0; j < kKeysPerThread; ++j) v[j] = __float_as_uint(wt[j]);
        pass_on(v, reinterpret_cast<unsigned*>(w_out));
    }
}

// One digit pass over tiles of kThreads * kKeysPerThread keys.  FIRST: keys
// come from J and the index is the position.  LAST: only the values (and
// weights) are written.  CARRY: weights travel with the keys; pass 0 also
// checks them and stores the smallest ulp exponent of each tile in qtile[tile].
//
// The input of passes 0-2 is split into 8 segments (the last pass's is one),
// each cut into tiles from its start with a ticket counter and a look-back
// chain of its own; the runs a segment's keys form start at offsets the
// histogram kernel counted.  A block takes a tile of
// segment blockIdx % 8 and of the next segments once that one is used up, so
// consecutive tiles, whose digit runs meet inside cache lines, are written
// from the same XCD's L2 (blocks are dealt to the 8 XCDs round robin) while
// there is work for it.  A tile waits only on earlier tiles of its segment,
// which took earlier tickets and are already running, so every wait ends.
// The grid has a block for every look-back id of every pass (tiles + 8);
// block b clears id b's entries of the next passes.
template <int kThreads, bool FIRST, bool LAST, bool CARRY, int KIN = 4, int KOUT = 4>
__global__ __launch_bounds__(kThreads) void k_onesweep(
    const float* __restrict__ J, const void* __restrict__ keys_in_v, const unsigned* __restrict__ vals_in,
    const float* __restrict__ w_in, void* __restrict__ keys_out_v, unsigned* __restrict__ vals_out,
    float* __restrict__ w_out, unsigned* __restrict__ lb, unsigned* __restrict__ lb_next,
    unsigned* __restrict__ lb_next2, int* __restrict__ qtile, Ctrl* ctrl, int pass, long long n) {
    constexpr int kWaves = kThreads / 64;
    constexpr int kTile = kThreads * kKeysPerThread;
    static_assert(kThreads >= 256 && kThreads % 64 == 0 && kTile <= 65535, "tile geometry");
    __shared__ unsigned s_seg, s_j;
    // per-wave digit counts, then wave offsets (the last pass: entry 256 is a
    // spare counter for lanes past the end of the last tile)
    constexpr int kRow = LAST ? 257 : 256;
    __shared__ unsigned short wcnt[kWaves][kRow];
    // Peer matching in the passes whose digits are spread: per wave and digit
    // a 64-bit mask that the lanes of one key round OR their bits into, read
    // back and clear (entry 256 takes the lanes past the end of the last
    // tile).  The last pass, whose top digit takes few values (so the atomics
    // of one instruction would mostly hit one address), matches by ballots.
    constexpr bool kPeerLds = !LAST;
    __shared__ unsigned long long pmask[kPeerLds ? kWaves : 1][kPeerLds ? 257 : 1];
    __shared__ unsigned loff[256];                // tile-local start of each digit
    __shared__ unsigned gbase[256];               // global start of each digit's run of this tile
    __shared__ unsigned scan_sh[4];
    // keys, then indices, then weights, in digit order (the last pass: one
    // spare slot per lane for the lanes past the end of the last tile)
    __shared__ unsigned stage[kTile + (LAST ? 64 : 0)];
    __shared__ int s_qmin[kWaves];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // keys travel with only the digits later passes still need: KIN / KOUT
    // bytes, the top bytes of the 32-bit key
    auto load_key = [&](unsigned i) -> unsigned {
        if (KIN == 4) return reinterpret_cast<const unsigned*>(keys_in_v)[i];
        if (KIN == 2) return (unsigned)reinterpret_cast<const unsigned short*>(keys_in_v)[i] << 16;
        return (unsigned)reinterpret_cast<const unsigned char*>(keys_in_v)[i] << 24;
    };
    auto store_key = [&](unsigned i, unsigned k) {
        if (KOUT == 4) reinterpret_cast<unsigned*>(keys_out_v)[i] = k;
        else if (KOUT == 2) reinterpret_cast<unsigned short*>(keys_out_v)[i] = (unsigned short)(k >> 16);
        else reinterpret_cast<unsigned char*>(keys_out_v)[i] = (unsigned char)(k >> 24);
    };
    if (tid == 0) {
        unsigned seg = 8u, jj = 0u;
        for (int t = 0; t < 8; ++t) {
            const unsigned sg = (blockIdx.x + (unsigned)t) & 7u;
            const unsigned cnt = ctrl->seg_tile0[pass][sg + 1] - ctrl->seg_tile0[pass][sg];
            if (cnt == 0u) continue;
            const unsigned j = atomicAdd(&ctrl->seg_ticket[pass][sg], 1u);
            if (j < cnt) {
                seg = sg;
                jj = j;
                break;
            }
        }
        s_seg = seg;
        s_j = jj;
    }
    for (int i = tid; i < kWaves * kRow; i += kThreads) (&wcnt[0][0])[i] = 0;
    if (kPeerLds)
        for (int i = tid; i < kWaves * 257; i += kThreads) (&pmask[0][0])[i] = 0ull;
    // The next passes' look-back entries start cleared.
    if (tid < 256) {
        if (lb_next) lb_next[(long long)blockIdx.x * 256 + tid] = 0u;
        if (lb_next2) lb_next2[(long long)blockIdx.x * 256 + tid] = 0u;
    }
    __syncthreads();
    const unsigned seg = s_seg, seg_j = s_j;
    if (seg >= 8u) return;  // every tile is taken
    const unsigned tile = ctrl->seg_tile0[pass][seg] + seg_j;  // look-back id
    // element positions fit in 32 bits (n <= 2^30)
    const unsigned tile_base = ctrl->seg_start[pass][seg] + seg_j * (unsigned)kTile;
    const unsigned seg_end = ctrl->seg_start[pass][seg + 1];
    const unsigned tend = tile_base + kTile < seg_end ? tile_base + kTile : seg_end;
    const int shift = 8 * pass;

    unsigned key[kKeysPerThread], val[kKeysPerThread], lrank[kKeysPerThread];
    float wt[kKeysPerThread];
    bool bad_w = false;
    int qmin = 0x7fffffff;
    const unsigned wbase = tile_base + (unsigned)wave * (64 * kKeysPerThread);
    // All loads first (no branch around a load, so they are all in flight
    // together).  Element indices fit in 32 bits (n <= 2^30): a full tile
    // loads at one lane offset plus constant strides; the last tile clamps
    // its positions, and its out-of-range lanes are masked after.
    const unsigned lane0 = wbase + (unsigned)lane;
    if (tile_base + kTile <= tend) {
#pragma unroll
        for (int j = 0; j < kKeysPerThread; ++j) {
            const unsigned pos = lane0 + 64u * j;
            if (FIRST) {
                key[j] = __float_as_uint(J[pos]);
                val[j] = pos;
            } else {
                key[j] = load_key(pos);
                val[j] = vals_in[pos];
            }
            if (CARRY) wt[j] = w_in[pos];
        }
    } else {
        const unsigned last = tend - 1u;
#pragma unroll
        for (int j = 0; j < kKeysPerThread; ++j) {
            const unsigned pos = lane0 + 64u * j;
            const unsigned pc = pos < last ? pos : last;
            if (FIRST) {
                key[j] = __float_as_uint(J[pc]);
                val[j] = pos;
            } else {
                key[j] = load_key(pc);
                val[j] = vals_in[pc];
            }
            if (CARRY) wt[j] = w_in[pc];
        }
    }
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        const bool ok = lane0 + 64u * j < tend;
        if (FIRST) key[j] = desc_key(__uint_as_float(key[j]));
        if (!ok) key[j] = 0xffffffffu;
        if (CARRY && FIRST && ok) {
            const unsigned b = __float_as_uint(wt[j]);
            const bool good = (b - 1u) < 0x7f7fffffu;  // 0 < w < inf, not NaN
            bad_w |= !good;
            const int q = weight_q(b);
            qmin = q < qmin ? q : qmin;
        }
    }

    // Rank each key among the wave's keys with the same digit, in input order.
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        const bool ok = lane0 + 64u * j < tend;
        const unsigned d = (key[j] >> shift) & 255u;
        if constexpr (kPeerLds) {
            // the lanes with this lane's digit: one LDS atomic OR per lane, one
            // read, one clear (a wave's LDS operations complete in order)
            const unsigned dd = ok ? d : 256u;
            atomicOr(&pmask[wave][dd], 1ull << lane);
            const unsigned long long peers = pmask[wave][dd];
            pmask[wave][dd] = 0ull;
            unsigned r = 0;
            if (ok) {
                const unsigned before = (unsigned)__popcll(peers & lt);
                const unsigned cnt = (unsigned)__popcll(peers);
                const unsigned old = wcnt[wave][d];
                r = old + before;
                if (before == 0) wcnt[wave][d] = (unsigned short)(old + cnt);  // lowest peer updates
            }
            lrank[j] = r;
        } else {
            // The top digit takes few values, so peer groups are large: lanes
            // whose digit equals this lane's, bit by bit on 32-bit halves (the
            // all-ones-where-set word a signed one-bit extract of the key, each
            // step one 3-input bit operation per half), and no branch: every
            // peer writes the same new count (lanes past the end of the last
            // tile use the spare counter).
            const unsigned long long ok_mask = __ballot(ok);
            unsigned plo = (unsigned)ok_mask, phi = (unsigned)(ok_mask >> 32);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const unsigned ext = (unsigned)__builtin_amdgcn_sbfe((int)key[j], shift + b, 1);
                const unsigned long long m = __ballot(ext != 0u);
                plo = and_xnor(plo, ext, (unsigned)m);
                phi = and_xnor(phi, ext, (unsigned)(m >> 32));
            }
            const unsigned long long peers = ((unsigned long long)phi << 32) | plo;
            const unsigned before = (unsigned)__popcll(peers & lt);
            const unsigned cnt = (unsigned)__popcll(peers);
            const unsigned dd = ok ? d : (unsigned)(kRow - 1);
            const unsigned old = wcnt[wave][dd];
            lrank[j] = old + before;
            wcnt[wave][dd] = (unsigned short)(old + cnt);
        }
    }
    __syncthreads();

    // Per digit (threads 0..255): wave offsets, tile count, look-back.
    unsigned tcnt = 0;
    if (tid < 256) {
        const int d = tid;
        unsigned run = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const unsigned c = wcnt[w][d];
            wcnt[w][d] = (unsigned short)run;
            run += c;
        }
        tcnt = run;
        unsigned* me = lb + (long long)tile * 256 + d;
        const unsigned seg_base = LAST ? ctrl->digit_off[3][d] : ctrl->segcnt[pass][seg][d];
        if (seg_j == 0) {
            st_release(me, kFlagPre | tcnt);
            gbase[d] = seg_base;
        } else {
            st_release(me, kFlagAgg | tcnt);
            const unsigned excl = lb_walk(lb, (long long)tile, d, (long long)ctrl->seg_tile0[pass][seg]);
            st_release(me, kFlagPre | (excl + tcnt));
            gbase[d] = seg_base + excl;
        }
    }
    const unsigned lo = digit_excl_scan(tcnt, scan_sh);
    if (tid < 256) loff[tid] = lo;
    // block-level reductions of the weight checks (pass 0)
    if (CARRY && FIRST) {
        int q = qmin;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int oq = __shfl_xor(q, o, 64);
            q = oq < q ? oq : q;
        }
        if (lane == 0) s_qmin[wave] = q;
        if (__any(bad_w) && lane == 0) report_status(ctrl, AMBER_STATUS_BAD_W);
    }
    __syncthreads();
    if (CARRY && FIRST && tid == 0) {  // a plain store: nothing in this block waits on it
        int q = s_qmin[0];
        for (int w = 1; w < kWaves; ++w) q = s_qmin[w] < q ? s_qmin[w] : q;
        qtile[tile] = q;
    }

    // Every load of this tile has arrived by now (the keys were ranked, the
    // look-back is done); saying so keeps the compiler from waiting on the
    // stores issued below before each later LDS staging step (the vector
    // memory counter counts loads and stores together).
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), expcnt and lgkmcnt unconstrained

    // Stage the keys in digit order; every thread then takes the slots
    // tid + k kThreads, finds each slot's destination from the staged key's
    // digit, and keeps it for the indices and weights staged after it.
    if constexpr (LAST) {
        last_pass_stores<kThreads, CARRY>(key, val, wt, lrank, wcnt[wave], loff, gbase, stage, vals_out, w_out,
                                          tile_base, tend, n, shift);
        return;
    }
    unsigned lpos[kKeysPerThread];
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j) {
        const bool ok = lane0 + 64u * j < tend;
        const unsigned dd = (key[j] >> shift) & 255u;
        const unsigned p = ok ? loff[dd] + wcnt[wave][dd] + lrank[j] : 0xffffffffu;
        lpos[j] = p < (unsigned)kTile ? p : 0xffffffffu;  // out of range is unreachable for consistent counts
        if (lpos[j] != 0xffffffffu) stage[p] = key[j];
    }
    __syncthreads();
    const int valid = (int)(tend - tile_base);  // <= kTile
    unsigned dst[kKeysPerThread];
#pragma unroll
    for (int k = 0; k < kKeysPerThread; ++k) {
        const int i = tid + k * kThreads;
        dst[k] = 0xffffffffu;
        if (i < valid) {
            const unsigned kk = stage[i];
            const unsigned dd = (kk >> shift) & 255u;
            const unsigned t = gbase[dd] + ((unsigned)i - loff[dd]);  // i >= loff[dd] inside the digit's run
            if (t < (unsigned)n) {
                dst[k] = t;
                if (!LAST) store_key(t, kk);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kKeysPerThread; ++j)
        if (lpos[j] != 0xffffffffu) stage[lpos[j]] = val[j];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kKeysPerThread; ++k)
        if (dst[k] != 0xffffffffu) vals_out[dst[k]] = stage[tid + k * kThreads];
    if (CARRY) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kKeysPerThread; ++j)
            if (lpos[j] != 0xffffffffu) stage[lpos[j]] = __float_as_uint(wt[j]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kKeysPerThread; ++k)
            if (dst[k] != 0xffffffffu) w_out[dst[k]] = __uint_as_float(stage[tid + k * kThreads]);
    }
}

// Status bits of the last matching call into a caller's per-box word.
__global__ void k_status_collect(const Ctrl* ctrl, unsigned* dst, int first) {
    if (threadIdx.x == 0) dst[0] = first ? 0u : (dst[0] | ctrl->status);
}

}  // namespace

int status_collect(const amber_plan_s* p, unsigned char* ws, const WsLayout& L, unsigned* dst, bool first,
                   hipStream_t s) {
    const Ctrl* ctrl = reinterpret_cast<const Ctrl*>(ws + L.ctrl);
    AMBER_LAUNCH(p, "status_collect", k_status_collect, dim3(1), dim3(64), s, ctrl, dst, first ? 1 : 0);
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}

template <int T>
static void launch_passes(const amber_plan_s* p, const float* d_J, const float* d_w, hipStream_t s, int carry,
                          unsigned* const* keys, unsigned* const* vals, float* const* wts, unsigned* const* lb,
                          uint32_t* final_vals, int* qtile, Ctrl* ctrl, long long n, long long n_tiles) {
    // a block for every look-back id of every pass: segments cut at most 8
    // more tiles than n_tiles (pass 0's exactly n_tiles)
    const dim3 grid((unsigned)(n_tiles + 8)), blk(T);
    // pass 0: J, w -> buffers 1; pass 1: 1 -> 0; pass 2: 0 -> 1; pass 3: 1 -> 0 (values, weights)
    if (carry) {
        AMBER_LAUNCH(p, "rank_pass0", (k_onesweep<T, true, false, true>), grid, blk, s, d_J, nullptr, nullptr, d_w,
                     keys[1], vals[1], wts[1], lb[0], lb[1], nullptr, qtile, ctrl, 0, n);
        AMBER_LAUNCH(p, "rank_qmin", k_qmin, dim3(1), dim3(1024), s, qtile, n_tiles, ctrl);
        AMBER_LAUNCH(p, "rank_pass1", (k_onesweep<T, false, false, true, 4, 2>), grid, blk, s, nullptr, keys[1],
                     vals[1], wts[1], keys[0], vals[0], wts[0], lb[1], lb[0], nullptr, nullptr, ctrl, 1, n);
        AMBER_LAUNCH(p, "rank_pass2", (k_onesweep<T, false, false, true, 2, 1>), grid, blk, s, nullptr, keys[0],
                     vals[0], wts[0], keys[1], vals[1], wts[1], lb[0], lb[1], nullptr, nullptr, ctrl, 2, n);
        AMBER_LAUNCH(p, "rank_pass3", (k_onesweep<T, false, true, true, 1, 4>), grid, blk, s, nullptr, keys[1],
                     vals[1], wts[1], nullptr, final_vals, wts[0], lb[1], lb[0], lb[2], nullptr, ctrl, 3, n);
    } else {
        AMBER_LAUNCH(p, "rank_pass0", (k_onesweep<T, true, false, false>), grid, blk, s, d_J, nullptr, nullptr,
                     nullptr, keys[1], vals[1], nullptr, lb[0], lb[1], nullptr, nullptr, ctrl, 0, n);
        AMBER_LAUNCH(p, "rank_pass1", (k_onesweep<T, false, false, false, 4, 2>), grid, blk, s, nullptr, keys[1],
                     vals[1], nullptr, keys[0], vals[0], nullptr, lb[1], lb[0], nullptr, nullptr, ctrl, 1, n);
        AMBER_LAUNCH(p, "rank_pass2", (k_onesweep<T, false, false, false, 2, 1>), grid, blk, s, nullptr, keys[0],
                     vals[0], nullptr, keys[1], vals[1], nullptr, lb[0], lb[1], nullptr, nullptr, ctrl, 2, n);
        AMBER_LAUNCH(p, "rank_pass3", (k_onesweep<T, false, true, false, 1, 4>), grid, blk, s, nullptr, keys[1],
                     vals[1], nullptr, nullptr, final_vals, nullptr, lb[1], lb[0], lb[2], nullptr, ctrl, 3, n);
    }
}

int rank_sort(const amber_plan_s* p, const float* d_J, const float* d_w, unsigned char* ws, const WsLayout& L,
              hipStream_t s, int carry, uint32_t* d_perm_out) {
    const long long n = (long long)p->n * p->n * p->n;
    const bool big = n >= kBigTileFrom;
    const long long tile = (long long)(big ? kBigThreads : kSmallThreads) * kKeysPerThread;
    const long long n_tiles = (n + tile - 1) / tile;
    Ctrl* ctrl = reinterpret_cast<Ctrl*>(ws + L.ctrl);
    unsigned* keys[2] = {reinterpret_cast<unsigned*>(ws + L.keys[0]), reinterpret_cast<unsigned*>(ws + L.keys[1])};
    unsigned* vals[2] = {reinterpret_cast<unsigned*>(ws + L.vals[0]), reinterpret_cast<unsigned*>(ws + L.vals[1])};
    float* wts[2] = {reinterpret_cast<float*>(ws + L.wts[0]), reinterpret_cast<float*>(ws + L.wts[1])};
    const long long lbw = lb_words(n);
    unsigned* lb[3] = {reinterpret_cast<unsigned*>(ws + L.lookback),
                       reinterpret_cast<unsigned*>(ws + L.lookback) + lbw,
                       reinterpret_cast<unsigned*>(ws + L.lookback) + 2 * lbw};

    AMBER_LAUNCH(p, "rank_init", k_ctrl_init, dim3(1), dim3(256), s, ctrl, p->d_sticky);
    const unsigned hist_blocks =
        (unsigned)std::min<long long>(2048, (n + kHistThreads * 16 - 1) / (kHistThreads * 16));
    // the histogram's per-lane top-digit counters are 16 bits wide
    const long long hist_step = (long long)hist_blocks * kHistThreads * 4;
    if ((long long)kHistWaves * 16 * ((n / 4 + hist_step - 1) / hist_step) > 65535) return AMBER_E_SIZE;
    // pass 0's segments: ranges of tps tiles; tile / tps = (tile * seg_mul) >> 32
    // with seg_mul = ceil(2^32 / tps) = (2^32 + r) / tps, r < tps: exact while
    // tile * r < 2^32, which n_tiles * tps < 2^32 ensures
    const unsigned tps = (unsigned)((n_tiles + 7) / 8);
    const unsigned long long seg_mul = ((1ULL << 32) + tps - 1) / tps;
    int tile_shift = 0;
    while ((1LL << tile_shift) < tile) ++tile_shift;
    if ((unsigned long long)n_tiles * tps >= (1ULL << 32)) return AMBER_E_SIZE;
    // The blocks' segment counts go through the first key buffer (free until
    // pass 1) where it holds them, else straight into the control block.
    constexpr long long kSegWords = 3 * 8 * 256;
    unsigned* part = (long long)hist_blocks * kSegWords <= n ? keys[0] : nullptr;
    AMBER_LAUNCH(p, "rank_hist", k_hist, dim3(hist_blocks), dim3(kHistThreads), s, d_J, n, ctrl, lb[0], n_tiles * 256,
                 part, tile_shift, seg_mul);
    if (part)
        AMBER_LAUNCH(p, "rank_seg_reduce", k_seg_reduce, dim3((unsigned)(kSegWords / 256), std::min(64u, hist_blocks)),
                     dim3(256), s, part, (long long)hist_blocks, ctrl);
    AMBER_LAUNCH(p, "rank_digit_offsets", k_digit_offsets, dim3(1), dim3(256), s, ctrl, n, (int)tile, tps);
    uint32_t* final_vals = d_perm_out ? d_perm_out : vals[0];
    // the per-tile ulp exponents of pass 0 live in the third look-back region
    // until the last pass clears it
    int* qtile = reinterpret_cast<int*>(lb[2]);
    if (big)
        launch_passes<kBigThreads>(p, d_J, d_w, s, carry, keys, vals, wts, lb, final_vals, qtile, ctrl, n, n_tiles);
    else
        launch_passes<kSmallThreads>(p, d_J, d_w, s, carry, keys, vals, wts, lb, final_vals, qtile, ctrl, n, n_tiles);
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}
