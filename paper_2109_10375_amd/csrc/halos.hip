// Source field from a halo catalogue on gfx950 (Sec. 3.2.1, Eqs. interlace and
// Wofk), feeding the radiation field of Sec. 3.4.1.
//
// Halo masses are assigned to two N^3 meshes with a window of order p (1 NGP,
// 2 CIC, 3 TSC): cell i spans [i, i+1) cells with its node at the centre,
// positions are in length units in [0, L) and wrap periodically; the second
// mesh takes the positions shifted by half a cell on every axis.  Both meshes
// are transformed, and every stored mode of the half spectrum becomes
//   S(k) = [A(k) + phi(k) B(k)] / (2 W(k)),  W(k) = prod_d sinc(pi m~_d / N)^p,
// phi = e^{i k.dx} except on the Nyquist planes, where it is the Hermitian
// average e^{i alpha} cos(beta) (alpha the phase of the non-Nyquist axes,
// beta = pi/2 per Nyquist axis), so that the real transform back gives the
// real part of the full-grid inverse.  Without interlacing S = A / W.
//
// Deposit: on grids that 16 divides, halos are binned by 16^3 mesh tile (a
// halo joins the bin of every tile its window touches on either mesh: one to
// eight) in two levels: blocks of the catalogue count and copy their halos
// per superbin of up to 8^3 tiles with LDS counters (offsets from a scan of
// the per-block counts), then one workgroup per superbin counts and copies its
// halos into its tiles' bins.  One workgroup per tile then sums its bin into
// the tile's cells in LDS and writes the block with plain stores, so the
// meshes need neither zeroing nor global atomics.  The LDS sums are exact: every term m w_x w_y w_z
// (FP64 from the FP32 position and mass) is rounded once to a 64-bit integer
// multiple of 2^-s, s chosen from the largest |mass| and the largest bin so
// that no cell sum can overflow, and added with integer atomics; each cell is
// then rounded once to FP32.  The mesh therefore does not depend on the order
// of the halos or of the atomics, and repeated calls give identical fields.
// The superbin copies and the tile bins live in the two spectrum regions,
// which the forward transforms only write afterwards; when they would not fit
// there (or on other grids) every halo adds its FP32 terms with global atomics
// instead, whose last bits depend on the order of the additions.
#include <algorithm>

#include "internal.h"

// The bin counts, the bin fill and the tile deposit must locate every halo's
// cells identically, so no FP64 operation here is fused.
#pragma clang fp contract(off)

namespace {

constexpr double kPiD = 3.14159265358979323846;

__global__ void k_zero_f32(float* __restrict__ p, long long count) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

template <int P>
__device__ __forceinline__ int assign_1d(double x, long long& i0, double* w) {
    if (P == 1) {
        i0 = (long long)floor(x);
        w[0] = 1.0;
        return 1;
    } else if (P == 2) {
        const double d = x - 0.5;
        const double f = floor(d);
        i0 = (long long)f;
        w[1] = d - f;
        w[0] = 1.0 - w[1];
        return 2;
    } else {
        const double c = floor(x);
        const double u = x - (c + 0.5);
        i0 = (long long)c - 1;
        w[0] = 0.5 * (0.5 - u) * (0.5 - u);
        w[1] = 0.75 - u * u;
        w[2] = 0.5 * (0.5 + u) * (0.5 + u);
        return 3;
    }
}

// Periodic cell index.  In-range positions reach at most one cell past either
// end, which one add or subtract folds back; the 64-bit remainder (slow on the
// GPU) only runs for positions outside the box.
__device__ __forceinline__ long long wrap(long long i, int n) {
    if (i < 0) i += n;
    else if (i >= n) i -= n;
    if ((unsigned long long)i >= (unsigned long long)n) {
        i %= n;
        if (i < 0) i += n;
    }
    return i;
}

// One halo per thread, onto mesh0 (positions as given) and, when interlacing,
// mesh1 (shifted by half a cell).  With a gate word it runs only when the gate
// is set (the binned deposit overflowed and left the meshes zeroed).
template <int P>
__global__ __launch_bounds__(256) void k_deposit(const float* __restrict__ pos, const float* __restrict__ mass,
                                                 long long n_halo, int n, double to_cell, float* __restrict__ mesh0,
                                                 float* __restrict__ mesh1, const unsigned* __restrict__ gate) {
    if (gate && *gate == 0u) return;
    for (long long h = (long long)blockIdx.x * blockDim.x + threadIdx.x; h < n_halo;
         h += (long long)gridDim.x * blockDim.x) {
    const double m = (double)mass[h];
    const double x[3] = {(double)pos[3 * h] * to_cell, (double)pos[3 * h + 1] * to_cell,
                         (double)pos[3 * h + 2] * to_cell};
    for (int mesh = 0; mesh < (mesh1 ? 2 : 1); ++mesh) {
        float* out = mesh ? mesh1 : mesh0;
        const double shift = mesh ? 0.5 : 0.0;
        long long i0[3];
        double w[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d) assign_1d<P>(x[d] + shift, i0[d], w[d]);
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
            for (int b = 0; b < P; ++b)
#pragma unroll
                for (int c = 0; c < P; ++c) {
                    const long long ix = wrap(i0[0] + a, n), iy = wrap(i0[1] + b, n), iz = wrap(i0[2] + c, n);
                    atomicAdd(&out[(ix * n + iy) * n + iz], (float)(m * w[0][a] * w[1][b] * w[2][c]));
                }
    }
    }
}

// Tiles touched by a halo along one axis: the union of both meshes' windows
// is a run of at most P + 1 cells, so at most two tiles (t0 and t1 == t0 when
// the run stays inside one).
template <int P>
__device__ __forceinline__ void axis_tiles(double x, int n, bool interlace, int& t0, int& t1) {
    long long i0, i1;
    double w[3];
    assign_1d<P>(x, i0, w);
    long long lo = i0, hi = i0;
    if (interlace) {
        assign_1d<P>(x + 0.5, i1, w);
        lo = i0 < i1 ? i0 : i1;
        hi = i0 < i1 ? i1 : i0;
    }
    t0 = (int)(wrap(lo, n) / kHaloTile);
    t1 = (int)(wrap(hi + (P - 1), n) / kHaloTile);
}

// Geometry of the two-level binning: 16^3-cell tiles, nt per axis, grouped
// into superbins of sb^3 tiles, ns = nt / sb per axis.
struct Geo {
    int n, nt, sb, ns;
    double to_cell;
    int interlace;
};

// The tiles a halo touches along each axis (a[d][0], a[d][1], equal when one).
template <int P>
__device__ __forceinline__ void halo_axes(float px, float py, float pz, const Geo& g, int (*a)[2]) {
    const double x[3] = {(double)px * g.to_cell, (double)py * g.to_cell, (double)pz * g.to_cell};
#pragma unroll
    for (int d = 0; d < 3; ++d) axis_tiles<P>(x[d], g.n, g.interlace != 0, a[d][0], a[d][1]);
}

// Visits every superbin the halo touches (1 to 8).
template <typename F>
__device__ __forceinline__ void for_each_superbin(int (*a)[2], const Geo& g, F f) {
    int sv[3][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sv[d][0] = a[d][0] / g.sb;
        sv[d][1] = a[d][1] / g.sb;
    }
    for (int i = 0; i < (sv[0][1] != sv[0][0] ? 2 : 1); ++i)
        for (int j = 0; j < (sv[1][1] != sv[1][0] ? 2 : 1); ++j)
            for (int k = 0; k < (sv[2][1] != sv[2][0] ? 2 : 1); ++k)
                f((sv[0][i] * g.ns + sv[1][j]) * g.ns + sv[2][k]);
}

// Visits the touched tiles inside superbin (sx, sy, sz), with the tile's index
// inside the superbin and its global index.
template <typename F>
__device__ __forceinline__ void for_each_tile_in(int (*a)[2], const Geo& g, int sx, int sy, int sz, F f) {
    const int s3[3] = {sx, sy, sz};
    int lo[3][2], cnt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        cnt[d] = 0;
        const int m = (a[d][1] != a[d][0]) ? 2 : 1;
        for (int i = 0; i < m; ++i)
            if (a[d][i] / g.sb == s3[d]) lo[d][cnt[d]++] = a[d][i];
    }
    for (int i = 0; i < cnt[0]; ++i)
        for (int j = 0; j < cnt[1]; ++j)
            for (int k = 0; k < cnt[2]; ++k) {
                const int tx = lo[0][i], ty = lo[1][j], tz = lo[2][k];
                const unsigned local = (unsigned)(((tx - sx * g.sb) * g.sb + (ty - sy * g.sb)) * g.sb + (tz - sz * g.sb));
                f(local, (unsigned)((tx * g.nt + ty) * g.nt + tz));
            }
}

__global__ __launch_bounds__(256) void k_zero_u32(unsigned* __restrict__ p, long long count) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned x = __shfl_xor(v, o, 64);
        v = x > v ? x : v;
    }
    return v;
}

// First level, counts: block b takes halos [b chunk, (b + 1) chunk) and counts
// per superbin in LDS; cmat[superbin * nb + b] receives the counts (no global
// atomics), mass_max the largest |mass| bits.
template <int P>
__global__ __launch_bounds__(256) void k_super_count(const float* __restrict__ pos, const float* __restrict__ mass,
                                                     long long n_halo, long long chunk, Geo g,
                                                     unsigned* __restrict__ cmat, int nb,
                                                     unsigned* __restrict__ mass_max) {
    __shared__ unsigned h[kHaloSuperMax];
    __shared__ unsigned wmax[4];
    const int nsup = g.ns * g.ns * g.ns;
    for (int i = threadIdx.x; i < nsup; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    const long long b0 = (long long)blockIdx.x * chunk;
    const long long b1 = b0 + chunk < n_halo ? b0 + chunk : n_halo;
    unsigned mx = 0u;
    for (long long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
        int a[3][2];
        halo_axes<P>(pos[3 * e], pos[3 * e + 1], pos[3 * e + 2], g, a);
        const unsigned mb = __float_as_uint(mass[e]) & 0x7fffffffu;
        mx = mb > mx ? mb : mx;
        for_each_superbin(a, g, [&](int sbid) { atomicAdd(&h[sbid], 1u); });
    }
    mx = wave_max_u32(mx);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned m = wmax[0];
        for (int w = 1; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
        atomicMax(mass_max, m);
    }
    for (int i = threadIdx.x; i < nsup; i += blockDim.x) cmat[(long long)i * nb + blockIdx.x] = h[i];
}

// First level, offsets in two steps.  One block per superbin row of cmat:
// exclusive prefix of its nb counts into loc[row (nb + 1) + b], the row total
// in loc[row (nb + 1) + nb] and in rowtot[row].
__global__ __launch_bounds__(256) void k_row_scan(const unsigned* __restrict__ cmat, int nb,
                                                  unsigned* __restrict__ loc, unsigned* __restrict__ rowtot) {
    __shared__ unsigned part[256];
    const int r = blockIdx.x, t = threadIdx.x;
    const unsigned* row = cmat + (long long)r * nb;
    unsigned* out = loc + (long long)r * (nb + 1);
    const int per = (nb + 255) / 256;
    const int b = t * per, e = min(nb, b + per);
    unsigned sum = 0u;
    for (int i = b; i < e; ++i) sum += row[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned run = part[t] - sum;
    for (int i = b; i < e; ++i) {
        out[i] = run;
        run += row[i];
    }
    if (t == 0) {
        out[nb] = part[255];
        rowtot[r] = part[255];
    }
}

// One block: exclusive prefix of the row totals into base[0, nsup], base[nsup]
// = total; gate_a = 1 when the total exceeds the first level's capacity.
__global__ __launch_bounds__(1024) void k_rows_scan(const unsigned* __restrict__ rowtot, int nsup,
                                                    unsigned* __restrict__ base, unsigned long long capacity,
                                                    unsigned* __restrict__ gate_a) {
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const unsigned long long v0 = t < nsup ? rowtot[t] : 0ull;
    part[t] = v0;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned long long v = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const unsigned long long total = part[1023];
    const bool fits = total <= capacity;
    if (t < nsup) base[t] = fits ? (unsigned)(part[t] - v0) : 0u;
    if (t == 0) {
        base[nsup] = fits ? (unsigned)total : 0u;
        *gate_a = fits ? 0u : 1u;
    }
}

// First level, fill: the same blocks copy (position, mass) into every touched
// superbin, at offsets reserved by the prefix of cmat (LDS cursors).
template <int P>
__global__ __launch_bounds__(256) void k_super_fill(const float* __restrict__ pos, const float* __restrict__ mass,
                                                    long long n_halo, long long chunk, Geo g,
                                                    const unsigned* __restrict__ base,
                                                    const unsigned* __restrict__ loc, int nb,
                                                    const unsigned* __restrict__ gate_a, float4* __restrict__ ent) {
    __shared__ unsigned cur[kHaloSuperMax];
    __shared__ unsigned lim[kHaloSuperMax];
    if (*gate_a != 0u) return;
    const int nsup = g.ns * g.ns * g.ns;
    for (int i = threadIdx.x; i < nsup; i += blockDim.x) {
        const unsigned* rl = loc + (long long)i * (nb + 1) + blockIdx.x;
        cur[i] = base[i] + rl[0];
        lim[i] = base[i] + rl[1];
    }
    __syncthreads();
    const long long b0 = (long long)blockIdx.x * chunk;
    const long long b1 = b0 + chunk < n_halo ? b0 + chunk : n_halo;
    for (long long e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
        const float px = pos[3 * e], py = pos[3 * e + 1], pz = pos[3 * e + 2];
        const float4 v = make_float4(px, py, pz, mass[e]);
        int a[3][2];
        halo_axes<P>(px, py, pz, g, a);
        for_each_superbin(a, g, [&](int sbid) {
            const unsigned slot = atomicAdd(&cur[sbid], 1u);
            if (slot < lim[sbid]) ent[slot] = v;  // the counts bound every run
        });
    }
}

// Second level, counts: one block per superbin counts its entries per tile of
// the superbin (LDS) and writes the tiles' counts (every tile belongs to one
// superbin, so every count is written).
template <int P>
__global__ __launch_bounds__(1024) void k_tile_count(const float4* __restrict__ ent, const unsigned* __restrict__ base,
                                                     Geo g, const unsigned* __restrict__ gate_a,
                                                     unsigned* __restrict__ tile_count) {
    __shared__ unsigned h[kHaloSuperMax];
    const int sid = blockIdx.x;
    const int sx = sid / (g.ns * g.ns), sy = (sid / g.ns) % g.ns, sz = sid % g.ns;
    const int tps = g.sb * g.sb * g.sb;
    for (int i = threadIdx.x; i < tps; i += blockDim.x) h[i] = 0u;
    __syncthreads();
    if (*gate_a == 0u) {
        const unsigned e0 = base[sid], e1 = base[sid + 1];
        for (unsigned e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const float4 v = ent[e];
            int a[3][2];
            halo_axes<P>(v.x, v.y, v.z, g, a);
            for_each_tile_in(a, g, sx, sy, sz, [&](unsigned local, unsigned) { atomicAdd(&h[local], 1u); });
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < tps; i += blockDim.x) {
        const int lx = i / (g.sb * g.sb), ly = (i / g.sb) % g.sb, lz = i % g.sb;
        tile_count[((sx * g.sb + lx) * g.nt + (sy * g.sb + ly)) * g.nt + (sz * g.sb + lz)] = h[i];
    }
}

// Second level, fill: the superbin's entries go to their tiles' bins (LDS
// cursors from the tile starts).
template <int P>
__global__ __launch_bounds__(1024) void k_tile_fill(const float4* __restrict__ ent, const unsigned* __restrict__ base,
                                                    Geo g, const unsigned* __restrict__ gate,
                                                    const unsigned* __restrict__ start, float4* __restrict__ out) {
    __shared__ unsigned cur[kHaloSuperMax];
    if (*gate != 0u) return;
    const int sid = blockIdx.x;
    const int sx = sid / (g.ns * g.ns), sy = (sid / g.ns) % g.ns, sz = sid % g.ns;
    const int tps = g.sb * g.sb * g.sb;
    for (int i = threadIdx.x; i < tps; i += blockDim.x) {
        const int lx = i / (g.sb * g.sb), ly = (i / g.sb) % g.sb, lz = i % g.sb;
        cur[i] = start[((sx * g.sb + lx) * g.nt + (sy * g.sb + ly)) * g.nt + (sz * g.sb + lz)];
    }
    __syncthreads();
    const unsigned e0 = base[sid], e1 = base[sid + 1];
    for (unsigned e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const float4 v = ent[e];
        int a[3][2];
        halo_axes<P>(v.x, v.y, v.z, g, a);
        for_each_tile_in(a, g, sx, sy, sz, [&](unsigned local, unsigned gid) {
            const unsigned slot = atomicAdd(&cur[local], 1u);
            if (slot < start[gid + 1]) out[slot] = v;  // the counts bound every bin
        });
    }
}

// Words of the bins region: the largest |mass| (FP32 bits), the tile counts,
// the bin starts (tiles + 1), the gate (1: the bins do not fit), the
// fixed-point exponent s, the first level's gate, count matrix, row
// prefixes, superbin totals and superbin starts.
struct Bins {
    unsigned* mass_max;
    unsigned* count;
    unsigned* start;
    unsigned* gate;
    int* sexp;
    unsigned* gate_a;
    unsigned* cmat;    // counts per (superbin, first-level block)
    unsigned* loc;     // their prefixes within each superbin row (nb + 1 per row)
    unsigned* rowtot;  // superbin totals
    unsigned* base;    // superbin starts (nsup + 1)
};

// One block: exclusive prefix of the tile counts into start[], start[tiles] =
// total, the gate word set when the total exceeds the binned-entry capacity or
// the first level did not fit, and the fixed-point exponent s = 62 - E with
// |mass| < 2^e and every bin holding at most 2^(E - e) entries, so that every
// cell's integer sum stays below 2^62 in magnitude (weights are at most 1).
__global__ __launch_bounds__(1024) void k_bin_scan(Bins bn, int tiles, unsigned long long capacity) {
    __shared__ unsigned long long part[1024];
    __shared__ unsigned cmax[16];
    const unsigned* __restrict__ count = bn.count;
    const int t = threadIdx.x;
    const int per = (tiles + 1023) / 1024;
    const int b = t * per, e = min(tiles, b + per);
    unsigned long long sum = 0;
    unsigned mc = 0u;
    for (int i = b; i < e; ++i) {
        sum += count[i];
        mc = count[i] > mc ? count[i] : mc;
    }
    mc = wave_max_u32(mc);
    if ((t & 63) == 0) cmax[t >> 6] = mc;
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned long long v = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned long long run = part[t] - sum;
    const unsigned long long total = part[1023];
    const bool fits = total <= capacity;
    for (int i = b; i < e; ++i) {
        bn.start[i] = fits ? (unsigned)run : 0u;
        run += count[i];
    }
    if (t == 0) {
        bn.start[tiles] = fits ? (unsigned)total : 0u;
        *bn.gate = (fits && *bn.gate_a == 0u) ? 0u : 1u;
        unsigned c = cmax[0];
        for (int w = 1; w < 16; ++w) c = cmax[w] > c ? cmax[w] : c;
        const unsigned eb = *bn.mass_max >> 23;  // biased exponent of the largest |mass|
        const int e_mass = eb == 0u ? -126 : (int)eb - 126;
        const int e_count = c > 1u ? 32 - __clz(c - 1u) : 0;
        *bn.sexp = 62 - (e_mass + e_count);
    }
}

// One workgroup per tile, one mesh after the other: the bin's halos are added
// into the tile's cells in LDS as 64-bit fixed-point integers (contributions
// to other tiles are dropped: those tiles hold the halo in their own bins),
// then the 16^3 block is rounded to FP32 and written out.  With the gate set
// the blocks are written as zeros for the direct deposit.
template <int P>
__global__ __launch_bounds__(256) void k_tile_deposit(const float4* __restrict__ entries,
                                                      const unsigned* __restrict__ start,
                                                      const unsigned* __restrict__ gate,
                                                      const int* __restrict__ sexp, int n, int nt,
                                                      double to_cell, float* __restrict__ mesh0,
                                                      float* __restrict__ mesh1) {
    constexpr int T = kHaloTile, T3 = T * T * T;
    __shared__ __align__(16) unsigned long long acc[T3];
    const unsigned tile = blockIdx.x;
    const int tc[3] = {(int)(tile / (unsigned)(nt * nt)), (int)((tile / (unsigned)nt) % (unsigned)nt),
                       (int)(tile % (unsigned)nt)};
    const bool live = *gate == 0u;
    const double scale = ldexp(1.0, *sexp), unscale = ldexp(1.0, -*sexp);
    const unsigned b = start[tile], e = live ? start[tile + 1] : b;
    for (int mesh = 0; mesh < (mesh1 ? 2 : 1); ++mesh) {
        for (int i = threadIdx.x; i < T3; i += blockDim.x) acc[i] = 0ull;
        __syncthreads();
        const double shift = mesh ? 0.5 : 0.0;
        for (unsigned k = b + threadIdx.x; k < e; k += blockDim.x) {
            const float4 v = entries[k];
            const double m = (double)v.w;
            const double x[3] = {(double)v.x * to_cell, (double)v.y * to_cell, (double)v.z * to_cell};
            int loc[3][3];
            double w[3][3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                long long i0;
                assign_1d<P>(x[d] + shift, i0, w[d]);
#pragma unroll
                for (int a = 0; a < P; ++a) loc[d][a] = (int)wrap(i0 + a, n) - tc[d] * T;
            }
#pragma unroll
            for (int a = 0; a < P; ++a) {
                if ((unsigned)loc[0][a] >= (unsigned)T) continue;
#pragma unroll
                for (int bb = 0; bb < P; ++bb) {
                    if ((unsigned)loc[1][bb] >= (unsigned)T) continue;
#pragma unroll
                    for (int c = 0; c < P; ++c) {
                        if ((unsigned)loc[2][c] >= (unsigned)T) continue;
                        const long long q = __double2ll_rn((m * w[0][a] * w[1][bb] * w[2][c]) * scale);
                        atomicAdd(&acc[(loc[0][a] * T + loc[1][bb]) * T + loc[2][c]], (unsigned long long)q);
                    }
                }
            }
        }
        __syncthreads();
        // rows of 16 cells as 4 float4 per row: 1024 float4 per mesh
        float* out = mesh ? mesh1 : mesh0;
        for (int q = threadIdx.x; q < T3 / 4; q += blockDim.x) {
            const int row = q / (T / 4), part = q % (T / 4);
            const int lx = row / T, ly = row % T;
            const long long g = ((long long)(tc[0] * T + lx) * n + (tc[1] * T + ly)) * n + tc[2] * T + part * 4;
            const unsigned long long* a4 = &acc[row * T + part * 4];
            *reinterpret_cast<float4*>(out + g) =
                make_float4((float)((double)(long long)a4[0] * unscale), (float)((double)(long long)a4[1] * unscale),
                            (float)((double)(long long)a4[2] * unscale), (float)((double)(long long)a4[3] * unscale));
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int signed_freq(int m, int n) { return (2 * m <= n) ? m : m - n; }

// Per-axis factors of the combined spectrum, for frequency index m in [0, n):
// {sinc(pi s / n)^p, cos(pi s / n), sin(pi s / n), 0} with s the signed
// frequency, and {sinc^p, 1, 0, 1} on the Nyquist index (its phase enters
// through the Hermitian average instead).
__global__ __launch_bounds__(256) void k_axis_table(double4* __restrict__ tab, int n, int p) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int s = signed_freq(m, n);
    const double a = kPiD * (double)s / (double)n;
    double w = 1.0;
    if (s != 0) {
        const double v = sin(a) / a;
        w = p == 1 ? v : (p == 2 ? v * v : v * v * v);
    }
    tab[m] = (2 * s == n) ? make_double4(w, 1.0, 0.0, 1.0) : make_double4(w, cos(a), sin(a), 0.0);
}

// kCombineRows rows (x, y) of the main half spectrum per block (threads over
// kz < n/2), then one block per x of the Nyquist plane (threads over y,
// kz = n/2).
//   S = [A + phi B] / (2 W),  phi = e^{i alpha} cos(n_nyq pi / 2),
// W and e^{i alpha} being products of the per-axis factors.
constexpr unsigned kCombineRows = 8;
__global__ __launch_bounds__(256) void k_combine(float2* __restrict__ spec_a, float2* __restrict__ nyq_a,
                                                 const float2* __restrict__ spec_b, const float2* __restrict__ nyq_b,
                                                 const double4* __restrict__ tab, int n, int interlace) {
    const int h = n / 2;
    const unsigned b = blockIdx.x;
    const unsigned main_blocks = (unsigned)n * (unsigned)n / kCombineRows;
    const bool nyq_plane = b >= main_blocks;
    auto mode = [&](float2* a, const float2* bp, const double4& tx, const double4& ty, const double4& tz) {
        const float2 av = *a;
        double re = av.x, im = av.y;
        const double W = tx.x * ty.x * tz.x;
        if (interlace) {
            const float2 bv = *bp;
            // e^{i alpha} over the non-Nyquist axes (the Nyquist entries are 1)
            const double c1 = tx.y * ty.y - tx.z * ty.z, s1 = tx.y * ty.z + tx.z * ty.y;
            double c = c1 * tz.y - s1 * tz.z, sn = c1 * tz.z + s1 * tz.y;
            const int n_nyq = (int)(tx.w + ty.w + tz.w);
            const double cb = (n_nyq & 1) ? 0.0 : ((n_nyq & 2) ? -1.0 : 1.0);  // cos(n_nyq pi / 2)
            c *= cb;
            sn *= cb;
            re = 0.5 * (re + c * bv.x - sn * bv.y);
            im = 0.5 * (im + c * bv.y + sn * bv.x);
        }
        *a = make_float2((float)(re / W), (float)(im / W));
    };
    if (!nyq_plane) {
        for (unsigned r = 0; r < kCombineRows; ++r) {
            const unsigned row = b * kCombineRows + r;
            const double4 tx = tab[row / (unsigned)n], ty = tab[row % (unsigned)n];
            for (int i = threadIdx.x; i < h; i += blockDim.x) {
                const size_t off = (size_t)row * h + i;
                mode(spec_a + off, spec_b + off, tx, ty, tab[i]);
            }
        }
    } else {
        const int x = (int)(b - main_blocks);
        const double4 tx = tab[x], tz = tab[h];
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const size_t off = (size_t)x * n + i;
            mode(nyq_a + off, nyq_b + off, tx, tab[i], tz);
        }
    }
}

}  // namespace

int halo_source_spectrum(const amber_plan_s* p, const float* d_pos, const float* d_mass, long long n_halo,
                         int scheme, int interlace, unsigned char* ws, const WsLayout& L, hipStream_t s) {
    const int n = p->n;
    const long long n3 = (long long)n * n * n;
    float* mesh0 = reinterpret_cast<float*>(ws + L.mesh[0]);
    float* mesh1 = reinterpret_cast<float*>(ws + L.mesh[1]);
    float2* sa = reinterpret_cast<float2*>(ws + L.spec_a);
    float2* na = reinterpret_cast<float2*>(ws + L.nyq_a);
    float2* sb = reinterpret_cast<float2*>(ws + L.spec_b);
    float2* nb = reinterpret_cast<float2*>(ws + L.nyq_b);
    const double to_cell = (double)n / p->box_len;
    float* m1 = interlace ? mesh1 : nullptr;
    const size_t tiles = halo_tiles(n);
    // binned entries fit in u32 indices: at most 8 per halo
    const bool binned = tiles > 0 && n_halo < (1ll << 29);
    const unsigned* gate = nullptr;
    if (binned) {
        Geo g;
        g.n = n;
        g.nt = n / kHaloTile;
        g.sb = (g.nt % 8 == 0) ? 8 : (g.nt % 4 == 0) ? 4 : (g.nt % 2 == 0) ? 2 : 1;
        g.ns = g.nt / g.sb;
        g.to_cell = to_cell;
        g.interlace = interlace;
        const int nsup = g.ns * g.ns * g.ns;  // <= 512 for N <= 1024
        unsigned* words = reinterpret_cast<unsigned*>(ws + L.bins);
        Bins bn;
        bn.mass_max = words;
        bn.count = words + 1;
        bn.start = bn.count + tiles;
        bn.gate = bn.start + tiles + 1;
        bn.sexp = reinterpret_cast<int*>(bn.gate + 1);
        bn.gate_a = bn.gate + 2;
        bn.cmat = bn.gate + 3;
        bn.loc = bn.cmat + (size_t)kHaloSuperMax * kHaloSuperBlocks;
        bn.rowtot = bn.loc + (size_t)kHaloSuperMax * (kHaloSuperBlocks + 1);
        bn.base = bn.rowtot + kHaloSuperMax;
        gate = bn.gate;
        // first-level copies in the second spectrum, tile bins in the first:
        // both are written by the forward transforms only after the deposit
        float4* ent_a = reinterpret_cast<float4*>(ws + L.spec_b);
        float4* ent_b = reinterpret_cast<float4*>(ws + L.spec_a);
        const unsigned long long cap_a = (L.mesh[0] - L.spec_b) / sizeof(float4);
        const unsigned long long cap_b = (L.spec_b - L.spec_a) / sizeof(float4);
        const int nb = (int)std::max<long long>(1, std::min<long long>(kHaloSuperBlocks, (n_halo + 16383) / 16384));
        const long long chunk = (n_halo + nb - 1) / nb;
        AMBER_LAUNCH(p, "halo_bin_zero", k_zero_u32, dim3(1), dim3(256), s, words, 1ll);
#define AMBER_BINNING(PV)                                                                                          \
    AMBER_LAUNCH(p, "halo_super_count", k_super_count<PV>, dim3(nb), dim3(256), s, d_pos, d_mass, n_halo, chunk, g,  \
                 bn.cmat, nb, bn.mass_max);                                                                          \
    AMBER_LAUNCH(p, "halo_super_scan", k_row_scan, dim3(nsup), dim3(256), s, bn.cmat, nb, bn.loc, bn.rowtot);       \
    AMBER_LAUNCH(p, "halo_super_scan", k_rows_scan, dim3(1), dim3(1024), s, bn.rowtot, nsup, bn.base, cap_a,        \
                 bn.gate_a);                                                                                         \
    AMBER_LAUNCH(p, "halo_super_fill", k_super_fill<PV>, dim3(nb), dim3(256), s, d_pos, d_mass, n_halo, chunk, g,    \
                 bn.base, bn.loc, nb, bn.gate_a, ent_a);                                                             \
    AMBER_LAUNCH(p, "halo_tile_count", k_tile_count<PV>, dim3(nsup), dim3(1024), s, ent_a, bn.base, g, bn.gate_a,   \
                 bn.count);                                                                                          \
    AMBER_LAUNCH(p, "halo_bin_scan", k_bin_scan, dim3(1), dim3(1024), s, bn, (int)tiles, cap_b);                    \
    AMBER_LAUNCH(p, "halo_tile_fill", k_tile_fill<PV>, dim3(nsup), dim3(1024), s, ent_a, bn.base, g, gate,          \
                 bn.start, ent_b);                                                                                   \
    AMBER_LAUNCH(p, "halo_deposit", k_tile_deposit<PV>, dim3((unsigned)tiles), dim3(256), s, ent_b, bn.start, gate, \
                 bn.sexp, n, g.nt, to_cell, mesh0, m1);
        if (scheme == 1) {
            AMBER_BINNING(1)
        } else if (scheme == 2) {
            AMBER_BINNING(2)
        } else {
            AMBER_BINNING(3)
        }
#undef AMBER_BINNING
    } else {
        const unsigned zero_blocks = (unsigned)std::min<long long>(4096, (n3 + 255) / 256);
        AMBER_LAUNCH(p, "halo_zero", k_zero_f32, dim3(zero_blocks), dim3(256), s, mesh0, n3);
        if (interlace) AMBER_LAUNCH(p, "halo_zero", k_zero_f32, dim3(zero_blocks), dim3(256), s, mesh1, n3);
    }
    // direct deposit: always without bins, and behind the gate with them
    if (n_halo > 0) {
        const dim3 grid((unsigned)std::min<long long>(65536, (n_halo + 255) / 256)), blk(256);
        if (scheme == 1) AMBER_LAUNCH(p, "halo_deposit_direct", k_deposit<1>, grid, blk, s, d_pos, d_mass, n_halo, n, to_cell, mesh0, m1, gate);
        else if (scheme == 2) AMBER_LAUNCH(p, "halo_deposit_direct", k_deposit<2>, grid, blk, s, d_pos, d_mass, n_halo, n, to_cell, mesh0, m1, gate);
        else AMBER_LAUNCH(p, "halo_deposit_direct", k_deposit<3>, grid, blk, s, d_pos, d_mass, n_halo, n, to_cell, mesh0, m1, gate);
    }
    int rc = fft_forward(p, mesh0, sa, na, s);
    if (rc == AMBER_OK && interlace) rc = fft_forward(p, mesh1, sb, nb, s);
    if (rc != AMBER_OK) return rc;
    double4* tab = reinterpret_cast<double4*>(ws + L.halo_tab);
    AMBER_LAUNCH(p, "halo_axis_table", k_axis_table, dim3((unsigned)((n + 255) / 256)), dim3(256), s, tab, n, scheme);
    AMBER_LAUNCH(p, "halo_combine", k_combine, dim3((unsigned)((long long)n * n / kCombineRows + n)), dim3(256), s, sa,
                 na, sb, nb, tab, n, interlace);
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}
