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
// eight), then one workgroup per tile sums its bin into the tile's cells in
// LDS and writes the block with plain stores, so the meshes need neither
// zeroing nor global atomics.  The LDS sums are exact: every term m w_x w_y w_z
// (FP64 from the FP32 position and mass) is rounded once to a 64-bit integer
// multiple of 2^-s, s chosen from the largest |mass| and the largest bin so
// that no cell sum can overflow, and added with integer atomics; each cell is
// then rounded once to FP32.  The mesh therefore does not depend on the order
// of the halos or of the atomics, and repeated calls give identical fields.
// The binned copies live in the spectrum region, which the forward transforms
// only write afterwards; when they would not fit there (or on other grids)
// every halo adds its FP32 terms with global atomics instead, whose last bits
// depend on the order of the additions.
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

// Visits every tile a halo touches (1 to 8), calling f(tile id).
template <int P, typename F>
__device__ __forceinline__ void for_each_tile(const double* x, int n, int nt, bool interlace, F f) {
    int a[3][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) axis_tiles<P>(x[d], n, interlace, a[d][0], a[d][1]);
    for (int i = 0; i < (a[0][1] != a[0][0] ? 2 : 1); ++i)
        for (int j = 0; j < (a[1][1] != a[1][0] ? 2 : 1); ++j)
            for (int k = 0; k < (a[2][1] != a[2][0] ? 2 : 1); ++k)
                f((unsigned)((a[0][i] * nt + a[1][j]) * nt + a[2][k]));
}

__global__ __launch_bounds__(256) void k_zero_u32(unsigned* __restrict__ p, long long count) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Words of the bins region: the largest |mass| (FP32 bits), the tile counts,
// the fill cursors, the bin starts (tiles + 1), the gate (1: the bins do not
// fit), the fixed-point exponent s.
struct Bins {
    unsigned* mass_max;
    unsigned* count;
    unsigned* cursor;
    unsigned* start;
    unsigned* gate;
    int* sexp;
};

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned x = __shfl_xor(v, o, 64);
        v = x > v ? x : v;
    }
    return v;
}

template <int P>
__global__ __launch_bounds__(256) void k_bin_count(const float* __restrict__ pos, const float* __restrict__ mass,
                                                   long long n_halo, int n, int nt, double to_cell, int interlace,
                                                   unsigned* __restrict__ count, unsigned* __restrict__ mass_max) {
    __shared__ unsigned wmax[4];
    unsigned mx = 0u;
    for (long long h = (long long)blockIdx.x * blockDim.x + threadIdx.x; h < n_halo;
         h += (long long)gridDim.x * blockDim.x) {
        const double x[3] = {(double)pos[3 * h] * to_cell, (double)pos[3 * h + 1] * to_cell,
                             (double)pos[3 * h + 2] * to_cell};
        const unsigned mb = __float_as_uint(mass[h]) & 0x7fffffffu;
        mx = mb > mx ? mb : mx;
        for_each_tile<P>(x, n, nt, interlace != 0, [&](unsigned t) { atomicAdd(&count[t], 1u); });
    }
    mx = wave_max_u32(mx);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned m = wmax[0];
        for (int w = 1; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
        atomicMax(mass_max, m);
    }
}

// One block: exclusive prefix of the tile counts into start[] and cursor[],
// start[tiles] = total, the gate word set when the total exceeds the
// binned-entry capacity, and the fixed-point exponent s = 62 - E with
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
        const unsigned v = fits ? (unsigned)run : 0u;
        bn.start[i] = v;
        bn.cursor[i] = v;
        run += count[i];
    }
    if (t == 0) {
        bn.start[tiles] = fits ? (unsigned)total : 0u;
        *bn.gate = fits ? 0u : 1u;
        unsigned c = cmax[0];
        for (int w = 1; w < 16; ++w) c = cmax[w] > c ? cmax[w] : c;
        const unsigned eb = *bn.mass_max >> 23;  // biased exponent of the largest |mass|
        const int e_mass = eb == 0u ? -126 : (int)eb - 126;
        const int e_count = c > 1u ? 32 - __clz(c - 1u) : 0;
        *bn.sexp = 62 - (e_mass + e_count);
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_bin_fill(const float* __restrict__ pos, const float* __restrict__ mass,
                                                  long long n_halo, int n, int nt, double to_cell, int interlace,
                                                  unsigned* __restrict__ cursor, const unsigned* __restrict__ start,
                                                  const unsigned* __restrict__ gate, float4* __restrict__ entries) {
    if (*gate != 0u) return;
    for (long long h = (long long)blockIdx.x * blockDim.x + threadIdx.x; h < n_halo;
         h += (long long)gridDim.x * blockDim.x) {
        const float px = pos[3 * h], py = pos[3 * h + 1], pz = pos[3 * h + 2];
        const float4 v = make_float4(px, py, pz, mass[h]);
        const double x[3] = {(double)px * to_cell, (double)py * to_cell, (double)pz * to_cell};
        for_each_tile<P>(x, n, nt, interlace != 0, [&](unsigned t) {
            const unsigned slot = atomicAdd(&cursor[t], 1u);
            if (slot < start[t + 1]) entries[slot] = v;   // the counts bound every bin
        });
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

// One block per row (x, y) of the main half spectrum (threads over kz < n/2),
// then one block per x of the Nyquist plane (threads over y, kz = n/2).
//   S = [A + phi B] / (2 W),  phi = e^{i alpha} cos(n_nyq pi / 2),
// W and e^{i alpha} being products of the per-axis factors.
__global__ __launch_bounds__(256) void k_combine(float2* __restrict__ spec_a, float2* __restrict__ nyq_a,
                                                 const float2* __restrict__ spec_b, const float2* __restrict__ nyq_b,
                                                 const double4* __restrict__ tab, int n, int interlace) {
    const int h = n / 2;
    const unsigned b = blockIdx.x;
    const unsigned rows = (unsigned)n * (unsigned)n;
    const bool nyq_plane = b >= rows;
    const int x = nyq_plane ? (int)(b - rows) : (int)(b / (unsigned)n);
    const int y_row = nyq_plane ? 0 : (int)(b % (unsigned)n);
    const double4 tx = tab[x];
    const int cnt = nyq_plane ? n : h;
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int y = nyq_plane ? i : y_row, kz = nyq_plane ? h : i;
        const double4 ty = tab[y], tz = tab[kz];
        const size_t off = nyq_plane ? (size_t)x * n + i : (size_t)b * h + i;
        float2* a = (nyq_plane ? nyq_a : spec_a) + off;
        const float2 av = *a;
        double re = av.x, im = av.y;
        const double W = tx.x * ty.x * tz.x;
        if (interlace) {
            const float2 bv = (nyq_plane ? nyq_b : spec_b)[off];
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
        const int nt = n / kHaloTile;
        unsigned* words = reinterpret_cast<unsigned*>(ws + L.bins);
        Bins bn;
        bn.mass_max = words;
        bn.count = words + 1;
        bn.cursor = bn.count + tiles;
        bn.start = bn.cursor + tiles;
        bn.gate = bn.start + tiles + 1;
        bn.sexp = reinterpret_cast<int*>(bn.gate + 1);
        unsigned* count = bn.count;
        unsigned* cursor = bn.cursor;
        unsigned* start = bn.start;
        gate = bn.gate;
        float4* entries = reinterpret_cast<float4*>(ws + L.spec_a);
        const unsigned long long capacity = (L.mesh[0] - L.spec_a) / sizeof(float4);
        const unsigned hb = (unsigned)std::max<long long>(1, std::min<long long>(16384, (n_halo + 255) / 256));
        AMBER_LAUNCH(p, "halo_bin_zero", k_zero_u32, dim3((unsigned)((tiles + 256) / 256)), dim3(256), s, words,
                     (long long)tiles + 1);
        if (scheme == 1) {
            AMBER_LAUNCH(p, "halo_bin_count", k_bin_count<1>, dim3(hb), dim3(256), s, d_pos, d_mass, n_halo, n, nt, to_cell, interlace, count, bn.mass_max);
        } else if (scheme == 2) {
            AMBER_LAUNCH(p, "halo_bin_count", k_bin_count<2>, dim3(hb), dim3(256), s, d_pos, d_mass, n_halo, n, nt, to_cell, interlace, count, bn.mass_max);
        } else {
            AMBER_LAUNCH(p, "halo_bin_count", k_bin_count<3>, dim3(hb), dim3(256), s, d_pos, d_mass, n_halo, n, nt, to_cell, interlace, count, bn.mass_max);
        }
        AMBER_LAUNCH(p, "halo_bin_scan", k_bin_scan, dim3(1), dim3(1024), s, bn, (int)tiles, capacity);
        if (scheme == 1) {
            AMBER_LAUNCH(p, "halo_bin_fill", k_bin_fill<1>, dim3(hb), dim3(256), s, d_pos, d_mass, n_halo, n, nt, to_cell, interlace, cursor, start, gate, entries);
            AMBER_LAUNCH(p, "halo_deposit", k_tile_deposit<1>, dim3((unsigned)tiles), dim3(256), s, entries, start, gate, bn.sexp, n, nt, to_cell, mesh0, m1);
        } else if (scheme == 2) {
            AMBER_LAUNCH(p, "halo_bin_fill", k_bin_fill<2>, dim3(hb), dim3(256), s, d_pos, d_mass, n_halo, n, nt, to_cell, interlace, cursor, start, gate, entries);
            AMBER_LAUNCH(p, "halo_deposit", k_tile_deposit<2>, dim3((unsigned)tiles), dim3(256), s, entries, start, gate, bn.sexp, n, nt, to_cell, mesh0, m1);
        } else {
            AMBER_LAUNCH(p, "halo_bin_fill", k_bin_fill<3>, dim3(hb), dim3(256), s, d_pos, d_mass, n_halo, n, nt, to_cell, interlace, cursor, start, gate, entries);
            AMBER_LAUNCH(p, "halo_deposit", k_tile_deposit<3>, dim3((unsigned)tiles), dim3(256), s, entries, start, gate, bn.sexp, n, nt, to_cell, mesh0, m1);
        }
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
    AMBER_LAUNCH(p, "halo_combine", k_combine, dim3((unsigned)((long long)n * n + n)), dim3(256), s, sa, na, sb, nb,
                 tab, n, interlace);
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}
