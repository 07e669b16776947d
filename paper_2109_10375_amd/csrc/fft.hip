// Radiation field on gfx950: J = IDFT[ DFT(S) * atan(k l)/k ] / N^3 (Sec. 3.4.1,
// Eq. intensity, evaluated as a periodic convolution through FFTs).
//
// Spectrum layout (device workspace, complex FP32):
//   main[x][y][kz] for kz in [0, N/2)   (row pitch N/2, 256-byte aligned rows)
//   nyq[x][y]      for kz = N/2          (the real-input Nyquist plane)
// Five streaming passes per l_mfp, each reading and writing the array once:
//   1. z  : real-to-complex along the contiguous axis (lines of N reals)
//   2. y  : complex FFT down columns of the (x, kz) planes, tiles of C columns
//   3. x  : forward FFT, multiply by Khat/N^3, inverse FFT, in one kernel
//   4. y  : inverse
//   5. z  : complex-to-real
// Every length-L transform inside a pass is split L = L1 x L2 over L1 threads:
// each thread does an L2-point DFT in registers on a decimated subsequence,
// applies the inter-step twiddles, exchanges through LDS (padded against bank
// conflicts), and finishes with L1-point DFTs in registers.  A thread ends up
// holding the same element positions it loaded, so every pass reads and writes
// with the same coalesced pattern.  Twiddles come from an FP64-generated table;
// the in-register DFT constants are exact compile-time values.
#include <cmath>
#include <type_traits>

#include "internal.h"

namespace {

// ---------------------------------------------------------------------------
// Compile-time roots of unity: cos/sin(2 pi m / R) with the quadrant removed
// exactly in integers and a Taylor series on |r| <= pi/4.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / double((2 * k) * (2 * k + 1));
        sum += term;
    }
    return sum;
}

constexpr double taylor_cos(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / double((2 * k - 1) * (2 * k));
        sum += term;
    }
    return sum;
}

struct Root {
    double c, s;
};

constexpr Root root_of_unity(long m, long R) {
    m %= R;
    if (m < 0) m += R;
    long q = (8 * m + R) / (2 * R);  // nearest multiple of pi/2
    long rn = 4 * m - q * R;         // |rn| <= R/2
    double r = (kPi / 2.0) * double(rn) / double(R);
    double c = taylor_cos(r), s = taylor_sin(r);
    switch (q & 3) {
        case 0: return Root{c, s};
        case 1: return Root{-s, c};
        case 2: return Root{-c, -s};
        default: return Root{s, -c};
    }
}

template <int R>
struct RootTable {
    float c[R];
    float s[R];
    constexpr RootTable() : c(), s() {
        for (int m = 0; m < R; ++m) {
            Root t = root_of_unity(m, R);
            c[m] = float(t.c);
            s[m] = float(t.s);
        }
    }
};

template <int R>
__device__ constexpr RootTable<R> kRoots = RootTable<R>();

// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 v) {
    return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
}

// v * W_R^e with W_R = exp(-2 pi i / R) (forward) or its conjugate (inverse);
// e is a compile-time constant after unrolling.
template <int R, bool INV>
__device__ __forceinline__ float2 twc(float2 v, int e) {
    e %= R;
    if (e == 0) return v;
    if (4 * e == R) return mul_mi<INV>(v);
    if (2 * e == R) return make_float2(-v.x, -v.y);
    if (4 * e == 3 * R) return mul_mi<!INV>(v);
    const float c = kRoots<R>.c[e];
    const float s = INV ? kRoots<R>.s[e] : -kRoots<R>.s[e];
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
}

// W_N^k for k = t + S j (S | N, j < N / S): one table read W_N^t per thread
// times the compile-time root W_{N/S}^j (one extra rounding of a complex
// product instead of a table read per k).
template <int N, int S>
__device__ __forceinline__ float2 tw_split(float2 wt, int j) {
    constexpr int R = N / S;
    const int m = j % R;
    if (m == 0) return wt;
    return cmul(wt, make_float2(kRoots<R>.c[m], -kRoots<R>.s[m]));
}

// In-register DFT of R points, natural order in and out.
template <int R>
struct Split {  // R = A * B
    static constexpr int A = R == 6 ? 2 : R == 8 ? 4 : R == 12 ? 4 : R == 16 ? 4 : R == 24 ? 8 : R == 32 ? 8 : 0;
    static constexpr int B = A ? R / A : 0;
};

template <int R, bool INV>
struct Dft {
    __device__ __forceinline__ static void run(float2* x) {
        constexpr int A = Split<R>::A, B = Split<R>::B;
        static_assert(A * B == R && A > 1, "unsupported in-register DFT size");
        float2 t[R];
#pragma unroll
        for (int a = 0; a < A; ++a) {
            float2 col[B];
#pragma unroll
            for (int b = 0; b < B; ++b) col[b] = x[a + A * b];
            Dft<B, INV>::run(col);
#pragma unroll
            for (int kb = 0; kb < B; ++kb) t[a * B + kb] = twc<R, INV>(col[kb], a * kb);
        }
#pragma unroll
        for (int kb = 0; kb < B; ++kb) {
            float2 row[A];
#pragma unroll
            for (int a = 0; a < A; ++a) row[a] = t[a * B + kb];
            Dft<A, INV>::run(row);
#pragma unroll
            for (int ka = 0; ka < A; ++ka) x[kb + B * ka] = row[ka];
        }
    }
};

template <bool INV>
struct Dft<1, INV> {
    __device__ __forceinline__ static void run(float2*) {}
};

template <bool INV>
struct Dft<2, INV> {
    __device__ __forceinline__ static void run(float2* x) {
        float2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};

template <bool INV>
struct Dft<3, INV> {
    __device__ __forceinline__ static void run(float2* x) {
        const float h = 0.8660254037844386f;  // sin(2 pi / 3)
        float2 s = cadd(x[1], x[2]);
        float2 d = csub(x[1], x[2]);
        float2 m = make_float2(x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y);
        float2 r = mul_mi<INV>(cscale(d, h));  // -i h d forward
        x[0] = cadd(x[0], s);
        x[1] = cadd(m, r);
        x[2] = csub(m, r);
    }
};

template <bool INV>
struct Dft<4, INV> {
    __device__ __forceinline__ static void run(float2* x) {
        float2 a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        float2 c = cadd(x[1], x[3]), d = mul_mi<INV>(csub(x[1], x[3]));
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        x[1] = cadd(b, d);
        x[3] = csub(b, d);
    }
};

// ---------------------------------------------------------------------------
// One length-L transform spread over L1 threads, L2 = L / L1 elements each,
// L1 | L2.  On entry v[j] = x[t + L1 j]; on exit v[j] = X[t + L1 j].
// lds points at this transform's LDS region: element (n1, k2) lives at
// lds[n1 * SN1 + k2 * SK2].  tw is the table of exp(-2 pi i j / (L * TS)).
// Inter-step twiddles W^(t k2), k2 = 1 .. L2 - 1.  Read from the table one
// by one (TWP = false), or (TWP = true) as products W^(t a) W^(t S b) of
// table entries, k2 = a + S b with S^2 >= L2: S - 1 + L2/S - 1 reads instead
// of L2 - 1 (10 instead of 31 for L2 = 32), so far fewer values are held in
// registers while the reads are in flight, at about one extra rounding of a
// complex product on the entries with a, b > 0.
template <int L2>
struct TwSplit {
    static constexpr int S = L2 <= 4 ? L2 : (L2 <= 16 ? 4 : 8);
    static_assert(L2 % S == 0, "twiddle split");
};

// SPLIT: the LDS exchange moves the real parts, then the imaginary parts,
// through a float array of the same layout (half the LDS of a float2 one).
template <int L, int L1, bool INV, int TS, int SN1, int SK2, bool TWP = false, bool SPLIT = false, class E = float2>
__device__ __forceinline__ void fft_2step(float2* v, int t, E* lds, const float2* __restrict__ tw) {
    static_assert(std::is_same<E, float>::value == SPLIT, "the LDS element type follows SPLIT");
    constexpr int L2 = L / L1;
    constexpr int RR = L2 / L1;
    static_assert(L1 * L2 == L && RR * L1 == L2, "bad split");
    Dft<L2, INV>::run(v);
    if constexpr (TWP) {
        constexpr int S = TwSplit<L2>::S, B = L2 / S;
        float2 wa[S], wb[B];
        wa[0] = wb[0] = make_float2(1.0f, 0.0f);
#pragma unroll
        for (int a = 1; a < S; ++a) wa[a] = tw[(t * a) * TS];
#pragma unroll
        for (int b = 1; b < B; ++b) wb[b] = tw[(t * S * b) * TS];
#pragma unroll
        for (int k2 = 1; k2 < L2; ++k2) {
            const int a = k2 % S, b = k2 / S;
            float2 w = (a == 0) ? wb[b] : (b == 0 ? wa[a] : cmul(wa[a], wb[b]));
            if (INV) w.y = -w.y;
            v[k2] = cmul(v[k2], w);
        }
    } else {
#pragma unroll
        for (int k2 = 1; k2 < L2; ++k2) {
            float2 w = tw[(t * k2) * TS];
            if (INV) w.y = -w.y;
            v[k2] = cmul(v[k2], w);
        }
    }
    if constexpr (SPLIT) {
        float re[L2];  // this thread's real parts after the exchange, RR groups of L1
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < L2; ++k2) lds[t * SN1 + k2 * SK2] = v[k2].x;
        __syncthreads();
#pragma unroll
        for (int b = 0; b < RR; ++b)
#pragma unroll
            for (int n1 = 0; n1 < L1; ++n1) re[b * L1 + n1] = lds[n1 * SN1 + (t + L1 * b) * SK2];
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < L2; ++k2) lds[t * SN1 + k2 * SK2] = v[k2].y;
        __syncthreads();
#pragma unroll
        for (int b = 0; b < RR; ++b) {
            const int k2 = t + L1 * b;
            float2 u[L1];
#pragma unroll
            for (int n1 = 0; n1 < L1; ++n1) u[n1] = make_float2(re[b * L1 + n1], lds[n1 * SN1 + k2 * SK2]);
            Dft<L1, INV>::run(u);
#pragma unroll
            for (int k1 = 0; k1 < L1; ++k1) v[b + RR * k1] = u[k1];
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < L2; ++k2) lds[t * SN1 + k2 * SK2] = v[k2];
        __syncthreads();
#pragma unroll
        for (int b = 0; b < RR; ++b) {
            const int k2 = t + L1 * b;
            float2 u[L1];
#pragma unroll
            for (int n1 = 0; n1 < L1; ++n1) u[n1] = lds[n1 * SN1 + k2 * SK2];
            Dft<L1, INV>::run(u);
#pragma unroll
            for (int k1 = 0; k1 < L1; ++k1) v[b + RR * k1] = u[k1];
        }
    }
}

// Launch schedules.  A column pass splits L = N into N1 x N2 and takes tiles
// of C columns (C * N1 threads); a z pass splits M = N/2 into M1 x M2 and takes
// ZL lines per block (ZL * M1 threads).  Each grid size has a list of
// candidates; the first is the default and a plan may pick any of them (the
// tuner times them on the device).  Every candidate keeps L1 | L2 with both
// factors among the in-register DFT sizes.
template <int N1_, int C_>
struct ColS {
    static constexpr int N1 = N1_, C = C_;
};
template <int M1_, int ZL_>
struct ZS {
    static constexpr int M1 = M1_, ZL = ZL_;
};
template <class... T>
struct List {
    static constexpr int size = sizeof...(T);
};
template <int N>
struct Scheds;
template <> struct Scheds<8>    { using col = List<ColS<2, 4>>;   using z = List<ZS<2, 64>>; };
template <> struct Scheds<16>   { using col = List<ColS<4, 8>>;   using z = List<ZS<2, 64>>; };
template <> struct Scheds<32>   { using col = List<ColS<4, 16>>;  using z = List<ZS<4, 64>>; };
template <> struct Scheds<64>   { using col = List<ColS<8, 32>>;  using z = List<ZS<4, 64>>; };
template <> struct Scheds<96>   { using col = List<ColS<4, 16>>;  using z = List<ZS<4, 64>>; };
template <> struct Scheds<128>  { using col = List<ColS<8, 32>, ColS<8, 16>, ColS<4, 32>>;
                                  using z = List<ZS<8, 32>, ZS<4, 64>, ZS<8, 64>>; };
template <> struct Scheds<192>  { using col = List<ColS<8, 32>, ColS<8, 16>, ColS<8, 48>>;
                                  using z = List<ZS<4, 64>, ZS<4, 32>, ZS<4, 16>>; };
template <> struct Scheds<256>  { using col = List<ColS<16, 16>, ColS<8, 32>, ColS<16, 8>>;
                                  using z = List<ZS<8, 32>, ZS<4, 64>, ZS<8, 16>>; };
template <> struct Scheds<512>  { using col = List<ColS<16, 16>, ColS<16, 8>, ColS<16, 32>>;
                                  using z = List<ZS<16, 16>, ZS<8, 32>, ZS<16, 8>>; };
template <> struct Scheds<1024> { using col = List<ColS<32, 8>, ColS<32, 4>, ColS<32, 16>>;
                                  using z = List<ZS<16, 16>, ZS<16, 8>, ZS<16, 32>>; };

// Tile geometry of a column pass: element (row r, column c) of tile (ta, tb)
// is at ta * sa + tb * sb + r * row + c * col (complex elements).
struct ColGeom {
    long long row, col, sa, sb;
    int tiles_b;
};

struct MulArgs {
    float c2;     // (2 pi l_mfp / box_len)^2: x^2 = c2 |m~|^2 with x = k l_mfp
    float ls;     // l_mfp / N^3
    int nyq;      // 1: the Nyquist plane (kz = N/2, columns are ky)
};

MulArgs mul_args(double box_len, double l_mfp, int n, int nyq) {
    const double kl = 2.0 * kPi * l_mfp / box_len;
    return MulArgs{(float)(kl * kl), (float)(l_mfp / ((double)n * n * n)), nyq};
}

// Khat(k)/N^3 = (l/N^3) g(x), g(x) = atan(x)/x, x = k l, from x^2 = c2 |m~|^2.
// On x <= 1, g = P(x^2); above, atan(x) = pi/2 - atan(1/x) gives
// g(x) = r (pi/2 - r P(r^2)) with r = 1/x.  P is a degree-9 polynomial with
// P(0) = 1, fitted to atan(sqrt t)/sqrt t on [0, 1] for relative error
// (csrc/fit_atan.py; 8e-8 relative in FP32); the reciprocal and reciprocal
// square root are the hardware's (about 1 ulp).
__device__ __forceinline__ float khat_scaled(float x2, float ls) {
    constexpr float kP[10] = {-1.744857524e-03f, 1.069426350e-02f, -3.076297976e-02f, 5.753647164e-02f,
                              -8.378560096e-02f, 1.094356626e-01f, -1.426257640e-01f, 1.999839097e-01f,
                              -3.333329260e-01f, 1.000000000e+00f};
    const bool big = x2 > 1.0f;
    const float t = big ? __builtin_amdgcn_rcpf(x2) : x2;
    float p = kP[0];
#pragma unroll
    for (int i = 1; i < 10; ++i) p = __builtin_fmaf(p, t, kP[i]);
    const float r = __builtin_amdgcn_rsqf(big ? x2 : 1.0f);
    const float g = big ? r * (1.57079632679489662f - r * p) : p;
    return g * ls;
}

__device__ __forceinline__ int signed_freq(int m, int n) { return (2 * m <= n) ? m : m - n; }

// Workgroups are dispatched to the 8 XCDs round robin (block b runs on XCD
// b % 8, each XCD with its own L2).  Neighbouring tiles read the two 64-byte
// halves of the same 128-byte lines, so each XCD takes one contiguous run of
// tiles instead of every eighth tile.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned grid) {
    if (grid % 8u != 0u) return b;
    return (b % 8u) * (grid / 8u) + b / 8u;
}

// Column pass.  MODE 0: one transform (INV selects the direction).
// MODE 1: forward transform, multiply by Khat(|k|)/N^3, inverse transform.
// MODE 2: the input is already transformed along x: multiply, inverse.
template <int N, class CS, int MODE, bool INV>
__global__ __launch_bounds__(CS::C * CS::N1, MODE != 0 ? 4 : 2) void k_fft_cols(
    const float2* __restrict__ in, float2* __restrict__ out, const float2* __restrict__ tw,
    ColGeom g, MulArgs m) {
    constexpr int N1 = CS::N1, C = CS::C, N2 = N / N1;
    // A column pass exchanges real and imaginary parts separately (half the
    // LDS, so more blocks share a compute unit) and forms its twiddles as
    // products (fewer registers); the x pass, which holds a column through
    // two transforms and the multiply, is held to four waves per SIMD.
    __shared__ float lds[N1 * (N2 + 1) * C];
    const int tid = threadIdx.x;
    const int c = tid % C, t = tid / C;
    const unsigned bid = xcd_tile(blockIdx.x, gridDim.x);
    const int tb = bid % g.tiles_b, ta = bid / g.tiles_b;
    const long long base = (long long)ta * g.sa + (long long)tb * g.sb + (long long)c * g.col;
    float2 v[N2];
#pragma unroll
    for (int j = 0; j < N2; ++j) v[j] = in[base + (long long)(t + N1 * j) * g.row];
    float* col = lds + c;
    if constexpr (MODE == 0) {
        fft_2step<N, N1, INV, 1, (N2 + 1) * C, C, true, true>(v, t, col, tw);
    } else {
        if (MODE == 1) fft_2step<N, N1, false, 1, (N2 + 1) * C, C, true, true>(v, t, col, tw);
        int my, mz;
        if (m.nyq) {
            my = tb * C + c;
            mz = N / 2;
        } else {
            my = ta;
            mz = tb * C + c;
        }
        const int sy = signed_freq(my, N), sz = mz;
        const int s2yz = sy * sy + sz * sz;
#pragma unroll
        for (int j = 0; j < N2; ++j) {
            const int sx = signed_freq(t + N1 * j, N);
            v[j] = cscale(v[j], khat_scaled(m.c2 * (float)(sx * sx + s2yz), m.ls));
        }
        fft_2step<N, N1, true, 1, (N2 + 1) * C, C, true, true>(v, t, col, tw);
    }
    // The store addresses are recomputed here rather than kept from the loads
    // (kept, they are spilled to scratch in the fused passes at N = 1024).
    long long obase = base + (long long)t * g.row;
    asm volatile("" : "+v"(obase));
#pragma unroll
    for (int j = 0; j < N2; ++j) out[obase + (long long)(N1 * j) * g.row] = v[j];
}

// z pass, real to complex: N reals per line -> N/2 + 1 complex (N/2 in main,
// the Nyquist value in nyq).  Packs x[2n] + i x[2n+1], does an N/2-point FFT
// and separates even and odd halves:
//   X[k] = (Z[k] + conj Z[M-k])/2 - i W_N^k (Z[k] - conj Z[M-k])/2.
template <int N, class ZSc>
__global__ __launch_bounds__(ZSc::ZL * ZSc::M1) void k_fft_z_r2c(
    const float* __restrict__ src, float2* __restrict__ main_out, float2* __restrict__ nyq_out,
    const float2* __restrict__ tw, long long n_lines) {
    constexpr int M = N / 2, M1 = ZSc::M1, M2 = M / M1, ZL = ZSc::ZL;
    constexpr int LS = M1 * (M2 + 1);  // per-line LDS stride (>= M + 1)
    // real and imaginary parts go through LDS one after the other (half the
    // LDS of a complex exchange, so more blocks share a compute unit)
    __shared__ float lds[ZL * LS];
    const int tid = threadIdx.x;
    const int t = tid % M1, l = tid / M1;
    const long long line = (long long)blockIdx.x * ZL + l;
    const bool live = line < n_lines;
    const float2* row = reinterpret_cast<const float2*>(src + (live ? line : 0) * N);
    float2 v[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) v[j] = live ? row[t + M1 * j] : make_float2(0.f, 0.f);
    float* mine = lds + l * LS;
    fft_2step<M, M1, false, 2, M2 + 1, 1, true, true>(v, t, mine, tw);
    // X[k] from Z[k] and Z[M-k]: the real parts first (a.x, b.x), then the
    // imaginary parts (a.y, b.y)
    float ax[M2], bx[M2], z0x = 0.0f;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M2; ++j) mine[t + M1 * j] = v[j].x;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M2; ++j) {
        const int k = t + M1 * j;
        const float zk = mine[k], zc = mine[(M - k) % M];
        ax[j] = 0.5f * (zk + zc);
        bx[j] = 0.5f * (zk - zc);
    }
    if (t == 0) z0x = mine[0];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M2; ++j) mine[t + M1 * j] = v[j].y;
    __syncthreads();
    float2* orow = main_out + (live ? line : 0) * M;
    const float2 wt = tw[t];  // W_N^t; tw[k] = W_N^t W_{N/M1}^j
#pragma unroll
    for (int j = 0; j < M2; ++j) {
        const int k = t + M1 * j;
        const float zk = mine[k], zc = mine[(M - k) % M];
        const float2 a = make_float2(ax[j], 0.5f * (zk - zc));
        const float2 b = make_float2(bx[j], 0.5f * (zk + zc));
        const float2 wb = cmul(tw_split<N, M1>(wt, j), b);
        if (live) orow[k] = make_float2(a.x + wb.y, a.y - wb.x);
    }
    if (live && t == 0) nyq_out[line] = make_float2(z0x - mine[0], 0.0f);
}

// z pass, complex to real (unnormalised inverse):
//   Z'[k] = (X[k] + conj X[M-k]) + i W_N^-k (X[k] - conj X[M-k]),
//   z = IDFT_M(Z'),  x[2n] = Re z[n], x[2n+1] = Im z[n].
template <int N, class ZSc>
__global__ __launch_bounds__(ZSc::ZL * ZSc::M1) void k_fft_z_c2r(
    const float2* __restrict__ main_in, const float2* __restrict__ nyq_in, float* __restrict__ dst,
    const float2* __restrict__ tw, long long n_lines) {
    constexpr int M = N / 2, M1 = ZSc::M1, M2 = M / M1, ZL = ZSc::ZL;
    constexpr int LS = M1 * (M2 + 1);
    // real and imaginary parts go through LDS one after the other
    __shared__ float lds[ZL * LS];
    const int tid = threadIdx.x;
    const int t = tid % M1, l = tid / M1;
    const long long line = (long long)blockIdx.x * ZL + l;
    const bool live = line < n_lines;
    const float2* irow = main_in + (live ? line : 0) * M;
    float* mine = lds + l * LS;
    // all loads in flight before the LDS writes (a dead line reads line 0 and
    // is never stored)
    float2 in[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) in[j] = irow[t + M1 * j];
    const float2 nq = nyq_in[live ? line : 0];
    // X[k] and X[M-k]: the real parts first (e.x, d.x), then the imaginary
    // parts (e.y, d.y)
    float ex[M2], dx[M2];
#pragma unroll
    for (int j = 0; j < M2; ++j) mine[t + M1 * j] = in[j].x;
    if (t == 0) mine[M] = nq.x;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M2; ++j) {
        const int k = t + M1 * j;
        const float xk = mine[k], xm = mine[M - k];
        ex[j] = xk + xm;
        dx[j] = xk - xm;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M2; ++j) mine[t + M1 * j] = in[j].y;
    if (t == 0) mine[M] = nq.y;
    __syncthreads();
    float2 v[M2];
    const float2 wt = tw[t];  // W_N^t; tw[k] = W_N^t W_{N/M1}^j
#pragma unroll
    for (int j = 0; j < M2; ++j) {
        const int k = t + M1 * j;
        const float xk = mine[k], xm = mine[M - k];
        const float2 e = make_float2(ex[j], xk - xm);              // X[k] + conj X[M-k]
        const float2 d = make_float2(dx[j], xk + xm);              // X[k] - conj X[M-k]
        const float2 w = tw_split<N, M1>(wt, j);
        const float2 o = cmul(d, make_float2(w.x, -w.y));          // * W_N^-k
        v[j] = make_float2(e.x - o.y, e.y + o.x);                  // e + i o
    }
    fft_2step<M, M1, true, 2, M2 + 1, 1, true, true>(v, t, mine, tw);
    if (live) {
        float2* orow = reinterpret_cast<float2*>(dst + line * N);
#pragma unroll
        for (int j = 0; j < M2; ++j) orow[t + M1 * j] = v[j];
    }
}

template <int N, class CS, class ZSc>
int run_radiation(const amber_plan_s* p, const float* d_src, const double* l_mfp, int n_lmfp,
                  float* const* d_J, unsigned char* ws, const WsLayout& L, hipStream_t s) {
    constexpr int H = N / 2, C = CS::C, N1 = CS::N1, ZL = ZSc::ZL, M1 = ZSc::M1;
    static_assert(H % C == 0 && N % C == 0, "tile width must divide the spectrum rows");
    const long long n_lines = (long long)N * N;
    float2* spec_a = reinterpret_cast<float2*>(ws + L.spec_a);
    float2* nyq_a = reinterpret_cast<float2*>(ws + L.nyq_a);
    float2* spec_b = reinterpret_cast<float2*>(ws + L.spec_b);
    float2* nyq_b = reinterpret_cast<float2*>(ws + L.nyq_b);
    const float2* tw = p->d_tw;
    const dim3 zblk(ZL * M1), cblk(C * N1);
    const unsigned zgrid = (unsigned)((n_lines + ZL - 1) / ZL);

    // geometry of the four kinds of column pass
    const ColGeom y_main{H, 1, (long long)N * H, C, H / C};
    const ColGeom y_nyq{1, N, 0, (long long)C * N, N / C};
    const ColGeom x_main{(long long)N * H, 1, H, C, H / C};
    const ColGeom x_nyq{N, 1, 0, C, N / C};
    const unsigned g_main = (unsigned)N * (H / C), g_nyq = (unsigned)(N / C);
    const MulArgs none{0.f, 0.f, 0};

    AMBER_LAUNCH(p, "fft_z_r2c", (k_fft_z_r2c<N, ZSc>), dim3(zgrid), zblk, s, d_src, spec_a, nyq_a, tw, n_lines);
    AMBER_LAUNCH(p, "fft_y", (k_fft_cols<N, CS, 0, false>), dim3(g_main), cblk, s, spec_a, spec_a, tw, y_main, none);
    AMBER_LAUNCH(p, "fft_nyq_y", (k_fft_cols<N, CS, 0, false>), dim3(g_nyq), cblk, s, nyq_a, nyq_a, tw, y_nyq, none);
    for (int i = 0; i < n_lmfp; ++i) {
        float2* so = (n_lmfp == 1) ? spec_a : spec_b;
        float2* no = (n_lmfp == 1) ? nyq_a : nyq_b;
        const MulArgs mm = mul_args(p->box_len, l_mfp[i], N, 0);
        const MulArgs mn = mul_args(p->box_len, l_mfp[i], N, 1);
        AMBER_LAUNCH(p, "fft_x_mul", (k_fft_cols<N, CS, 1, false>), dim3(g_main), cblk, s, spec_a, so, tw, x_main, mm);
        AMBER_LAUNCH(p, "fft_nyq_x_mul", (k_fft_cols<N, CS, 1, false>), dim3(g_nyq), cblk, s, nyq_a, no, tw, x_nyq, mn);
        AMBER_LAUNCH(p, "fft_y_inv", (k_fft_cols<N, CS, 0, true>), dim3(g_main), cblk, s, so, so, tw, y_main, none);
        AMBER_LAUNCH(p, "fft_nyq_y_inv", (k_fft_cols<N, CS, 0, true>), dim3(g_nyq), cblk, s, no, no, tw, y_nyq, none);
        AMBER_LAUNCH(p, "fft_z_c2r", (k_fft_z_c2r<N, ZSc>), dim3(zgrid), zblk, s, so, no, d_J[i], tw, n_lines);
    }
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}


// Runs f(integral_constant<N>, column schedule, z schedule) for the plan's grid
// size and chosen candidates.
template <class F, class T0, class... T>
int pick(List<T0, T...>, int idx, F&& f) {
    if (idx == 0) return f(T0{});
    if constexpr (sizeof...(T) > 0) {
        return pick(List<T...>{}, idx - 1, f);
    } else {
        return AMBER_E_ARG;
    }
}

template <int N, class F>
int with_scheds(int col, int z, F&& f) {
    return pick(typename Scheds<N>::col{}, col, [&](auto cs) {
        return pick(typename Scheds<N>::z{}, z, [&](auto zs) { return f(std::integral_constant<int, N>{}, cs, zs); });
    });
}

template <class F>
int with_size(int n, F&& f) {
    switch (n) {
        case 8: return f(std::integral_constant<int, 8>{});
        case 16: return f(std::integral_constant<int, 16>{});
        case 32: return f(std::integral_constant<int, 32>{});
        case 64: return f(std::integral_constant<int, 64>{});
        case 96: return f(std::integral_constant<int, 96>{});
        case 128: return f(std::integral_constant<int, 128>{});
        case 192: return f(std::integral_constant<int, 192>{});
        case 256: return f(std::integral_constant<int, 256>{});
        case 512: return f(std::integral_constant<int, 512>{});
        case 1024: return f(std::integral_constant<int, 1024>{});
        default: return AMBER_E_SIZE;
    }
}

template <class F>
int dispatch(const amber_plan_s* p, F&& f) {
    return with_size(p->n, [&](auto n) { return with_scheds<decltype(n)::value>(p->col_sched, p->z_sched, f); });
}

}  // namespace

// Forward real 3D FFT only (unnormalised): main[x][y][kz < N/2] and nyq[x][y].
template <int N, class CS, class ZSc>
int run_forward(const amber_plan_s* p, const float* d_src, float2* spec, float2* nyq, hipStream_t s) {
    constexpr int H = N / 2, C = CS::C, N1 = CS::N1, ZL = ZSc::ZL, M1 = ZSc::M1;
    const long long n_lines = (long long)N * N;
    const float2* tw = p->d_tw;
    const dim3 zblk(ZL * M1), cblk(C * N1);
    const unsigned zgrid = (unsigned)((n_lines + ZL - 1) / ZL);
    const ColGeom y_main{H, 1, (long long)N * H, C, H / C};
    const ColGeom y_nyq{1, N, 0, (long long)C * N, N / C};
    const ColGeom x_main{(long long)N * H, 1, H, C, H / C};
    const ColGeom x_nyq{N, 1, 0, C, N / C};
    const unsigned g_main = (unsigned)N * (H / C), g_nyq = (unsigned)(N / C);
    const MulArgs none{0.f, 0.f, 0};
    AMBER_LAUNCH(p, "fft_z_r2c", (k_fft_z_r2c<N, ZSc>), dim3(zgrid), zblk, s, d_src, spec, nyq, tw, n_lines);
    AMBER_LAUNCH(p, "fft_y", (k_fft_cols<N, CS, 0, false>), dim3(g_main), cblk, s, spec, spec, tw, y_main, none);
    AMBER_LAUNCH(p, "fft_nyq_y", (k_fft_cols<N, CS, 0, false>), dim3(g_nyq), cblk, s, nyq, nyq, tw, y_nyq, none);
    AMBER_LAUNCH(p, "fft_x", (k_fft_cols<N, CS, 0, false>), dim3(g_main), cblk, s, spec, spec, tw, x_main, none);
    AMBER_LAUNCH(p, "fft_nyq_x", (k_fft_cols<N, CS, 0, false>), dim3(g_nyq), cblk, s, nyq, nyq, tw, x_nyq, none);
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}

int fft_forward(const amber_plan_s* p, const float* d_src, float2* spec, float2* nyq, hipStream_t s) {
    return dispatch(p, [&](auto n, auto cs, auto zs) {
        return run_forward<decltype(n)::value, decltype(cs), decltype(zs)>(p, d_src, spec, nyq, s);
    });
}

// J_l from a spectrum already transformed along all three axes (main + Nyquist
// plane): per l_mfp, multiply by Khat/N^3 and inverse x in one pass (into the
// scratch spectrum when there are several l_mfp, in place otherwise), inverse y,
// complex-to-real.
template <int N, class CS, class ZSc>
int run_from_spectrum(const amber_plan_s* p, float2* spec, float2* nyq, const double* l_mfp, int n_lmfp,
                      float* const* d_J, float2* spec_tmp, float2* nyq_tmp, hipStream_t s) {
    constexpr int H = N / 2, C = CS::C, N1 = CS::N1, ZL = ZSc::ZL, M1 = ZSc::M1;
    const long long n_lines = (long long)N * N;
    const float2* tw = p->d_tw;
    const dim3 zblk(ZL * M1), cblk(C * N1);
    const unsigned zgrid = (unsigned)((n_lines + ZL - 1) / ZL);
    const ColGeom y_main{H, 1, (long long)N * H, C, H / C};
    const ColGeom y_nyq{1, N, 0, (long long)C * N, N / C};
    const ColGeom x_main{(long long)N * H, 1, H, C, H / C};
    const ColGeom x_nyq{N, 1, 0, C, N / C};
    const unsigned g_main = (unsigned)N * (H / C), g_nyq = (unsigned)(N / C);
    const MulArgs none{0.f, 0.f, 0};
    for (int i = 0; i < n_lmfp; ++i) {
        float2* so = (n_lmfp == 1) ? spec : spec_tmp;
        float2* no = (n_lmfp == 1) ? nyq : nyq_tmp;
        const MulArgs mm = mul_args(p->box_len, l_mfp[i], N, 0);
        const MulArgs mn = mul_args(p->box_len, l_mfp[i], N, 1);
        AMBER_LAUNCH(p, "fft_x_mul_inv", (k_fft_cols<N, CS, 2, false>), dim3(g_main), cblk, s, spec, so, tw, x_main, mm);
        AMBER_LAUNCH(p, "fft_nyq_x_mul_inv", (k_fft_cols<N, CS, 2, false>), dim3(g_nyq), cblk, s, nyq, no, tw, x_nyq, mn);
        AMBER_LAUNCH(p, "fft_y_inv", (k_fft_cols<N, CS, 0, true>), dim3(g_main), cblk, s, so, so, tw, y_main, none);
        AMBER_LAUNCH(p, "fft_nyq_y_inv", (k_fft_cols<N, CS, 0, true>), dim3(g_nyq), cblk, s, no, no, tw, y_nyq, none);
        AMBER_LAUNCH(p, "fft_z_c2r", (k_fft_z_c2r<N, ZSc>), dim3(zgrid), zblk, s, so, no, d_J[i], tw, n_lines);
    }
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}

int fft_from_spectrum(const amber_plan_s* p, float2* spec, float2* nyq, const double* l_mfp, int n_lmfp,
                      float* const* d_J, float2* spec_tmp, float2* nyq_tmp, hipStream_t s) {
    return dispatch(p, [&](auto n, auto cs, auto zs) {
        return run_from_spectrum<decltype(n)::value, decltype(cs), decltype(zs)>(p, spec, nyq, l_mfp, n_lmfp, d_J, spec_tmp,
                                                                                   nyq_tmp, s);
    });
}

int fft_radiation(const amber_plan_s* p, const float* d_src, const double* l_mfp, int n_lmfp,
                  float* const* d_J, unsigned char* ws, const WsLayout& L, hipStream_t s) {
    return dispatch(p, [&](auto n, auto cs, auto zs) {
        return run_radiation<decltype(n)::value, decltype(cs), decltype(zs)>(p, d_src, l_mfp, n_lmfp, d_J, ws, L, s);
    });
}

int fft_schedule_count(int n, int* n_col, int* n_z) {
    return with_size(n, [&](auto nc) {
        using S = Scheds<decltype(nc)::value>;
        *n_col = S::col::size;
        *n_z = S::z::size;
        return AMBER_OK;
    });
}

int fft_schedule_info(int n, int kind, int idx, int* a, int* b) {
    return with_size(n, [&](auto nc) {
        using S = Scheds<decltype(nc)::value>;
        if (kind == 0) return pick(typename S::col{}, idx, [&](auto cs) {
            *a = decltype(cs)::N1;
            *b = decltype(cs)::C;
            return AMBER_OK;
        });
        if (kind == 1) return pick(typename S::z{}, idx, [&](auto zs) {
            *a = decltype(zs)::M1;
            *b = decltype(zs)::ZL;
            return AMBER_OK;
        });
        return AMBER_E_ARG;
    });
}
