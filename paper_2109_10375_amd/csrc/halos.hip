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
// The deposit uses FP32 atomics (the last bits of a cell's sum depend on the
// order of the halos); weights are formed in FP64 from the FP32 positions.
#include <algorithm>

#include "internal.h"

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

__device__ __forceinline__ long long wrap(long long i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// One halo per thread, onto mesh0 (positions as given) and, when interlacing,
// mesh1 (shifted by half a cell).
template <int P>
__global__ __launch_bounds__(256) void k_deposit(const float* __restrict__ pos, const float* __restrict__ mass,
                                                 long long n_halo, int n, double to_cell, float* __restrict__ mesh0,
                                                 float* __restrict__ mesh1) {
    const long long h = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n_halo) return;
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

__device__ __forceinline__ int signed_freq(int m, int n) { return (2 * m <= n) ? m : m - n; }

// sinc(pi s / n)^p for one axis
__device__ __forceinline__ double window_1d(int s, int n, int p) {
    if (s == 0) return 1.0;
    const double a = kPiD * (double)s / (double)n;
    const double v = sin(a) / a;
    return p == 1 ? v : (p == 2 ? v * v : v * v * v);
}

// Main half spectrum (rows (x, y) of n/2 modes, kz < n/2) then the Nyquist
// plane (kz = n/2), one mode per thread.
__global__ __launch_bounds__(256) void k_combine(float2* __restrict__ spec_a, float2* __restrict__ nyq_a,
                                                 const float2* __restrict__ spec_b, const float2* __restrict__ nyq_b,
                                                 int n, int p, int interlace) {
    const long long h = n / 2;
    const long long main_modes = (long long)n * n * h;
    const long long total = main_modes + (long long)n * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        int x, y, kz;
        float2* a;
        const float2* b;
        if (e < main_modes) {
            const long long r = e / h;
            kz = (int)(e % h);
            x = (int)(r / n);
            y = (int)(r % n);
            a = spec_a + e;
            b = spec_b + e;
        } else {
            const long long r = e - main_modes;
            kz = (int)h;
            x = (int)(r / n);
            y = (int)(r % n);
            a = nyq_a + r;
            b = nyq_b + r;
        }
        const int s[3] = {signed_freq(x, n), signed_freq(y, n), kz};
        double W = 1.0;
        long long phase_num = 0;  // alpha = pi * phase_num / n over the non-Nyquist axes
        int n_nyq = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            W *= window_1d(s[d], n, p);
            if (2 * s[d] == n) ++n_nyq;
            else phase_num += s[d];
        }
        const float2 av = *a;
        double re = av.x, im = av.y;
        if (interlace) {
            const float2 bv = *b;
            const double alpha = kPiD * (double)phase_num / (double)n;
            const double cb = (n_nyq & 1) ? 0.0 : ((n_nyq & 2) ? -1.0 : 1.0);  // cos(n_nyq pi / 2)
            const double c = cos(alpha) * cb, sn = sin(alpha) * cb;
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
    const unsigned zero_blocks = (unsigned)std::min<long long>(4096, (n3 + 255) / 256);
    AMBER_LAUNCH(p, "halo_zero", k_zero_f32, dim3(zero_blocks), dim3(256), s, mesh0, n3);
    if (interlace) AMBER_LAUNCH(p, "halo_zero", k_zero_f32, dim3(zero_blocks), dim3(256), s, mesh1, n3);
    if (n_halo > 0) {
        const dim3 grid((unsigned)((n_halo + 255) / 256)), blk(256);
        const double to_cell = (double)n / p->box_len;
        float* m1 = interlace ? mesh1 : nullptr;
        if (scheme == 1) AMBER_LAUNCH(p, "halo_deposit", k_deposit<1>, grid, blk, s, d_pos, d_mass, n_halo, n, to_cell, mesh0, m1);
        else if (scheme == 2) AMBER_LAUNCH(p, "halo_deposit", k_deposit<2>, grid, blk, s, d_pos, d_mass, n_halo, n, to_cell, mesh0, m1);
        else AMBER_LAUNCH(p, "halo_deposit", k_deposit<3>, grid, blk, s, d_pos, d_mass, n_halo, n, to_cell, mesh0, m1);
    }
    int rc = fft_forward(p, mesh0, sa, na, s);
    if (rc == AMBER_OK && interlace) rc = fft_forward(p, mesh1, sb, nb, s);
    if (rc != AMBER_OK) return rc;
    const long long modes = n3 / 2 + (long long)n * n;
    AMBER_LAUNCH(p, "halo_combine", k_combine, dim3((unsigned)std::min<long long>(8192, (modes + 255) / 256)),
                 dim3(256), s, sa, na, sb, nb, n, scheme, interlace);
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}
