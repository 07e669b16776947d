// Two-point statistics on gfx950 (Sec. 2.3: Eqs. deltaz, Pk, Dk, bias, rcc):
// shell-averaged auto and cross power spectra of two fields from their
// forward real 3D FFTs.
//
// A field enters as given, as the overdensity f/mean - 1, or as the
// normalised redshift (f - mean)/(1 + mean) of Eq. (deltaz).  Both derived
// forms only rescale the non-zero modes and zero the mean mode, the mean being
// the transform's zero mode divided by N^3.  Shell i holds the modes with
// i - 1/2 <= |m~| < i + 1/2 over the full N^3 grid, decided in integers from
// |m~|^2; P = (L^3/N^6) <Re(A_m conj B_m)> and k = (2 pi/L) <|m~|>.
//
// The half spectrum stores kz in [0, N/2]; a stored mode with 0 < kz < N/2
// also stands for its conjugate partner (same |m~|, same product), so it
// counts twice.  Blocks accumulate a row range into LDS bins and add them to
// the FP64 output once; the sums are then divided by the mode counts.
#include "internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBins = 1024;
constexpr int kRowsPerBlock = 16;

__device__ __forceinline__ int signed_freq(int m, int n) { return (2 * m <= n) ? m : m - n; }

__device__ __forceinline__ int shell_of(long long s2) {
    long long i = (long long)sqrt((double)s2);
    while (i * i > s2) --i;
    while ((i + 1) * (i + 1) <= s2) ++i;
    if (4 * s2 >= (2 * i + 1) * (2 * i + 1)) ++i;
    return (int)i;
}

// Scale of the non-zero modes for a field kind, from the zero mode A0 = sum f.
__device__ __forceinline__ double mode_scale(int kind, double a0, double n3) {
    if (kind == 1) return n3 / a0;                  // f/mean - 1
    if (kind == 2) return 1.0 / (1.0 + a0 / n3);    // (f - mean)/(1 + mean)
    return 1.0;
}

__global__ void k_zero(double* __restrict__ p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

// rows: the N*N (x, y) rows of the main half spectrum (kz < N/2), then one
// more group for the Nyquist plane kz = N/2 handled as rows of length 1.
__global__ __launch_bounds__(kThreads) void k_bins(const float2* __restrict__ spec_a, const float2* __restrict__ nyq_a,
                                                   int kind_a, const float2* __restrict__ spec_b,
                                                   const float2* __restrict__ nyq_b, int kind_b, int n, int n_bins,
                                                   double* __restrict__ out) {
    __shared__ double acc[5][kMaxBins];  // modes, sum |m~|, aa, bb, ab
    for (int i = threadIdx.x; i < 5 * kMaxBins; i += kThreads) (&acc[0][0])[i] = 0.0;
    __syncthreads();
    const int h = n / 2;
    const double n3 = (double)n * n * n;
    const double sa = mode_scale(kind_a, (double)spec_a[0].x, n3);
    const double sb = mode_scale(kind_b, (double)spec_b[0].x, n3);
    const long long rows = (long long)n * n;
    const long long r0 = (long long)blockIdx.x * kRowsPerBlock;
    // main half spectrum: kRowsPerBlock rows of h modes
    for (int e = threadIdx.x; e < kRowsPerBlock * h; e += kThreads) {
        const long long r = r0 + e / h;
        if (r >= rows) break;
        const int kz = e % h;
        const int x = (int)(r / n), y = (int)(r % n);
        const long long sx = signed_freq(x, n), sy = signed_freq(y, n);
        const long long s2 = sx * sx + sy * sy + (long long)kz * kz;
        const int sh = shell_of(s2);
        if (sh >= n_bins) continue;
        const bool zero = s2 == 0;
        const float2 a = spec_a[r * h + kz], b = spec_b[r * h + kz];
        const double ax = zero && kind_a ? 0.0 : sa * a.x, ay = zero && kind_a ? 0.0 : sa * a.y;
        const double bx = zero && kind_b ? 0.0 : sb * b.x, by = zero && kind_b ? 0.0 : sb * b.y;
        const double wgt = kz == 0 ? 1.0 : 2.0;
        atomicAdd(&acc[0][sh], wgt);
        atomicAdd(&acc[1][sh], wgt * sqrt((double)s2));
        atomicAdd(&acc[2][sh], wgt * (ax * ax + ay * ay));
        atomicAdd(&acc[3][sh], wgt * (bx * bx + by * by));
        atomicAdd(&acc[4][sh], wgt * (ax * bx + ay * by));
    }
    // Nyquist plane kz = n/2 (all its (x, y) modes), split over the blocks
    for (long long r = r0 + threadIdx.x; r < r0 + kRowsPerBlock && r < rows; r += kThreads) {
        const int x = (int)(r / n), y = (int)(r % n);
        const long long sx = signed_freq(x, n), sy = signed_freq(y, n);
        const long long s2 = sx * sx + sy * sy + (long long)h * h;
        const int sh = shell_of(s2);
        if (sh >= n_bins) continue;
        const float2 a = nyq_a[r], b = nyq_b[r];
        const double ax = sa * a.x, ay = sa * a.y, bx = sb * b.x, by = sb * b.y;
        atomicAdd(&acc[0][sh], 1.0);
        atomicAdd(&acc[1][sh], sqrt((double)s2));
        atomicAdd(&acc[2][sh], ax * ax + ay * ay);
        atomicAdd(&acc[3][sh], bx * bx + by * by);
        atomicAdd(&acc[4][sh], ax * bx + ay * by);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_bins; i += kThreads) {
        if (acc[0][i] == 0.0) continue;
#pragma unroll
        for (int q = 0; q < 5; ++q) atomicAdd(&out[q * n_bins + i], acc[q][i]);
    }
}

// Sums (rows: modes, sum |m~|, aa, bb, ab) -> shell averages in the output
// order k, modes, P_aa, P_bb, P_ab, then the dimensionless
// Delta^2_aa = k^3 P_aa / (2 pi^2) (Eq. Dk), b_ab = sqrt(P_aa / P_bb) (Eq. bias)
// and r_ab = P_ab / sqrt(P_aa P_bb) (Eq. rcc).
__global__ void k_finish(double* __restrict__ out, int n_bins, double k0, double vol) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_bins) return;
    const double m = out[i];
    double k = 0.0, paa = 0.0, pbb = 0.0, pab = 0.0, d2 = 0.0, b = 0.0, r = 0.0;
    if (m > 0.0) {
        k = k0 * out[1 * n_bins + i] / m;
        paa = vol * out[2 * n_bins + i] / m;
        pbb = vol * out[3 * n_bins + i] / m;
        pab = vol * out[4 * n_bins + i] / m;
        d2 = k * k * k * paa / (2.0 * 3.14159265358979323846 * 3.14159265358979323846);
        b = pbb > 0.0 ? sqrt(paa / pbb) : 0.0;
        r = (paa > 0.0 && pbb > 0.0) ? pab / sqrt(paa * pbb) : 0.0;
    }
    out[0 * n_bins + i] = k;  // the documented row order: k, then the mode count
    out[1 * n_bins + i] = m;
    out[2 * n_bins + i] = paa;
    out[3 * n_bins + i] = pbb;
    out[4 * n_bins + i] = pab;
    out[5 * n_bins + i] = d2;
    out[6 * n_bins + i] = b;
    out[7 * n_bins + i] = r;
}

}  // namespace

int spectra_bins(const amber_plan_s* p, const float2* spec_a, const float2* nyq_a, int kind_a, const float2* spec_b,
                 const float2* nyq_b, int kind_b, int n_bins, double* d_out, hipStream_t s) {
    if (n_bins < 1 || n_bins > kMaxBins) return AMBER_E_ARG;
    const int n = p->n;
    const long long rows = (long long)n * n;
    AMBER_LAUNCH(p, "spectra_zero", k_zero, dim3(8), dim3(256), s, d_out, 5 * n_bins);
    AMBER_LAUNCH(p, "spectra_bins", k_bins, dim3((unsigned)((rows + kRowsPerBlock - 1) / kRowsPerBlock)),
                 dim3(kThreads), s, spec_a, nyq_a, kind_a, spec_b, nyq_b, kind_b, n, n_bins, d_out);
    const double L = p->box_len;
    const double n3 = (double)n * n * n;
    AMBER_LAUNCH(p, "spectra_finish", k_finish, dim3((unsigned)((n_bins + 255) / 256)), dim3(256), s, d_out, n_bins,
                 2.0 * 3.14159265358979323846 / L, L * L * L / (n3 * n3));
    AMBER_HIP_CHECK(hipGetLastError());
    return AMBER_OK;
}
