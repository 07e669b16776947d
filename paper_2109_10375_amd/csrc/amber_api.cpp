// Host side of the C-ABI: argument checks, plans, workspace layout, the
// reionization-history fit (Sec. 3.1, Appendix A) and the inversion table.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.h"

namespace {

bool supported_n(int n) {
    switch (n) {
        case 8: case 16: case 32: case 64: case 96: case 128: case 192: case 256: case 512: case 1024:
            return true;
        default:
            return false;
    }
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// g(c) = (p_e - p_m) - A_z (p_m - p_l) with p = |ln x|^(1/c): zero exactly when
// the Weibull curve through the mid and late points also passes the early one
// (Eqs. (asymmetry), (weibull)); positive for small c, negative for large c.
double asym_residual(double c, double le, double lm, double ll, double az) {
    const double pe = std::pow(le, 1.0 / c), pm = std::pow(lm, 1.0 / c), pl = std::pow(ll, 1.0 / c);
    return (pe - pm) - az * (pm - pl);
}

// Brent's method (R. P. Brent, Algorithms for Minimization without
// Derivatives, 1973, ch. 4) on s = ln c over a sign-change bracket.
bool solve_c(double le, double lm, double ll, double az, double* c_out) {
    double a = std::log(1.0 / 64.0), b = std::log(4096.0);
    double fa = asym_residual(std::exp(a), le, lm, ll, az), fb = asym_residual(std::exp(b), le, lm, ll, az);
    if (!(fa > 0.0) || !(fb < 0.0)) {
        // narrow the upper end: the residual tends to 0- only slowly
        return false;
    }
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 300; ++it) {
        if ((fb > 0.0) == (fc > 0.0)) {
            c = a; fc = fa; d = b - a; e = d;
        }
        if (std::fabs(fc) < std::fabs(fb)) {
            a = b; b = c; c = a;
            fa = fb; fb = fc; fc = fa;
        }
        const double tol = 2.0 * 2.220446049250313e-16 * std::fabs(b) + 1e-300;
        const double m = 0.5 * (c - b);
        if (std::fabs(m) <= tol || fb == 0.0) break;
        if (std::fabs(e) >= tol && std::fabs(fa) > std::fabs(fb)) {
            double p, q, r;
            const double s = fb / fa;
            if (a == c) {
                p = 2.0 * m * s;
                q = 1.0 - s;
            } else {
                q = fa / fc;
                r = fb / fc;
                p = s * (2.0 * m * q * (q - r) - (b - a) * (r - 1.0));
                q = (q - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0.0) q = -q; else p = -p;
            if (2.0 * p < std::min(3.0 * m * q - std::fabs(tol * q), std::fabs(e * q))) {
                e = d;
                d = p / q;
            } else {
                d = m;
                e = d;
            }
        } else {
            d = m;
            e = d;
        }
        a = b;
        fa = fb;
        b += (std::fabs(d) > tol) ? d : (m > 0 ? tol : -tol);
        fb = asym_residual(std::exp(b), le, lm, ll, az);
    }
    *c_out = std::exp(b);
    return std::isfinite(*c_out);
}

}  // namespace

WsLayout ws_layout(int n, int n_lmfp, bool halo_meshes) {
    WsLayout L{};
    const size_t N = (size_t)n, n3 = N * N * N;
    const size_t n_tiles = (n3 + 4095) / 4096;
    size_t off = 0;
    L.ctrl = off;
    off = align256(off + sizeof(Ctrl));
    const size_t region = off;
    // radiation
    size_t f = region;
    L.spec_a = f; f = align256(f + N * N * (N / 2) * sizeof(float2));
    L.nyq_a = f;  f = align256(f + N * N * sizeof(float2));
    if (n_lmfp > 1) {
        L.spec_b = f; f = align256(f + N * N * (N / 2) * sizeof(float2));
        L.nyq_b = f;  f = align256(f + N * N * sizeof(float2));
    } else {
        L.spec_b = L.spec_a;
        L.nyq_b = L.nyq_a;
    }
    L.mesh[0] = L.mesh[1] = f;
    if (halo_meshes) {
        L.mesh[0] = f; f = align256(f + n3 * 4);
        L.mesh[1] = f; f = align256(f + n3 * 4);
        L.bins = f; f = align256(f + halo_bin_words(n) * 4);
        L.halo_tab = f; f = align256(f + N * 32);
    }
    // ranking and matching (same region: the stages never overlap on a stream)
    size_t r = region;
    for (int i = 0; i < 2; ++i) { L.keys[i] = r; r = align256(r + n3 * 4); }
    for (int i = 0; i < 2; ++i) { L.vals[i] = r; r = align256(r + n3 * 4); }
    for (int i = 0; i < 2; ++i) { L.wts[i] = r; r = align256(r + n3 * 4); }
    for (int i = 0; i < 2; ++i) { L.part2[i] = r; r = align256(r + n3 * 4); }
    L.lookback = r;
    r = align256(r + (size_t)lb_words((long long)n3) * 4 * 3 + n_tiles * 16);
    L.total = std::max(f, r);
    return L;
}

extern "C" {

const char* amber_version(void) { return "amber-mi355x 0.1 (gfx950)"; }

const char* amber_strerror(int code) {
    switch (code) {
        case AMBER_OK: return "ok";
        case AMBER_E_ARG: return "invalid argument";
        case AMBER_E_SIZE: return "unsupported grid size";
        case AMBER_E_HISTORY: return "no valid Weibull history for these parameters";
        case AMBER_E_WORKSPACE: return "workspace too small";
        case AMBER_E_HIP: return "HIP runtime error";
        case AMBER_E_UNIMPL: return "not implemented";
        default: return "unknown error";
    }
}

int amber_weibull_from_coeffs(double a_w, double b_w, double c_w, amber_weibull* out) {
    if (!out) return AMBER_E_ARG;
    if (!(a_w > 0.0) || !(b_w > 0.0) || !(c_w > 0.0) || !std::isfinite(a_w) || !std::isfinite(b_w) ||
        !std::isfinite(c_w))
        return AMBER_E_HISTORY;
    const double top = a_w + b_w * std::pow(64.0 * 0.69314718055994530942, 1.0 / c_w);
    const double span = top - a_w;
    const double r = span / 4194304.0;
    int e = 0;
    const double f = std::frexp(r, &e);
    const double h = (f == 0.5) ? r : std::ldexp(1.0, e);
    out->a_w = a_w;
    out->b_w = b_w;
    out->c_w = c_w;
    out->h = h;
    out->z_top = top;
    out->table_n = (int64_t)std::ceil(span / h) + 1;
    out->d_table = nullptr;
    out->d_growth = nullptr;
    return AMBER_OK;
}

int amber_weibull_fit(const amber_history* hist, amber_weibull* out) {
    if (!hist || !out) return AMBER_E_ARG;
    const double xe = hist->x_ear == 0.0 ? 0.05 : hist->x_ear;
    const double xm = hist->x_mid == 0.0 ? 0.5 : hist->x_mid;
    const double xl = hist->x_lat == 0.0 ? 0.95 : hist->x_lat;
    if (!(0.0 < xe && xe < xm && xm < xl && xl < 1.0)) return AMBER_E_ARG;
    if (!std::isfinite(hist->z_mid) || !(hist->delta_z > 0.0) || !(hist->a_z > 0.0) || !std::isfinite(hist->delta_z) ||
        !std::isfinite(hist->a_z))
        return AMBER_E_ARG;
    if (hist->a_z > 15.0) return AMBER_E_HISTORY;
    // Sec. 3.1.1: the early and late points
    const double z_ear = hist->z_mid + hist->delta_z * hist->a_z / (1.0 + hist->a_z);
    const double z_lat = z_ear - hist->delta_z;
    const double le = std::fabs(std::log(xe)), lm = std::fabs(std::log(xm)), ll = std::fabs(std::log(xl));
    double c = 0.0;
    if (!solve_c(le, lm, ll, hist->a_z, &c)) return AMBER_E_HISTORY;
    // Appendix A: the two algebraic coefficients
    const double pe = std::pow(le, 1.0 / c), pm = std::pow(lm, 1.0 / c), pl = std::pow(ll, 1.0 / c);
    const double a = (z_ear * pl - z_lat * pe) / (pl - pe);
    const double b = (hist->z_mid - a) / pm;
    return amber_weibull_from_coeffs(a, b, c, out);
}

// X_j = x_i(z_j), z_j = a_w + j h (Sec. 3.1.2, Eq. weibull).
static double weibull_node(const amber_weibull* w, int64_t j) {
    const double a = w->a_w, z = a + (double)j * w->h;
    return std::exp(-std::pow((z - a) / w->b_w, w->c_w));
}

// A fitted history as amber_zre uses it: positive coefficients, the table
// geometry that amber_weibull_from_coeffs gives for them (the kernels rely on
// T >= 2^21 nodes), a device table and a 16-byte aligned growth table.
static int check_weibull(const amber_weibull& w) {
    amber_weibull ref{};
    if (amber_weibull_from_coeffs(w.a_w, w.b_w, w.c_w, &ref) != AMBER_OK) return AMBER_E_HISTORY;
    if (!(w.h == ref.h) || !(w.z_top == ref.z_top) || w.table_n != ref.table_n) return AMBER_E_ARG;
    if (!w.d_table) return AMBER_E_ARG;
    if (reinterpret_cast<uintptr_t>(w.d_growth) % 16 != 0) return AMBER_E_ARG;
    return AMBER_OK;
}

int amber_weibull_table(const amber_weibull* w, double* host_table, int64_t n_entries) {
    if (!w || !host_table || n_entries != w->table_n || n_entries < 2) return AMBER_E_ARG;
    for (int64_t j = 0; j < n_entries; ++j) host_table[j] = weibull_node(w, j);
    return AMBER_OK;
}

// Growing mode of flat Lambda-CDM, normalised to a early: a 2F1(1/3, 1; 11/6; x),
// x = -(1 - om)/om a^3, summed after Pfaff's transformation as
// a / (1 - x) * sum_k (3/2)_k / (11/6)_k y^k, y = x / (x - 1), until a term no
// longer changes the sum.
static double growth_factor(double z, double om) {
#pragma clang fp contract(off)
    const double a = 1.0 / (1.0 + z);
    const double x = -(1.0 - om) / om * (a * a * a);
    const double y = x / (x - 1.0);
    double term = 1.0, sum = 1.0;
    for (int k = 0; k < 100000; ++k) {
        term = term * ((1.5 + (double)k) / (11.0 / 6.0 + (double)k)) * y;
        const double next = sum + term;
        if (next == sum) break;
        sum = next;
    }
    return a * (sum / (1.0 - x));
}

int amber_growth_table(const amber_weibull* w, double z_mid, double omega_m, double* host_table,
                       int64_t n_entries) {
    if (!w || !host_table || n_entries != w->table_n || n_entries < 2) return AMBER_E_ARG;
    if (!(omega_m > 0.0) || !(omega_m <= 1.0) || !std::isfinite(z_mid) || !(z_mid > -1.0)) return AMBER_E_ARG;
    const double dmid = growth_factor(z_mid, omega_m);
    for (int64_t j = 0; j < n_entries; ++j) {
        host_table[2 * j] = weibull_node(w, j);
        host_table[2 * j + 1] = growth_factor(w->a_w + (double)j * w->h, omega_m) / dmid;
    }
    return AMBER_OK;
}

int amber_history_prepare(const amber_history* hist, amber_weibull* out, void* d_table_buf, size_t buf_bytes,
                          void* stream) {
    if (!hist || !out) return AMBER_E_ARG;
    amber_weibull w{};
    const int rc = amber_weibull_fit(hist, &w);
    if (rc != AMBER_OK) return rc;
    if (!d_table_buf) {  // size query
        *out = w;
        return AMBER_OK;
    }
    const size_t bytes = (size_t)w.table_n * sizeof(double);
    if (buf_bytes < bytes) return AMBER_E_WORKSPACE;
    double* host = new (std::nothrow) double[(size_t)w.table_n];
    if (!host) return AMBER_E_ARG;
    amber_weibull_table(&w, host, w.table_n);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(d_table_buf, host, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    delete[] host;
    if (e != hipSuccess) return AMBER_E_HIP;
    w.d_table = static_cast<const double*>(d_table_buf);
    *out = w;
    return AMBER_OK;
}

int amber_growth_prepare(amber_weibull* w, double z_mid, double omega_m, void* d_pairs_buf, size_t buf_bytes,
                         void* stream) {
    if (!w || !d_pairs_buf) return AMBER_E_ARG;
    if (reinterpret_cast<uintptr_t>(d_pairs_buf) % 16 != 0) return AMBER_E_ARG;
    amber_weibull ref{};
    if (amber_weibull_from_coeffs(w->a_w, w->b_w, w->c_w, &ref) != AMBER_OK) return AMBER_E_HISTORY;
    if (!(w->h == ref.h) || !(w->z_top == ref.z_top) || w->table_n != ref.table_n) return AMBER_E_ARG;
    const size_t bytes = 2 * (size_t)w->table_n * sizeof(double);
    if (buf_bytes < bytes) return AMBER_E_WORKSPACE;
    double* host = new (std::nothrow) double[2 * (size_t)w->table_n];
    if (!host) return AMBER_E_ARG;
    int rc = amber_growth_table(w, z_mid, omega_m, host, w->table_n);
    if (rc == AMBER_OK) {
        const hipStream_t s = static_cast<hipStream_t>(stream);
        hipError_t e = hipMemcpyAsync(d_pairs_buf, host, bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = AMBER_E_HIP;
    }
    delete[] host;
    if (rc == AMBER_OK) w->d_growth = static_cast<const double*>(d_pairs_buf);
    return rc;
}

int amber_plan_create(amber_plan* out, int n, double box_len) {
    if (!out) return AMBER_E_ARG;
    *out = nullptr;
    if (!supported_n(n)) return AMBER_E_SIZE;
    if (!(box_len > 0.0) || !std::isfinite(box_len)) return AMBER_E_ARG;
    amber_plan_s* p = new (std::nothrow) amber_plan_s();
    if (!p) return AMBER_E_ARG;
    p->n = n;
    p->box_len = box_len;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return AMBER_E_HIP;
    }
    float2* host = new (std::nothrow) float2[n];
    if (!host) {
        delete p;
        return AMBER_E_ARG;
    }
    for (int j = 0; j < n; ++j) {
        // exp(-2 pi i j / n) from long-double (64-bit significand) cos/sin
        const long double t = 2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)n;
        host[j] = make_float2((float)cosl(t), (float)(-sinl(t)));
    }
    // one allocation: the twiddles, then the accumulated status word
    const size_t tw_bytes = align256(sizeof(float2) * (size_t)n);
    hipError_t e = hipMalloc(&p->d_tw, tw_bytes + 256);
    if (e == hipSuccess) e = hipMemcpy(p->d_tw, host, sizeof(float2) * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        p->d_sticky = reinterpret_cast<unsigned*>(reinterpret_cast<unsigned char*>(p->d_tw) + tw_bytes);
        e = hipMemset(p->d_sticky, 0, sizeof(unsigned));
    }
    delete[] host;
    if (e != hipSuccess) {
        if (p->d_tw) (void)hipFree(p->d_tw);
        delete p;
        return AMBER_E_HIP;
    }
    // the no-allocation matching call's scratch on this device (a failed
    // lookup leaves it NULL: that call then reports AMBER_E_HIP)
    if (n <= AMBER_NOALLOC_MAX_N) (void)noalloc_scratch_address(p->device, &p->d_scratch);
    *out = p;
    return AMBER_OK;
}

static void profiler_free(amber_plan_s* p) {
    Profiler* f = p->prof;
    if (!f) return;
    for (int i = 0; i < 2 * f->capacity; ++i)
        if (f->ev[i]) (void)hipEventDestroy(f->ev[i]);
    delete[] f->ev;
    delete[] f->names;
    delete f;
    p->prof = nullptr;
}

void amber_plan_destroy(amber_plan plan) {
    if (!plan) return;
    profiler_free(plan);
    if (plan->d_tw) (void)hipFree(plan->d_tw);
    delete plan;
}

int amber_profile_begin(amber_plan plan, int capacity) {
    if (!plan || capacity < 1 || capacity > (1 << 20)) return AMBER_E_ARG;
    profiler_free(plan);
    Profiler* f = new (std::nothrow) Profiler();
    if (!f) return AMBER_E_ARG;
    f->ev = new (std::nothrow) hipEvent_t[2 * (size_t)capacity]();
    f->names = new (std::nothrow) const char*[(size_t)capacity]();
    plan->prof = f;
    if (!f->ev || !f->names) {
        profiler_free(plan);
        return AMBER_E_ARG;
    }
    f->capacity = capacity;
    for (int i = 0; i < 2 * capacity; ++i) {
        if (hipEventCreate(&f->ev[i]) != hipSuccess) {
            f->capacity = i / 2;
            profiler_free(plan);
            return AMBER_E_HIP;
        }
    }
    return AMBER_OK;
}

int amber_profile_end(amber_plan plan, amber_kernel_time* out, int max_entries, int* n_entries) {
    if (!plan || !plan->prof || (!out && max_entries > 0) || !n_entries) return AMBER_E_ARG;
    Profiler* f = plan->prof;
    int n = 0;
    int rc = AMBER_OK;
    for (int slot = 0; slot < f->used; ++slot) {
        if (hipEventSynchronize(f->ev[2 * slot + 1]) != hipSuccess) {
            rc = AMBER_E_HIP;
            break;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, f->ev[2 * slot], f->ev[2 * slot + 1]) != hipSuccess) {
            rc = AMBER_E_HIP;
            break;
        }
        int k = 0;
        while (k < n && std::strncmp(out[k].name, f->names[slot], sizeof(out[k].name)) != 0) ++k;
        if (k == n) {
            if (n >= max_entries) continue;
            std::memset(&out[n], 0, sizeof(out[n]));
            std::strncpy(out[n].name, f->names[slot], sizeof(out[n].name) - 1);
            ++n;
        }
        out[k].launches += 1;
        out[k].total_ms += (double)ms;
    }
    *n_entries = n;
    profiler_free(plan);
    return rc;
}

size_t amber_workspace_bytes(amber_plan plan, int n_lmfp, int n_hist) {
    if (!plan || n_lmfp < 0 || n_lmfp > 64 || n_hist < 0 || n_hist > 8) return 0;
    // histories are matched in groups that reuse the ranking's buffers, so
    // their count does not change the size
    return ws_layout(plan->n, n_lmfp < 1 ? 1 : n_lmfp).total;
}

int amber_radiation(amber_plan plan, const float* d_src, const double* l_mfp, int n_lmfp, float* const* d_J,
                    void* d_ws, size_t ws_bytes, void* stream) {
    if (!plan || !d_src || !l_mfp || !d_J || !d_ws || n_lmfp < 1 || n_lmfp > 64) return AMBER_E_ARG;
    for (int i = 0; i < n_lmfp; ++i) {
        if (!(l_mfp[i] > 0.0) || !std::isfinite(l_mfp[i]) || !d_J[i]) return AMBER_E_ARG;
        if ((const void*)d_J[i] == (const void*)d_src) return AMBER_E_ARG;
    }
    const WsLayout L = ws_layout(plan->n, n_lmfp);
    if (ws_bytes < L.total) return AMBER_E_WORKSPACE;
    return fft_radiation(plan, d_src, l_mfp, n_lmfp, d_J, static_cast<unsigned char*>(d_ws), L,
                         static_cast<hipStream_t>(stream));
}

int amber_fft_schedules(int n, int* n_col, int* n_z) {
    if (!n_col || !n_z) return AMBER_E_ARG;
    return fft_schedule_count(n, n_col, n_z);
}

int amber_fft_schedule_info(int n, int kind, int idx, int* split, int* width) {
    if (!split || !width || idx < 0) return AMBER_E_ARG;
    return fft_schedule_info(n, kind, idx, split, width);
}

int amber_plan_set_schedule(amber_plan plan, int col, int z) {
    if (!plan) return AMBER_E_ARG;
    int nc = 0, nz = 0;
    const int rc = fft_schedule_count(plan->n, &nc, &nz);
    if (rc != AMBER_OK) return rc;
    if (col < 0 || col >= nc || z < 0 || z >= nz) return AMBER_E_ARG;
    plan->col_sched = col;
    plan->z_sched = z;
    return AMBER_OK;
}

int amber_plan_get_schedule(amber_plan plan, int* col, int* z) {
    if (!plan || !col || !z) return AMBER_E_ARG;
    *col = plan->col_sched;
    *z = plan->z_sched;
    return AMBER_OK;
}

namespace {

// Mean time of one radiation pass (one l_mfp) under the plan's current
// schedule: one untimed pass, then reps passes between two events.
int time_radiation(amber_plan_s* p, const float* d_src, float* d_J, unsigned char* ws, const WsLayout& L, int reps,
                   hipEvent_t e0, hipEvent_t e1, hipStream_t s, float* ms) {
    const double l = p->box_len / 16.0;
    float* out[1] = {d_J};
    int rc = fft_radiation(p, d_src, &l, 1, out, ws, L, s);
    if (rc != AMBER_OK) return rc;
    AMBER_HIP_CHECK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) {
        rc = fft_radiation(p, d_src, &l, 1, out, ws, L, s);
        if (rc != AMBER_OK) return rc;
    }
    AMBER_HIP_CHECK(hipEventRecord(e1, s));
    AMBER_HIP_CHECK(hipEventSynchronize(e1));
    float t = 0.f;
    AMBER_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
    *ms = t / (float)reps;
    return AMBER_OK;
}

}  // namespace

int amber_plan_tune(amber_plan plan, const float* d_src, float* d_J, void* d_ws, size_t ws_bytes, int reps,
                    float* ms_out, int* col, int* z, void* stream) {
    if (!plan || !d_src || !d_J || !d_ws || (const void*)d_J == (const void*)d_src) return AMBER_E_ARG;
    if (reps < 1 || reps > 1000) return AMBER_E_ARG;
    const WsLayout L = ws_layout(plan->n, 1);
    if (ws_bytes < L.total) return AMBER_E_WORKSPACE;
    int nc = 0, nz = 0;
    int rc = fft_schedule_count(plan->n, &nc, &nz);
    if (rc != AMBER_OK) return rc;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char* ws = static_cast<unsigned char*>(d_ws);
    const int keep_col = plan->col_sched, keep_z = plan->z_sched;
    Profiler* keep_prof = plan->prof;  // tuning launches are not traced
    plan->prof = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best_ms[64 * 64];
    const int n_all = nc * nz;
    if (n_all > 64 * 64) rc = AMBER_E_ARG;
    if (rc == AMBER_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = AMBER_E_HIP;
    // Three rounds over every candidate pair; a pair's figure is its fastest
    // round, which discounts clock ramps and one-off stalls.
    for (int round = 0; rc == AMBER_OK && round < 3; ++round) {
        for (int k = 0; rc == AMBER_OK && k < n_all; ++k) {
            plan->col_sched = k / nz;
            plan->z_sched = k % nz;
            float ms = 0.f;
            rc = time_radiation(plan, d_src, d_J, ws, L, reps, e0, e1, s, &ms);
            if (rc == AMBER_OK) best_ms[k] = (round == 0) ? ms : std::min(best_ms[k], ms);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    plan->prof = keep_prof;
    if (rc != AMBER_OK) {
        plan->col_sched = keep_col;
        plan->z_sched = keep_z;
        return rc;
    }
    // The default pair stays unless another is faster by more than 2 %: a
    // change of schedule changes the FP32 rounding of J, so it has to pay.
    // Among the pairs that do, the first (lowest index) within 1 % of the
    // fastest is taken, so timing noise between near-equal pairs does not
    // decide.
    int fastest = 0;
    for (int k = 1; k < n_all; ++k)
        if (best_ms[k] < best_ms[fastest]) fastest = k;
    int best = 0;
    if (best_ms[fastest] < 0.98f * best_ms[0]) {
        for (int k = 1; k < n_all; ++k)
            if (best_ms[k] < 0.98f * best_ms[0] && best_ms[k] <= 1.01f * best_ms[fastest]) {
                best = k;
                break;
            }
    }
    plan->col_sched = best / nz;
    plan->z_sched = best % nz;
    if (ms_out) std::memcpy(ms_out, best_ms, sizeof(float) * (size_t)n_all);
    if (col) *col = plan->col_sched;
    if (z) *z = plan->z_sched;
    return AMBER_OK;
}

size_t amber_halo_workspace_bytes(amber_plan plan) {
    if (!plan) return 0;
    return ws_layout(plan->n, 2, true).total;
}

int amber_radiation_from_halos(amber_plan plan, const float* d_pos, const float* d_mass, int64_t n_halo,
                               int scheme, int interlace, const double* l_mfp, int n_lmfp, float* const* d_J,
                               void* d_ws, size_t ws_bytes, void* stream) {
    if (!plan || !l_mfp || !d_J || !d_ws || n_lmfp < 1 || n_lmfp > 64 || n_halo < 0) return AMBER_E_ARG;
    if (n_halo > 0 && (!d_pos || !d_mass)) return AMBER_E_ARG;
    if (n_halo > (int64_t)1 << 40 || scheme < 1 || scheme > 3 || (interlace != 0 && interlace != 1)) return AMBER_E_ARG;
    for (int i = 0; i < n_lmfp; ++i)
        if (!(l_mfp[i] > 0.0) || !std::isfinite(l_mfp[i]) || !d_J[i]) return AMBER_E_ARG;
    const WsLayout L = ws_layout(plan->n, 2, true);
    if (ws_bytes < L.total) return AMBER_E_WORKSPACE;
    unsigned char* ws = static_cast<unsigned char*>(d_ws);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = halo_source_spectrum(plan, d_pos, d_mass, n_halo, scheme, interlace, ws, L, s);
    if (rc != AMBER_OK) return rc;
    return fft_from_spectrum(plan, reinterpret_cast<float2*>(ws + L.spec_a), reinterpret_cast<float2*>(ws + L.nyq_a),
                             l_mfp, n_lmfp, d_J, reinterpret_cast<float2*>(ws + L.spec_b),
                             reinterpret_cast<float2*>(ws + L.nyq_b), s);
}

int amber_rank(amber_plan plan, const float* d_J, uint32_t* d_perm, void* d_ws, size_t ws_bytes, void* stream) {
    if (!plan || !d_J || !d_perm || !d_ws) return AMBER_E_ARG;
    const WsLayout L = ws_layout(plan->n, 1);
    if (ws_bytes < L.total) return AMBER_E_WORKSPACE;
    return rank_sort(plan, d_J, nullptr, static_cast<unsigned char*>(d_ws), L, static_cast<hipStream_t>(stream), 0,
                     d_perm);
}

int amber_zre(amber_plan plan, const float* d_J, const float* d_w, const amber_weibull* hist, int n_hist,
              float* const* d_zre, void* d_ws, size_t ws_bytes, void* stream) {
    if (!plan || !d_J || !d_w || !hist || !d_zre || !d_ws || n_hist < 1 || n_hist > 8) return AMBER_E_ARG;
    for (int i = 0; i < n_hist; ++i) {
        if (!d_zre[i]) return AMBER_E_ARG;
        const int rc = check_weibull(hist[i]);
        if (rc != AMBER_OK) return rc;
    }
    const WsLayout L = ws_layout(plan->n, 1);
    if (ws_bytes < L.total) return AMBER_E_WORKSPACE;
    unsigned char* ws = static_cast<unsigned char*>(d_ws);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = rank_sort(plan, d_J, d_w, ws, L, s, 1, nullptr);
    if (rc != AMBER_OK) return rc;
    return match_scan(plan, hist, n_hist, d_zre, ws, L, s);
}

static int check_item(const amber_batch_item& it) {
    if (!it.plan || !it.d_w || !it.d_J || !it.d_zre || !it.hist) return AMBER_E_ARG;
    if (it.n_lmfp < 1 || it.n_lmfp > 64 || it.n_hist < 1 || it.n_hist > 8) return AMBER_E_ARG;
    for (int i = 0; i < it.n_lmfp; ++i) {
        if (!it.d_J[i]) return AMBER_E_ARG;
        if (it.d_src) {
            if (!it.l_mfp || !(it.l_mfp[i] > 0.0) || !std::isfinite(it.l_mfp[i])) return AMBER_E_ARG;
            if ((const void*)it.d_J[i] == (const void*)it.d_src) return AMBER_E_ARG;
        }
    }
    for (int h = 0; h < it.n_hist; ++h) {
        const int rc = check_weibull(it.hist[h]);
        if (rc != AMBER_OK) return rc;
    }
    return AMBER_OK;
}

// Workspace of one box of a batch (radiation with all its fields, or matching only).
static size_t item_ws_bytes(const amber_batch_item& it) {
    const int nl = it.d_src ? std::max(1, it.n_lmfp) : 1;
    return ws_layout(it.plan->n, nl).total;
}

// One box: its radiation fields, then each field's wanted histories
// (consecutive non-NULL outputs share one ranking), on one stream and one
// workspace slice.
static int run_item(const amber_batch_item& it, unsigned* d_status, unsigned char* ws, hipStream_t s) {
    const amber_plan_s* p = it.plan;
    if (it.d_src) {
        const WsLayout LR = ws_layout(p->n, it.n_lmfp);
        const int rc = fft_radiation(p, it.d_src, it.l_mfp, it.n_lmfp, it.d_J, ws, LR, s);
        if (rc != AMBER_OK) return rc;
    }
    const WsLayout L = ws_layout(p->n, 1);
    if (d_status) {
        const int rc = status_collect(p, ws, L, d_status, true, s);
        if (rc != AMBER_OK) return rc;
    }
    for (int l = 0; l < it.n_lmfp; ++l) {
        amber_weibull hs[8];
        float* zs[8];
        int k = 0;
        for (int h = 0; h < it.n_hist; ++h) {
            float* z = it.d_zre[(size_t)l * it.n_hist + h];
            if (!z) continue;
            hs[k] = it.hist[h];
            zs[k] = z;
            ++k;
        }
        if (k == 0) continue;
        int rc = rank_sort(p, it.d_J[l], it.d_w, ws, L, s, 1, nullptr);
        if (rc == AMBER_OK) rc = match_scan(p, hs, k, zs, ws, L, s);
        if (rc == AMBER_OK && d_status) rc = status_collect(p, ws, L, d_status, false, s);
        if (rc != AMBER_OK) return rc;
    }
    return AMBER_OK;
}

int amber_executor_create(amber_executor* out, int n_lanes) {
    if (!out || n_lanes < 1 || n_lanes > 16) return AMBER_E_ARG;
    *out = nullptr;
    amber_executor_s* ex = new (std::nothrow) amber_executor_s();
    if (!ex) return AMBER_E_ARG;
    ex->n_lanes = n_lanes;
    hipError_t e = hipGetDevice(&ex->device);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ex->fork, hipEventDisableTiming);
    for (int l = 1; e == hipSuccess && l < n_lanes; ++l) {
        e = hipStreamCreateWithFlags(&ex->side[l], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ex->join[l], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        amber_executor_destroy(ex);
        return AMBER_E_HIP;
    }
    *out = ex;
    return AMBER_OK;
}

void amber_executor_destroy(amber_executor ex) {
    if (!ex) return;
    for (int l = 1; l < 16; ++l) {
        if (ex->side[l]) {
            (void)hipStreamSynchronize(ex->side[l]);
            (void)hipStreamDestroy(ex->side[l]);
        }
        if (ex->join[l]) (void)hipEventDestroy(ex->join[l]);
    }
    if (ex->fork) (void)hipEventDestroy(ex->fork);
    delete ex;
}

size_t amber_batch_workspace_bytes(const amber_batch_item* items, int n_items, int n_lanes) {
    if (!items || n_items < 1 || n_lanes < 1 || n_lanes > 16) return 0;
    size_t need = 0;
    for (int i = 0; i < n_items; ++i) {
        if (!items[i].plan) return 0;
        need = std::max(need, item_ws_bytes(items[i]));
    }
    return align256(need) * (size_t)std::min(n_lanes, n_items);
}

int amber_batch_run(const amber_batch_item* items, int n_items, unsigned* d_status, void* d_ws, size_t ws_bytes,
                    void* stream, amber_executor ex) {
    if (!items || n_items < 1 || n_items > (1 << 20) || !d_ws) return AMBER_E_ARG;
    for (int i = 0; i < n_items; ++i) {
        const int rc = check_item(items[i]);
        if (rc != AMBER_OK) return rc;
    }
    const int lanes = ex ? std::min(ex->n_lanes, n_items) : 1;
    if (ws_bytes < amber_batch_workspace_bytes(items, n_items, lanes)) return AMBER_E_WORKSPACE;
    unsigned char* ws = static_cast<unsigned char*>(d_ws);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (lanes == 1) {
        for (int i = 0; i < n_items; ++i) {
            const int rc = run_item(items[i], d_status ? d_status + i : nullptr, ws, s);
            if (rc != AMBER_OK) return rc;
        }
        return AMBER_OK;
    }
    // Deal the boxes to the lanes: largest first, each to the least loaded lane.
    const size_t slice = align256(amber_batch_workspace_bytes(items, n_items, 1));
    int* order = new (std::nothrow) int[(size_t)n_items];
    int* lane_of = new (std::nothrow) int[(size_t)n_items];
    if (!order || !lane_of) {
        delete[] order;
        delete[] lane_of;
        return AMBER_E_ARG;
    }
    auto cost = [&](int i) {
        const double n3 = (double)items[i].plan->n * items[i].plan->n * items[i].plan->n;
        return n3 * (double)items[i].n_lmfp;
    };
    for (int i = 0; i < n_items; ++i) order[i] = i;
    std::stable_sort(order, order + n_items, [&](int a, int b) { return cost(a) > cost(b); });
    double load[16] = {};
    for (int k = 0; k < n_items; ++k) {
        int best = 0;
        for (int l = 1; l < lanes; ++l)
            if (load[l] < load[best]) best = l;
        lane_of[order[k]] = best;
        load[best] += cost(order[k]);
    }
    int rc = AMBER_OK;
    if (hipEventRecord(ex->fork, s) != hipSuccess) rc = AMBER_E_HIP;
    for (int l = 1; rc == AMBER_OK && l < lanes; ++l)
        if (hipStreamWaitEvent(ex->side[l], ex->fork, 0) != hipSuccess) rc = AMBER_E_HIP;
    // each lane's boxes in the order they were dealt
    for (int k = 0; rc == AMBER_OK && k < n_items; ++k) {
        const int i = order[k], l = lane_of[i];
        rc = run_item(items[i], d_status ? d_status + i : nullptr, ws + (size_t)l * slice, l == 0 ? s : ex->side[l]);
    }
    // join every side lane back into the caller's stream (also after an error,
    // so that no captured fork is left open)
    for (int l = 1; l < lanes; ++l) {
        if (hipEventRecord(ex->join[l], ex->side[l]) != hipSuccess || hipStreamWaitEvent(s, ex->join[l], 0) != hipSuccess)
            if (rc == AMBER_OK) rc = AMBER_E_HIP;
    }
    delete[] order;
    delete[] lane_of;
    return rc;
}

size_t amber_spectra_workspace_bytes(amber_plan plan) {
    if (!plan) return 0;
    return ws_layout(plan->n, 2).total;
}

int amber_spectra(amber_plan plan, const float* d_a, int kind_a, const float* d_b, int kind_b, int n_bins,
                  double* d_out, void* d_ws, size_t ws_bytes, void* stream) {
    if (!plan || !d_a || !d_out || !d_ws || n_bins < 1 || n_bins > 1024) return AMBER_E_ARG;
    if (kind_a < 0 || kind_a > 2 || kind_b < 0 || kind_b > 2) return AMBER_E_ARG;
    const WsLayout L = ws_layout(plan->n, 2);
    if (ws_bytes < L.total) return AMBER_E_WORKSPACE;
    unsigned char* ws = static_cast<unsigned char*>(d_ws);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    float2* sa = reinterpret_cast<float2*>(ws + L.spec_a);
    float2* na = reinterpret_cast<float2*>(ws + L.nyq_a);
    float2* sb = reinterpret_cast<float2*>(ws + L.spec_b);
    float2* nb = reinterpret_cast<float2*>(ws + L.nyq_b);
    int rc = fft_forward(plan, d_a, sa, na, s);
    if (rc != AMBER_OK) return rc;
    if (d_b && d_b != d_a) {
        rc = fft_forward(plan, d_b, sb, nb, s);
        if (rc != AMBER_OK) return rc;
    } else {
        sb = sa;
        nb = na;
    }
    return spectra_bins(plan, sa, na, kind_a, sb, nb, kind_b, n_bins, d_out, s);
}

int amber_status(amber_plan plan, void* stream, unsigned* status) {
    if (!plan || !status) return AMBER_E_ARG;
    AMBER_HIP_CHECK(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    unsigned v = 0, zero = 0;
    AMBER_HIP_CHECK(hipMemcpy(&v, plan->d_sticky, sizeof(unsigned), hipMemcpyDeviceToHost));
    AMBER_HIP_CHECK(hipMemcpy(plan->d_sticky, &zero, sizeof(unsigned), hipMemcpyHostToDevice));
    *status = v;
    return AMBER_OK;
}

}  // extern "C"
