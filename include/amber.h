/*
 * amber.h -- C-ABI of the MI355X (gfx950) library for the reionization-redshift
 * hot path of AMBER (Trac et al., "AMBER: A Semi-numerical Abundance Matching
 * Box for the Epoch of Reionization", arXiv:2109.10375).
 *
 * Two device stages, each a single asynchronous call on a HIP stream:
 *   amber_radiation : J = S * [exp(-r/l_mfp) / (4 pi r^2)] on a periodic N^3
 *                     grid (Sec. 3.4.1, Eq. intensity), by forward real 3D FFT,
 *                     multiplication by the kernel transform atan(k l_mfp)/k and
 *                     inverse FFT;
 *   amber_zre       : abundance matching (Sec. 3.4.2): cells ranked by J
 *                     (higher first), gas mass 1+delta summed in that order,
 *                     z_re assigned so that the ionized mass fraction equals the
 *                     Weibull history x_i(z) (Sec. 3.1.2, Eq. weibull).
 * plus host-side helpers for the history (Sec. 3.1, Appendix A).
 *
 * Conventions for every call:
 *   - fields are N^3 FP32 arrays in row-major order, z fastest: cell (x, y, z)
 *     is element (x * N + y) * N + z.  "d_" pointers are device pointers on the
 *     device that was current when the plan was created; "host" pointers are
 *     ordinary host memory.
 *   - the caller owns every buffer and stream; the library owns plans.  Compute
 *     calls never allocate: all scratch comes from a caller-provided device
 *     workspace of at least amber_workspace_bytes() bytes, which may be reused
 *     once the stream has passed the call.  Calls sharing one workspace must be
 *     ordered on one stream.
 *   - compute calls return after enqueueing work on `stream` (a hipStream_t; NULL
 *     is the default stream).  Results are deterministic and do not depend on
 *     the launch order of other work.
 *   - errors are returned as negative codes and never abort.  Argument errors
 *     are found on the host before anything is enqueued.  Data errors found on
 *     the device (NaN intensity, non-positive or non-finite weights, a mass sum
 *     wider than 127 bits) set bits of the plan's status word, which keeps them
 *     until amber_status() reads and clears it; the outputs of such a call are
 *     unspecified.
 */
#ifndef AMBER_H
#define AMBER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define AMBER_OK 0
#define AMBER_E_ARG (-1)        /* null pointer, bad count, non-finite parameter   */
#define AMBER_E_SIZE (-2)       /* grid size not supported                          */
#define AMBER_E_HISTORY (-3)    /* no positive Weibull coefficients for a history   */
#define AMBER_E_WORKSPACE (-4)  /* workspace too small                              */
#define AMBER_E_HIP (-5)        /* a HIP runtime call failed                        */
#define AMBER_E_UNIMPL (-6)     /* not implemented                                  */

/* Device status bits reported by amber_status(). */
#define AMBER_STATUS_NAN_J 1u   /* an intensity was NaN (no rank order exists)      */
#define AMBER_STATUS_BAD_W 2u   /* a weight was <= 0, NaN or infinite               */
#define AMBER_STATUS_RANGE 4u   /* exact mass sum needs more than 127 bits          */

typedef struct amber_plan_s* amber_plan;

/* Reionization-history parameters, Sec. 3.1.1: midpoint, duration, asymmetry and
 * the ionization fractions at the early, middle and late redshifts.  An x_* of 0
 * selects the paper's default (0.05, 0.5, 0.95). */
typedef struct {
    double z_mid, delta_z, a_z;
    double x_ear, x_mid, x_lat;
} amber_history;

/* A fitted history: Weibull coefficients (Sec. 3.1.2) and the geometry of the
 * inversion table used by amber_zre.
 *   z_top   = a_w + b_w (64 ln 2)^(1/c_w)        (x_i(z_top) = 2^-64)
 *   h       = smallest power of two >= (z_top - a_w) / 2^22
 *   table_n = T + 1 with T = ceil((z_top - a_w) / h); node j is z_j = a_w + j h
 *             and holds X_j = exp(-((z_j - a_w)/b_w)^c_w) (FP64)
 * d_table must point to T + 1 doubles on the device holding exactly the values
 * written by amber_weibull_table() for this struct (amber_history_prepare
 * fills such a buffer).  amber_zre rejects a struct whose h, z_top or table_n
 * differ from what amber_weibull_from_coeffs gives for its coefficients.
 * d_growth selects the matching equation (Sec. 3.4.2): NULL weights every cell
 * by its gas mass 1 + delta at z_mid; otherwise it points to T + 1 pairs
 * (X_j, G_j) of device doubles (2 (T + 1) doubles, 16-byte aligned, as written
 * by amber_growth_table), G_j = D(z_j)/D(z_mid), and the overdensities are
 * extrapolated linearly to each redshift, delta(z) = G delta.  The pairs keep
 * a node's two values in one 16-byte read for the bisection. */
typedef struct {
    double a_w, b_w, c_w;
    double h, z_top;
    int64_t table_n;
    const double* d_table;
    const double* d_growth;
} amber_weibull;

/* ---- history helpers (host work; the two prepare calls also copy to the device) -- */

const char* amber_version(void);
const char* amber_strerror(int code);

/* Appendix A: z_ear = z_mid + Delta_z A_z/(1 + A_z), z_lat = z_ear - Delta_z
 * (Sec. 3.1.1), then the root c_w of the Appendix-A equation and the algebraic
 * a_w, b_w.  Fills everything except d_table.  AMBER_E_HISTORY when a
 * coefficient would not be positive or A_z > 15 (Sec. 3.1.2's stated range);
 * AMBER_E_ARG for Delta_z <= 0, A_z <= 0 or unordered ionization points. */
int amber_weibull_fit(const amber_history* hist, amber_weibull* out);

/* Table geometry for given coefficients (all > 0); d_table is set to NULL. */
int amber_weibull_from_coeffs(double a_w, double b_w, double c_w, amber_weibull* out);

/* Writes the T + 1 inversion-table values X_j into host_table (n_entries must
 * equal w->table_n).  The caller copies them to the device and sets d_table. */
int amber_weibull_table(const amber_weibull* w, double* host_table, int64_t n_entries);

/* Sec. 3.1 and Sec. 3.1.2 on the device: amber_weibull_fit of hist, then the
 * T + 1 inversion-table values of amber_weibull_table copied into the caller's
 * device buffer d_table_buf (buf_bytes >= 8 table_n bytes) on `stream`; *out
 * receives the fitted history with d_table = d_table_buf (d_growth NULL).
 * Blocks the host until the copy has completed (the values are built in
 * library-owned host memory that is freed before returning).  With d_table_buf
 * NULL only *out is filled (d_table NULL): table_n gives the buffer size.
 * Errors: those of amber_weibull_fit; AMBER_E_WORKSPACE when buf_bytes is too
 * small; AMBER_E_HIP when the copy fails (nothing is written to *out). */
int amber_history_prepare(const amber_history* hist, amber_weibull* out, void* d_table_buf, size_t buf_bytes,
                          void* stream);

/* Sec. 3.4.2 with growth-rescaled overdensities: the (X_j, G_j) pairs of
 * amber_growth_table for the fitted history *w copied into the caller's device
 * buffer d_pairs_buf (16-byte aligned, buf_bytes >= 16 table_n) on `stream`;
 * sets w->d_growth = d_pairs_buf.  Blocks the host until the copy has
 * completed.  AMBER_E_ARG for a misaligned buffer or a table geometry that is
 * not amber_weibull_from_coeffs(a_w, b_w, c_w)'s; AMBER_E_WORKSPACE when the
 * buffer is too small; AMBER_E_HIP when the copy fails (w is left unchanged). */
int amber_growth_prepare(amber_weibull* w, double z_mid, double omega_m, void* d_pairs_buf, size_t buf_bytes,
                         void* stream);

/* Linear growth factor ratio at the table nodes, G_j = D(a_w + j h)/D(z_mid),
 * j = 0..T, for a flat universe of matter density omega_m (0 < omega_m <= 1)
 * and a cosmological constant; D is the growing mode, D = a while matter
 * dominates: D(a) = a 2F1(1/3, 1; 11/6; -(1 - omega_m)/omega_m a^3) (the paper's
 * cosmology, Sec. 2, has omega_m = 0.3).  Written as pairs: host_table[2j] =
 * X_j (the value amber_weibull_table writes) and host_table[2j + 1] = G_j, so
 * host_table holds 2 n_entries doubles; n_entries must equal w->table_n. */
int amber_growth_table(const amber_weibull* w, double z_mid, double omega_m, double* host_table,
                       int64_t n_entries);

/* ---- plans and workspace ------------------------------------------------ */

/* Plan for an N^3 periodic box of side box_len (same length unit as l_mfp).
 * N must be one of 8, 16, 32, 64, 96, 128, 192, 256, 512, 1024.  Allocates the
 * plan's twiddle tables on the current device (the only allocation the library
 * makes).  AMBER_E_SIZE for other N. */
int amber_plan_create(amber_plan* out, int n, double box_len);
void amber_plan_destroy(amber_plan plan);

/* Device workspace needed by amber_radiation (with n_lmfp mean free paths),
 * amber_rank and amber_zre (with n_hist histories; 0 for radiation or rank
 * only) on this plan.  0 for a NULL plan, n_lmfp outside 0..64 or n_hist
 * outside 0..8. */
size_t amber_workspace_bytes(amber_plan plan, int n_lmfp, int n_hist);

/* ---- device stages ------------------------------------------------------ */

/* Radiation field, Sec. 3.4.1 (Eq. intensity):
 *   J_l = IDFT[ DFT(S) * Khat(|k|; l) ] / N^3,  Khat(k; l) = atan(k l)/k, Khat(0) = l,
 *   k = (2 pi / box_len) |m~| with m~ the signed integer frequency.
 * d_src: N^3 FP32 source field S (read only).  l_mfp: host array of n_lmfp
 * mean free paths (> 0, finite).  d_J: host array of n_lmfp device pointers,
 * each to N^3 FP32 outputs (must not alias d_src or the workspace).  The
 * forward transform of S is computed once and shared by all l_mfp. */
int amber_radiation(amber_plan plan, const float* d_src, const double* l_mfp, int n_lmfp,
                    float* const* d_J, void* d_ws, size_t ws_bytes, void* stream);

/* ---- FFT launch schedules and the tuner ---------------------------------- */

/* The FFTs inside amber_radiation, amber_radiation_from_halos and
 * amber_spectra (the DFTs of Sec. 3.4.1 and Sec. 3.2.1) run as column passes,
 * which split a length-N transform into N1 x (N/N1) over N1 threads and take
 * tiles of C columns, and z passes, which split the length-N/2 complex
 * transform of the real lines into M1 x (N/2/M1) over M1 threads and take ZL
 * lines per block.  Several (N1, C) and (M1, ZL) candidates are compiled per
 * grid size; candidate 0 is the default.  All candidates compute the same
 * transforms; they differ in FP32 rounding order only.
 *
 * Number of column-pass and z-pass candidates for grid size n (host only, no
 * device call).  AMBER_E_SIZE for an unsupported n. */
int amber_fft_schedules(int n, int* n_col, int* n_z);

/* Split of candidate idx: kind 0 gives (N1, C) of a column pass, kind 1
 * (M1, ZL) of a z pass.  Host only.  AMBER_E_ARG for a bad kind or idx. */
int amber_fft_schedule_info(int n, int kind, int idx, int* split, int* width);

/* Chooses the candidates later calls on this plan use (not thread-safe with
 * calls in flight on other host threads).  AMBER_E_ARG when out of range. */
int amber_plan_set_schedule(amber_plan plan, int col, int z);
int amber_plan_get_schedule(amber_plan plan, int* col, int* z);

/* Autotuner: times one radiation pass (one mean free path) of d_src into d_J
 * under every (column, z) candidate pair, `reps` passes per pair after one
 * untimed pass, in three rounds (a pair's figure is its fastest round), and
 * sets the plan to the fastest pair.  The default pair is kept unless another
 * is faster by more than 2 %; among those, the lowest-index pair within 1 % of
 * the fastest is taken.  d_src: N^3 FP32 (read only); d_J: N^3 FP32
 * scratch, overwritten; d_ws: amber_workspace_bytes(plan, 1) bytes.
 * ms_out: host array of n_col * n_z floats (row-major [col][z], mean ms per
 * pass), may be NULL; col, z: the chosen pair, may be NULL.  Creates and
 * destroys two HIP events and blocks the host until the timing passes end;
 * launches are not traced by amber_profile_begin.  On error the plan keeps
 * the schedule it had. */
int amber_plan_tune(amber_plan plan, const float* d_src, float* d_J, void* d_ws, size_t ws_bytes, int reps,
                    float* ms_out, int* col, int* z, void* stream);

/* Mass-assignment windows for halo sources (Sec. 3.2.1, Eq. Wofk: p = 1, 2, 3). */
#define AMBER_ASSIGN_NGP 1
#define AMBER_ASSIGN_CIC 2
#define AMBER_ASSIGN_TSC 3

/* Workspace needed by amber_radiation_from_halos on this plan. */
size_t amber_halo_workspace_bytes(amber_plan plan);

/* Radiation field of a halo catalogue (Sec. 3.2.1 and Sec. 3.4.1):
 *   the halo masses are assigned with window p (scheme) to mesh 1 and, when
 *   interlace is set, with the positions shifted by +l_c/2 on every axis to
 *   mesh 2 (cell i spans [i, i+1) l_c, node at its centre, periodic);
 *   S(k) = [A(k) + e^{i k.dx} B(k)] / 2 / W(k) (Eq. interlace), or A(k)/W(k)
 *   without interlacing, W(k) = prod_d [sin(k_d l_c/2)/(k_d l_c/2)]^p (Eq. Wofk),
 *   k_d = (2 pi/L) m~_d (m~ the signed frequency, +N/2 at the Nyquist index);
 *   J_l = Re IDFT[S(k) Khat(|k|; l)] / N^3 for each l_mfp, as amber_radiation.
 * d_pos: device, n_halo x 3 FP32 positions in [0, box_len) (others wrap);
 * d_mass: device, n_halo finite FP32 masses.  When 16 divides N and the
 * binned copies of the catalogue fit in the workspace's two spectrum regions
 * (up to (4 N^3 + 8 N^2) / 16 halo-superbin pairs, about 1.05 per halo, and as
 * many halo-tile pairs, about 1.4 per halo for CIC with interlacing), each
 * mesh cell is the exact sum of its terms rounded once to FP32 and J is
 * identical from call to call; otherwise the deposit falls back to FP32
 * global atomics, whose last bits depend on their order. */
int amber_radiation_from_halos(amber_plan plan, const float* d_pos, const float* d_mass, int64_t n_halo,
                               int scheme, int interlace, const double* l_mfp, int n_lmfp, float* const* d_J,
                               void* d_ws, size_t ws_bytes, void* stream);

/* Rank order of Sec. 3.4.2: d_perm[n] = index of the cell of rank n, ranking by
 * d_J descending, ties by ascending cell index, -0 equal to +0.  NaN sets
 * AMBER_STATUS_NAN_J.  d_perm: N^3 uint32 outputs. */
int amber_rank(amber_plan plan, const float* d_J, uint32_t* d_perm,
               void* d_ws, size_t ws_bytes, void* stream);

/* Abundance matching, Sec. 3.4.2:
 *   C_n = exact sum of d_w over the cells of rank <= n (inclusive),
 *   F_n = RN(C_n) / RN(C_N)  (FP64, round-to-nearest-even conversions),
 *   z_n = the table inversion of x_i(z) = F_n:
 *         j = max{ j in [0, T] : X_j >= F_n } clamped to T - 1,
 *         t = (X_j - F_n) / (X_j - X_{j+1})  (0 when the two are equal),
 *         z = z_j + t (z_{j+1} - z_j),  z = min(z, z_top),
 *         all in FP64 without fused multiply-add,
 *   d_zre[h][perm[n]] = (float) z_n for each history h.
 * With a growth table (d_growth), rank n (k = n + 1 cells ionized) instead
 * solves m_j / M_j = X_j with the growth-weighted masses
 *   m_j = (k s)(1 - G_j) + G_j RN(C_n),  M_j = (N s)(1 - G_j) + G_j RN(C_N),
 *   s = the unit of the exact sums (the cell count in the same units),
 * h_j = m_j / M_j - X_j: z = a_w if h_0 > 0, z_top if h_T <= 0, otherwise
 * bisection on the node index keeps h_lo <= 0 < h_hi down to adjacent nodes and
 * z = z_lo + t (z_hi - z_lo), t = -h_lo / (h_hi - h_lo), min z_top (FP64,
 * this operation order, no fused multiply-add).
 * d_J: N^3 FP32 intensities; d_w: N^3 FP32 gas-mass weights (1 + delta, > 0);
 * hist: host array of n_hist fitted histories with device tables; d_zre: host
 * array of n_hist device pointers to N^3 FP32 outputs.  The rank order and the
 * cumulative mass are computed once and shared by all histories. */
int amber_zre(amber_plan plan, const float* d_J, const float* d_w,
              const amber_weibull* hist, int n_hist, float* const* d_zre,
              void* d_ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): amber_zre
 * without a workspace.  Its scratch is a static device array of
 * AMBER_NOALLOC_SCRATCH_BYTES (68 MiB) in the library, one copy per device,
 * held until the process ends; it suffices for plans of N <= AMBER_NOALLOC_MAX_N
 * (128).  Arguments and results as amber_zre (bit-identical z_re).  The call
 * allocates nothing and enqueues only kernels.  Every call on a device shares
 * that device's array, which keeps the last call's contents: calls that
 * overlap in time on one device race and must be ordered by the caller.
 * AMBER_E_SIZE for a plan with N > AMBER_NOALLOC_MAX_N; AMBER_E_HIP when the
 * array's device address could not be looked up at plan creation. */
#define AMBER_NOALLOC_MAX_N 128
#define AMBER_NOALLOC_SCRATCH_BYTES (68u << 20)
int amber_zre_noalloc(amber_plan plan, const float* d_J, const float* d_w, const amber_weibull* hist, int n_hist,
                      float* const* d_zre, void* stream);

/* Waits for `stream`, then returns in *status and clears the device status
 * bits (AMBER_STATUS_*) of every ranking and matching call on this plan since
 * the plan was created or amber_status last cleared them, whatever workspace
 * the calls used.  Calls still in flight on other streams are reported by a
 * later amber_status once they have completed. */
int amber_status(amber_plan plan, void* stream, unsigned* status);

/* ---- two-point statistics (Sec. 2.3) ------------------------------------- */

/* How a field enters the spectra: as given, as the overdensity f/mean - 1
 * (mean != 0), or as the normalised redshift (f - mean)/(1 + mean) of
 * Eq. (deltaz); the mean is the volume average. */
#define AMBER_FIELD_RAW 0
#define AMBER_FIELD_OVERDENSITY 1
#define AMBER_FIELD_REDSHIFT 2

/* Workspace needed by amber_spectra on this plan. */
size_t amber_spectra_workspace_bytes(amber_plan plan);

/* Shell-averaged auto and cross power spectra of two N^3 FP32 fields
 * (Eq. Pk; Dk, bias and rcc follow from them):
 *   shell i (0 <= i < n_bins <= 1024) holds the modes of the full N^3 DFT grid
 *   with i - 1/2 <= |m~| < i + 1/2 (m~ the signed integer frequency);
 *   P_xy = (L^3/N^6) <Re(X_m conj Y_m)> over the shell, X the unnormalised DFT
 *   of field x after its kind_x normalisation; k_i = (2 pi/L) <|m~|>.
 * d_out: device, 8 * n_bins doubles, each row n_bins long: k | number of modes
 * | P_aa | P_bb | P_ab | Delta^2_aa = k^3 P_aa/(2 pi^2) (Eq. Dk) | b_ab =
 * sqrt(P_aa/P_bb) (Eq. bias) | r_ab = P_ab/sqrt(P_aa P_bb) (Eq. rcc); empty
 * shells (and undefined ratios) are zero.  d_b may be NULL or equal to
 * d_a (one transform).  Modes beyond the last shell are left out.  The sums
 * are accumulated with FP64 atomics, so the last bits may differ between runs. */
int amber_spectra(amber_plan plan, const float* d_a, int kind_a, const float* d_b, int kind_b, int n_bins,
                  double* d_out, void* d_ws, size_t ws_bytes, void* stream);

/* ---- batches (several boxes, mean free paths and histories) ------------- */

/* One box of a batch: the radiation field for each of its n_lmfp mean free
 * paths (Sec. 3.4.1), then abundance matching of every J against each of its
 * n_hist histories (Sec. 3.4.2), exactly as amber_radiation followed by one
 * amber_zre per J.  Boxes may have different plans (sizes). */
typedef struct {
    amber_plan plan;             /* grid size and box side of this box                     */
    const float* d_src;          /* N^3 source field; NULL: d_J already holds the fields   */
    const float* d_w;            /* N^3 gas-mass weights (1 + delta, > 0)                  */
    int n_lmfp;                  /* 1..64                                                  */
    const double* l_mfp;         /* host array of n_lmfp mean free paths (unused if no src) */
    float* const* d_J;           /* host array of n_lmfp device pointers to N^3 FP32       */
    int n_hist;                  /* 1..8                                                   */
    const amber_weibull* hist;   /* host array of n_hist fitted histories (device tables)  */
    float* const* d_zre;         /* host array of n_lmfp * n_hist device pointers, entry
                                    l * n_hist + h is z_re of J_l under history h, or NULL
                                    when that pair is not wanted                           */
} amber_batch_item;

/* Side streams and events on which amber_batch_run runs boxes concurrently
 * ("lanes"): lane 0 is the caller's stream, lanes 1..n_lanes-1 are streams the
 * executor creates (default priority, non-blocking) with one event each, plus
 * one fork event.  Created once, outside any timed or captured region, on the
 * device that is current; destroyed by amber_executor_destroy.  n_lanes in
 * 1..16.  An executor must not be used by two host threads at once. */
typedef struct amber_executor_s* amber_executor;
int amber_executor_create(amber_executor* out, int n_lanes);
void amber_executor_destroy(amber_executor ex);

/* Workspace for amber_batch_run over these items on n_lanes lanes: n_lanes
 * slices of the largest single-box requirement (each lane runs its boxes one
 * after another in its own slice). 0 on bad input. */
size_t amber_batch_workspace_bytes(const amber_batch_item* items, int n_items, int n_lanes);

/* Runs every box of the batch (Sec. 3.4: each box's radiation fields, then
 * the matching of each field against its histories).  With ex NULL the boxes
 * run in order on `stream`.  With an executor of L lanes the boxes are dealt
 * to the lanes, largest first (cost N^3 times the number of fields), each lane
 * taking the box with the least accumulated cost; the lanes fork from `stream`
 * (an event recorded on it) and join back into it (one event per side lane),
 * so the work after the call on `stream` sees every result, and the whole
 * call can be captured into a HIP graph from `stream`.  Results do not depend
 * on the lanes: each box computes exactly what its single calls compute.
 * Entries of d_zre may be NULL: that (l, h) pair is not matched, and a field
 * with no requested history is not ranked (a sparse set of pairs per box).
 * All items are checked on the host before anything is enqueued (the first
 * error is returned and nothing runs).  d_status (optional, device, n_items
 * unsigned) receives the OR of each box's device status bits (AMBER_STATUS_*).
 * Only kernels and event records/waits are enqueued (no allocation, copy,
 * memset or synchronisation); per-kernel timing (amber_profile_begin) must be
 * off while capturing. */
int amber_batch_run(const amber_batch_item* items, int n_items, unsigned* d_status, void* d_ws, size_t ws_bytes,
                    void* stream, amber_executor ex);

/* ---- per-kernel timing (tracing aid, not needed for results) ------------ */

typedef struct {
    char name[48];      /* kernel name, e.g. "fft_x_mul", "rank_pass1"          */
    int32_t launches;   /* launches timed                                       */
    double total_ms;    /* summed HIP-event time between each launch's start and
                           stop events, recorded on the launch's own stream    */
} amber_kernel_time;

/* Starts timing the kernels that later compute calls on this plan launch:
 * creates `capacity` pairs of HIP events (besides the tuner's two, the only
 * events the library creates); launches beyond capacity are not timed.  Calls
 * on several streams are timed each on its own stream. */
int amber_profile_begin(amber_plan plan, int capacity);

/* Waits for the recorded events, writes up to max_entries per-kernel totals
 * (aggregated by name, in first-launch order) and their count, releases the
 * events and stops timing. */
int amber_profile_end(amber_plan plan, amber_kernel_time* out, int max_entries, int* n_entries);

#ifdef __cplusplus
}
#endif

#endif /* AMBER_H */
