/*
 * rlbm.h -- C ABI of the MI355X (gfx950) relativistic lattice Boltzmann library.
 *
 * The method is the forced relativistic lattice Boltzmann model of
 * M. Watson, "Two Dimensional Turbulence in a Massless Fluid with a
 * Relativistic Lattice Boltzmann Model" (arXiv:2101.06187):
 *   Sec. III A  relativistic Boltzmann equation with the Anderson-Witting
 *               collision term, Juettner equilibrium, T^{mu nu}, Landau frame,
 *               massless equation of state P = eps/3;
 *   Sec. III B  angular-polynomial expansion (App. A), spherical off-lattice
 *               momentum set streamed by linear interpolation;
 *   Sec. III C  algorithm (a)-(f) and the projected stirring-force term (App. B);
 *   Sec. IV     energy spectrum and vorticity;
 *   Sec. V      2D periodic N x N x 1 lattice, spherical 26+1 momentum set,
 *               random forcing on a band of the Fourier lattice.
 *
 * Units: lattice spacing 1, c = 1, time step dt = cfl, T0 = 1.  Populations
 * F_q are the energy-weighted angular distribution, so T^{mu nu} =
 * sum_q w_q F_q v_q^mu v_q^nu with v^0 = 1 (constant prefactor dropped).
 *
 * Conventions common to every call
 *   - Every function returns an int status: RLBM_OK (0) or a negative code.
 *     No C++ exception crosses this boundary.  rlbm_status_string() names a
 *     code; rlbm_last_error() gives the text of the last failure on the
 *     calling thread.
 *   - Pointers named d_* are device pointers, h_* are host pointers.
 *   - The caller owns all device memory (the workspace, field buffers, the
 *     spectrum scratch) and the HIP stream.  The library never allocates or
 *     frees device memory for user data; it allocates only its host-side
 *     context, and graph-replay state inside the HIP runtime.
 *   - Work is enqueued asynchronously on the stream given to *_init, except
 *     calls that write h_* pointers (they synchronise that stream).
 *   - Field arrays are FP64, row-major [ny][nx], x fastest, no padding.
 *   - A context is used by one host thread at a time; contexts are independent.
 */
#ifndef RLBM_H
#define RLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define RLBM_OK            0
#define RLBM_EINVAL       -1  /* invalid argument (null pointer, size, range) */
#define RLBM_ENOSPACE     -2  /* workspace / buffer too small */
#define RLBM_EHIP         -3  /* a HIP runtime call failed (see rlbm_last_error) */
#define RLBM_EUNSTABLE    -4  /* a site became unphysical: eps <= 0, |beta| >= 1,
                                 non-finite, or the Landau solve did not converge */
#define RLBM_EUNSUPPORTED -5  /* valid request the library does not support */

/* ---- enumerations --------------------------------------------------------- */
/* Momentum stencil.
 * SPH26: the paper's spherical set (Sec. V: "D3Q27" made spherical, Sec. III B:
 *   off-lattice, from the angular quadrature).  The 26 non-zero directions of
 *   the 3x3x3 cube normalised to unit length, weights of the 26-point Lebedev
 *   rule (faces 1/21, edges 4/105, corners 9/280; exact to degree 7).  The
 *   zero momentum has weight 0 (a massless particle cannot be at rest) and is
 *   not stored.  P = eps/3.
 * CIRC8: 2+1-dimensional analogue, 8 in-plane directions at 2 pi q/8, weights
 *   1/8, P = eps/2 (the 2D massless ideal gas).  Not the paper's stencil.
 * SPH26_ZFOLD: SPH26 with each z-mirror pair (a, b, +c) / (a, b, -c) stored
 *   once at the summed weight (17 populations).  Every state of the one-layer
 *   lattice of Sec. V is mirror symmetric, so the dynamics are those of SPH26
 *   exactly; bytes per site drop from 26 to 17 populations.               */
enum { RLBM_STENCIL_SPH26 = 0, RLBM_STENCIL_CIRC8 = 1, RLBM_STENCIL_SPH26_ZFOLD = 2 };

/* Population storage in HBM.  Arithmetic: FP64 for RLBM_F64, FP32 otherwise;
 * the Landau-frame solve is FP64 in every form.  F32, F16S and BF16S store the
 * deviation F_q - 1 from the rest equilibrium at eps = 1 (F_q = 1 for every q),
 * rounded to nearest even; F64 stores F_q.  rlbm_get/set_populations convert,
 * so callers always see F_q.                                                */
enum { RLBM_F64 = 0, RLBM_F32 = 1, RLBM_F16S = 2, RLBM_BF16S = 3 };

/* ---- parameter blocks ----------------------------------------------------- */
typedef struct {
    int32_t nx, ny;   /* lattice sites, 2 <= nx, ny <= 65536, periodic */
    double  cfl;      /* c dt / dx in (0, 2]; a population moves cfl * v_q per step.
                         cfl <= 1 reads the nearest nodes; 1 < cfl <= 2 (the paper's
                         dt = 0.05 on its finest grid, spacing 0.04, is cfl 1.25)
                         reads up to two nodes upstream, tile kernel form only */
} rlbm_lattice;

/* Stirring force (Sec. III C / Sec. V).  Driven modes: integer (kx, ky) with
 * k_lo <= |k| <= k_hi, half plane ky > 0 or (ky == 0, kx > 0), numbered in
 * (ky, kx) lexicographic order; all strictly below Nyquist.  Each step s and
 * mode m draws Philox4x32-10(counter = (m, s, realization, 0), key = seed)
 * -> magnitude r, direction theta, phase phi, and
 *   F(x, y) = amplitude * sum_m r_m (cos theta_m, sin theta_m)
 *                              * cos(2 pi (kx x/nx + ky y/ny) + phi_m).
 * amplitude == 0 means unforced.                                          */
typedef struct {
    double   amplitude;
    double   k_lo, k_hi;
    uint64_t seed;
} rlbm_forcing;

typedef struct rlbm_ctx rlbm_ctx;       /* one lattice; host-allocated by the library */
typedef struct rlbm_batch rlbm_batch;   /* an ensemble of independent lattices        */

/* ---- library info --------------------------------------------------------- */
const char* rlbm_status_string(int status);
const char* rlbm_last_error(void);

/* Direction table of a stencil in the library's storage order.
 * *h_q receives Q (26, 8 or 17); h_v (3*Q doubles, may be NULL) the unit vectors
 * (vx, vy, vz) per direction; h_w (Q doubles, may be NULL) the weights.
 * Pure host function.                                                      */
int rlbm_stencil_info(int stencil, int32_t* h_q, double* h_v, double* h_w);

/* Driven forcing modes for a lattice (host logic only, no device work).
 * Writes up to cap (kx, ky) pairs into h_kx/h_ky (either may be NULL when cap
 * is 0) and the total count into *h_n.  EINVAL if the shell reaches Nyquist.   */
int rlbm_forcing_modes(const rlbm_lattice* lat, const rlbm_forcing* forcing,
                       int32_t* h_kx, int32_t* h_ky, int32_t cap, int32_t* h_n);

/* ---- one lattice ------------------------------------------------------------ */

/* Bytes of device workspace rlbm_init needs (two population buffers of
 * Q * ny * pitch elements, pitch = nx rounded up to 64, plus forcing tables
 * and a few KB of control data).
 * forcing may be NULL (unforced).                                          */
int rlbm_workspace_bytes(const rlbm_lattice* lat, int stencil, int storage,
                         const rlbm_forcing* forcing, size_t* h_bytes);

/* Create a context on caller memory.  tau = tau_R / dt (> 0.5), the
 * relaxation time of the Anderson-Witting term (Sec. III A).  d_workspace
 * must stay valid until rlbm_destroy; hip_stream (hipStream_t, may be NULL
 * for the null stream) is where all work is enqueued.  The populations are
 * undefined until rlbm_set_state / rlbm_set_populations / rlbm_load.
 * Errors: EINVAL (bad lattice, tau <= 0.5, cfl outside (0, 2], k_lo > k_hi,
 * shell at or above Nyquist, unknown enum, null pointer), ENOSPACE, EHIP.  */
int rlbm_init(rlbm_ctx** out, const rlbm_lattice* lat, double tau, int stencil,
              const rlbm_forcing* forcing, int storage,
              void* d_workspace, size_t ws_bytes, void* hip_stream);

/* Relaxation time of the Anderson-Witting term (Sec. III A: tau_R =
 * 5 (eta/s) / T).
 *   RLBM_TAU_CONSTANT (default) -- tau_R / dt = tau at every site.
 *   RLBM_TAU_ETA_S              -- eta/s constant instead: the temperature of
 *     the massless gas is T = T0 (eps / eps_ref)^(1/4) with T0 = eps_ref = 1,
 *     so the local relaxation time is tau(eps) = tau * eps^(-1/4), tau being
 *     its value at eps = 1, i.e. tau = 5 (eta/s) / (T0 dt) (the paper's runs,
 *     eta/s = 0.01 and dt = 0.05 time units, give tau = 1).  The scheme needs
 *     tau(eps) > 1/2, i.e. eps < (2 tau)^4, everywhere.
 * Takes effect from the next step; recorded in checkpoints.  EINVAL for an
 * unknown mode.  Synchronises.                                             */
enum { RLBM_TAU_CONSTANT = 0, RLBM_TAU_ETA_S = 1 };
int rlbm_set_relaxation(rlbm_ctx* ctx, int32_t mode);

/* Step (a) of Sec. III C: F_q := F_eq,q(eps, beta) at every site (the
 * truncated Juettner equilibrium of Sec. III B), step counter := 0, stability
 * flag cleared.  d_e, d_ux, d_uy: FP64 [ny][nx] device arrays of the Landau
 * energy density and the 3-velocity beta (u^mu = gamma (1, beta)).        */
int rlbm_set_state(rlbm_ctx* ctx, const double* d_e, const double* d_ux,
                   const double* d_uy);

/* Advance n >= 0 time steps, each: stream (linear interpolation, periodic),
 * moments, FP64 Landau frame, equilibrium, Anderson-Witting collision, force
 * term, store (Sec. III C (b)-(e)).  Asynchronous; never synchronises.  The
 * stability flag is only read by rlbm_check.                               */
int rlbm_step(rlbm_ctx* ctx, int64_t n);

/* Synchronise the stream and return RLBM_EUNSTABLE if any site of any step
 * since the last set_state/load became unphysical, else RLBM_OK.           */
int rlbm_check(rlbm_ctx* ctx);

/* Steps taken since the last set_state (restored by rlbm_load).           */
int rlbm_step_count(const rlbm_ctx* ctx, int64_t* h_steps);

/* Macroscopic fields at the current time: stage (c) of Sec. III C applied to
 * the current populations -- stream them, form T^{mu nu}, solve the Landau
 * frame in FP64 (the moments the next step computes).  Any output pointer may
 * be NULL.  d_e, d_ux, d_uy: [ny][nx]; d_T: 6 planes [6][ny][nx] holding
 * T^00, T^0x, T^0y, T^xx, T^xy, T^yy.                                     */
int rlbm_fields(rlbm_ctx* ctx, double* d_e, double* d_ux, double* d_uy,
                double* d_T);

/* Sum over the lattice of T^00, T^0x, T^0y of the stored populations, FP64,
 * deterministic order.  Synchronises.                                      */
int rlbm_conserved(rlbm_ctx* ctx, double h_out[3]);

/* Populations as FP64 planes [Q][ny][nx] in the order of rlbm_stencil_info
 * (converted from / to the storage type).  For tests and tooling.
 * The paper's lattice is one layer thick (Sec. V, N x N x 1), so its states
 * are even under v_z -> -v_z, and the 26-direction step never forms the
 * moments with a single z index (T^{0z}, T^{xz}, T^{yz}, which vanish on
 * such states).  rlbm_set_populations therefore accepts only z-mirror
 * symmetric input for RLBM_STENCIL_SPH26: F of direction (a, b, c) must equal
 * F of (a, b, -c) at every site, bit for bit.  It checks this on the device
 * first and returns RLBM_EINVAL, leaving the state unchanged, if any pair
 * differs (or holds a NaN); the check synchronises the stream.  The folded
 * stencil stores one population per mirror pair, and CIRC8 has no z
 * component, so neither needs the check.                                   */
int rlbm_get_populations(rlbm_ctx* ctx, double* d_out);
int rlbm_set_populations(rlbm_ctx* ctx, const double* d_in);

/* Energy spectrum and enstrophy of the current fields (Sec. IV):
 *   E(k_b) = sum over integer k with round(|k|) = k_b of 1/2 |beta_hat(k)|^2,
 *   beta_hat = DFT(beta)/(nx ny), k in [-n/2, n/2)^2, b = 0 .. nbins-1;
 *   Z = 1/2 sum_k |i (2 pi kx/nx) beta_hat_y - i (2 pi ky/ny) beta_hat_x|^2.
 * nx and ny must be powers of two (EUNSUPPORTED otherwise).  d_scratch must
 * hold rlbm_spectrum_scratch_bytes() bytes.  h_Ek: nbins doubles;
 * h_enstrophy may be NULL.  Synchronises.                                  */
int rlbm_spectrum_scratch_bytes(const rlbm_ctx* ctx, size_t* h_bytes);
int rlbm_spectrum(rlbm_ctx* ctx, void* d_scratch, size_t scratch_bytes,
                  double* h_Ek, int32_t nbins, double* h_enstrophy);

/* rlbm_spectrum without caller scratch, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid allocation): the scratch is a 33 MiB array in the library's device
 * memory, one copy per GPU, held until the process ends.  Lattices up to
 * 2^20 sites (nx * ny, both powers of two, e.g. 1024 x 1024); larger ones
 * get RLBM_ENOSPACE.  The call allocates nothing; it must be made with the
 * context's device current (EINVAL otherwise).  Calls on one GPU share the
 * array: calls that overlap on one GPU (other threads, other contexts'
 * streams) race and must be serialised by the caller.  Nothing in the array
 * needs to start at zero; each call overwrites what it reads.  Same results
 * as rlbm_spectrum, synchronises.                                           */
int rlbm_spectrum_static(rlbm_ctx* ctx, double* h_Ek, int32_t nbins, double* h_enstrophy);

/* Velocity with the driven band removed (Sec. V: the recorded velocities are
 * filtered in Fourier space so that the driven wave numbers do not
 * contribute).  beta of the current fields (as rlbm_fields) is transformed,
 * every mode with k_lo^2 <= kx^2 + ky^2 <= k_hi^2 (integer k in
 * [-n/2, n/2)^2, the shell test of the forcing modes) is set to zero, and the
 * field is transformed back.  d_ux, d_uy: [ny][nx] FP64 device outputs, either
 * may be NULL.  h_mean_speed, if not NULL, receives the lattice average of
 * |beta_filtered| (the filtered average fluid velocity by which the paper
 * tunes the forcing amplitude) and the call synchronises.  k_hi may be
 * +infinity (remove everything from k_lo up, the paper's k_f <= k < k_max).
 * Same scratch and power-of-two requirement as rlbm_spectrum.  EINVAL unless
 * 0 <= k_lo <= k_hi.                                                       */
int rlbm_filtered_velocity(rlbm_ctx* ctx, void* d_scratch, size_t scratch_bytes,
                           double k_lo, double k_hi, double* d_ux, double* d_uy,
                           double* h_mean_speed);

/* Number of integer wave vectors in each shell of rlbm_spectrum:
 *   h_counts[b] = #{ k : round(|k|) = b },  b = 0 .. nbins-1,
 * k running over the DFT's integer wave numbers of an nx x ny lattice (per
 * axis k = i for 2i < n, else i - n: [-n/2, n/2) for even n).  Sec. IV
 * defines the spectral energy density as half the squared velocity amplitude
 * averaged over the directions of k; on the lattice that average is the
 * shell sum E(k_b) of rlbm_spectrum divided by h_counts[b].  Any nx, ny >= 1.
 * Pure host function (integer arithmetic, work of order ny times the shells
 * a row crosses).  EINVAL for nx, ny or nbins < 1 or a NULL h_counts.       */
int rlbm_shell_modes(int32_t nx, int32_t ny, int32_t nbins, int64_t* h_counts);

/* Time-averaged spectrum and its error estimate (the paper's appendix on the
 * minimum simulation time): from M spectra sampled every N steps, N being a
 * decorrelation interval,
 *   <E(k)> = (1/M) sum_i E_i(k),
 *   err(k) = (1/M) sum_i sqrt(| <E(k)>^2 - E_i(k)^2 |)
 * (reading: the printed expression under the root can be negative, so its
 * magnitude is taken).  h_samples: M x nbins, row-major (sample i at
 * h_samples + i * nbins); h_mean, h_err: nbins doubles (h_err may be NULL).
 * Pure host function.  EINVAL for M < 1, nbins < 1 or NULL pointers.       */
int rlbm_spectrum_average(const double* h_samples, int32_t n_samples, int32_t nbins,
                          double* h_mean, double* h_err);

/* Checkpoint: a self-describing host blob (header: lattice, stencil,
 * storage, tau and relaxation mode, forcing, step counter; then the
 * population buffer as the library stores it, in the storage type: rows of
 * Q * pitch elements, pitch = nx rounded up to 64, each row made of 64-column
 * bricks holding population 0 .. Q-1 in turn; the padding columns carry no
 * data).  A run resumed from it continues bit for bit, because the forcing
 * is counter-based.  rlbm_load rejects a blob of another configuration
 * (EINVAL).  Both synchronise.                                             */
int rlbm_state_bytes(const rlbm_ctx* ctx, size_t* h_bytes);
int rlbm_save(rlbm_ctx* ctx, void* h_buf, size_t bytes);
int rlbm_load(rlbm_ctx* ctx, const void* h_buf, size_t bytes);

/* Streaming copy of `bytes` bytes from d_src to d_dst on hip_stream (NULL:
 * the null stream), `reps` times after one untimed copy, with 16-byte loads
 * and stores and four loads in flight per thread, 8 blocks per compute unit,
 * each copying one contiguous chunk.  *h_ms receives the mean duration of one copy in
 * milliseconds (HIP events around the reps; synchronises).  A copy moves
 * 2 * bytes through HBM when both buffers are larger than the caches: the
 * practical streaming ceiling against which the step's bandwidth is read.
 * EINVAL: NULL pointers, bytes or a pointer not a multiple of 16, reps < 1,
 * overlapping buffers.  The buffers belong to the caller.                  */
int rlbm_stream_copy(const void* d_src, void* d_dst, size_t bytes, int32_t reps,
                     void* hip_stream, double* h_ms);

/* Kernel form and launch shape.  Results never depend on them (bitwise).
 *   RLBM_KERNEL_TILE   -- every thread streams one site from global memory;
 *                         param = tile height th in {1, 2, 4, 8} rows of 64 sites.
 *   RLBM_KERNEL_MARCH  -- each wavefront marches down a 64-column strip, loading
 *                         every population row once into a rolling register
 *                         window, and writes with non-temporal stores (this
 *                         form is for lattices far larger than the caches);
 *                         param = rows per strip segment (0: chosen from the
 *                         lattice size and the GPU's resident waves).
 *   RLBM_KERNEL_STAGED -- a block of 4 wavefronts stages the population rows
 *                         of its 64 x 4 tile (its own rows, the needed
 *                         populations of the rows above and below, and the
 *                         halo columns) into LDS with aligned row loads, then
 *                         every site streams from LDS; param = 4 (or 0).
 *   RLBM_KERNEL_MARCH_PAIRS -- F16S and BF16S storage only: as RLBM_KERNEL_MARCH
 *                         with every lane on two adjacent columns, so that
 *                         each load and store moves a 32-bit pair of a
 *                         128-column strip; param as for RLBM_KERNEL_MARCH.
 *                         Needs an even nx on every lattice (EUNSUPPORTED
 *                         otherwise; the autotuner then skips it).
 *   RLBM_KERNEL_MARCH2 -- two time steps per launch: each wavefront marches
 *                         down a 62-column strip computing the first step
 *                         into registers and the second from them, so every
 *                         population is read and written once per two steps;
 *                         param = rows per strip segment, 0 = 12 rows.  An
 *                         odd step count ends with one launch of the
 *                         one-step form.  Needs ny >= 3 on every lattice
 *                         (EUNSUPPORTED otherwise; the autotuner then skips
 *                         it).
 * By default the library uses RLBM_KERNEL_MARCH (param 0) for FP32, F16S and
 * BF16S storage when every resident wavefront gets a segment of at least 8
 * rows, and RLBM_KERNEL_TILE with th = 4 otherwise; RLBM_KERNEL_STAGED and
 * RLBM_KERNEL_MARCH2 are used only when requested or chosen by the autotuner
 * (the two-step form moves half the bytes per step but, holding two steps'
 * rows in registers, runs fewer wavefronts: with short segments, param 0 =
 * 12 rows, it is faster than the one-step form for FP32 lattices much larger
 * than the caches, slower elsewhere).  With
 * cfl > 1 only the tile form exists (the other forms give EUNSUPPORTED).
 * rlbm_set_tile(th) is rlbm_set_kernel(RLBM_KERNEL_TILE, th).
 * rlbm_get_kernel reports the form that advances the bulk of the steps.
 * rlbm_autotune times the tile heights, the staged form, five segment lengths
 * of the row-marching form (the automatic one and 1/2, 3/4, 3/2 and 2 times
 * it; a length two of them share is timed once), the same five of the paired
 * form for 16-bit storage, and the two-step form with segments of 8, 10, 12,
 * 16, 18, 20, 24 and 32 rows, for `steps` steps each (advancing the state) and keeps
 * the fastest; *h_th receives th, or minus the segment length for a
 * marching form.                                                           */
enum {
    RLBM_KERNEL_TILE = 0,
    RLBM_KERNEL_MARCH = 1,
    RLBM_KERNEL_MARCH2 = 2,
    RLBM_KERNEL_STAGED = 3,
    RLBM_KERNEL_MARCH_PAIRS = 4
};
int rlbm_set_kernel(rlbm_ctx* ctx, int32_t kind, int32_t param);
int rlbm_get_kernel(const rlbm_ctx* ctx, int32_t* h_kind, int32_t* h_param);
int rlbm_set_tile(rlbm_ctx* ctx, int32_t th);
int rlbm_autotune(rlbm_ctx* ctx, int32_t steps, int32_t* h_th);

/* Replay rlbm_step in chunks of `chunk` steps through a captured HIP graph
 * (0 = direct launches).  Results are identical either way.               */
int rlbm_set_graph_chunk(rlbm_ctx* ctx, int32_t chunk);

/* n >= 1 launches of the form rlbm_get_kernel reports (n steps, or 2 n for
 * RLBM_KERNEL_MARCH2), directly, with a HIP event recorded on the context's
 * stream just before and just after every launch; synchronises and writes
 * the mean duration of one launch in milliseconds to *h_ms.  For roofline
 * measurement.                                                             */
int rlbm_profile_step_kernel(rlbm_ctx* ctx, int64_t n, double* h_ms);

void rlbm_destroy(rlbm_ctx* ctx);

/* ---- ensemble of independent lattices --------------------------------------- */
/* n_real realizations, each with its own lattice, tau and forcing
 * (forcings may be NULL: all unforced); realization r draws its forcing with
 * Philox counter word 2 = r.  All share the stencil and the storage.  One
 * persistent kernel advances every lattice per step.                       */
int rlbm_batch_workspace_bytes(int32_t n_real, const rlbm_lattice* lats,
                               int stencil, int storage,
                               const rlbm_forcing* forcings, size_t* h_bytes);
int rlbm_batch_init(rlbm_batch** out, int32_t n_real, const rlbm_lattice* lats,
                    const double* taus, int stencil,
                    const rlbm_forcing* forcings, int storage,
                    void* d_workspace, size_t ws_bytes, void* hip_stream);
int rlbm_batch_set_state(rlbm_batch* b, int32_t r, const double* d_e,
                         const double* d_ux, const double* d_uy);
int rlbm_batch_step(rlbm_batch* b, int64_t n);
int rlbm_batch_step_count(const rlbm_batch* b, int64_t* h_steps);
int rlbm_batch_check(rlbm_batch* b);
int rlbm_batch_fields(rlbm_batch* b, int32_t r, double* d_e, double* d_ux,
                      double* d_uy, double* d_T);
int rlbm_batch_get_populations(rlbm_batch* b, int32_t r, double* d_out);
int rlbm_batch_set_graph_chunk(rlbm_batch* b, int32_t chunk);
/* rlbm_set_relaxation for every lattice of the ensemble.                   */
int rlbm_batch_set_relaxation(rlbm_batch* b, int32_t mode);
/* rlbm_set_kernel, rlbm_get_kernel and rlbm_autotune for the ensemble's
 * launches (the autotuner advances every lattice by the steps it times).   */
int rlbm_batch_set_kernel(rlbm_batch* b, int32_t kind, int32_t param);
int rlbm_batch_get_kernel(const rlbm_batch* b, int32_t* h_kind, int32_t* h_param);
int rlbm_batch_autotune(rlbm_batch* b, int32_t steps, int32_t* h_th);
void rlbm_batch_destroy(rlbm_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* RLBM_H */
