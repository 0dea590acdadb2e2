/*
 * pin.h -- C ABI of libpin: the collapse-time path of PINOCCHIO (Monaco et al. 2013,
 * arXiv:1305.1505) on AMD Instinct MI355X (gfx950).
 *
 * The path (section "Collapse times" of the paper):
 *   1. a Gaussian linear density field delta_l on an N^3 Lagrangian grid of side L, normalised so
 *      that its top-hat variance at 8 Mpc/h is sigma_8^2 (eq. deltal and the paragraph after it);
 *   2. for each Gaussian smoothing radius R, the deformation tensor T_ij = d_i d_j phi with
 *      lap(phi) = delta_l, obtained with FFTs;
 *   3. for each grid point, the inverse collapse time F = 1/D(t_coll) (eq. F) of the ellipsoidal
 *      collapse model (truncated 3rd-order LPT with a quasi-spherical correction);
 *   4. for each grid point, the maximum F over the radii, F_max, and the radius R_max where it
 *      was reached (the trajectory maximum);
 *   5. the closing Zel'dovich and 2LPT displacement fields.
 *
 * Conventions shared by every entry point
 *   - Grids are C order, z fastest.  A "half spectrum" is complex [N][N][N/2+1] (the layout of a
 *     real-to-complex 3D FFT); a "real field" is [N][N][N].  Complex numbers are interleaved
 *     (re, im) pairs of the plan's precision: float for PIN_FP32, double for PIN_FP64.
 *   - The forward transform is unnormalised: a real field x has spectrum
 *     X(k) = sum_q x(q) exp(-2 pi i k.q/N); the inverse carries 1/N^3.
 *   - Integer frequencies f = 0..N/2-1, -N/2..-1 on x and y, 0..N/2 on z; k = 2 pi f / L (h/Mpc).
 *     Every mode with a Nyquist index carries no derivative and is treated as zero.
 *   - Radii are in grid cells (R_phys = R * L / N); the window is W(kR) = exp(-k^2 R^2 / 2).
 *   - Device pointers are caller-owned (the library never frees them) and must stay valid until
 *     the work queued on `stream` completes.  Every call is ordered on `stream` (NULL = the null
 *     stream) and returns without waiting for the GPU.
 *   - Arguments are validated before anything is queued: on an error status nothing was written.
 *     A plan is not thread-safe; distinct plans may be used from distinct threads.
 *   - Errors: every function returns a pin_status; pin_last_error() returns a thread-local
 *     message for the last failure on the calling thread.
 */
#ifndef PIN_H
#define PIN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIN_OK = 0,
  PIN_ERR_INVALID_ARG = 1,      /* a NULL pointer, a bad size, an unordered radius list, ... */
  PIN_ERR_UNSUPPORTED_SIZE = 2, /* N not in the supported set (pin_size_supported)           */
  PIN_ERR_OUT_OF_MEMORY = 3,    /* device allocation failed                                  */
  PIN_ERR_DEVICE = 4,           /* a HIP call or kernel launch failed                        */
  PIN_ERR_NOT_READY = 5,        /* serving: the result is not ready yet                      */
  PIN_ERR_BUDGET = 6,           /* serving: the request can never fit the HBM budget         */
  PIN_ERR_CANCELLED = 7,        /* serving: the request was cancelled                        */
  PIN_ERR_SHUTDOWN = 8,         /* serving: the server is shutting down                      */
  PIN_ERR_TIMEOUT = 9           /* serving: a wait timed out                                 */
} pin_status;

typedef enum {
  PIN_FP32 = 0, /* complex64 FFTs and spectral multiplies (FP64-computed twiddles and windows);
                   float64 for the eigenvalue near degeneracy and for the collapse root        */
  PIN_FP64 = 1  /* complex128 FFTs, float64 throughout                                        */
} pin_precision;

typedef struct pin_plan_s* pin_plan;

/* Problem description (section "Collapse times"): grid, box, radii and spectrum. */
typedef struct {
  int n;                     /* grid points per side: 8, 12, 16, 24, 32, 48, 64, 96, 128,
                                192, 256, 384, 512, 768 or 1024 (pin_size_supported)         */
  double box;                /* side L in Mpc/h, > 0                                          */
  int n_radii;               /* 1..254                                                        */
  const double* radii_cells; /* host array of n_radii radii in cells, > 0, strictly decreasing
                                (largest first); copied by pin_plan_create                     */
  double sigma8;             /* top-hat rms at 8 Mpc/h, > 0 (workloads: 0.8)                  */
  double gamma;              /* BBKS shape parameter, > 0 (workloads: 0.21)                   */
  double ns;                 /* primordial slope of P(k) = A k^ns T_BBKS(k/gamma)^2 (1.0)     */
  pin_precision prec;
} pin_plan_desc;

/* Whether N is a supported grid size (1) or not (0). Host only. */
int pin_size_supported(int n);

/* Device bytes pin_plan_create allocates for `desc` (workspace, tables); host only. */
pin_status pin_plan_workspace_bytes(const pin_plan_desc* desc, size_t* bytes);

/* Validate `desc` without touching the GPU. */
pin_status pin_plan_validate(const pin_plan_desc* desc);

/* Create a plan on the current HIP device: computes the sigma_8 amplitude, the FP64 twiddle and
 * window tables, and allocates the FFT workspace.  *out receives the handle. */
pin_status pin_plan_create(const pin_plan_desc* desc, pin_plan* out);

/* Replace the plan's radius list (section "Collapse times": the smoothing radii): n_radii must
 * not exceed the count the plan was created with; the radii follow the rules of pin_plan_desc
 * (copied).  The new window tables are uploaded on `stream` and the call returns once the copy
 * is done; work queued earlier on other streams must not be using this plan. */
pin_status pin_plan_set_radii(pin_plan plan, const double* radii_cells, int n_radii, hipStream_t stream);

/* Free the plan and its device memory (waits for the device to go idle first). */
pin_status pin_plan_destroy(pin_plan plan);

/* eq. deltal: write the seeded Gaussian linear field's half spectrum to `dk` (device,
 * N*N*(N/2+1) complex).  Each half-space mode (i, j, l) takes two uniforms from Philox4x32-10
 * (Salmon et al., SC'11) with counter (i*N + j)*(N/2+1) + l split into (low, high) 32-bit words
 * and key = seed split likewise; a uniform is (2*(w >> 12) + 1)*2^-53 from the 64-bit words
 * w = c1:c0 and c3:c2; Box-Muller gives g1 + i g2 and dk = sqrt(P(k) N^6 / (2 L^3)) (g1 + i g2).
 * On the l = 0 plane the member of each (f, -f) pair with the larger i*N + j is drawn and the
 * other is its conjugate; k = 0 and every Nyquist mode are zero. */
pin_status pin_generate_field(pin_plan plan, uint64_t seed, void* dk, hipStream_t stream);

/* Set F (device, N^3 of the plan's real type) to 0 and ridx (device, N^3 bytes) to 255. */
pin_status pin_collapse_reset(pin_plan plan, void* F, uint8_t* ridx, hipStream_t stream);

/* Trajectory maximum over radii [r_begin, r_end) (0 <= r_begin < r_end <= n_radii), updating
 * the running state (F, ridx) in place: for each radius r in order and each grid point, if the
 * inverse collapse time F(q; R_r) is strictly larger than F[q], F[q] <- F(q; R_r) and
 * ridx[q] <- r.  dk is the half spectrum (device).  Splitting [0, n_radii) into consecutive
 * ranges gives the same result as one call. */
pin_status pin_collapse_times_range(pin_plan plan, const void* dk, void* F, uint8_t* ridx,
                                    int r_begin, int r_end, hipStream_t stream);

/* pin_collapse_reset followed by pin_collapse_times_range over all radii: F_max and the index
 * of R_max (255 where no radius gives a positive F). */
pin_status pin_collapse_times(pin_plan plan, const void* dk, void* F, uint8_t* ridx,
                              hipStream_t stream);

/* Velocity at the trajectory maximum (section "Collapse times", last paragraph: with F_max the
 * code records v_max, computed from the first derivative of the peculiar potential smoothed on
 * R_max each time F_max is updated).  v_max is [3][N^3] (x, y, z; plan precision, device,
 * caller-owned): the Zel'dovich displacement of the field smoothed on the radius of the last
 * update of F_max, psi1_R(k) = i k W(kR) dk / k^2 in Mpc/h at D = 1 (times a H f D for a
 * peculiar velocity), 0 where F_max was never set.  F and ridx are exactly those of the calls
 * without _v.  The first _v call on a plan allocates pin_plan_velocity_workspace_bytes of
 * device memory more, kept until pin_plan_destroy. */
pin_status pin_plan_velocity_workspace_bytes(const pin_plan_desc* desc, size_t* bytes);
/* pin_collapse_reset, and v_max <- 0. */
pin_status pin_collapse_reset_v(pin_plan plan, void* F, uint8_t* ridx, void* vmax, hipStream_t stream);
/* pin_collapse_times_range, also setting v_max[.][q] wherever F[q] is updated. */
pin_status pin_collapse_times_range_v(pin_plan plan, const void* dk, void* F, uint8_t* ridx, void* vmax,
                                      int r_begin, int r_end, hipStream_t stream);
/* pin_collapse_reset_v followed by pin_collapse_times_range_v over all radii. */
pin_status pin_collapse_times_v(pin_plan plan, const void* dk, void* F, uint8_t* ridx, void* vmax,
                                hipStream_t stream);

/* Growing-mode clock (section "Collapse times": the linear growing mode D, normalised to 1 at
 * z = 0, is the time coordinate; F = 1/D at collapse; section "Simulations": flat LambdaCDM).
 * pin_plan_set_growth tabulates D for a flat LambdaCDM universe without radiation,
 * D(a) ~ E(a) Int_0^a da'/(a' E(a'))^3 with E^2 = omega_m a^-3 + 1 - omega_m (0 < omega_m <= 1;
 * 1 is Einstein-de Sitter, D = a), in float64 on the host, and keeps it on the device with the
 * plan (stream-ordered upload; returns when done).  pin_collapse_redshift writes, for each of
 * count values F (device, plan precision), the redshift z_c with D(z_c) = 1/F to zc (device, plan
 * precision); z_c = -1 where F <= 0 or where 1/F is beyond D(a = 1e6) (no collapse).  Computed
 * in float64 (relative error of 1 + z_c below 1e-12, besides the rounding of z_c itself).
 * PIN_ERR_INVALID_ARG without a table. */
pin_status pin_plan_set_growth(pin_plan plan, double omega_m, hipStream_t stream);
pin_status pin_collapse_redshift(pin_plan plan, const void* F, size_t count, void* zc, hipStream_t stream);

/* Smoothing-radius ladder (section "Collapse times": radii chosen so that the mass variances of
 * the smoothed field are logarithmically spaced by 0.15 dex).  Host only.  sigma^2(R) is the
 * variance of the field smoothed with the plan's Gaussian window, 1/(2 pi^2) Int k^2 P(k)
 * exp(-k^2 R^2) dk for the BBKS spectrum (gamma, ns; the amplitude cancels), R = cells * box / n
 * Mpc/h.  From r_max_cells the ladder descends with sigma^2 growing by 10^dex per step while the
 * radius stays >= r_min_cells; *count receives its length, radii_cells (host, capacity entries;
 * may be NULL to query the length) the radii, largest first. */
pin_status pin_radius_ladder(int n, double box, double r_max_cells, double r_min_cells, double dex, double gamma,
                             double ns, double* radii_cells, int capacity, int* count);

/* The six deformation-tensor components at radius index r (r = -1: unsmoothed), written to T6
 * (device, [6][N][N][N] real, order xx, xy, xz, yy, yz, zz). */
pin_status pin_deformation_tensor(pin_plan plan, const void* dk, int r, void* T6,
                                  hipStream_t stream);

/* Closing displacements at D = 1 in Mpc/h, each [3][N][N][N] real (components x, y, z):
 * psi1 = Zel'dovich, psi1(k) = i k dk / k^2;  psi2 = EdS 2LPT, psi2(k) = (3/7) i k mu2~(k) / k^2
 * with mu2 = sum_{i<j} (T_ii T_jj - T_ij^2) of the unsmoothed tensor and mu2~ its forward
 * transform (k = 0 and Nyquist modes zeroed).  Either output may be NULL to skip it. */
pin_status pin_displacements(pin_plan plan, const void* dk, void* psi1, void* psi2,
                             hipStream_t stream);

/* Third-order displacement at D = 1 in Mpc/h (conclusions: halo positions from 3rd-order LPT;
 * the terms are those of standard Einstein-de Sitter 3LPT, x = q + D psi1 + D^2 psi2 + D^3 psi3),
 * psi3 [3][N][N][N] real (device, plan precision, caller-owned; components x, y, z):
 *     div psi3 = det(T1)/3 - (10/21) ((tr T1)(tr T2) - tr(T1 T2))/2,  curl psi3 = C/7,
 *     C_i = eps_ijk (T1 T2)_jk,
 * T1 the unsmoothed tensor of pin_displacements, T2 the Hessian of phi2 with lap phi2 = mu2(T1);
 * i.e. psi3(k) = i (-k S(k) + k x c(k)) / k^2 with S and c the forward transforms of the
 * divergence and of C/7 (k = 0 and Nyquist modes zeroed in every spectrum, no dealiasing).  The first call on a plan allocates
 * pin_plan_lpt3_workspace_bytes of device memory more, kept until pin_plan_destroy;
 * PIN_ERR_OUT_OF_MEMORY if that fails.  dk is the half spectrum (device). */
pin_status pin_plan_lpt3_workspace_bytes(const pin_plan_desc* desc, size_t* bytes);
pin_status pin_lpt3_displacement(pin_plan plan, const void* dk, void* psi3, hipStream_t stream);

/* Fragmentation of the collapsed medium into halos (section "Fragmentation").  Particles (grid
 * points) with F[q] >= f_min (f_min = 1/D at the output time, > 0) are taken in decreasing F
 * (ties in increasing linear index) at D = 1/F; each looks at its six neighbours:
 *   (i) none collapsed: a new halo; (ii) one halo touched: accreted if d < f_a R + f_ra +
 *   f_s (R sigma(R) D)^1.7 (eq. accretion), then neighbouring filament particles join it, else a
 *   filament particle; (iii) several halos: accretion on the halo of smallest d/R, then every
 *   pair merged if d < f_m max(R1, R2) + f_rm (eq. merging), accretion retried after the mergers
 *   if it failed; (iv) filaments only: a filament particle.
 * d is the distance after Zel'dovich displacement, x = q + D vmax (vmax from pin_collapse_times_v,
 * Mpc/h, converted to grid units), periodic minimum image; a halo sits at its founder's position
 * plus the mean offset of its members plus D times their mean displacement; R = (3 N_h/4 pi)^(1/3)
 * grid units; sigma(R) is the top-hat rms of the plan's linear field at R box/n Mpc/h (64 nodes per
 * octave, linear in ln R); merged halos keep the id of the larger (smaller id on equal sizes).
 * The result equals that of taking the particles one by one in this order (the GPU runs them in
 * parallel rounds of particles whose neighbourhoods and halos do not overlap).
 * F [N^3] and vmax [3][N^3] are device arrays of the plan's precision; label [N^3] (device,
 * int32) receives -2 (F < f_min), -1 (filament) or the halo id (linear index of its founding
 * particle); halo_size [N^3] (device, int32, may be NULL) receives N_h at each halo id and 0
 * elsewhere; *n_halos (host) the number of halos.  params NULL means Table 1's values
 * (pin_fragment_default_params).  Synchronous: returns when done (rounds are driven from the
 * host).  The first call on a plan allocates pin_plan_fragment_workspace_bytes of device memory
 * more, kept until pin_plan_destroy. */
typedef struct {
  double f_a, f_ra, f_s; /* eq. accretion */
  double f_m, f_rm;      /* eq. merging   */
} pin_fragment_params;
void pin_fragment_default_params(pin_fragment_params* out);
pin_status pin_plan_fragment_workspace_bytes(const pin_plan_desc* desc, size_t* bytes);
pin_status pin_fragment(pin_plan plan, const void* F, const void* vmax, double f_min, const pin_fragment_params* params,
                        int32_t* label, int32_t* halo_size, int* n_halos, hipStream_t stream);
/* Halo catalogue of the last pin_fragment call on this plan (section "Fragmentation": halos are
 * output with their masses, Lagrangian centres of mass and Zel'dovich displacements).  For each
 * halo in increasing id: id[k], its particle count n_particles[k], its Lagrangian centre of mass
 * centre[a*capacity + k] (founder position plus the mean minimum-image offset of the members from
 * it, wrapped into [0, box), Mpc/h) and the mean of its members' vmax, displacement[a*capacity + k]
 * (Mpc/h at D = 1; times D at the output time for positions).  Device arrays (int32, int32, float64
 * [3][capacity], float64 [3][capacity]); capacity >= the n_halos of that call.  PIN_ERR_INVALID_ARG
 * without a completed pin_fragment.  Synchronous. */
pin_status pin_fragment_catalog(pin_plan plan, int32_t* id, int32_t* n_particles, double* centre, double* displacement,
                                int capacity, hipStream_t stream);
/* Merger history of the last pin_fragment call on this plan (section "Fragmentation": reported at
 * the final time, the masses of the merging halos at each merger), in the order the mergers
 * happened: f[k] the F_max of the particle whose step merged the halos (D = 1/f), keep[k] the id
 * of the halo that keeps its id and n_keep[k] its particle count before the merger, gone[k] and
 * n_gone[k] those of the halo absorbed.  Device arrays of `capacity` entries (float64, int32 x 4);
 * *count (host) receives the number of mergers.  With capacity 0 and every array NULL the call
 * only sets *count; otherwise capacity below the count is PIN_ERR_INVALID_ARG.  Synchronous. */
pin_status pin_fragment_mergers(pin_plan plan, double* f, int32_t* keep, int32_t* gone, int32_t* n_keep,
                                int32_t* n_gone, int capacity, int* count, hipStream_t stream);

/* eq. F per point: the inverse collapse time of the ellipsoidal collapse model (the per-point
 * step of pin_collapse_times) for caller-given tensors.  T6 (device, [6][count] of the plan's
 * real type, components xx, xy, xz, yy, yz, zz) -> F (device, [count]).  Model: lambda_1 = the
 * largest eigenvalue, delta = tr T, mu2 = sum_{i<j} lambda_i lambda_j, mu3 = det T; F_E3 = the
 * largest positive root of F^3 - lambda_1 F^2 - (mu2/7) F + (mu3/9 - 10 delta mu2/189) (0 if
 * none), the first-axis orbit crossing of 3rd-order LPT with the higher-order traces shared
 * equally by the axes; F = F_E3 (1 + (X3/delta_c - 1) s) with s = clamp(1 - 3p/delta, 0, 1) for
 * delta > 0 (else 0), p^2 = tr((T - delta/3)^2)/6, X3 = 2.05008... the root of
 * 1 - x/3 - x^2/21 - 23x^3/1701, delta_c = (3/20)(12 pi)^(2/3).  count = 0 is a no-op. */
pin_status pin_inverse_collapse_time(pin_plan plan, const void* T6, size_t count, void* F, hipStream_t stream);

/* pin_collapse_times for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): no plan, no hipMalloc/hipFree,
 * no copy from host memory and no host wait -- only kernel launches on `stream`.  The workspace a
 * plan would allocate (11 half-spectrum slots, twiddle and window tables) is one static device
 * array of 96 MiB that the library holds on each device it runs on until the process ends; its
 * device address is looked up once per device on the first call there, so make that first call
 * outside stream capture: later calls queue kernels only and can be captured into a HIP graph
 * whose replays recompute the result.  desc as for
 * pin_plan_create (the spectrum fields are not used); dk, F and ridx as for pin_collapse_times
 * (device, caller-owned), with the same results.  Sizes: N <= 128 in PIN_FP32 and N <= 96 in
 * PIN_FP64 (any radius count); larger ones return PIN_ERR_UNSUPPORTED_SIZE before anything is
 * queued.  Every call on a device shares that device's array: calls that overlap on one device
 * (on different streams, or from different threads) race and give undefined results; calls
 * ordered on one stream are safe.  Each call rewrites every part of the array it reads. */
pin_status pin_collapse_times_noalloc(const pin_plan_desc* desc, const void* dk, void* F, uint8_t* ridx,
                                      hipStream_t stream);

/* Per-kernel timing with HIP events recorded around every launch of the plan on its stream.
 * Kernel classes are numbered 0..pin_kernel_class_count()-1 and named by pin_kernel_class_name. */
int pin_kernel_class_count(void);
const char* pin_kernel_class_name(int cls);
pin_status pin_plan_set_timing(pin_plan plan, int enable); /* enabling also resets the totals   */
/* Waits for the recorded events, then returns the summed duration (ms) and launch count. */
pin_status pin_plan_kernel_time(pin_plan plan, int cls, double* total_ms, long long* launches);

/* ------------------------------------------------------------------------------------------
 * Serving: continuous batching of realization requests (seed, grid size, box, radii) of uneven
 * sizes as they arrive.  A server owns per-size-class "slots" (a plan workspace, the field and
 * the outputs of one request, and a stream of its own); a request is admitted when a slot of its
 * class is idle or a new one fits the device-memory budget (idle slots of other classes are
 * evicted, least recently used first), and its whole path -- field, collapse times over its
 * radii, optionally ZA and 2LPT displacements -- is then queued on that slot's stream as one
 * captured hipGraph (cached per slot for each radius count, box and displacement choice).
 * Admitted requests therefore run concurrently; within a size class admission is first come,
 * first served.  Every request's result is computed by the same kernels with the same inputs
 * whatever else is in flight, so it is bitwise identical alone and in a mix.  All server calls
 * are thread-safe.  Results are device pointers owned by the server until pin_serve_release. */
typedef struct pin_server_s* pin_server;

typedef struct {
  uint64_t seed;             /* field seed (pin_generate_field)                            */
  int n;                     /* grid size (pin_size_supported)                              */
  double box;                /* Mpc/h, > 0                                                  */
  int n_radii;               /* 1..254                                                      */
  const double* radii_cells; /* host, strictly decreasing, > 0; copied by pin_serve_submit  */
  int want_disp;             /* 1: also psi1 and psi2                                       */
} pin_request;

typedef struct {
  const void* F;             /* device [N^3] F_max (server precision)                       */
  const uint8_t* ridx;       /* device [N^3] radius index of F_max, 255 = never             */
  const void* psi1;          /* device [3][N^3] or NULL                                     */
  const void* psi2;          /* device [3][N^3] or NULL                                     */
  int n, n_radii;
  double t_submit, t_admit, t_done;   /* seconds since the server was created              */
  pin_status status;
} pin_result;

typedef struct {
  double hbm_budget_bytes;   /* device bytes all slots together may hold                   */
  int max_slots_per_class;   /* concurrent requests per grid size, >= 1                     */
  int device;                /* HIP device ordinal                                          */
  pin_precision prec;
  double sigma8, gamma, ns;  /* spectrum, as in pin_plan_desc                               */
} pin_serve_config;

typedef struct {
  double p50_s, p99_s, mean_s;   /* latency submit -> done of completed requests            */
  double updates_per_s;          /* sum of N^3 n_radii completed / (last done - first submit) */
  double hbm_in_use;             /* bytes held by slots                                     */
  long long completed, failed, cancelled, queued, running, slots;
} pin_serve_stats_t;

/* Device bytes one slot of grid size n holds (host only; the admission unit). */
pin_status pin_serve_slot_bytes(const pin_serve_config* cfg, int n, size_t* bytes);
pin_status pin_serve_create(const pin_serve_config* cfg, pin_server* out);
/* Validate and copy the request, return a ticket; never blocks.  PIN_ERR_BUDGET if a slot of
 * this size can never fit the budget; PIN_ERR_SHUTDOWN after pin_serve_destroy began. */
pin_status pin_serve_submit(pin_server srv, const pin_request* req, uint64_t* ticket);
/* PIN_ERR_NOT_READY while queued or running; PIN_OK with *out filled when done; the request's
 * failure status (PIN_ERR_DEVICE, PIN_ERR_CANCELLED, ...) otherwise. */
pin_status pin_serve_poll(pin_server srv, uint64_t ticket, pin_result* out);
/* As poll, blocking up to timeout_s seconds (PIN_ERR_TIMEOUT after that). */
pin_status pin_serve_wait(pin_server srv, uint64_t ticket, double timeout_s, pin_result* out);
/* Queued: removed (PIN_ERR_CANCELLED).  Running: its result is discarded when the device work
 * ends.  Finished: no effect. */
pin_status pin_serve_cancel(pin_server srv, uint64_t ticket);
/* Forget a finished request and free its slot for the next one (invalidates its pointers). */
pin_status pin_serve_release(pin_server srv, uint64_t ticket);
pin_status pin_serve_stats(pin_server srv, pin_serve_stats_t* out);
pin_status pin_serve_reset_stats(pin_server srv);
/* Stop admitting, cancel queued requests, wait for running ones, free all device memory. */
pin_status pin_serve_destroy(pin_server srv);

const char* pin_status_string(pin_status status);
const char* pin_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PIN_H */
