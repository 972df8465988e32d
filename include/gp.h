/*
 * gp.h -- C-ABI of the MI355X (gfx950) split-step Crank-Nicolson solver for the 3D
 * Gross-Pitaevskii equation in a fully anisotropic harmonic trap,
 *
 *     i dpsi/dt = [ -1/2 lap + 1/2 (nux^2 x^2 + nuy^2 y^2 + nuz^2 z^2) + g |psi|^2 ] psi,
 *
 * propagated in imaginary time (ground states, renormalised every step) or real time
 * (dynamics).  Method: paper, program summary "Solution method" and program summaries
 * (i) imagtime3d / (ii) realtime3d: discretise space and time, split the Hamiltonian into
 * the potential+nonlinear part (calcnu) and one Crank-Nicolson solve per axis (calclux,
 * calcluy, calcluz), and propagate over small steps; norm, rms sizes, chemical potential
 * and energy (calcrms, calcmuen) are global sums.
 *
 * Layout (paper, "Summary of revisions"): psi is ONE contiguous device array
 * [nx][ny][nz] with z stride 1, y stride nz, x stride ny*nz; complex values interleaved
 * (re, im): complex64 = 2 x float, complex128 = 2 x double.
 *
 * Grid: x_i = (i - (nx-1)/2) dx, i = 0..nx-1 (centred at 0), homogeneous Dirichlet
 * ghosts at i = -1 and i = nx; same for y and z.  One step (split = GP_SPLIT_LIE):
 *   psi <- exp(-tau (V + g|psi|^2)) psi     (tau = dt imaginary, i dt real)
 *   then one Crank-Nicolson solve along x, y, z with c = dt/(4 d^2) (imaginary) or
 *   i dt/(4 d^2) (real):  -c u_{i-1} + (1+2c) u_i - c u_{i+1} = c p_{i-1} + (1-2c) p_i + c p_{i+1}
 *   imaginary time then renormalises psi to dx dy dz sum|psi|^2 = 1.
 * GP_SPLIT_STRANG uses half potential steps before and after the sweeps.
 *
 * Ownership: psi is caller-owned device memory (e.g. a torch tensor); the library keeps
 * a non-owning pointer and never frees it.  The context owns its coefficient tables,
 * reduction scratch, device-side parameters and graphs.  The HIP stream is borrowed;
 * every call is ordered on it.  Step calls do not synchronise; gp_norm, gp_energy_mu,
 * gp_rms, gp_raw_sums, gp_status and gp_converge_imag synchronise the stream.  A context
 * is not thread-safe; use one context per stream.
 *
 * Errors: every function returns GP_OK (0) or a negative GP_ERR_* code; nothing aborts
 * or prints.  An asynchronous kernel fault surfaces at the next synchronising call as
 * GP_ERR_HIP; gp_last_error(ctx) returns the runtime's message.
 */
#ifndef GP_H
#define GP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GP_OK = 0,
  GP_ERR_INVALID = -1,     /* bad parameter, null pointer, psi not device memory */
  GP_ERR_HIP = -2,         /* HIP runtime error (message: gp_last_error) */
  GP_ERR_OOM = -3,         /* device allocation failed */
  GP_ERR_NONFINITE = -4,   /* a norm or observable came out NaN/Inf */
  GP_ERR_ZERO_NORM = -5,   /* psi has zero norm */
  GP_ERR_UNSUPPORTED = -6  /* grid too large for the kernels' line mapping */
};

enum { GP_C64 = 0, GP_C128 = 1 };                 /* storage / sweep precision */
enum { GP_SPLIT_LIE = 0, GP_SPLIT_STRANG = 1 };
enum { GP_FLAG_NONFINITE = 1, GP_FLAG_ZERO_NORM = 2 }; /* gp_status flags */

typedef struct gp_ctx gp_ctx;

typedef struct {
  int32_t nx, ny, nz;     /* 3 <= n <= 2048 grid points per axis (gp_batch: <= 1024);
                           * gp_init returns GP_ERR_UNSUPPORTED where no kernel mapping
                           * covers a line (z lines: a block's 4 lines must fit 64 KiB
                           * of LDS, <= 2032 points complex64, <= 1016 complex128; x and
                           * y lines of complex128 <= 1024) or a wavefront's rows of an x/y sweep would
                           * span 2 GiB or more (x: 64-128 planes of ny*nz points) */
  double dx, dy, dz;      /* > 0 spacings */
  double nux, nuy, nuz;   /* >= 0 trap frequencies */
  double g;               /* nonlinearity, any finite real */
  double dt;              /* > 0 time step, used by both step kinds */
  int32_t precision;      /* GP_C64 (complex64 storage, FP32 sweeps, FP64 sums) or GP_C128 */
  int32_t split;          /* GP_SPLIT_LIE (default) or GP_SPLIT_STRANG */
} gp_params;

/* Create a context for psi (device pointer, nx*ny*nz complex values of the chosen
 * precision) on hip_stream (a hipStream_t; NULL = default stream). */
int gp_init(const gp_params* p, void* psi_dev, void* hip_stream, gp_ctx** out);
int gp_destroy(gp_ctx* c);

/* nsteps imaginary-time steps (paper: program summary (i)); psi is renormalised every
 * step and is normalised to dx dy dz sum|psi|^2 = 1 on return. Does not synchronise. */
int gp_step_imag(gp_ctx* c, int32_t nsteps);
/* nsteps real-time steps (paper: program summary (ii)); no renormalisation. */
int gp_step_real(gp_ctx* c, int32_t nsteps);

/* dx dy dz sum |psi|^2 in FP64.  Synchronises. */
int gp_norm(gp_ctx* c, double* norm);
/* Energy and chemical potential of the normalised state phi = psi/sqrt(N) (calcmuen):
 *   E = (T+U)/N + (g/2) I/N^2,  mu = (T+U)/N + g I/N^2, with T the kinetic link sum
 *   1/2 dV sum_a sum_links |dpsi|^2/da^2 over all +1 links including the ghost links,
 *   U = dV sum V|psi|^2, I = dV sum |psi|^4, N = dV sum |psi|^2.  Synchronises. */
int gp_energy_mu(gp_ctx* c, double* energy, double* mu);
/* rms[4] = <x^2>^1/2, <y^2>^1/2, <z^2>^1/2, <r^2>^1/2 of the normalised state (calcrms). */
int gp_rms(gp_ctx* c, double rms[4]);
/* raw[9] = { N, Tx, Ty, Tz, U, I, dV sum x^2|psi|^2, dV sum y^2|psi|^2, dV sum z^2|psi|^2 } */
int gp_raw_sums(gp_ctx* c, double raw[9]);

/* Change g (quench).  Stream-ordered device-side update; no graph rebuild. */
int gp_set_g(gp_ctx* c, double g);
/* Point the context at another caller buffer of the same shape and precision. */
int gp_set_psi(gp_ctx* c, void* psi_dev);
/* Steps done so far, the last cheap chemical-potential estimate -ln(N_pre)/(2 dt) from
 * the imaginary-time renormalisation, and GP_FLAG_* bits.  Synchronises. */
int gp_status(gp_ctx* c, int64_t* steps_done, double* mu_est, int32_t* flags);

/* Imaginary-time propagation to the ground state at relative tolerance tol, checking every
 * check_every = K steps (K <= 0 selects ceil(0.25/dt)), at most max_steps steps.
 * Stopping rule, on the sequence of checked values m_n with d_n = m_n - m_{n-1} and
 * q_n = d_n / d_{n-1}: while m approaches its limit geometrically (q_n and q_{n-1} in
 * (0, 1) and within q_n / 10 of each other), stop when |d_n| <= tol |m_n|, the
 * extrapolated distance to the limit |d_n| r / (1 - r) with r = max(q_n, q_{n-1})
 * (Aitken) is <= tol |m_n| / 2 and the extrapolated limit agrees within tol |m_n| / 2 with
 * the previous check's; otherwise (m(t) turning, as from an already close start,
 * alternating, or at its rounding floor) when |d| <= tol |m| / 10 at three successive
 * checks (gp_stop_rule_eval replays the rule on a given sequence).  complex64: m = mu (the
 * observables pass) at every check.  complex128: m = mu_est = -ln(N_pre)/(2 dt) from the
 * renormalisation (no extra pass); when it stops, mu is evaluated and must change by at
 * most tol |mu| (with the same predicted tail) over one more interval, else monitoring
 * resumes.
 * Returns the steps taken and the final mu.  GP_OK also when max_steps is reached;
 * *converged tells which.  Synchronises at every check. */
int gp_converge_imag(gp_ctx* c, double tol, int32_t check_every, int64_t max_steps,
                     int64_t* steps_taken, double* mu, int32_t* converged);
/* The stopping rule of gp_converge_imag and gp_batch_converge_imag on a host sequence
 * values[0..n) (one value per check, in order): *stop_index = the first index at which the
 * rule is met, -1 if it never is.  Host only (no device, no context); n >= 0, values and
 * stop_index non-null when n > 0, else GP_ERR_INVALID. */
int gp_stop_rule_eval(const double* values, int32_t n, double tol, int32_t* stop_index);


/* Per-kernel timing: while enabled, eager launches are bracketed by HIP events on the
 * context's stream (graphs are not used).  gp_get_timing returns the mean duration in ms
 * of each kernel kind { x sweep, y sweep, z sweep, norm finalize, other } and the number
 * of launches of each, accumulated since enabling.  Synchronises. */
int gp_set_timing(gp_ctx* c, int32_t enable);
int gp_get_timing(gp_ctx* c, double ms_mean[5], int64_t launches[5]);

/* Line mapping in use: {m_x, sw_x, m_y, sw_y, segments_z, m_z}.  m = points per thread
 * along a line, sw = line segments per wavefront for the x and y sweeps (a wavefront then
 * covers 64/sw lines), segments_z = threads per z line (power of two <= 64).
 * gp_set_mapping overrides it (0 = keep / choose); combinations the kernels do not cover
 * return GP_ERR_INVALID and leave the mapping unchanged.  Synchronises. */
int gp_get_mapping(gp_ctx* c, int32_t map[6]);
int gp_set_mapping(gp_ctx* c, const int32_t map[6]);

/* Halo-truncated Crank-Nicolson inverse (an opt-in variant of the sweeps).  The solution
 * of a line is u_i = sum_m a^m d_{i+m} (the back-substitution of the constant-pivot
 * elimination, |a| = |c gamma| < 1); mode 1 keeps only the first H + 1 terms, with H the
 * smallest length whose dropped tail |a|^(H+1)/(1-|a|) max|d| is below 1/100 of the storage
 * precision's unit roundoff, so results agree with the exact sweeps to rounding.  Then each
 * thread streams one whole x or y line (forward elimination exact from the line start,
 * u_{j-H} emitted at step j): one coalesced read and write of psi per sweep, no LDS, no
 * barriers; the z sweep stays exact.  mode 2 keeps the exact x sweep, writing its result
 * to a work array the context allocates (psi's size), and fuses the y and z sweeps into
 * one pass from that array back into psi: a block walks the rows of one plane (chunks of
 * rows, each started H rows early), and every row the truncated y solve emits is a whole
 * z line, solved at once in LDS; psi crosses HBM twice per step instead of three times
 * (32 instead of 48 B per point in complex64).  mode 2 needs z lines of at most 1024
 * points, one group of rows of z lines ((H + 1) ceil(ceil(nz/64) / (H + 1)) rows) within
 * 160 KiB of LDS (complex128 960-point lines with H = 6 need 261 KB: unsupported), and
 * psi-sized free device memory (else GP_ERR_OOM, mode unchanged).  mode 0: exact sweeps
 * (default).  Returns GP_ERR_UNSUPPORTED (mode unchanged) when H exceeds 15 (dt/dx^2
 * large) or the grid does not fit the fused pass.
 * gp_get_truncation: the mode and H per [imaginary, real][x, y, z].  Synchronises. */
int gp_set_truncation(gp_ctx* c, int32_t mode);
int gp_get_truncation(gp_ctx* c, int32_t* mode, int32_t hlen[6]);

/* Project autotuner: times every line mapping the kernels cover on this context's grid
 * (each axis independently, `steps` steps of kind mode = 0 imaginary / 1 real, HIP-event
 * kernel durations), keeps the fastest and returns it in map_out (nullable).  psi, the
 * device state and the step count are restored afterwards (one temporary device copy of
 * psi).  cache_path (nullable): a text file of earlier results keyed by grid, precision
 * and step kind; a hit applies the stored mapping without timing, a miss appends the new
 * result.  Synchronises. */
int gp_autotune(gp_ctx* c, int32_t mode, int32_t steps, const char* cache_path, int32_t map_out[6]);

/* ---------------------------------------------------------------------------------------
 * Batched form: n independent grids (different sizes, traps, g and dt allowed; one
 * precision and one splitting) advanced by the same launches, four per step whatever n
 * is.  psi_dev is ONE caller-owned device buffer; instance i occupies
 * nx_i*ny_i*nz_i complex values from element offsets[i] on (same layout as a single
 * grid); regions must not overlap.  Each instance's psi must stay below 4 GiB.
 * `active` (nullable, n bytes): instances with 0 are left untouched by the step calls
 * (and stay masked until a later call passes them as 1).  Step calls do not
 * synchronise; the observables, status and convergence calls do.
 * ------------------------------------------------------------------------------------- */
typedef struct gp_batch gp_batch;

int gp_batch_init(const gp_params* p, int32_t n, void* psi_dev, const int64_t* offsets,
                  void* hip_stream, gp_batch** out);
int gp_batch_destroy(gp_batch* b);
int gp_batch_step_imag(gp_batch* b, int32_t nsteps, const uint8_t* active);
int gp_batch_step_real(gp_batch* b, int32_t nsteps, const uint8_t* active);
/* per instance, arrays of length n (rms4 and raw: 4n and 9n, instance-major) */
int gp_batch_norm(gp_batch* b, double* norm);
int gp_batch_energy_mu(gp_batch* b, double* energy, double* mu);
int gp_batch_rms(gp_batch* b, double* rms4);
int gp_batch_raw_sums(gp_batch* b, double* raw);
int gp_batch_status(gp_batch* b, int64_t* steps_done, double* mu_est, int32_t* flags);
/* Residual of the stationary equation for the normalised state phi = psi / sqrt(N):
 * res[i] = || H[phi] phi - mu phi || with H[phi] = -1/2 lap_h + V + g |phi|^2 (lap_h the
 * 3-point Laplacian with zero ghosts, the operator whose energy gp_batch_energy_mu
 * evaluates), mu = <phi, H[phi] phi> (returned in mu, nullable), norms dx dy dz sum|.|^2.
 * Zero exactly at a discrete ground state; used to judge a starting state before
 * imaginary-time propagation.  Synchronises. */
int gp_batch_residual(gp_batch* b, double* res, double* mu);
/* Imaginary time until every instance meets gp_converge_imag's stopping rule on its mu
 * (observables every K steps, K <= 0 selects ceil(0.25/min dt)); converged instances are
 * masked off
 * while the rest continue.  Per-instance steps taken, final mu and converged flag. */
int gp_batch_converge_imag(gp_batch* b, double tol, int32_t check_every, int64_t max_steps,
                           int64_t* steps_taken, double* mu, int32_t* converged);
/* Mapping shared by all instances: {m_x, sw_x, m_y, sw_y, m_z}; the z threads per line
 * follow per instance.  gp_batch_autotune times the candidates on the batch (psi and
 * state restored) and keeps the fastest. */
/* Fused y and z sweeps (default off): for instances whose x-plane (ny x (nz+1) values)
 * fits in one block's LDS and whose splitting is Lie, one kernel loads each x-plane once,
 * solves its y and z lines in LDS and stores it: psi crosses HBM twice for y and z
 * together instead of four times.  Same arithmetic per point, different rounding order
 * from the separate sweeps (results agree to rounding, not bitwise).  gp_batch_autotune
 * times both and keeps the faster.  get: whether fusion is enabled and how many instances
 * use it; the z entry of gp_batch_get_timing covers the fused kernel. */
int gp_batch_set_yz_fusion(gp_batch* b, int32_t enable);
int gp_batch_get_yz_fusion(gp_batch* b, int32_t* enabled, int32_t* fused_instances);
int gp_batch_get_mapping(gp_batch* b, int32_t map[5]);
int gp_batch_set_mapping(gp_batch* b, const int32_t map[5]);
/* cache_path (nullable): a text file of earlier results keyed by the instances' grid sizes
 * (in order), their count, precision, splitting and step kind mode (0 imaginary, 1 real);
 * a hit applies the stored mapping and y+z fusion choice without timing, a miss appends
 * the new result. */
int gp_batch_autotune(gp_batch* b, int32_t mode, int32_t steps, const char* cache_path, int32_t map_out[5]);
int gp_batch_set_timing(gp_batch* b, int32_t enable);
int gp_batch_get_timing(gp_batch* b, double ms_mean[5], int64_t launches[5]);
const char* gp_batch_last_error(gp_batch* b);

const char* gp_strerror(int code);
const char* gp_last_error(gp_ctx* c);

/* ---------------------------------------------------------------------------------------
 * Test and measurement support (not part of the method).
 * ------------------------------------------------------------------------------------- */
/* Failure injection: every later device allocation the library makes for its own buffers
 * (contexts, batches, networks, autotuner copies) that asks for more than `bytes` fails
 * with GP_ERR_OOM (networks: GPNN_ERR_OOM) without reaching the runtime.  bytes < 0
 * removes the cap (the default).  Process-wide; not thread-safe against concurrent
 * init calls. */
int gp_set_alloc_cap(int64_t bytes);
/* The sin and cos the real-time potential step uses for its phase factor, on n device
 * arguments x_dev (float for GP_C64, double for GP_C128), written to sin_dev and cos_dev
 * (same type and length; caller-owned device buffers).  Stream-ordered, no sync. */
int gp_eval_sincos(int32_t precision, const void* x_dev, int64_t n, void* sin_dev, void* cos_dev, void* hip_stream);
/* Plain device-to-device copy of `bytes` (a multiple of 16; both pointers 16-byte
 * aligned) with the 16-byte raw buffer loads and stores the sweeps use for their rows: the
 * practical HBM ceiling the sweep bandwidths are compared with.  Stream-ordered. */
int gp_stream_copy(const void* src_dev, void* dst_dev, int64_t bytes, void* hip_stream);

/* ---------------------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gp_raw_sums without a context.
 * raw_dev (caller-owned device memory, 9 doubles) receives gp_raw_sums' raw[9] for the
 * grid p describes (nx, ny, nz, dx, dy, dz, nux, nuy, nuz, precision; g, dt and split are
 * not used) and psi_dev; the values are bitwise those of gp_raw_sums on a context of the
 * same grid.  Stream-ordered: no synchronisation, no host copy, no allocation, no
 * hipMemset; NaN/Inf/zero norms are returned as values, not as error codes.  The
 * reduction scratch is one file-scope device array per GPU (147,584 bytes: 2048 blocks x
 * 9 partial sums + the final sums), held until the process ends; its address is looked up
 * on the first call on each device.  Grids up to 2048 points per axis (larger:
 * GP_ERR_UNSUPPORTED).  All calls on one GPU share that array: calls that overlap in time
 * on one GPU (different streams, or host threads) race and may return each other's sums;
 * serialise them. */
int gp_raw_sums_noalloc(const gp_params* p, const void* psi_dev, double* raw_dev, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
