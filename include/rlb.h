/*
 * rlb.h -- C ABI of librlb, an MI355X (gfx950) implementation of the
 * relativistic lattice-Boltzmann (RLB) time step of Watson, "Turbulence in
 * Two-Dimensional Relativistic Hydrodynamic Systems with a Lattice Boltzmann
 * Model" (arXiv:2205.04658).
 *
 * The step (Ch. 3 "The Standard/Classical LBM" procedure with the
 * relativistic pieces of Ch. 3 "Relativistic Lattice Boltzmann" and
 * "Boltzmann to Lattice Boltzmann", the driving term of Ch. 4 eq. forceTerm
 * and the impurity bounce-back of Ch. 5 "Model and Methods") is:
 *   pull-stream with bilinear interpolation -> moments T^{mu nu}, J^mu ->
 *   Landau matching (eps, u^mu), n = u_mu J^mu -> truncated Juttner
 *   equilibrium -> Anderson-Witting relaxation + projected driving term
 *   (body force + random k-shell stirring) -> bounce-back at solid nodes.
 *
 * Conventions
 *   - Every pointer named d_* is device memory on the lattice's device;
 *     h_* is host memory.  Device pointers must be 256-byte aligned.
 *   - The library never allocates device memory: the caller passes one
 *     workspace of rlb_workspace_bytes() bytes to rlb_create and keeps it
 *     alive until rlb_destroy (which never frees it).
 *   - All device work is enqueued on the stream given at creation (a
 *     hipStream_t passed as void*, NULL = the null stream).  Calls that
 *     return data to the host (rlb_conserved, rlb_sync, rlb_get_status)
 *     synchronise that stream.
 *   - Fields are float32 arrays [ny][nx], x fastest.
 *   - Errors are status codes; nothing is thrown across the ABI.  Argument
 *     checks happen before any device work and nothing is written when they
 *     fail (RLB_EINVAL).  Device-side failures (a node with no timelike
 *     Landau frame, a non-finite population) set a sticky flag that the next
 *     synchronising call reports (RLB_ELANDAU / RLB_ENONFINITE).
 *     rlb_last_error() gives a thread-local message for the last failure.
 */
#ifndef RLB_H
#define RLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RLB_OK = 0,
  RLB_EINVAL = 1,       /* bad argument (shape, range, null, alignment)     */
  RLB_EDEVICE = 2,      /* HIP runtime error or no usable gfx950 device      */
  RLB_ENOMEM = 3,       /* workspace or buffer too small                     */
  RLB_ENONFINITE = 4,   /* a population became non-finite                    */
  RLB_ELANDAU = 5,      /* Landau matching found no timelike frame           */
  RLB_ESTATE = 6,       /* state buffer has the wrong header / shape         */
  RLB_EUNSUPPORTED = 7  /* valid request outside what the library implements */
} rlb_status;

/* rlb_params.flags */
#define RLB_WALLS_Y 0x1u  /* rows y = 0 and y = ny-1 are solid (channel)      */
#define RLB_FULL26  0x2u  /* store all 26 populations per family instead of  */
                          /* the 17 z-mirror-folded planes (see rlb_create)   */
#define RLB_OPEN_X  0x4u  /* open x borders: velocity inlet at x = 0,        */
                          /* pressure outlet at x = nx-1 (rlb_set_open_borders) */
#define RLB_PLANAR  0x8u  /* planar (2+1) momentum set: 12 in-plane unit     */
                          /* momenta, P = eps/2, c_s^2 = 1/2 (see rlb_create)  */

/* Lattice parameters.
 *   nx, ny   lattice nodes (one z node); 4 <= nx, ny; ny * (nx rounded up
 *            to 64) < 2^30, and one lattice row of state (nx rounded up to
 *            64, times 4 bytes per plane, 2 x 17, 2 x 26 or 2 x 12 planes)
 *            < 2^32 bytes: nx <= 31,580,608 folded, 20,648,832 with
 *            RLB_FULL26, 44,739,200 with RLB_PLANAR.
 *   tau      relaxation time in time steps, tau > 1/2 (Ch. 3: eta =
 *            tau_R (eps + P) / 5; the scheme's shear viscosity is
 *            (tau - 1/2)/5 + nu_interp).
 *   cfl      dt/dx in (0, 2]; populations move cfl * (v_x, v_y) per step,
 *            interpolated bilinearly between the two nodes that bracket the
 *            departure point along each axis (Ch. 3, linear interpolation;
 *            the paper's time steps give cfl up to 1.25, Ch. 4).  cfl > 1
 *            reaches two nodes and needs a periodic lattice (RLB_WALLS_Y and
 *            RLB_OPEN_X give RLB_EUNSUPPORTED); rlb_adjoint_run and
 *            rlb_column_current support cfl <= 1.
 *   flags    RLB_WALLS_Y | RLB_FULL26 | RLB_OPEN_X | RLB_PLANAR.  RLB_PLANAR
 *            replaces the paper's 3D momentum set (P = eps/3, c_s^2 = 1/3 on
 *            the one-z-node lattice) by 12 in-plane momenta at 30 degrees for
 *            particles confined to the plane (traceless T over t, x, y:
 *            P = eps/2, c_s^2 = 1/2; equilibrium
 *            w eps (1 - 3/2 |u|^2 + 3 u^0 u.v + 6 (u.v)^2), w n (u^0 + 2 u.v)).
 *            It has no driving term (rlb_set_body_force / rlb_set_stirring
 *            give RLB_EUNSUPPORTED), no open borders, no adjoint; it cannot
 *            be combined with RLB_FULL26.
 *   eps_ref, n_ref  shifted-storage references: populations are stored as
 *            F_i - w_i eps_ref and G_i - w_i n_ref in float32 (the float32
 *            rounding then acts on the deviation only).  Any finite value is
 *            valid; the mean of the initial fields is the best choice.
 */
typedef struct {
  int32_t nx, ny;
  double tau;
  double cfl;
  uint32_t flags;
  double eps_ref;
  double n_ref;
} rlb_params;

typedef struct rlb_lattice rlb_lattice;   /* opaque, host heap */

/* Field identifiers for rlb_read_fields (bit k of field_mask = field k).
 * Fields are those of the current state: the populations are streamed, then
 * moments and Landau matching are taken, with no collision (Ch. 3 LBM
 * procedure, step 3).  Solid nodes report 0. */
enum {
  RLB_FIELD_EPS = 0,     /* Landau energy density eps                      */
  RLB_FIELD_BETA_X = 1,  /* 3-velocity u^x / u^0                            */
  RLB_FIELD_BETA_Y = 2,
  RLB_FIELD_N = 3,       /* charge density n = u_mu J^mu                    */
  RLB_FIELD_T00 = 4, RLB_FIELD_T0X = 5, RLB_FIELD_T0Y = 6,
  RLB_FIELD_TXX = 7, RLB_FIELD_TXY = 8, RLB_FIELD_TYY = 9,
  RLB_FIELD_J0 = 10, RLB_FIELD_JX = 11, RLB_FIELD_JY = 12,
  RLB_FIELD_COUNT = 13
};

/* Bytes of workspace a lattice with these parameters needs. */
rlb_status rlb_workspace_bytes(const rlb_params* p, size_t* bytes);

/* Create a lattice on the current HIP device.  The state is undefined until
 * rlb_init_fields or rlb_load_state.  Populations are stored per family as
 * planes [i][ny][nx]: 17 planes by default -- the 26 directions of the
 * momentum set with each z-mirror pair (v_x, v_y, +v_z) / (v_x, v_y, -v_z)
 * folded into one plane holding the pair's sum, which is exact because the
 * lattice has one z node and no z force, so mirror populations stay equal --
 * or 26 planes with RLB_FULL26.  Errors: RLB_EINVAL (params, pointer,
 * alignment), RLB_ENOMEM (bytes too small), RLB_EDEVICE (not gfx950). */
rlb_status rlb_create(const rlb_params* p, void* d_workspace, size_t bytes,
                      void* hip_stream, rlb_lattice** out);

/* Release the handle.  Does not free the workspace.  NULL is a no-op. */
rlb_status rlb_destroy(rlb_lattice* lat);

/* F = F_eq(eps, u), G = G_eq(n, u) at every node, u^mu = gamma (1, beta)
 * (Ch. 3 LBM procedure step 1).  Resets the step counter to 0.
 * d_eps, d_bx, d_by, d_n: float32 [ny][nx]; eps > 0, bx^2 + by^2 < 1
 * (violations raise the device flag, reported as RLB_ELANDAU). */
rlb_status rlb_init_fields(rlb_lattice* lat, const float* d_eps,
                           const float* d_bx, const float* d_by,
                           const float* d_n);

/* Mark solid (bounce-back) nodes: every nonzero byte of d_mask [ny][nx]
 * becomes solid, in addition to walls and discs already set. */
rlb_status rlb_set_obstacles(rlb_lattice* lat, const uint8_t* d_mask);

/* Add discs (Ch. 5 impurities): node (x, y) is solid when dx^2 + dy^2 <= r^2
 * with dx, dy the periodic minimum-image distances to the centre.
 * h_cx_cy_r: host array of count triples (cx, cy, r), r > 0, finite. */
rlb_status rlb_add_disks(rlb_lattice* lat, int32_t count,
                         const double* h_cx_cy_r);

/* Remove every obstacle except the RLB_WALLS_Y rows. */
rlb_status rlb_clear_obstacles(rlb_lattice* lat);

/* Uniform body force (F^x, F^y) added to the stirring force in the driving
 * term of every fluid node (Ch. 4 eq. forceTerm with T_0 = 1). */
rlb_status rlb_set_body_force(rlb_lattice* lat, double fx, double fy);

/* Random k-shell stirring (Ch. 4 "Model and Methods"): every step, each
 * integer mode kmin <= |k| <= kmax on the half plane (ky > 0 or ky = 0,
 * kx > 0; ordered by ky then kx, index m) gets complex coefficients
 *   Fx_hat = amplitude (z0 + i z1),  Fy_hat = amplitude (z2 + i z3)
 * where z0..z3 are Box-Muller normals from the Philox4x64-10 block with
 * counter (m, step, 0, 0) and key (seed, 0); the conjugate fills -k and the
 * real-space force is F_c(x,y) = sum_shell F_c_hat e^{2 pi i (kx x/nx +
 * ky y/ny)}.  amplitude = 0 disables stirring.  0 <= kmin <= kmax <= 63,
 * kmax < min(nx, ny) / 2, at least one mode in the shell. */
rlb_status rlb_set_stirring(rlb_lattice* lat, double kmin, double kmax,
                            double amplitude, uint64_t seed);

/* Advance nsteps >= 0 steps (asynchronous on the stream). */
rlb_status rlb_step(rlb_lattice* lat, int64_t nsteps);

/* Replay the kernels of steps_per_graph consecutive steps (the stirring
 * draw and synthesis, the step, the open borders) as one HIP graph, for
 * lattices small enough that launch overhead shows.  0 (the default) turns
 * graphs off; otherwise steps_per_graph is even, 2..4096.  rlb_step uses
 * the graph only on a non-null stream, with kernel timing off and for at
 * least steps_per_graph steps (plus one if the current state is the second
 * copy); the rest runs kernel by kernel.  Results are bitwise those of
 * direct launches.  The graph is captured on first use and again whenever
 * a setting its kernels take by value changes (force, stirring, tau,
 * eta/s, open borders, obstacles, launch shape, stream).  EINVAL for an
 * odd or out-of-range count. */
rlb_status rlb_use_graph(rlb_lattice* lat, int32_t steps_per_graph);

/* Write the fields selected by field_mask (bits of RLB_FIELD_*) to d_out as
 * consecutive float32 planes [k][ny][nx] in increasing field order. */
rlb_status rlb_read_fields(rlb_lattice* lat, uint32_t field_mask, float* d_out);

/* Global totals over all nodes of the current (post-collision) state:
 * h_out = {E = sum F, P^x = sum F v_x, P^y = sum F v_y, Q = sum G}, summed
 * in float64 in a fixed order (deterministic).  Synchronises. */
rlb_status rlb_conserved(rlb_lattice* lat, double h_out[4]);

/* Energy and momentum the driving term (Ch. 4 eq. forceTerm, discretised as
 * in the appendix on the forcing term) adds in the lattice's next step:
 *   h_out = {sum F.T^{0k} / 6, sum F^x T^{00} / 6, sum F^y T^{00} / 6}
 * over fluid nodes, with T^{0 mu} from the current state streamed as the
 * step streams it and F the next step's force (body force + the stirring
 * field of step rlb_get_step).  On a periodic lattice without obstacles the
 * totals of rlb_conserved change by exactly these amounts over that step
 * (up to the float32 rounding of the state).  Summed in float64 in a fixed
 * order; overwrites the lattice's stirring planes (every step synthesises
 * its own).  RLB_EUNSUPPORTED for the planar set, RLB_EINVAL for a batch
 * member.  Synchronises. */
rlb_status rlb_force_injection(rlb_lattice* lat, double h_out[3]);

/* Wait for queued work; report sticky device failures. */
rlb_status rlb_sync(rlb_lattice* lat);

/* Number of steps taken since rlb_init_fields / rlb_load_state. */
rlb_status rlb_get_step(const rlb_lattice* lat, int64_t* step);

/* Bytes of a saved state (header + raw float32 planes). */
rlb_status rlb_state_bytes(const rlb_lattice* lat, size_t* bytes);

/* Copy the state (raw shifted float32 planes, step counter, parameters) to
 * d_buf / restore it.  A save followed by a load and N steps is bitwise
 * identical to N steps.  Load checks the header (RLB_ESTATE on mismatch). */
rlb_status rlb_save_state(rlb_lattice* lat, void* d_buf, size_t bytes);
rlb_status rlb_load_state(rlb_lattice* lat, const void* d_buf, size_t bytes);

/* Layout of the populations in saved states (and on the device): `planes`
 * per family (17 or 26; F planes 0..planes-1 first, then G), stored as node
 * bricks.  row_pitch = nx rounded up to 64 (columns nx.. are unused);
 * row_stride = 2 * planes * row_pitch.  Plane k of node (x, y) is the
 * float32 at element
 *   y * row_stride + (x / 64) * (2 * planes * 64) + k * 64 + x % 64
 * after header_bytes: each run of 64 columns of a row keeps its 2 * planes
 * planes together, 256 bytes per plane. */
rlb_status rlb_layout(const rlb_lattice* lat, int32_t* planes, int32_t* row_pitch,
                      int64_t* row_stride, size_t* header_bytes);

/* Open x borders of a lattice created with RLB_OPEN_X (Ch. 5, "Model and
 * Methods": a fixed velocity enters along the inflow border, the lateral
 * borders are periodic).  After every step:
 *   - velocity inlet, column x = 0: equilibrium at 3-velocity (bx, by) and
 *     charge density n_in, with the energy density of column 1;
 *   - pressure outlet, column x = nx-1: equilibrium at energy density
 *     eps_out (pressure eps_out / 3), with the velocity and charge density
 *     of column nx-2;
 * the adjacent columns' eps, u, n from Landau matching of their stored
 * moments (the step kernel sets the borders itself; for nx % 64 == 1 a
 * kernel of their own follows it).  Streaming stays periodic (the wrapped
 * values only reach the border columns, which are overwritten), so fields
 * read at x = 0 and x = nx-1 mix the two borders.  Defaults at creation: beta = 0,
 * n_in = n_ref, eps_out = eps_ref.  RLB_EINVAL without RLB_OPEN_X, for
 * |beta| >= 1, non-finite n_in or eps_out <= 0, and on a batch member
 * (members share rlb_batch_set_open_borders).  rlb_adjoint_run does not
 * support open borders (RLB_EUNSUPPORTED). */
rlb_status rlb_set_open_borders(rlb_lattice* lat, double bx, double by, double n_in,
                                double eps_out);

/* Current density at column x (Ch. 5: j recorded at the outflow border and
 * along the channel): d_out[0] = (1/ny) sum_y J^x(x, y) of the current step
 * (streamed populations, as rlb_read_fields; solid nodes count as zero),
 * float64, written asynchronously on the lattice stream.  Collect a time
 * series by passing d_out + t at successive steps. */
rlb_status rlb_column_current(rlb_lattice* lat, int32_t x, double* d_out);

/* Bytes of the rlb_record_current workspace that holds `chunk` steps
 * (1 <= chunk <= 65536): chunk * ny float64, rounded up to 256. */
rlb_status rlb_record_workspace_bytes(const rlb_lattice* lat, int32_t chunk, size_t* bytes);

/* nsteps steps that also record the current density at column x: d_series[t]
 * = j of the state before step t+1, t = 0 .. nsteps-1.  In open channels
 * (RLB_OPEN_X, nx % 64 != 1) and with RLB_FULL26 the step kernel writes
 * each row's J^x while it streams and one workgroup per chunk of steps
 * averages the rows in a fixed order: the value rlb_column_current gives
 * for that state up to float32 rounding.  Otherwise each step is preceded
 * by rlb_column_current (bitwise its values).  d_work: a 256-byte aligned
 * device workspace of `bytes` (rlb_record_workspace_bytes); it holds
 * bytes / (8 ny) steps at a time (RLB_ENOMEM below one).  Steps launch
 * kernel by kernel, never as graphs.  Errors as rlb_step and
 * rlb_column_current; nothing is checked past them when nsteps == 0. */
rlb_status rlb_record_current(rlb_lattice* lat, int64_t nsteps, int32_t x, double* d_series,
                              void* d_work, size_t bytes);

/* rlb_record_current without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid allocation): the per-row currents go to a fixed device scratch of
 * 4 MiB inside the library (one per device, held until the process ends),
 * so a chunk holds min(65536, 4 MiB / (8 ny)) steps.  Same steps, kernels
 * and results as rlb_record_current (bitwise).  It calls no allocating
 * routine.  RLB_ENOMEM when one step's rows do not fit (ny > 524288); other
 * errors as rlb_record_current.  Every call on a device shares that
 * device's scratch: calls that overlap on one device (two streams, two
 * threads) race and must be serialised by the caller. */
rlb_status rlb_record_current_noalloc(rlb_lattice* lat, int64_t nsteps, int32_t x,
                                      double* d_series);

/* One-sided power spectrum of the fluctuations of a float64 device series
 * s[0..n), 2 <= n <= 2^26: d_out[k] = |sum_t (s_t - mean) e^{-2 pi i k t/n}|^2
 * / n^2 for k = 0 .. n/2 (n/2 + 1 doubles; a plain sum, angles reduced
 * exactly), on hip_stream.  j(omega) from a j(t) series, j(k_x) from a j(x)
 * line.  d_out must not overlap d_series. */
rlb_status rlb_power_spectrum(const double* d_series, int64_t n, double* d_out, void* hip_stream);

/* Spectral analysis of the current velocity field (Ch. 2 "Turbulence":
 * E(k) = dE/dk from 1/2 |v~(k)|^2 over integer shells; Ch. 4 "Model and
 * Methods": velocities filtered to remove the driven range).  nx and ny
 * must be powers of two in [4, 4096] (RLB_EUNSUPPORTED otherwise).
 * rlb_energy_spectrum reads beta (as rlb_read_fields), transforms it in
 * float64 and writes, on the lattice stream:
 *   d_out[s] = E(s) = 1/2 sum_{s-1/2 <= |k| < s+1/2} |beta~(k)|^2 / (nx ny)^2,
 *              s = 0 .. kmax (numpy.fft conventions, integer wave numbers);
 *   d_out[kmax+1] = rms |beta_f|, d_out[kmax+2] = mean |beta_f|, beta_f the
 *              velocity keeping only the modes with |k| < k_cut;
 *   d_out[kmax+3] = enstrophy Z = sum over nodes of omega^2, omega =
 *              d_x beta_y - d_y beta_x by periodic central differences
 *              (Ch. 2 "Turbulence"; solid nodes read as beta = 0);
 * (d_out holds kmax + 4 doubles)
 * and, if d_acc is not null, adds E(s) to d_acc[s] and E(s)^2 to
 * d_acc[kmax+1+s] (running sums for time averages).  d_work: a 256-byte
 * aligned device buffer of rlb_spectrum_workspace_bytes.  Deterministic. */
rlb_status rlb_spectrum_workspace_bytes(const rlb_lattice* lat, int32_t kmax, size_t* bytes);
rlb_status rlb_energy_spectrum(rlb_lattice* lat, int32_t kmax, double k_cut, double* d_out,
                               double* d_acc, void* d_work, size_t bytes);

/* Host helpers of the analysis (no device work).  rlb_spectrum_average: mean
 * and standard error sqrt(sum (E - mean)^2 / (M (M-1))) per shell from the
 * running sums of M = count samples taken a decorrelation stride apart
 * (h_acc as d_acc above, copied to the host).  rlb_power_law_fit:
 * least-squares log y = intercept + slope log k over n > 1 points (k, y > 0),
 * e.g. the inertial range of E(k) against the k^-5/3 law. */
rlb_status rlb_spectrum_average(const double* h_acc, int32_t kmax, int64_t count, double* h_mean,
                                double* h_err);
rlb_status rlb_power_law_fit(const double* h_k, const double* h_y, int32_t n, double* h_slope,
                             double* h_intercept);

/* Stirring coefficients of a given step without advancing anything:
 * d_out[4m .. 4m+3] = (Re Fx_hat, Im Fx_hat, Re Fy_hat, Im Fy_hat) of mode
 * m, float64.  *count receives the number of half-shell modes. */
rlb_status rlb_stirring_coefficients(rlb_lattice* lat, int64_t step,
                                     double* d_out, int32_t* count);

/* The real-space stirring field of a given step, float32 [2][ny][nx]
 * (F^x then F^y), evaluated exactly as the step evaluates it. */
rlb_status rlb_stirring_field(rlb_lattice* lat, int64_t step, float* d_out);

/* Raw Philox4x64-10 blocks: d_out[4m + j] = word j of the block with
 * counter (m, c1, 0, 0) and key (k0, k1), m < count.  For testing the
 * generator bit for bit. */
rlb_status rlb_philox(uint64_t k0, uint64_t k1, uint64_t c1, int64_t count,
                      uint64_t* d_out, void* hip_stream);

/* Per-launch timing of the main step kernel with HIP events on the lattice
 * stream.  rlb_timing(lat, k), k >= 1, starts recording the step kernel of
 * every k-th step launched kernel by kernel (k = 1: every step; events
 * around a launch keep the next kernel from starting early, so sampling
 * disturbs the timed run less) and clears the totals; rlb_timing(lat, 0)
 * stops.  rlb_timing_read synchronises and returns the summed kernel time
 * in ms and the number of timed launches.  RLB_EINVAL for k < 0. */
rlb_status rlb_timing(rlb_lattice* lat, int32_t enable);
rlb_status rlb_timing_read(rlb_lattice* lat, double* total_ms, int64_t* launches);

/* Launch shape of the step kernel: tiles of 64 x tile_rows nodes (one
 * wavefront per row; tile_rows in {1, 2, 4, 8} for the folded layout, 2 or 4
 * for RLB_FULL26 (its plain step; its other kernels keep 4), 4 for
 * RLB_PLANAR, else RLB_EUNSUPPORTED); the grid: grid_per_cu = 0 launches one workgroup per
 * tile, k > 0 launches about k resident workgroups of 4 wavefronts per CU
 * that walk the tile list; and the tile order: a lattice's tiles are
 * visited in vertical strips `strip` tiles wide (1..65536; the last strip
 * may be narrower), row by row inside a strip, the eight XCDs each taking
 * a contiguous share of that order.  Results do not depend on the shape
 * (bitwise). */
rlb_status rlb_set_launch_shape(rlb_lattice* lat, int32_t tile_rows, int32_t grid_per_cu,
                                int32_t strip);
rlb_status rlb_get_launch_shape(const rlb_lattice* lat, int32_t* tile_rows, int32_t* grid_per_cu,
                                int32_t* strip);

/* Autotuner: time `trials` step-kernel launches for every candidate shape
 * (the tile_rows the layout accepts x grid_per_cu in {0, 4} x strip in
 * {4, 8, 16, 32}) on the
 * current state -- each launch reads the current copy and overwrites the
 * other, so the state does not advance -- and keep the fastest.  If h_ms
 * is not null, up to max_results rows (tile_rows, grid_per_cu, strip, ms
 * per launch) of 4 doubles are written.  Synchronises. */
rlb_status rlb_autotune(rlb_lattice* lat, int32_t trials, double* h_ms, int32_t max_results);

/* ------------------------------------------------------------------------
 * Batched lattices: many lattices of uneven sizes that share tau, cfl,
 * flags and references advance together, one launch per step over the
 * concatenated tile lists of all members (a persistent or one-workgroup-
 * per-tile grid), replayed from a captured hipGraph.  Each member evolves
 * bitwise as the same lattice stepped alone.
 * ------------------------------------------------------------------------ */
typedef struct rlb_batch rlb_batch;   /* opaque, host heap */

/* Workspace bytes for `count` members of sizes h_nx[b] x h_ny[b] (host
 * arrays); p supplies tau, cfl, flags, eps_ref, n_ref (p->nx, p->ny are
 * ignored). */
rlb_status rlb_batch_workspace_bytes(const rlb_params* p, int32_t count,
                                     const int32_t* h_nx, const int32_t* h_ny,
                                     size_t* bytes);

/* Create the batch and its members inside d_workspace.  Graph replay needs a
 * non-null stream; with the null stream every step is a direct launch. */
rlb_status rlb_batch_create(const rlb_params* p, int32_t count,
                            const int32_t* h_nx, const int32_t* h_ny,
                            void* d_workspace, size_t bytes, void* hip_stream,
                            rlb_batch** out);
rlb_status rlb_batch_destroy(rlb_batch* batch);

/* Handle of member b for every single-lattice call except stepping and
 * the settings the batch holds for all members (rlb_init_fields,
 * rlb_add_disks, rlb_set_obstacles, rlb_read_fields, rlb_conserved,
 * rlb_column_current, rlb_save_state, ...).  On a member, rlb_step,
 * rlb_record_current, rlb_set_body_force, rlb_set_stirring,
 * rlb_set_relaxation_time/_eta_s, rlb_set_open_borders,
 * rlb_set_launch_shape, rlb_autotune, rlb_use_graph and rlb_timing return
 * RLB_EINVAL.  The handle is owned by the batch. */
rlb_status rlb_batch_member(rlb_batch* batch, int32_t b, rlb_lattice** out);

/* Uniform body force of every member (Ch. 4 eq. forceTerm). */
rlb_status rlb_batch_set_body_force(rlb_batch* batch, double fx, double fy);

/* Open x borders of every member of a batch created with RLB_OPEN_X (as
 * rlb_set_open_borders; e.g. one Part II channel per impurity placement).
 * Such batches need nx % 64 != 1 for every member (RLB_EUNSUPPORTED at
 * creation): the step kernel sets the borders itself.  Errors as
 * rlb_set_open_borders; RLB_EINVAL without RLB_OPEN_X. */
rlb_status rlb_batch_set_open_borders(rlb_batch* batch, double bx, double by, double n_in,
                                      double eps_out);

/* Advance every member nsteps steps.  All members must be at the same
 * ping-pong phase (they are unless a member was re-initialised alone):
 * otherwise RLB_ESTATE.  Members may be advanced group by group (see
 * rlb_batch_use_graph), so after RLB_EDEVICE from a launch the members'
 * states and step counts are undefined; re-initialise them. */
rlb_status rlb_batch_step(rlb_batch* batch, int64_t nsteps);

/* Bytes of the rlb_batch_record_current workspace that holds `chunk` steps
 * (1 <= chunk <= 32768): chunk * (sum of the members' ny) float64,
 * rounded up to 256. */
rlb_status rlb_batch_record_workspace_bytes(const rlb_batch* batch, int32_t chunk, size_t* bytes);

/* nsteps batched steps that also record every member's current density
 * (Ch. 5: j(t) of each impurity placement): d_series[b * stride + t] = j
 * of member b's state before step t+1 at column x, t = 0 .. nsteps-1,
 * bitwise the series rlb_record_current gives for an open-channel member
 * stepped alone, and otherwise rlb_column_current before each step.  x >= 0 names the same column in every member; x < 0 counts
 * from each member's last column (-2: the column before the outlet,
 * x + nx_b).  Open-channel batches (RLB_OPEN_X) record in the step kernel
 * (one launch per step, plus one averaging launch per chunk of steps);
 * otherwise a column launch (one workgroup per member) precedes each
 * step.  Steps launch kernel by kernel, never as graphs.
 * d_work: a 256-byte aligned device workspace of `bytes`
 * (rlb_batch_record_workspace_bytes), holding up to 32768 steps at a time
 * (RLB_ENOMEM below one).  RLB_EINVAL for a column outside a member,
 * stride < nsteps, or a null or misaligned d_series (8 bytes) or d_work;
 * RLB_EUNSUPPORTED for cfl > 1; RLB_ESTATE as rlb_batch_step.  Nothing is
 * checked past the column when nsteps == 0. */
rlb_status rlb_batch_record_current(rlb_batch* batch, int64_t nsteps, int32_t x,
                                    double* d_series, int64_t stride, void* d_work, size_t bytes);

/* Wait for queued work; report device failures of batched steps. */
rlb_status rlb_batch_sync(rlb_batch* batch);

/* Members, total nodes, planes per family and steps taken. */
rlb_status rlb_batch_info(const rlb_batch* batch, int32_t* count, int64_t* cells,
                          int32_t* planes, int64_t* step);

/* Launch shape (as rlb_set_launch_shape, except that a batch of the full
 * set keeps tile_rows 4) and autotuner (as rlb_autotune) of the batched
 * step; graph replay of steps_per_graph (even, 0 = off, default 64) steps
 * per launch.  Members whose state together exceeds 224 MiB are stepped in
 * consecutive groups of at most that size, each group through all the
 * steps of a graph (or of one rlb_batch_step call's direct launches)
 * before the next, so that a group's state stays in the last-level cache;
 * the first step of each group reads it from HBM, so longer graphs pay
 * that read less often. */
rlb_status rlb_batch_set_launch_shape(rlb_batch* batch, int32_t tile_rows, int32_t grid_per_cu,
                                      int32_t strip);
rlb_status rlb_batch_get_launch_shape(const rlb_batch* batch, int32_t* tile_rows,
                                      int32_t* grid_per_cu, int32_t* strip);
rlb_status rlb_batch_autotune(rlb_batch* batch, int32_t trials, double* h_ms, int32_t max_results);
rlb_status rlb_batch_use_graph(rlb_batch* batch, int32_t steps_per_graph);

/* Wall time of rlb_batch_step calls between HIP events on the batch stream
 * (each call synchronises while timing is on). */
rlb_status rlb_batch_timing(rlb_batch* batch, int32_t enable);
rlb_status rlb_batch_timing_read(rlb_batch* batch, double* total_ms, int64_t* steps);

/* ------------------------------------------------------------------------
 * Adjoint: gradients of a time-averaged objective of a driven run with
 * respect to theta = (F_b, tau, A_1..A_M), by the discrete adjoint of the
 * step with checkpoint-and-recompute.  The driving force is
 *   F(x) = F_b x_hat + sum_m A_m e_m cos(2 pi (kx x / nx + ky y / ny) + phase_m)
 * (a fixed stirring basis; Ch. 4 eq. forceTerm).  Objectives, averaged over
 * steps N/2 + 1 .. N and over fluid nodes, from the fields of each step
 * (post-stream moments): RLB_OBJ_CURRENT the charge current J^x;
 * RLB_OBJ_DISSIPATION pi^{kl} pi^{kl} with pi = T^{kl} - T_eq^{kl}(eps, u)
 * (k, l over x, y, z), a viscous-dissipation proxy.
 * ------------------------------------------------------------------------ */
enum { RLB_OBJ_CURRENT = 0, RLB_OBJ_DISSIPATION = 1 };

typedef struct {
  int64_t nsteps;          /* N: even, >= 2                                   */
  int32_t checkpoint;      /* K: states kept every K steps, >= 1               */
  int32_t objective;       /* RLB_OBJ_*                                        */
  int32_t nmodes;          /* M basis modes, 0..64                             */
  const double* h_modes;   /* host [M][5]: kx, ky (integers), ex, ey, phase    */
  const double* h_amps;    /* host [M]: amplitudes A_m                          */
  double body_force;       /* F_b                                              */
  int32_t resident;        /* segments of K states kept resident by the
                              forward pass (the last ones), which the
                              backward pass then does not recompute; 0 or 1
                              means the minimum (2, or 1 for a single
                              segment); values above ceil(N/K) keep all.
                              The gradient does not depend on it.          */
} rlb_adjoint_cfg;

/* Set the relaxation time (tau > 1/2) of an existing lattice; this also
 * returns a lattice set by rlb_set_relaxation_eta_s to a constant tau.
 * RLB_EINVAL for batch members (they share the batch's tau). */
rlb_status rlb_set_relaxation_time(rlb_lattice* lat, double tau);

/* Per-node relaxation time from a fixed shear viscosity to entropy ratio
 * (Ch. 3, "Relativistic Lattice Boltzmann": tau_R = 5 (eta/s) / T, and
 * "Boltzmann to Lattice Boltzmann": eps = 3 T^4 / pi^2 in natural units):
 * each fluid node relaxes with tau(x) = 5 (eta/s) / (T(x) dt), steps,
 * T(x) = (pi^2 eps(x) / 3)^(1/4) from its Landau energy density, dt the
 * time step in the units of T^-1.  Stability needs tau(x) > 1/2, i.e.
 * eps(x) < (3 / pi^2) (10 (eta/s) / dt)^4; the library does not clamp.
 * Applies to rlb_step of single lattices; rlb_adjoint_run rejects it
 * (RLB_EUNSUPPORTED).  RLB_EINVAL for non-positive or non-finite arguments
 * and for batch members. */
rlb_status rlb_set_relaxation_eta_s(rlb_lattice* lat, double eta_over_s, double dt);

/* Bytes of the adjoint workspace: R resident segments of K states each
 * (R = cfg->resident clamped to [2, ceil(N/K)], or 1 for a single segment:
 * a segment that is not resident is recomputed from its checkpoint into a
 * free segment buffer while the adjoint sweeps the one after it) +
 * ceil(N/K) - R checkpoints + 2 adjoint states + float64 per-node
 * accumulators + (K + 2) R launch descriptors (64 bytes each).  With all
 * segments resident nothing is recomputed: one
 * state is 2 Q row_stride ny floats (17.8 MB at 512 x 256 with Q = 17). */
rlb_status rlb_adjoint_workspace_bytes(const rlb_lattice* lat, const rlb_adjoint_cfg* cfg,
                                       size_t* bytes);

/* Run N steps from the lattice's current state with the force above
 * (overwriting the lattice's stirring-force planes), write J to
 * *h_objective and, if h_grad is not null, the gradient (2 + M doubles:
 * dJ/dF_b, dJ/dtau, dJ/dA_m) computed by the adjoint.  The lattice is left
 * at step N.  Synchronises.  d_ws: 256-byte aligned device memory.  The
 * backward pass also uses a second stream of the library's (created on
 * first use, default priority, ordered after the lattice stream's prior
 * work and joined back into it before return). */
rlb_status rlb_adjoint_run(rlb_lattice* lat, const rlb_adjoint_cfg* cfg, void* d_ws,
                           size_t bytes, double* h_objective, double* h_grad);

/* The two linear maps one reverse step of rlb_adjoint_run applies, on caller
 * buffers, for checking them by the dot-product identity
 * <A^T mu, v> = <mu, A v> against a tangent of the forward step:
 *   RLB_ADJ_PULL_T  d_out = P^T d_mu, P the bilinear pull of the streaming
 *                   step (Ch. 3, linear interpolation): the same weights
 *                   taken at x + delta;
 *   RLB_ADJ_STEP    d_out = (dC/dF~)^T P^T d_mu with F~ = P d_state: the
 *                   adjoint kernel of one step (C the local update: moments,
 *                   Landau matching, equilibrium, relaxation, the driving
 *                   term of Ch. 4 eq. forceTerm with the lattice's body
 *                   force and no stirring, bounce-back at the lattice's
 *                   obstacles) with no objective term; d_acc (float64,
 *                   3 nx ny) receives per node the adjoints with respect to
 *                   the force at the node and 1/tau: (d/dF^x, d/dF^y) pairs
 *                   at d_acc[2 (y nx + x)], d/d(1/tau) at
 *                   d_acc[2 nx ny + y nx + x].
 * d_state, d_mu, d_out: population copies in the lattice's layout
 * (rlb_layout: 2 * planes planes of node bricks, row_stride * ny floats, no
 * header; shifted storage for d_state).  All pointers 256-byte aligned;
 * d_out must not alias an input.  RLB_ADJ_STEP overwrites the lattice's
 * stirring-force planes (as rlb_adjoint_run does).  Asynchronous on the
 * lattice stream.  Errors as rlb_adjoint_run for the lattice (constant tau,
 * periodic x, cfl <= 1, 3D set); RLB_EINVAL for an unknown op or a bad
 * pointer. */
enum { RLB_ADJ_STEP = 0, RLB_ADJ_PULL_T = 1 };
rlb_status rlb_adjoint_apply(rlb_lattice* lat, int32_t op, const float* d_state,
                             const float* d_mu, float* d_out, double* d_acc);

/* A plain device copy of `bytes` (multiple of 16) for bandwidth calibration. */
rlb_status rlb_copy_probe(const void* d_src, void* d_dst, size_t bytes,
                          void* hip_stream);

/* Human-readable message of the last failure on this thread. */
const char* rlb_last_error(void);

/* Library version string. */
const char* rlb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RLB_H */
