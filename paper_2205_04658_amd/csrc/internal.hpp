// Host-side internals of librlb: the lattice handle, kernel argument blocks
// and the launchers each translation unit exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rlb.h"

namespace rlb {

constexpr int kMaxQ = 26;
constexpr int kMaxK = 63;            // largest stirring |k|
constexpr int kMaxModes = 8192;      // half-shell modes for |k| <= kMaxK
constexpr int kTileX = 64;           // one wavefront spans 64 x-nodes
constexpr int kTileY = 4;            // four wavefronts per workgroup
constexpr int kBlock = kTileX * kTileY;
constexpr int kRedBlocks = 1024;     // partial sums of the totals kernel
constexpr size_t kAlign = 256;
// Size of the fixed device scratch of rlb_record_current_noalloc (noalloc.hip).
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;

// Device error bits (sticky word in the workspace).
enum : uint32_t { ERR_LANDAU = 1u, ERR_NONFINITE = 2u };

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Step-kernel modes: a step; the field read-out; a step that also sets the
// open x borders of the new state (velocity inlet, pressure outlet); a step
// that also adds the adjoint objective's density of the state it streams
// to per-wavefront slots (StepShared::obj).
enum StepMode : int { MODE_STEP = 0, MODE_FIELDS = 1, MODE_OPEN = 2, MODE_OBJ = 3 };
// Force modes: none, uniform body force, body force + force planes (the
// k-shell stirring, or the adjoint's static basis).
enum ForceMode : int { FORCE_NONE = 0, FORCE_BODY = 1, FORCE_STIR = 2 };

// Parameters shared by every lattice of one step launch.
struct StepShared {
  float tap[kMaxQ][4];    // bilinear weights (w00, w10, w01, w11) per plane
  uint8_t shift[kMaxQ][2];  // whole-cell tap shifts (x, y) per plane (cfl > 1)
  float inv_tau;           // constant 1/tau (tau_k == 0)
  double tau_k;            // > 0: per-node 1/tau = tau_k * eps^(1/4) (eta/s relaxation)
  double eps_ref, n_ref;
  float fx, fy;           // uniform body force
  double o_bx, o_by, o_n; // open borders: inlet 3-velocity and charge density
  double o_eps;           // open borders: outlet energy density
  uint32_t* err;          // sticky device error word
  uint32_t field_mask;    // MODE_FIELDS selection
  double* rec;            // non-null (records_current): J^x of the streamed
  int32_t rec_x;          //   populations at column rec_x (x < 0: nx + rec_x) written
                          //   to rec[rec_row + y] (row y of the lattice)
  double* obj;            // MODE_OBJ: slot y * tiles_x + x / 64 += the wavefront's
  int32_t obj_kind;       //   sum of J^x (kind 0) or pi:pi (kind 1) over fluid nodes
};

// One lattice as the tile kernel sees it (device memory, read with scalar
// loads).  state[c] are the two ping-pong state copies (node bricks, see
// brick.hpp); the two stirring-force planes are plain [ny][row] arrays
// `pitch` elements apart.
struct LatDesc {
  const float* state[2];
  const uint8_t* mask;    // [ny][nx] solid flags (used when MASK)
  const float* force;     // two stirring-force planes (FORCE_STIR)
  int64_t pitch;          // force-plane pitch in elements
  int32_t nx, ny;
  int32_t tiles_x;        // tiles per row of tiles
  int32_t tile_begin;     // first global tile index of this lattice
  int32_t row;            // row pitch in elements (nx rounded up to 64)
  int32_t rec_row;        // first row of this lattice among recorded rows
                          // (0 alone; a batch's members follow each other)
};

// A step launch whose two state copies take at most this many bytes fits
// the 256 MB last-level cache: its kernels store with plain stores (the
// next step reads the state from that cache), larger launches with
// non-temporal ones (measured crossover between 214 MB, plain faster, and
// 285 MB, non-temporal faster).  Batches step members in groups of this
// size inside a captured graph.
constexpr double kCachedStateBytes = 224.0 * 1024 * 1024;

struct TileArgs {
  StepShared sh;
  const LatDesc* lats;
  const int32_t* tile_lat;  // lattice of each tile; null for a single lattice
  int32_t parity;           // read state[parity], write state[parity ^ 1]
  int32_t tile_first;       // tile range of this launch
  int32_t ntiles;
  int32_t tiles_per_xcd;    // ceil(ntiles / 8)
  int32_t strip;            // tile-order strip width in tiles (>= 1)
  float* fields;            // MODE_FIELDS output [k][ny][nx]
};

// Launch shape: tile height in rows (one wavefront per row of 64 nodes) and
// the grid: 0 = one workgroup per tile, k > 0 = k resident workgroups per CU
// walking the tile list (persistent).
struct LaunchShape {
  int32_t tile_rows;
  int32_t grid_per_cu;
  int32_t strip;          // tiles are ordered in vertical strips this many tiles wide
};

struct StirArgs {
  const int4* modes;      // binned list (m, kx, ky, 0), grouped by |kx|
  const int32_t* bins;    // [K+2] offsets of |kx| = 0..K in `modes`
  double* coef;           // [nmodes][4] (Re Fx, Im Fx, Re Fy, Im Fy)
  // series coefficients (a_k, b_k) of F^x, F^y times `scale`, as float16
  // hi + lo pairs in matrix-operand order: 16-byte items
  // [k / 8][(k / 4) % 2][component][hi | lo][ny] of 8 halves
  // (a_k, b_k for 4 consecutive k), zero past K: consecutive rows are
  // consecutive items, so the synthesis's operand loads are contiguous
  uint4* table;
  const double2* phase;   // [ny] (cos, sin)(2 pi m / ny)
  // (cos, sin)(2 pi k x / nx) as float16 hi + lo pairs: 16-byte items
  // [k / 8][(k / 4) % 2][hi | lo][nx] of 8 halves, zero past K
  const uint4* twiddle;
  float scale, inv_scale; // power of two keeping the coefficients in float16's normal range
  float* force;           // [2][force_pitch] synthesised force planes, rows padded
  int64_t force_pitch;
  int32_t row;
  int64_t* dstep;         // device step counter (draw reads and advances it)
  int32_t nmodes, K, nx, ny;
  double amplitude;
  uint64_t seed, stream;
};

// Adjoint kernels (adjoint.hip).
struct AdjArgs {
  StepShared sh;
  const float* state;     // s_t (node bricks)
  const float* mu_in;     // mu_{t+1} (null: zero)
  float* mu_out;          // mu_t
  const uint8_t* mask;    // solid flags [ny][nx] or null
  const float* force;     // static stirring-basis planes [2][pitch], rows of `row`
  double2* acc_f;         // per-node sum of dJ/dF(x), dense [ny][nx]
  double* acc_itau;       // per-node sum of dJ/d(1/tau)
  int64_t pitch;
  int32_t nx, ny, row, tiles_x, ntiles;
  int32_t tiles_per_xcd;  // ceil(ntiles / 8): the grid is 8 * tiles_per_xcd
  int32_t strip;          // tile-order strip width in tiles (as TileArgs)
  float obj_c;            // weight of J_t (0 outside the averaging window)
  int32_t kind;           // 0 current, 1 dissipation
};

struct ObjArgs {
  StepShared sh;
  const float* state;
  const uint8_t* mask;
  double* acc;            // per-block running sums [grid]
  int64_t pitch;
  int32_t nx, ny, row, kind;   // kind 2 counts fluid nodes
};

// Open x borders (boundary.hip): velocity inlet at x = 0, pressure outlet
// at x = nx - 1.
struct OpenArgs {
  double bx, by, n_in;    // inlet 3-velocity and charge density
  double eps_out;         // outlet energy density
  double eps_ref, n_ref;  // storage references (filled at launch)
  uint32_t* err;
};

// Spectral analysis scratch (spectral.hip), carved from a caller workspace.
struct SpectralLayout {
  size_t z_off, fields_off, twx_off, twy_off, part_off, speed_off, total;
};

struct Workspace {
  size_t state_off[2], mask_off, coef_off, modes_off, bins_off, table_off,
      phase_off, force_off, twiddle_off, partial_off, desc_off, misc_off, total;
};

}  // namespace rlb

struct rlb_lattice {
  rlb_params p;
  rlb::LaunchShape shape;
  rlb::LatDesc desc;      // host copy of the descriptor uploaded to ws
  rlb::LatDesc* d_desc;
  int num_cu;
  struct rlb_batch* owner;  // set when the lattice is a batch member
  int device;
  hipStream_t stream;
  int Q;                  // planes per family (17 or 26)
  int32_t row;            // row pitch in elements (nx rounded up to 64)
  int64_t pitch;          // plane pitch in elements (ny * row rounded up)
  char* ws;
  size_t ws_bytes;
  rlb::Workspace lay;
  float* state[2];
  int cur;                // index of the current state
  uint8_t* mask;
  bool any_solid;
  double* coef;
  int4* modes;
  int32_t* bins;
  uint4* table;
  double2* phase;
  uint4* twiddle;
  float* force;
  double* partials;
  uint32_t* err;
  int64_t* dstep;
  double* result;
  // forcing
  double fx, fy;
  double tau_k;           // per-node relaxation from eta/s (0 = constant tau)
  rlb::OpenArgs open;     // open x borders (RLB_OPEN_X)
  bool stir;
  double kmin, kmax, amp;
  float stir_scale;       // power of two applied to the series coefficients
  uint64_t seed;
  int nmodes, K;
  // bilinear tap weights per plane
  float tap[rlb::kMaxQ][4];
  uint8_t shift[rlb::kMaxQ][2];   // whole-cell tap shifts (cfl > 1)
  int64_t step;
  // timing of the main step kernel (of every timing_every-th step)
  bool timing;
  int32_t timing_every;
  int64_t timed_launches;
  double timed_ms;
  hipEvent_t ev[16][2];   // ring of (start, end) pairs
  uint32_t ev_pending;
  // graph replay of graph_steps steps (0 = off); the graph captures its
  // kernels' arguments by value, so it is tied to the configuration key
  int graph_steps;
  bool graph_valid;
  hipGraph_t graph;
  hipGraphExec_t exec;
  double graph_key[24];
  // second stream and events of the adjoint's backward pass (created on
  // first use)
  hipStream_t aux;
  hipEvent_t aux_ev[5];
  // saved-state header staging
  alignas(64) unsigned char header[256];
};

namespace rlb {

// api.cpp: thread-local message returned by rlb_last_error
void set_error_message(const char* msg);
// api.cpp: validate and store open-border settings (no batch-member check)
rlb_status set_open(rlb_lattice* lat, double bx, double by, double n_in, double eps_out);

// step.hip
StepShared shared_of(const rlb_lattice* lat);
// sm: streaming mode (SM_GENERAL / SM_UNIT / SM_WIDE, see brick.hpp), from
// stream_mode(cfl).
int stream_mode(double cfl);
hipError_t launch_tiles(int Q, int sm, bool mask, int mode, int force_mode,
                        const TileArgs& a, LaunchShape shape, int num_cu,
                        hipStream_t s);
int tiles_of(int nx, int ny, int tile_rows);
// The tile height the step kernels of a launch use for a shape's tile_rows:
// any of 1, 2, 4, 8 for the folded set (field read-out: 4), 2 or 4 for the
// full set's step (MODE_STEP), 4 otherwise.  Tile counts (tiles_of) must be
// taken with this height.
int kernel_tile_rows(int Q, int mode, int tile_rows);
// Launch shapes the autotuners time: tile heights 1, 2, 4, 8 for the folded
// set, 2 and 4 for a single full-set lattice, 4 otherwise (batches of the
// full set included).
std::vector<LaunchShape> launch_candidates(int Q, bool batch);
hipError_t launch_step(const rlb_lattice* lat, int mode, int force_mode,
                       int parity, float* fields, uint32_t field_mask,
                       double* rec = nullptr, int rec_x = 0, double* obj = nullptr,
                       int obj_kind = 0);
// The mode of a step of this lattice: MODE_OPEN when the open borders can be
// set inside the step kernel (the outlet column and the one before it share
// a 64-node tile, i.e. nx % 64 != 1), else MODE_STEP.
int step_mode(const rlb_lattice* lat);
// Whether the step kernels of this lattice can record a column's current
// (open-channel kernels and the full set's kernels).
bool records_current(const rlb_lattice* lat);
SpectralLayout spectral_layout(int nx, int ny, int kmax);
hipError_t launch_spectrum(rlb_lattice* lat, int kmax, double kcut, double* out, double* acc,
                           char* ws);
hipError_t launch_open_borders(const rlb_lattice* lat, float* state);
hipError_t launch_column_current(const rlb_lattice* lat, int x, double* out);
hipError_t launch_batch_column_current(const StepShared& sh, int Q, const LatDesc* lats, int count,
                                       int parity, bool unit, bool mask, int x, int64_t stride,
                                       double* out, hipStream_t stream);
hipError_t launch_power_spectrum(const double* s, int64_t n, double* out, hipStream_t st);
// out[t] = (1/ny) sum_y rows[t * ny + y], t < count, fixed summation order.
hipError_t launch_row_means(const double* rows, int ny, int count, double* out, hipStream_t st);
// out[b * stride + t] = (1/ny_b) sum_y rows[t * total + rec_row_b + y] for the
// `members` lattices of lats, t < count (<= 32768), in the order of
// launch_row_means.
hipError_t launch_batch_row_means(const LatDesc* lats, int members, const double* rows, int64_t total,
                                  int count, double* out, int64_t stride, hipStream_t st);
hipError_t launch_init(const rlb_lattice* lat, const float* eps,
                       const float* bx, const float* by, const float* n,
                       float* dst);
hipError_t launch_disks(const rlb_lattice* lat, const double* d_discs,
                        int count);
hipError_t launch_mask_or(const rlb_lattice* lat, const uint8_t* d_mask);
hipError_t launch_walls(const rlb_lattice* lat);
hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t s);

// forcing.hip
// Every mode's coefficients at `step` into a.coef.
hipError_t launch_stir_draw(const StirArgs& a, int64_t step, hipStream_t s);
// Draw and row series of the step on the device counter (fixed_step < 0)
// or of fixed_step; the synthesis, advancing the counter when `advance`.
hipError_t launch_stir_table(const StirArgs& a, int64_t fixed_step, hipStream_t s);
hipError_t launch_stir_synth(const StirArgs& a, bool advance, hipStream_t s);
hipError_t launch_phase(const rlb_lattice* lat);
hipError_t launch_twiddle(uint4* tw, int K, int nx, hipStream_t s);
hipError_t launch_philox(uint64_t k0, uint64_t k1, uint64_t c1, int64_t count,
                         uint64_t* out, hipStream_t s);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);

// adjoint.hip
hipError_t launch_adjoint(int Q, bool unit, bool mask, const AdjArgs& a, hipStream_t s);
hipError_t launch_objective(int Q, bool unit, bool mask, const ObjArgs& a, int grid, hipStream_t s);
// out = P^T mu (the adjoint kernel's transposed pull alone)
hipError_t launch_transpose_pull(int Q, bool unit, const float* mu, float* out, int nx, int ny,
                                 int row, const StepShared& sh, hipStream_t s);
hipError_t launch_basis_force(const double* modes, const double* amps, int M, int nx, int ny,
                              int row, int64_t pitch, float* force, hipStream_t s);
hipError_t launch_grad_reduce(const double2* acc_f, const double* acc_itau, const double* modes,
                              int M, int nx, int ny, double tau, double* partial, int cols,
                              double* out, hipStream_t s);
hipError_t launch_sum_rows(const double* partial, int cols, int rows, double scale, double* out,
                           hipStream_t s);
hipError_t launch_zero_f64(double* p, size_t n, hipStream_t s);

// noalloc.hip: device address of the fixed scratch (kStaticScratchBytes) on
// `device`, looked up on first use with that device current.
hipError_t static_scratch(int device, double** ptr);

// reduce.hip
hipError_t launch_totals(const rlb_lattice* lat, const float* state,
                         double* result);
// Energy and momentum the next step's driving term adds (result[0..2]);
// the stirring planes must hold the next step's field when `planes`.
hipError_t launch_injection(const rlb_lattice* lat, bool planes, double* result);
hipError_t launch_copy(const void* src, void* dst, size_t bytes,
                       hipStream_t s);

}  // namespace rlb
