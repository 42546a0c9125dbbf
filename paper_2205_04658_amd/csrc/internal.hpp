// Host-side internals of librlb: the lattice handle, kernel argument blocks
// and the launchers each translation unit exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

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

// Device error bits (sticky word in the workspace).
enum : uint32_t { ERR_LANDAU = 1u, ERR_NONFINITE = 2u };

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// Step-kernel modes.
enum StepMode : int { MODE_STEP = 0, MODE_FIELDS = 1 };
// Force modes: none, uniform body force, body force + k-shell stirring.
enum ForceMode : int { FORCE_NONE = 0, FORCE_BODY = 1, FORCE_STIR = 2 };

struct StepArgs {
  const float* src;       // current planes [2Q][pitch] (F then G)
  float* dst;             // next planes (MODE_STEP)
  int64_t pitch;          // plane pitch in elements
  int32_t nx, ny;
  int32_t tiles_x, ntiles, tiles_per_xcd;
  const uint8_t* mask;    // [ny][nx] solid flags or null
  float tap[kMaxQ][4];    // bilinear weights (w00, w10, w01, w11) per plane
  float inv_tau;
  double eps_ref, n_ref;
  float fx, fy;           // uniform body force
  const float4* table;    // stirring series table [ny][kMaxK+1]
  int32_t K;              // stirring series order (largest |kx|)
  float theta_scale;      // 2 / nx (angle of column x is pi * x * theta_scale)
  uint32_t* err;
  float* fields;          // MODE_FIELDS output [k][ny][nx]
  uint32_t field_mask;
};

struct StirArgs {
  const int4* modes;      // binned list (m, kx, ky, 0), grouped by |kx|
  const int32_t* bins;    // [K+2] offsets of |kx| = 0..K in `modes`
  double* coef;           // [nmodes][4] (Re Fx, Im Fx, Re Fy, Im Fy)
  float4* table;          // [ny][kMaxK+1]
  int64_t* dstep;         // device step counter (draw reads and advances it)
  int32_t nmodes, K, nx, ny;
  double amplitude;
  uint64_t seed, stream;
};

struct Workspace {
  size_t state_off[2], mask_off, coef_off, modes_off, bins_off, table_off,
      partial_off, misc_off, total;
};

}  // namespace rlb

struct rlb_lattice {
  rlb_params p;
  int device;
  hipStream_t stream;
  int Q;                  // planes per family (17 or 26)
  int64_t pitch;
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
  float4* table;
  double* partials;
  uint32_t* err;
  int64_t* dstep;
  double* result;
  // forcing
  double fx, fy;
  bool stir;
  double kmin, kmax, amp;
  uint64_t seed;
  int nmodes, K;
  // bilinear tap weights per plane
  float tap[rlb::kMaxQ][4];
  int64_t step;
  // timing of the main step kernel
  bool timing;
  int64_t timed_launches;
  double timed_ms;
  hipEvent_t ev[16][2];   // ring of (start, end) pairs
  uint32_t ev_pending;
  // saved-state header staging
  alignas(64) unsigned char header[256];
};

namespace rlb {

// step.hip
hipError_t launch_step(const rlb_lattice* lat, int mode, int force_mode,
                       const float* src, float* dst, float* fields,
                       uint32_t field_mask);
hipError_t launch_init(const rlb_lattice* lat, const float* eps,
                       const float* bx, const float* by, const float* n,
                       float* dst);
hipError_t launch_disks(const rlb_lattice* lat, const double* d_discs,
                        int count);
hipError_t launch_mask_or(const rlb_lattice* lat, const uint8_t* d_mask);
hipError_t launch_walls(const rlb_lattice* lat);
hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t s);

// forcing.hip
hipError_t launch_stir_draw(const StirArgs& a, int64_t fixed_step,
                            hipStream_t s);
hipError_t launch_stir_table(const StirArgs& a, hipStream_t s);
hipError_t launch_stir_field(const rlb_lattice* lat, float* out);
hipError_t launch_philox(uint64_t k0, uint64_t k1, uint64_t c1, int64_t count,
                         uint64_t* out, hipStream_t s);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);

// reduce.hip
hipError_t launch_totals(const rlb_lattice* lat, const float* state,
                         double* result);
hipError_t launch_copy(const void* src, void* dst, size_t bytes,
                       hipStream_t s);

}  // namespace rlb
