// Device state of one solve (internal to libpond.so).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/pond.h"
#include "pond_internal.h"

namespace pond {

constexpr size_t kStagingBytes = size_t(16) << 20;  // host<->device staging in the arena

struct Layout {
  int D = 2, QF = 16, QG = 9, NP = 25;
  bool fp64 = false;
  size_t cells = 0;
  size_t pop_bytes = 0, led_bytes = 0, red_bytes = 0, stage_bytes = 0, tab_bytes = 0;
  size_t stage_rows = 0, stage_cells = 0;
  int red_blocks = 256;
  bool ms = false;                 // per-cell f-lattices (D2Q9 or multiscale)
  size_t lat_bytes = 0, theta_bytes = 0;
  size_t wall_len = 0, wall_bytes = 0;  // wall ghost entries per side and layer; their bytes
  bool q25 = false;                // D2Q25 f-lattice: unfused kernels with HBM face data
  size_t q25_P = 0, q25_fr = 0, q25_nfx = 0, q25_nfy = 0, q25_bytes = 0;
  size_t total = 0;
};

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
int validate(const pond_config* c);
int upload_table(pond_state* s);
Layout layout_of(const pond_config* c);
// The launches of one step of s, from buffer `in` to buffer 1 - in, on st
// (no synchronisation, no allocation: safe under stream capture).
int step_launches(pond_state* s, int in, hipStream_t st);

}  // namespace pond

struct pond_state {
  pond_config cfg{};
  pond::Layout L;
  hipStream_t stream = nullptr;
  void* n[2] = {nullptr, nullptr};        // non-equilibrium population planes (ping-pong)
  long long* U[2] = {nullptr, nullptr};   // conserved-moment ledger planes (ping-pong)
  int* flag = nullptr;
  int* q16 = nullptr;                     // multiscale: per lattice plane, 0 if no cell is on D2Q16
  long long* inflow_dev = nullptr;        // [4][4] fixed-point moments of the inflow states
  pond::BatchEntry* tab = nullptr;        // one-entry step table (2D): the kernel serving uses
  long long* red = nullptr;
  double* stage = nullptr;
  unsigned char* lat[2] = {nullptr, nullptr};  // f-lattice per cell of n[0], n[1]
  double* theta = nullptr;                     // multiscale switch indicator
  long long* wU = nullptr;                     // wall ghosts: 4 ledger planes of 8 wall_len entries
  void* wN = nullptr;                          // wall ghosts: NP population planes
  // D2Q25 intermediates: phi-bar-plus and frames per cell; per x- and y-face
  // the face populations, frames and ledger fluxes
  void* qP = nullptr;
  double* qfr = nullptr;
  void* qfp[2] = {nullptr, nullptr};
  double* qff[2] = {nullptr, nullptr};
  long long* qps[2] = {nullptr, nullptr};
  int cur = 0;
  int64_t nstep = 0;
  bool initialized = false;
  double dt = 0.0, dx = 0.0, cv = 0.0, scale = 1.0;
  int scale_bits = 0;
  long long inflow_U[4][4] = {};
  pond::StepArgs args{};
};
