// Internal declarations of the learned warm-start network (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pdhot.h"

namespace pdhot {

// the library's one last-error slot (pd_last_error), shared with the solver
void set_last_error(const std::string& m);

constexpr int kMpnF = 16;                // node features
constexpr int kMpnH = 64;                // hidden width
constexpr int kMpnLayers = 2;            // message-passing layers
constexpr int kMpnKM = 2 * kMpnH + 6;    // message input width

struct MpnArgs {
  int nv, n_free, ne;
  double ell, L, h, s_out, kappa;
  double Xmin[3];
  const double* X;        // nv x 3 rest positions (caller order)
  const double* mass;     // nv lumped masses
  const uint8_t* pinned;  // nv
  const int* src;         // ne: source vertex of each directed edge (edges sorted by destination)
  const int* dst;         // ne
  const int* in_ptr;      // nv + 1: in-edges of each vertex
  const int* out_ptr;     // nv + 1: out-edge lists
  const int* out_eid;     // ne: edge ids grouped by source
  float* x0;              // nv x 16 features
  float* agg;             // nv x H aggregated messages (current layer)
  float* dagg;            // nv x H gradient of the aggregate
  const double* qt;       // nv x 3 current positions of the call
};

}  // namespace pdhot
