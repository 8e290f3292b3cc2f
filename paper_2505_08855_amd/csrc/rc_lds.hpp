// LDS-tiled table reads (RC_VARIANT_LDS).
//
// During a solve a cell's cooling-table coordinates along N and B and its
// Coulomb coordinate along n_e stay fixed; only the temperature coordinates
// move.  A workgroup therefore knows, after setup, the box of table nodes its
// cells can touch: [N range] x (whole T_e axis) x [B range] of the cooling
// tables and [n_e range] x (whole T_e, T_i plane) of the Coulomb table.  When
// the cooling box fits the workgroup's LDS budget it is staged there (the
// solver's {brem, se} pair per node), then the Coulomb box if the remainder
// allows.  A staged box holds
// every node any of the workgroup's cells can read, so the choice between LDS
// and global memory is made once per workgroup, and the solver is instantiated
// once per choice (a per-read choice costs registers the Newton solve does not
// have).  The results equal the GLOBAL variant's.  Spatially coherent inputs
// (a patch of a disk) give small boxes; independent random cells give boxes as
// large as the tables, which are then read from global memory.
#pragma once

#include "rc_kernels.hpp"

namespace rc {

// Reads the staged cooling box from LDS, and the staged Coulomb box when
// COUL (else the Coulomb table from global memory).  The cooling box holds the
// solver's {brem, se} pair per node (8 bytes); single-node reads of the three
// separate cooling quantities (diagnostic outputs only) go to global memory.
template <class Base, bool COUL>
struct LdsTab {
  Base g;                 // global-memory accessor (the staging source)
  const float2* cool_s;   // staged cooling box [dN][c1][dB] (LDS)
  const float* coul_s;    // staged Coulomb box [dn][k1][k2] (LDS)
  int n0, b0, dB;         // cooling box origin along N and B, extent along B
  int m0;                 // Coulomb box origin along n_e
  __device__ float4 cool_at(int i0, int i1, int i2) const { return g.cool_at(i0, i1, i2); }
  __device__ float coul_at(int i0, int i1, int i2) const {
    if constexpr (COUL) return coul_s[((i0 - m0) * g.k1 + i1) * g.k2 + i2];
    else return g.coul_at(i0, i1, i2);
  }
  __device__ void cool8(int i0, int i1, int i2, float2 (&v)[8]) const {
    const float2* p = cool_s + ((i0 - n0) * g.c1 + i1) * dB + (i2 - b0);
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[((k >> 2) * g.c1 + ((k >> 1) & 1)) * dB + (k & 1)];
  }
  __device__ void coul8(int i0, int i1, int i2, float (&v)[8]) const { corners8c(*this, i0, i1, i2, v); }
};

// Minimum and maximum of v over the 64 lanes of a wavefront (butterfly of
// lane exchanges; every lane receives the result).
__device__ inline int wave_min(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline int wave_max(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
  return v;
}

}  // namespace rc
