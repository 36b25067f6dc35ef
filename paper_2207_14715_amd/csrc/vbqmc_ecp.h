// Pseudopotential tables of a context (host and kernels).  Nothing here is
// part of the public C ABI (include/vbqmc.h).
#pragma once

#include <stdint.h>

namespace vbqmc {

constexpr int kEcpMaxL = 4;   // nonlocal channels l = 0 .. 3
constexpr int kEcpPts = 12;   // points of the angular rule (icosahedron vertices)

// Semilocal pseudopotentials, one record per pseudo-nucleus.  info[8 c ..]:
// nucleus, L (nonlocal channels), then L + 2 cumulative offsets into terms:
// the local part's terms, channel 0's, .., channel L-1's, end.  terms[3 k ..]
// = c, n, alpha of c r^(n-2) exp(-alpha r^2).  ncen = 0: no pseudopotential.
struct DevEcp {
  int ncen;
  const int* info;
  const double* rcut;
  const double* terms;
};

}  // namespace vbqmc
