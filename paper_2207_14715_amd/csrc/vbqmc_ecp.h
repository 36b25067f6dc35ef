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
// l_scr: LDS offset (doubles) of the scratch of the batched projection (the
// 12 points of one electron and centre at once), scr_doubles its size, or
// l_scr = -1 when it does not fit (then one point at a time); nPmax: the
// larger table-orbital count of the two spins.
struct DevEcp {
  int ncen;
  const int* info;
  const double* rcut;
  const double* terms;
  int l_scr, scr_doubles, nPmax;
};

}  // namespace vbqmc
