// Device-assembly descriptor shared by the host table builder
// (host_setup.cpp) and the assembly kernels (assemble.hip).
#pragma once

#include <cstdint>

namespace igamg {

// One patch of one level for device assembly (Sec. 4: Gauss quadrature with
// p+1 points per element and direction, sum-factorised over the tensor rule).
// Unused directions (2D) have n = nel = nq = 1, degree 0, value 1, derivative
// 0, weight 1 and geometry degree 0.  All table offsets index one pool of
// doubles.
struct AsmPatch {
  int n[3];          // local functions per direction
  int nel[3];        // elements per direction
  int pc[3];         // spline degree per direction
  int nq[3];         // Gauss points per element per direction
  int g[3];          // geometry (Bezier) degree per direction
  int pad;
  int64_t off;       // first local row of the patch on its level
  int64_t w[3];      // Gauss weights, nel*nq
  int64_t val[3];    // basis values [(e*nq + q)*(pc+1) + l] (function e + l)
  int64_t der[3];    // basis derivatives, same layout
  int64_t gv[3];     // Bernstein values of the geometry at the points [(e*nq + q)*(g+1) + a]
  int64_t gd[3];     // Bernstein derivatives, same layout
  int64_t ctrl;      // control points, d values each, first index fastest
};

}  // namespace igamg
