// Device view of a degree-1 level operator in colour-major stencil layout
// (shared by the kernels and the host code that builds it; the layout is
// described with the structured h-multigrid kernels).
#pragma once

namespace pmg {

struct GridLevel {
  int nx, n;            // nodes per axis, nodes
  int cnt[8], voff[8];  // per colour: nodes, offset of its values in v
  const double* v;
  // 2-D Poisson on the unit box: the 1-D stiffness and mass of the level as
  // bands (nx rows of 3), from which the tiled kernels form the values of v
  // bit for bit instead of reading them; null otherwise
  const double* kK;
  const double* kM;
};

}  // namespace pmg
