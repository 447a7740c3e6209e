// Dirichlet faces (internal to libhelm).  A face with u = 0 takes its nodes
// out of the unknowns: every vector is kept zero there, and every other row
// of an operator is the row of the all-Sommerfeld operator restricted to the
// remaining columns (the boundary integral of a face only couples that
// face's nodes).
#pragma once

#include "helm_common.h"

namespace helm {

// y = 0 on the nodes of the faces set in mask (x0=1, x1=2, y0=4, y1=8,
// z0=16, z1=32) of a mesh with n cells per side; a no-op for mask = 0.
template <typename T>
void mask_faces(hipStream_t st, int dim, int n, unsigned mask, Vec<cx<T>> Y, int nslots);

}  // namespace helm
