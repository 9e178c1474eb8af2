// Rigid-body modes of linear elasticity as spline coefficient fields
// (Section 4): d translations, then the infinitesimal rotations, evaluated
// at a control point X.  3D rotations (0, x3, -x2), (x3, 0, -x1),
// (x2, -x1, 0); 2D rotation (x2, -x1).  Shared by the host setup and the
// device kernels so both use one definition of the mode basis.
#pragma once

#if defined(__HIPCC__)
#define AFIETI_HD __host__ __device__
#else
#define AFIETI_HD
#endif

namespace afieti {

AFIETI_HD inline double rigid_mode_value(int dim, int m, int c, const double* X) {
    if (m < dim) return m == c ? 1.0 : 0.0;
    if (dim == 2) return c == 0 ? X[1] : -X[0];
    switch (m) {
        case 3: return c == 0 ? 0.0 : (c == 1 ? X[2] : -X[1]);
        case 4: return c == 0 ? X[2] : (c == 1 ? 0.0 : -X[0]);
        default: return c == 0 ? X[1] : (c == 1 ? -X[0] : 0.0);
    }
}

AFIETI_HD inline int rigid_mode_count(int dim) { return dim == 3 ? 6 : 3; }

}  // namespace afieti
