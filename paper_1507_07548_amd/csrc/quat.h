// Rotation matrix of a unit quaternion q = (w, x, y, z): the body-to-lab
// rotation of a rigid molecule, lab = A(q) body.  One definition for every
// kernel that rotates site offsets, axes or angular velocities.
#pragma once
#include <hip/hip_runtime.h>

namespace ms2 {

// Rounded exactly as written (no contraction into fused multiply-adds), so
// that site offsets built from it equal a plain FP64 evaluation of the same
// expressions bit for bit (the site-site cut-off decides on them).
__device__ __forceinline__ void quat_matrix(double w, double x, double y, double z, double A[3][3]) {
#pragma clang fp contract(off)
  A[0][0] = 1.0 - 2.0 * (y * y + z * z);
  A[0][1] = 2.0 * (x * y - w * z);
  A[0][2] = 2.0 * (x * z + w * y);
  A[1][0] = 2.0 * (x * y + w * z);
  A[1][1] = 1.0 - 2.0 * (x * x + z * z);
  A[1][2] = 2.0 * (y * z - w * x);
  A[2][0] = 2.0 * (x * z - w * y);
  A[2][1] = 2.0 * (y * z + w * x);
  A[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

}  // namespace ms2
