// Host stand-in for the HIP runtime header, used only when physics.h is
// compiled on the host to count its floating-point operations.
#pragma once
#define __device__
#define __host__
#define __forceinline__ inline
#define __all(x) (x)
// the sweep table's element type (declared after the counting scalar
// replaces double, so it holds counted values)
struct double2 {
  double x, y;
};
inline double2 make_double2(double x, double y) { return double2{x, y}; }
