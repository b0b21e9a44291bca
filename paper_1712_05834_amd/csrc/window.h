// Mass-assignment windows (Sec. 3.3.2): CIC, TSC and PCS are the centred
// cardinal B-splines of order p = 2, 3, 4 -- the windows whose Fourier
// transform is the sinc^p divided out by Eq. (2).
#pragma once

#include <hip/hip_runtime.h>

namespace pk {

// Cell coordinate u = (x mod L) N / L in float64: mesh node j sits at u = j.
// A position that wraps to exactly L is mapped to 0.
__device__ __forceinline__ double cell_coordinate(double x, int nmesh, double boxsize) {
  x = x - boxsize * floor(x / boxsize);
  if (x >= boxsize) x = 0.0;
  return x * (double)nmesh / boxsize;
}

// The same from the host-computed 1 / L and N / L: products instead of two
// float64 divisions per coordinate (the bucketing is 11-15% faster).  The
// cell chosen can differ from the divided form only where the position sits
// on a cell boundary to within an ulp, where the window weight of the far
// cell vanishes.
__device__ __forceinline__ double cell_coordinate_rcp(double x, double boxsize, double inv_box,
                                                     double cells_per_len) {
  x = x - boxsize * floor(x * inv_box);
  if (x >= boxsize) x = 0.0;
  return x * cells_per_len;
}

// First (unwrapped) cell touched by the order-P window at coordinate u and
// the P weights M_P(u - j), j = first .. first + P - 1.  The integer part is
// split off in float64; the fractional offset is then rounded once to T.
template <typename T, int P>
__device__ __forceinline__ void window_weights(double u, int& first, T* w) {
  if constexpr (P == 2) {
    const double f = floor(u);
    const T t = static_cast<T>(u - f);
    first = (int)f;
    w[0] = T(1) - t;
    w[1] = t;
  } else if constexpr (P == 3) {
    const double f = floor(u + 0.5);
    const T d = static_cast<T>(u - f);  // in [-1/2, 1/2)
    first = (int)f - 1;
    const T a = T(0.5) - d, b = T(0.5) + d;
    w[0] = T(0.5) * a * a;
    w[1] = T(0.75) - d * d;
    w[2] = T(0.5) * b * b;
  } else {
    const double f = floor(u);
    const T t = static_cast<T>(u - f);
    const T s = T(1) - t;
    first = (int)f - 1;
    const T one6 = T(1) / T(6);
    w[0] = s * s * s * one6;
    w[1] = (T(4) - T(6) * t * t + T(3) * t * t * t) * one6;
    w[2] = (T(4) - T(6) * s * s + T(3) * s * s * s) * one6;
    w[3] = t * t * t * one6;
  }
}

// The same windows from an integer cell `base` and a fraction t in [0, 1)
// (u = base + t), all in the mesh precision T.
template <typename T, int P>
__device__ __forceinline__ void window_frac(T t, int base, int& first, T* w) {
  if constexpr (P == 2) {
    first = base;
    w[0] = T(1) - t;
    w[1] = t;
  } else if constexpr (P == 3) {
    // centre cell floor(u + 1/2); d = u - centre in [-1/2, 1/2)
    const bool up = t >= T(0.5);
    const T d = up ? t - T(1) : t;
    first = base + (up ? 1 : 0) - 1;
    const T a = T(0.5) - d, b = T(0.5) + d;
    w[0] = T(0.5) * a * a;
    w[1] = T(0.75) - d * d;
    w[2] = T(0.5) * b * b;
  } else {
    const T s = T(1) - t;
    first = base - 1;
    const T one6 = T(1) / T(6);
    w[0] = s * s * s * one6;
    w[1] = (T(4) - T(6) * t * t + T(3) * t * t * t) * one6;
    w[2] = (T(4) - T(6) * s * s + T(3) * s * s * s) * one6;
    w[3] = t * t * t * one6;
  }
}

}  // namespace pk
