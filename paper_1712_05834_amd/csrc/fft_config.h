// Compile-time launch shapes of the FFT passes, shared by the plain FFT
// kernels and the fused x-pass + binning kernel.
#pragma once

#include "fft_core.h"

namespace pk {

// Points per thread: 16 complex floats or 8 complex doubles (32 VGPRs of data).
template <typename T>
__host__ __device__ constexpr int e_max() { return sizeof(T) == 4 ? 16 : 8; }

// z-pass: rows of M = N/2 complex points (the real row viewed as complex).
template <typename T, int N>
struct ZCfg {
  static constexpr int M = N / 2;
  static constexpr int E = M < e_max<T>() ? M : e_max<T>();
  static constexpr int TPL = M / E;
  static constexpr int RPB = TPL >= 256 ? 1 : 256 / TPL;  // rows per workgroup
  static constexpr int THREADS = RPB * TPL;
  static constexpr int LP = lds_pad_len<M>();
};

// y- and x-passes: lines of N complex points, C neighbouring packed columns
// per workgroup (C * 8 bytes contiguous per row for complex float), with the
// LDS footprint capped at 80 KB so two workgroups fit on a CU.  EM caps the
// points per thread (the fused x-pass + binning keeps two meshes' lines in
// registers and uses fewer points per thread).
template <typename T, int N, int EM = e_max<T>()>
struct ColCfg {
  static constexpr int L = N;
  static constexpr int E = L < EM ? L : EM;
  static constexpr int TPL = L / E;
  static constexpr int NC = N / 2;
  static constexpr int pick() {
    int c = 256 / TPL;
    if (c < 8) c = 8;
    while (c > 1 && c * TPL > 1024) c /= 2;
    while (c > 1 && (long)c * lds_pad_len<L>() * (long)sizeof(cpx<T>) > 80 * 1024) c /= 2;
    if (c > NC) c = NC;
    return c;
  }
  static constexpr int C = pick();
  static constexpr int CHUNKS = NC / C;
  static constexpr int THREADS = TPL * C;
  static constexpr int LDS_ELEMS = lds_pad_len<L>() * C;
};

// Tile order for passes whose workgroups read C-column chunks narrower than a
// 128-byte line: the two chunks sharing a line (tiles 2j and 2j + 1) are
// given to workgroups g and g + 8, which the dispatcher places on the same
// XCD (round robin over 8 XCDs) at about the same time, so the second read
// of each line hits that XCD's L2.  Identity unless `ntiles` is a multiple
// of 16.
__device__ __forceinline__ int xcd_pair_tile(int g, int ntiles) {
  if (ntiles & 15) return g;
  return (g & ~15) | ((g & 7) << 1) | ((g >> 3) & 1);
}

// Launch shape of the fused x-pass + binning kernel.
template <typename T, int N>
using XCfg = ColCfg<T, N, (sizeof(T) == 4 ? 8 : 4)>;

}  // namespace pk
