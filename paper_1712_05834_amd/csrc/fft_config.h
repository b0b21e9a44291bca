// Compile-time launch shapes of the FFT passes, shared by the plain FFT
// kernels and the fused x-pass + binning kernel.
#pragma once

#include <type_traits>

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
template <typename T, int N, int EM = e_max<T>(), int LDS_KB = 80, int CMIN = 8>
struct ColCfg {
  static constexpr int L = N;
  static constexpr int E = L < EM ? L : EM;
  static constexpr int TPL = L / E;
  static constexpr int NC = N / 2;
  static constexpr int pick() {
    int c = 256 / TPL;
    if (c < CMIN) c = CMIN;
    while (c > 1 && c * TPL > 1024) c /= 2;
    while (c > 1 && (long)c * lds_pad_len<L>() * (long)sizeof(cpx<T>) > LDS_KB * 1024) c /= 2;
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

// The same with groups of G tiles (G a power of two): tiles G j .. G j + G - 1
// go to workgroups g, g + 8, ..., g + 8 (G - 1).  Identity unless `ntiles`
// is a multiple of 8 G.
template <int G>
__device__ __forceinline__ int xcd_group_tile(int g, int ntiles) {
  if (ntiles % (8 * G)) return g;
  const int blk = g / (8 * G), off = g % (8 * G);
  return blk * 8 * G + (off % 8) * G + off / 8;
}

// Launch shape of the y-pass of the power-spectrum path (k_fft_y_relayout).
// Float32 at N = 1024: 16 points per thread and 16 columns per workgroup
// (1024 threads, 144 KB of LDS, one workgroup per CU), so that every row read
// and written is a whole 128-byte line: 1.80 ms per mesh against 2.04 ms with
// 8 columns of 8 points.  Elsewhere 8 points per thread (16 were 1-2% slower
// there, 4 were 60% slower at 1024^3) and up to 16 columns where they fit in
// 80 KB (N <= 512).
template <typename T, int N>
using YCfg = typename std::conditional<(sizeof(T) == 4 && N == 1024), ColCfg<T, N, 16, 160, 16>,
                                       ColCfg<T, N, 8, 80, 16>>::type;

// Launch shape of the fused x-pass + binning kernel.
// (Line buffers capped at 40 KB -- 4 columns per tile at N = 1024, two
// workgroups per CU -- made the x-pass 9% faster, but the y-pass writes of
// 64-byte layout rows cost more than that.)
template <typename T, int N>
using XCfg = ColCfg<T, N, (sizeof(T) == 4 ? 8 : 4), 80>;

// Layout of the y-transformed spectrum handed from the y-pass to the fused
// x-pass in the power-spectrum path.  The x-pass reads, for one ky and C
// neighbouring packed columns, all N values of kx; the y-pass writes, for one
// x and C columns, all N values of ky.  In the plain packed layout the x-pass
// reads would be N * N / 2 complex apart (4 MB at N = 1024), a different
// page for every kx.  Here the columns are grouped W at a time (two x-pass
// chunks) and x in blocks of BX:
//   (kx, ky, col) at (col / W) N^2 W + (kx / BX) N BX W + ky BX W
//                    + (kx % BX) W + col % W,
// so the y-pass of one x writes N values BX W apart (a 1 MB span at
// N = 1024), and the x-pass of one ky reads BX consecutive W-wide rows per
// block, blocks N BX W apart.  The G = W / C tiles of a column group run
// side by side on one XCD (xcd_group_tile) and read the parts of the same
// rows; the y-pass pairs its tiles so that the rows it writes fill lines.
template <typename T, int N>
struct YLayout {
  static constexpr int CX = XCfg<T, N>::C;
  static constexpr int W = 2 * CX <= N / 2 ? 2 * CX : N / 2;
  static constexpr int G = W / CX;  // x-pass tiles sharing a group
  static constexpr int BX = N < 8 ? N : 8;
  using Ix = typename std::conditional<((long)N * N * (N / 2) <= (1L << 31)), unsigned, size_t>::type;
  __host__ __device__ static constexpr Ix at(int kx, int ky, int col) {
    return (Ix)(col / W) * ((Ix)N * N * W) + (Ix)(kx / BX) * ((Ix)N * BX * W) +
           (Ix)ky * (BX * W) + (Ix)(kx % BX) * W + (Ix)(col % W);
  }
};

}  // namespace pk
