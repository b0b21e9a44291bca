// The 3-D forward r2c FFT (Sec. 3.3.1) as three passes over the mesh:
//   z-pass: each real row of N points is read as N/2 complex points, given an
//           N/2-point FFT and split into the N/2 + 1 outputs of the real DFT;
//           the two real outputs (kz = 0 and kz = N/2) are packed into one
//           complex slot, so a row stays N reals long and 4 KB aligned;
//   y-pass: N-point FFTs along y for C neighbouring packed columns at once;
//   x-pass: the same along x (here for the stand-alone transform; the
//           power-spectrum path fuses it with the binning).
// Every pass reads and writes each point once, coalesced along z.
#include "fft_config.h"
#include "internal.h"

namespace pk {

template <typename T, int N>
__global__ void __launch_bounds__((ZCfg<T, N>::THREADS))
    k_fft_z(T* __restrict__ mesh0, size_t mesh_stride, const cpx<T>* __restrict__ tw,
            const double* __restrict__ wsum) {
  using Z = ZCfg<T, N>;
  constexpr int M = Z::M, E = Z::E, TPL = Z::TPL, RPB = Z::RPB;
  __shared__ cpx<T> lds[RPB * Z::LP];
  __shared__ cpx<T> twq[N / 4];
  __shared__ cpx<T> tws[stage_table_size<M, E>() + 1];
  build_stage_table<T, M, E>(tws, TwGlobal<T>{tw, 2});
  load_quarter(twq, tw, N);
  const TwStage<T, M, E> tw2{tws};
  const TwQuarter<T> tw1{twq, 1, ilog2(N / 4)};
  const int r = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const size_t nrows = (size_t)N * N;
  const size_t row = (size_t)blockIdx.x * RPB + r;
  const bool active = row < nrows;
  cpx<T>* rowp = reinterpret_cast<cpx<T>*>(mesh0 + blockIdx.z * mesh_stride + row * N);
  // Subtracting the mean only changes the DC mode, which is never binned; it
  // keeps the float32 rounding of the other modes relative to the fluctuations.
  const T mean = wsum ? static_cast<T>(wsum[0] / ((double)N * N * N)) : T(0);
  cpx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (active) {
      v[e] = rowp[t + TPL * e];
      v[e].x -= mean;
      v[e].y -= mean;
    } else {
      v[e] = {T(0), T(0)};
    }
  }
  LdsLine<T> line{lds + r * Z::LP};
  stockham<T, M, E, 1>(v, t, tw2, line);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) line.template put_step<TPL>(t, e, v[e]);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = t + TPL * e;
    cpx<T> out;
    if (k == 0) {
      out = {v[e].x + v[e].y, v[e].x - v[e].y};  // {X_0, X_{N/2}}, both real
    } else {
      // X_k = (Z_k + conj Z_{M-k}) / 2 - (i / 2) W_N^k (Z_k - conj Z_{M-k});
      // M - k = (TPL - t) + TPL (E - 1 - e)
      const cpx<T> zc = cconj(line.template get_step<TPL>(TPL - t, E - 1 - e));
      const cpx<T> s = cadd(v[e], zc);
      const cpx<T> w = cmul(tw1(k), csub(v[e], zc));
      out = {T(0.5) * (s.x + w.y), T(0.5) * (s.y - w.x)};
    }
    if (active) rowp[k] = out;
  }
}

// Inverse z-pass (c2r of each row): the packed half spectrum X_0 .. X_{N/2}
// of a real row (slot 0 holding X_0 + i X_{N/2}) back to the N real values,
// unnormalised (x_n = sum_k X_k exp(+2 pi i n k / N) over the full row).  The
// row is rebuilt as the M-point complex sequence z_j = x_{2j} + i x_{2j+1}:
// with E_k = X_k + conj X_{M-k} and O_k = (X_k - conj X_{M-k}) W_N^{-k} (twice
// the transforms of the even and odd samples), Z_k = E_k + i O_k, and the
// unnormalised inverse M-point transform of Z -- conj(FFT(conj Z)) -- is
// 2 M z = N z.
template <typename T, int N>
__global__ void __launch_bounds__((ZCfg<T, N>::THREADS))
    k_ifft_z(T* __restrict__ mesh0, const cpx<T>* __restrict__ tw) {
  using Z = ZCfg<T, N>;
  constexpr int M = Z::M, E = Z::E, TPL = Z::TPL, RPB = Z::RPB;
  __shared__ cpx<T> lds[RPB * Z::LP];
  __shared__ cpx<T> twq[N / 4];
  __shared__ cpx<T> tws[stage_table_size<M, E>() + 1];
  build_stage_table<T, M, E>(tws, TwGlobal<T>{tw, 2});
  load_quarter(twq, tw, N);
  const TwStage<T, M, E> tw2{tws};
  const TwQuarter<T> tw1{twq, 1, ilog2(N / 4)};
  const int r = threadIdx.x / TPL, t = threadIdx.x % TPL;
  const size_t row = (size_t)blockIdx.x * RPB + r;
  const bool active = row < (size_t)N * N;
  cpx<T>* rowp = reinterpret_cast<cpx<T>*>(mesh0 + row * N);
  LdsLine<T> line{lds + r * Z::LP};
  cpx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = active ? rowp[t + TPL * e] : cpx<T>{T(0), T(0)};
    line.template put_step<TPL>(t, e, v[e]);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = t + TPL * e;
    cpx<T> zk;
    if (k == 0) {
      // X_0 and X_{N/2} are real: E_0 = X_0 + X_{N/2}, O_0 = X_0 - X_{N/2}
      zk = {v[e].x + v[e].y, v[e].x - v[e].y};
    } else {
      const cpx<T> xc = cconj(line.template get_step<TPL>(TPL - t, E - 1 - e));  // X_{M-k}
      const cpx<T> ev = cadd(v[e], xc);
      const cpx<T> od = cmul(cconj(tw1(k)), csub(v[e], xc));
      zk = {ev.x - od.y, ev.y + od.x};
    }
    v[e] = cconj(zk);
  }
  __syncthreads();  // every partner read before the line is reused
  stockham<T, M, E, 1>(v, t, tw2, line);
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (active) rowp[t + TPL * e] = cconj(v[e]);
}

template <typename T, int N>
__global__ void __launch_bounds__((ColCfg<T, N>::THREADS))
    k_fft_cols(T* __restrict__ mesh0, size_t mesh_stride, const cpx<T>* __restrict__ tw,
               int axis, int inverse) {
  using Cf = ColCfg<T, N>;
  constexpr int E = Cf::E, TPL = Cf::TPL, C = Cf::C, NC = Cf::NC;
  __shared__ cpx<T> lds[Cf::LDS_ELEMS];
  __shared__ cpx<T> tws[stage_table_size<N, E>() + 1];
  build_stage_table<T, N, E>(tws, TwGlobal<T>{tw, 1});
  const TwStage<T, N, E> tw1{tws};
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int tile = xcd_pair_tile(blockIdx.x, N * Cf::CHUNKS);
  const int outer = tile / Cf::CHUNKS, chunk = tile % Cf::CHUNKS;
  cpx<T>* mesh = reinterpret_cast<cpx<T>*>(mesh0 + blockIdx.z * mesh_stride);
  size_t base, step;
  if (axis == 1) {
    base = (size_t)outer * N * NC + (size_t)chunk * C + c;
    step = NC;
  } else {
    base = (size_t)outer * NC + (size_t)chunk * C + c;
    step = (size_t)N * NC;
  }
  cpx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    v[e] = mesh[base + (size_t)(t + TPL * e) * step];
    if (inverse) v[e] = cconj(v[e]);  // inverse transform: conj(FFT(conj x))
  }
  LdsCols<T, C> lc{lds, c};
  stockham<T, N, E, 1>(v, t, tw1, lc);
#pragma unroll
  for (int e = 0; e < E; ++e)
    mesh[base + (size_t)(t + TPL * e) * step] = inverse ? cconj(v[e]) : v[e];
}

// y-pass of the power-spectrum path: the same transform as k_fft_cols along
// y, read from the plain packed layout of one mesh and written out of place
// in the layout the fused x-pass reads (YLayout).  Each row of C columns that
// a workgroup writes is contiguous: a whole 128-byte line when C is 16
// complex floats; with 8 the sibling tile (next chunk, same x-plane, same
// XCD) writes the other half of its lines.
template <typename T, int N>
__global__ void __launch_bounds__((YCfg<T, N>::THREADS))
    k_fft_y_relayout(const T* __restrict__ src0, cpx<T>* __restrict__ dst,
                     const cpx<T>* __restrict__ tw) {
  using Cf = YCfg<T, N>;
  using YL = YLayout<T, N>;
  using Ix = typename YL::Ix;
  constexpr int E = Cf::E, TPL = Cf::TPL, C = Cf::C, NC = Cf::NC;
  __shared__ cpx<T> lds[Cf::LDS_ELEMS];
  __shared__ cpx<T> tws[stage_table_size<N, E>() + 1];
  build_stage_table<T, N, E>(tws, TwGlobal<T>{tw, 1});
  const TwStage<T, N, E> tw1{tws};
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int tile = xcd_pair_tile(blockIdx.x, N * Cf::CHUNKS);
  int x, chunk;
  if constexpr (C >= YL::W && YL::W * sizeof(cpx<T>) < 128) {
    // a tile writes whole rows of the layout, and the rows of x and x + 1
    // share a line: the sibling tiles are those two x-planes
    const int pair = tile >> 1;
    chunk = pair % Cf::CHUNKS;
    x = (pair / Cf::CHUNKS) * 2 + (tile & 1);
  } else {
    // siblings are neighbouring column chunks of one x-plane (same lines)
    x = tile / Cf::CHUNKS;
    chunk = tile % Cf::CHUNKS;
  }
  const int col = chunk * C + c;
  const cpx<T>* src = reinterpret_cast<const cpx<T>*>(src0);
  const Ix base = (Ix)x * ((Ix)N * NC) + (Ix)col;
  cpx<T> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[base + (Ix)(t + TPL * e) * NC];
  LdsCols<T, C> lc{lds, c};
  stockham<T, N, E, 1>(v, t, tw1, lc);
#pragma unroll
  for (int e = 0; e < E; ++e) dst[YL::at(x, t + TPL * e, col)] = v[e];
}

template <typename T, int N>
static hipError_t fft_y_relayout_t(const void* src, void* dst, const void* tw, hipStream_t s) {
  using Cf = YCfg<T, N>;
  const unsigned blocks = (unsigned)(N * Cf::CHUNKS);
  hipLaunchKernelGGL((k_fft_y_relayout<T, N>), dim3(blocks), dim3(Cf::THREADS), 0, s,
                     static_cast<const T*>(src), static_cast<cpx<T>*>(dst),
                     static_cast<const cpx<T>*>(tw));
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t fft_z_t(void* mesh, int nmeshes, size_t stride_bytes, const void* tw,
                          const double* wsum, hipStream_t s) {
  using Z = ZCfg<T, N>;
  const size_t nrows = (size_t)N * N;
  const unsigned blocks = (unsigned)((nrows + Z::RPB - 1) / Z::RPB);
  hipLaunchKernelGGL((k_fft_z<T, N>), dim3(blocks, 1, nmeshes), dim3(Z::THREADS), 0, s,
                     static_cast<T*>(mesh), stride_bytes / sizeof(T),
                     static_cast<const cpx<T>*>(tw), wsum);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t fft_cols_t(void* mesh, int nmeshes, size_t stride_bytes, const void* tw,
                             int axis, int inverse, hipStream_t s) {
  using Cf = ColCfg<T, N>;
  const unsigned blocks = (unsigned)(N * Cf::CHUNKS);
  hipLaunchKernelGGL((k_fft_cols<T, N>), dim3(blocks, 1, nmeshes), dim3(Cf::THREADS), 0, s,
                     static_cast<T*>(mesh), stride_bytes / sizeof(T),
                     static_cast<const cpx<T>*>(tw), axis, inverse);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t ifft_z_t(void* mesh, const void* tw, hipStream_t s) {
  using Z = ZCfg<T, N>;
  const unsigned blocks = (unsigned)(((size_t)N * N + Z::RPB - 1) / Z::RPB);
  hipLaunchKernelGGL((k_ifft_z<T, N>), dim3(blocks), dim3(Z::THREADS), 0, s,
                     static_cast<T*>(mesh), static_cast<const cpx<T>*>(tw));
  return hipGetLastError();
}

#define PK_DISPATCH_N(FN, T, ...)            \
  switch (nmesh) {                           \
    case 8: return FN<T, 8>(__VA_ARGS__);     \
    case 16: return FN<T, 16>(__VA_ARGS__);   \
    case 32: return FN<T, 32>(__VA_ARGS__);   \
    case 64: return FN<T, 64>(__VA_ARGS__);   \
    case 128: return FN<T, 128>(__VA_ARGS__); \
    case 256: return FN<T, 256>(__VA_ARGS__); \
    case 512: return FN<T, 512>(__VA_ARGS__); \
    case 1024: return FN<T, 1024>(__VA_ARGS__); \
    case 2048: return FN<T, 2048>(__VA_ARGS__); \
    default: return hipErrorInvalidValue;    \
  }

hipError_t launch_fft_z(int dtype, int nmesh, void* mesh, int nmeshes, size_t stride_bytes,
                        const void* tw, const double* wsum, hipStream_t s) {
  if (dtype == PK_F32) {
    PK_DISPATCH_N(fft_z_t, float, mesh, nmeshes, stride_bytes, tw, wsum, s)
  } else {
    PK_DISPATCH_N(fft_z_t, double, mesh, nmeshes, stride_bytes, tw, wsum, s)
  }
}

hipError_t launch_fft_cols(int dtype, int nmesh, void* mesh, int nmeshes, size_t stride_bytes,
                           const void* tw, int axis, hipStream_t s, int inverse) {
  if (dtype == PK_F32) {
    PK_DISPATCH_N(fft_cols_t, float, mesh, nmeshes, stride_bytes, tw, axis, inverse, s)
  } else {
    PK_DISPATCH_N(fft_cols_t, double, mesh, nmeshes, stride_bytes, tw, axis, inverse, s)
  }
}

hipError_t launch_ifft_z(int dtype, int nmesh, void* mesh, const void* tw, hipStream_t s) {
  if (dtype == PK_F32) {
    PK_DISPATCH_N(ifft_z_t, float, mesh, tw, s)
  } else {
    PK_DISPATCH_N(ifft_z_t, double, mesh, tw, s)
  }
}

hipError_t launch_fft_y_relayout(int dtype, int nmesh, const void* src, void* dst, const void* tw,
                                 hipStream_t s) {
  if (dtype == PK_F32) {
    PK_DISPATCH_N(fft_y_relayout_t, float, src, dst, tw, s)
  } else {
    PK_DISPATCH_N(fft_y_relayout_t, double, src, dst, tw, s)
  }
}

}  // namespace pk
