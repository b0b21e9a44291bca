// Painting (Sec. 3.3.1, Eq. 1; windows and interlacing, Sec. 3.3.2):
// scatter form.  One thread per particle computes its cell coordinates in
// float64, its p weights per axis, and adds the p^3 products into the mesh
// with float atomics (global_atomic_add_f32 / _f64 on gfx950).
#include "internal.h"
#include "window.h"

namespace pk {

__global__ void k_fill_zero(float4* __restrict__ p, size_t n4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_fill_zero_tail(float* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t n4 = bytes / 16;
  if (n4) {
    size_t blocks = (n4 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s,
                       reinterpret_cast<float4*>(p), n4);
  }
  const size_t rem = (bytes - n4 * 16) / 4;
  if (rem) {
    hipLaunchKernelGGL(k_fill_zero_tail, dim3(1), dim3(64), 0, s,
                       reinterpret_cast<float*>(static_cast<char*>(p) + n4 * 16), rem);
  }
  return hipGetLastError();
}

// Wave-level sum of a double (64 lanes), result valid in every lane.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T, int P>
__global__ void __launch_bounds__(256) k_paint_atomic(const T* __restrict__ pos,
                                                      const T* __restrict__ weight, int64_t n,
                                                      int nmesh, double boxsize, double shift_a,
                                                      T* __restrict__ mesh_a, double shift_b,
                                                      T* __restrict__ mesh_b,
                                                      double* __restrict__ wsums) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int mask = nmesh - 1;
  double ws = 0.0, ws2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = cell_coordinate((double)pos[3 * i + d], nmesh, boxsize);
    const T wp = weight ? weight[i] : T(1);
    ws += (double)wp;
    ws2 += (double)wp * (double)wp;
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      T* mesh = pass == 0 ? mesh_a : mesh_b;
      if (mesh == nullptr) continue;
      const double sh = pass == 0 ? shift_a : shift_b;
      int first[3];
      T w[3][P];
#pragma unroll
      for (int d = 0; d < 3; ++d) window_weights<T, P>(u[d] + sh, first[d], w[d]);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        const size_t ix = (size_t)((first[0] + a) & mask);
        const T wa = wp * w[0][a];
#pragma unroll
        for (int b = 0; b < P; ++b) {
          const size_t iy = (size_t)((first[1] + b) & mask);
          const T wab = wa * w[1][b];
          const size_t row = (ix * nmesh + iy) * nmesh;
#pragma unroll
          for (int c = 0; c < P; ++c) {
            const size_t iz = (size_t)((first[2] + c) & mask);
            atomicAdd(&mesh[row + iz], wab * w[2][c]);
          }
        }
      }
    }
  }
  if (wsums) {
    ws = wave_sum(ws);
    ws2 = wave_sum(ws2);
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&wsums[0], ws);
      atomicAdd(&wsums[1], ws2);
    }
  }
}

template <typename T, int P>
static hipError_t paint_atomic_t(int nmesh, double boxsize, const void* pos, const void* weight,
                                 int64_t n, double shift_a, void* mesh_a, double shift_b,
                                 void* mesh_b, double* wsums, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_paint_atomic<T, P>), dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<const T*>(pos), static_cast<const T*>(weight), n, nmesh,
                     boxsize, shift_a, static_cast<T*>(mesh_a), shift_b, static_cast<T*>(mesh_b),
                     wsums);
  return hipGetLastError();
}

hipError_t launch_paint_atomic(int dtype, int order, int nmesh, double boxsize, const void* pos,
                               const void* weight, int64_t n, double shift_a, void* mesh_a,
                               double shift_b, void* mesh_b, double* wsums, hipStream_t s) {
#define PK_PAINT_CASE(T, P)                                                                   \
  return paint_atomic_t<T, P>(nmesh, boxsize, pos, weight, n, shift_a, mesh_a, shift_b, mesh_b, \
                              wsums, s)
  if (dtype == PK_F32) {
    if (order == 2) PK_PAINT_CASE(float, 2);
    if (order == 3) PK_PAINT_CASE(float, 3);
    if (order == 4) PK_PAINT_CASE(float, 4);
  } else {
    if (order == 2) PK_PAINT_CASE(double, 2);
    if (order == 3) PK_PAINT_CASE(double, 3);
    if (order == 4) PK_PAINT_CASE(double, 4);
  }
#undef PK_PAINT_CASE
  return hipErrorInvalidValue;
}

}  // namespace pk
