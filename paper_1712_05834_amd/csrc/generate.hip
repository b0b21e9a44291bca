// Device-side field generation on packed spectra: the scaling of every mode
// by a real amplitude that depends on |n|^2 only (an isotropic transfer, such
// as the sqrt(P(k)) that turns white noise into a Gaussian field of spectrum
// P).  With the forward and backward transforms it generates Gaussian
// realisations on the device (Sec. 3.2: the catalogs built from Gaussian
// fields; Sec. 3.3.1: RealField <-> ComplexField).
#include "fft_core.h"
#include "internal.h"

namespace pk {

namespace {

__device__ __forceinline__ int signed_mode(int i, int n) { return i < n / 2 ? i : i - n; }

// c(k) *= table[|n|^2].  Column kz' >= 1 holds c(kx, ky, kz'); column 0
// packs Z = c0 + i c1 with c0 = c(kx, ky, 0), c1 = c(kx, ky, N/2), whose
// amplitudes t0 = table[nx^2 + ny^2] and t1 = table[nx^2 + ny^2 + N^2/4]
// differ: Z' = t0 c0 + i t1 c1 = a Z + b conj Z(-k) with a = (t0 + t1) / 2,
// b = (t0 - t1) / 2, and the partner (-kx, -ky) has the same t0, t1, so each
// pair is updated together by the thread of its lower index.
template <typename T>
__global__ void __launch_bounds__(256)
    k_shape_packed(int N, cpx<T>* __restrict__ cm, const double* __restrict__ table) {
  const int NC = N / 2, mask = N - 1;
  const size_t total = (size_t)N * N * NC;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(idx % NC);
    const size_t rest = idx / NC;
    const int ky = (int)(rest % N), kx = (int)(rest / N);
    const int nx = signed_mode(kx, N), ny = signed_mode(ky, N);
    const int n2xy = nx * nx + ny * ny;
    if (col != 0) {
      const T f = static_cast<T>(table[n2xy + col * col]);
      const cpx<T> v = cm[idx];
      cm[idx] = {f * v.x, f * v.y};
      continue;
    }
    const size_t me = (size_t)kx * N + ky;
    const size_t pa = (size_t)((N - kx) & mask) * N + ((N - ky) & mask);
    if (me > pa) continue;
    const double t0 = table[n2xy], t1 = table[n2xy + NC * NC];
    const T a = static_cast<T>(0.5 * (t0 + t1)), b = static_cast<T>(0.5 * (t0 - t1));
    const cpx<T> z = cm[me * NC], zp = cm[pa * NC];
    cm[me * NC] = {a * z.x + b * zp.x, a * z.y - b * zp.y};
    if (pa != me) cm[pa * NC] = {a * zp.x + b * z.x, a * zp.y - b * z.y};
  }
}

}  // namespace

hipError_t launch_shape_packed(int dtype, int nmesh, void* cmesh, const double* table,
                               hipStream_t s) {
  const size_t total = (size_t)nmesh * nmesh * (nmesh / 2);
  size_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_shape_packed<float>, dim3((unsigned)g), dim3(256), 0, s, nmesh,
                       static_cast<cpx<float>*>(cmesh), table);
  else
    hipLaunchKernelGGL(k_shape_packed<double>, dim3((unsigned)g), dim3(256), 0, s, nmesh,
                       static_cast<cpx<double>*>(cmesh), table);
  return hipGetLastError();
}

}  // namespace pk
