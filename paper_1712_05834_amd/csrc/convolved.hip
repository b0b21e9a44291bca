// Survey power multipoles with a line of sight that varies from particle to
// particle (ConvolvedFFTPower, Sec. 3.4.1).  The paper names the estimator
// (the FFT multipoles of Hand et al. 2017) without writing it out; the
// standard form is computed here:
//
//   F(x)     = sum_data w delta_D(x - x_i) - alpha sum_randoms w delta_D(x - x_j),
//              alpha = sum_data w / sum_randoms w,
//   A_lm(k)  = FFT of F painted with the extra factor Y_lm(r^), r^ the unit
//              vector from the observer to the particle, divided by the
//              window (Eq. 2),
//   F_ell(k) = 4 pi / (2 ell + 1) sum_m Y_lm(k^) A_lm(k),
//   P_ell(k) = (2 ell + 1) / I <Re F_0(k) conj F_ell(k)>_shell.
//
// Y_lm are the real orthonormal spherical harmonics, evaluated through the
// associated Legendre recurrence in z and the powers of (x + i y), so the
// same routine serves the positions (r^) and the wave vectors (k^).  The
// catalog (data and randoms in one) is bucketed by column once, with the
// amounts w s; one pass over the sorted records then writes the amounts
// times Y_lm(r^) of the record's position for every harmonic, and each
// harmonic paints (with the z-pass), runs the y-pass into the x-pass layout
// and an x-pass that adds its lines into F_ell.  This file holds the weight
// sums, the amounts and the fused x-pass + accumulation; bucketing, painting,
// the y-pass and the binning are the kernels of the FFTPower path.
#include "fft_config.h"
#include "internal.h"

namespace pk {

namespace {

// Q_ell^m(z) = P_ell^m(z) / (1 - z^2)^(m/2) (no Condon-Shortley phase) by
// the three-term recurrence in ell, started from Q_m^m = (2m - 1)!!.
__device__ __forceinline__ double legendre_q(int ell, int am, double z) {
  double q0 = 1.0;
  for (int i = 1; i <= am; ++i) q0 *= (double)(2 * i - 1);
  if (ell == am) return q0;
  double q1 = (double)(2 * am + 1) * z * q0;
  for (int l = am + 2; l <= ell; ++l) {
    const double q2 = ((double)(2 * l - 1) * z * q1 - (double)(l + am - 1) * q0) / (double)(l - am);
    q0 = q1;
    q1 = q2;
  }
  return q1;
}

// Real spherical harmonic at the unit vector (x, y, z): knorm * Q_ell^|m|(z)
// times Re (x + i y)^|m| (m >= 0) or Im (x + i y)^|m| (m < 0).  knorm is
// the normalisation sqrt((2 ell + 1) / 4 pi (ell - |m|)! / (ell + |m|)!),
// times sqrt(2) for m != 0.
__device__ __forceinline__ double real_harmonic(int ell, int am, int sine, double knorm, double x,
                                                double y, double z) {
  double re = 1.0, im = 0.0;
  for (int i = 0; i < am; ++i) {
    const double r2 = re * x - im * y;
    im = re * y + im * x;
    re = r2;
  }
  return knorm * legendre_q(ell, am, z) * (sine ? im : re);
}

constexpr int kSumGroups = 512;

// Per-group partial sums {sum_data w, sum_data w^2, sum_randoms w,
// sum_randoms w^2} in float64; weights NULL mean 1.
template <typename T>
__global__ void __launch_bounds__(256)
    k_survey_sums(const T* __restrict__ wd, int64_t nd, const T* __restrict__ wr, int64_t nr,
                  double* __restrict__ part) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += stride) {
    const double w = wd ? (double)wd[i] : 1.0;
    s[0] += w;
    s[1] += w * w;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += stride) {
    const double w = wr ? (double)wr[i] : 1.0;
    s[2] += w;
    s[3] += w * w;
  }
  __shared__ double sh[4][256];
  for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] = s[j];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

// Sums the group partials in a fixed order (reproducible).
__global__ void __launch_bounds__(256)
    k_survey_sums_final(const double* __restrict__ part, int groups, double* __restrict__ sums) {
  __shared__ double sh[4][256];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g = threadIdx.x; g < groups; g += blockDim.x)
    for (int j = 0; j < 4; ++j) s[j] += part[g * 4 + j];
  for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] = s[j];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int j = 0; j < 4; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) sums[threadIdx.x] = sh[threadIdx.x][0];
}

// value_i = w_i s_i Y_lm(r^_i): s = 1 for the nd data particles (first in
// pos), -alpha for the randoms after them; r = x - observer with the position
// as given, r^ = z^ where r = 0.  With Y_00 and knorm = 1 (the constant 1)
// this is the amount w s that the bucketing sorts.
template <typename T>
__global__ void __launch_bounds__(256)
    k_ylm_value(const T* __restrict__ pos, const T* __restrict__ wd, int64_t nd,
                const T* __restrict__ wr, int64_t nr, double ox, double oy, double oz, int ell,
                int am, int sine, double knorm, const double* __restrict__ sums,
                T* __restrict__ value) {
  const int64_t n = nd + nr;
  const double neg_alpha = -sums[0] / sums[2];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double w;
    if (i < nd) {
      w = wd ? (double)wd[i] : 1.0;
    } else {
      w = (wr ? (double)wr[i - nd] : 1.0) * neg_alpha;
    }
    if (ell == 0) {  // Y_00 is the constant knorm: the position is not read
      value[i] = static_cast<T>(w * knorm);
      continue;
    }
    double rx = (double)pos[3 * i] - ox, ry = (double)pos[3 * i + 1] - oy,
           rz = (double)pos[3 * i + 2] - oz;
    const double rn = sqrt(rx * rx + ry * ry + rz * rz);
    if (rn > 0.0) {
      const double inv = 1.0 / rn;
      rx *= inv;
      ry *= inv;
      rz *= inv;
    } else {
      rx = 0.0;
      ry = 0.0;
      rz = 1.0;
    }
    value[i] = static_cast<T>(w * real_harmonic(ell, am, sine, knorm, rx, ry, rz));
  }
}

// Sorted records of the painting: {t_x, t_y, t_z, iy << 16 | iz} per
// particle, t the offsets from the cell corner, grouped by column
// c = ix N + iy (offsets[c] .. offsets[c + 1]).
__device__ __forceinline__ unsigned record_cell_bits(float w) { return __float_as_uint(w); }
__device__ __forceinline__ unsigned record_cell_bits(double w) { return (unsigned)w; }

// Every real harmonic Y_lm with ell <= 4 at the unit vector (x, y, z), up to
// its normalisation, written to y[ell (ell + 1) + m]: Q_ell^|m|(z) times
// Re (x + i y)^|m| (m >= 0) or Im (x + i y)^|m| (m < 0) -- the terms of
// real_harmonic, with the powers and the recurrences shared by all 25.
template <typename U>
__device__ __forceinline__ void harmonics_to_4(U x, U y, U z, U* out) {
  U re[5], im[5];
  re[0] = U(1);
  im[0] = U(0);
#pragma unroll
  for (int m = 1; m <= 4; ++m) {
    re[m] = re[m - 1] * x - im[m - 1] * y;
    im[m] = re[m - 1] * y + im[m - 1] * x;
  }
#pragma unroll
  for (int m = 0; m <= 4; ++m) {
    U q0 = U(1);  // Q_m^m = (2m - 1)!!
#pragma unroll
    for (int i = 1; i <= m; ++i) q0 *= static_cast<U>(2 * i - 1);
    U q1 = U(0);
#pragma unroll
    for (int l = m; l <= 4; ++l) {
      U q;
      if (l == m) {
        q = q0;
      } else if (l == m + 1) {
        q = static_cast<U>(2 * m + 1) * z * q0;
        q1 = q;
      } else {
        q = (static_cast<U>(2 * l - 1) * z * q1 - static_cast<U>(l + m - 1) * q0) /
            static_cast<U>(l - m);
        q0 = q1;
        q1 = q;
      }
      out[l * (l + 1) + m] = q * re[m];
      if (m > 0) out[l * (l + 1) - m] = q * im[m];
    }
  }
}

// amount[k][j] = base_j Y_k(r^_j) for every harmonic k of the set, for the
// records of one column per wavefront: base holds w s of every record, r^
// points from the observer to the record's position (ix + t_x, iy + t_y,
// iz + t_z) h in the periodic box.  One pass writes all harmonics, so the
// records are read once rather than once per harmonic.  slot[q] (q =
// ell (ell + 1) + m) is the harmonic's index k in the set, or -1.
struct YlmSlots {
  int slot[kMaxHarmonics];
  double knorm[kMaxHarmonics];
};

// Unit vector from the observer to a record's position (float64), rounded
// to the field precision U; z^ at the observer itself.
template <typename U, typename R>
__device__ __forceinline__ void record_direction(const R& r, int ix, double h, double ox,
                                                 double oy, double oz, U* u) {
  const unsigned bits = record_cell_bits(r.w);
  const int iy = (int)(bits >> 16), iz = (int)(bits & 0xffffu);
  double rx = ((double)ix + (double)r.x) * h - ox, ry = ((double)iy + (double)r.y) * h - oy,
         rz = ((double)iz + (double)r.z) * h - oz;
  const double rn = sqrt(rx * rx + ry * ry + rz * rz);
  if (rn > 0.0) {
    const double inv = 1.0 / rn;
    u[0] = static_cast<U>(rx * inv);
    u[1] = static_cast<U>(ry * inv);
    u[2] = static_cast<U>(rz * inv);
  } else {
    u[0] = U(0);
    u[1] = U(0);
    u[2] = U(1);
  }
}

// The harmonics are evaluated in the field precision T (the amounts are T
// values); each lane takes two records per step, so that two chains of
// load, evaluation and stores are in flight.
template <typename T, typename R>
__global__ void __launch_bounds__(256)
    k_ylm_records(const R* __restrict__ rec, const T* __restrict__ base,
                  const int* __restrict__ offsets, int N, double h, double ox, double oy,
                  double oz, YlmSlots ys, size_t stride, T* __restrict__ amount) {
  const int col = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (col >= N * N) return;
  const int ix = col / N;
  const int lane = threadIdx.x & 63;
  const int end = offsets[col + 1];
  for (int j = offsets[col] + lane; j < end; j += 128) {
    const int j2 = j + 64;
    const bool two = j2 < end;
    const R r1 = rec[j];
    const R r2 = two ? rec[j2] : r1;
    const T b1 = base[j];
    const T b2 = two ? base[j2] : b1;
    T u1[3], u2[3], y1[kMaxHarmonics], y2[kMaxHarmonics];
    record_direction<T>(r1, ix, h, ox, oy, oz, u1);
    record_direction<T>(r2, ix, h, ox, oy, oz, u2);
    harmonics_to_4<T>(u1[0], u1[1], u1[2], y1);
    harmonics_to_4<T>(u2[0], u2[1], u2[2], y2);
#pragma unroll
    for (int q = 0; q < kMaxHarmonics; ++q) {
      if (ys.slot[q] >= 0) {
        const T kn = static_cast<T>(ys.knorm[q]);
        T* __restrict__ out = amount + (size_t)ys.slot[q] * stride;
        out[j] = b1 * (kn * y1[q]);
        if (two) out[j2] = b2 * (kn * y2[q]);
      }
    }
  }
}

__device__ __forceinline__ int signed_wave(int i, int n) { return i < n / 2 ? i : i - n; }

// Mode factor of the accumulation: coef Y_lm(k^) / W(k) (W the window's
// sinc^p, or 1 without compensation) at the signed mode (nx, ny, nz); at the
// DC mode k^ is taken as z^ (the DC mode is never binned).  Evaluated in the
// field's precision T (the factor multiplies a T value): the same recurrence
// as real_harmonic.
template <typename T>
__device__ __forceinline__ T mode_factor(int nx, int ny, int nz, int kx, int ky, int ell, int am,
                                         int sine, double knorm, double coef,
                                         const T* __restrict__ sinv) {
  const int n2 = nx * nx + ny * ny + nz * nz;
  T ux = T(0), uy = T(0), uz = T(1);
  if (n2 > 0) {
    const T inv = T(1) / sqrt(static_cast<T>(n2));
    ux = static_cast<T>(nx) * inv;
    uy = static_cast<T>(ny) * inv;
    uz = static_cast<T>(nz) * inv;
  }
  T re = T(1), im = T(0);
  for (int i = 0; i < am; ++i) {
    const T r2 = re * ux - im * uy;
    im = re * uy + im * ux;
    re = r2;
  }
  T q0 = T(1);
  for (int i = 1; i <= am; ++i) q0 *= static_cast<T>(2 * i - 1);
  T q = q0;
  if (ell > am) {
    T q1 = static_cast<T>(2 * am + 1) * uz * q0;
    for (int l = am + 2; l <= ell; ++l) {
      const T q2 = (static_cast<T>(2 * l - 1) * uz * q1 - static_cast<T>(l + am - 1) * q0) /
                   static_cast<T>(l - am);
      q0 = q1;
      q1 = q2;
    }
    q = q1;
  }
  T g = static_cast<T>(coef * knorm) * q * (sine ? im : re);
  if (sinv) g *= sinv[kx] * sinv[ky] * sinv[nz];
  return g;
}

// Last FFT pass (along x) of one harmonic's spectrum A_lm, fused with the
// accumulation F_ell (+)= coef Y_lm(k^) A_lm / W(k): the transformed lines are
// added into F instead of being written back.  A arrives from the y-pass in
// its output layout (YLayout: the kx lines of a tile lie in a few pages
// rather than one page per kx) and F is kept in the same layout, so the
// read-modify-write of F has the locality of the loads.  Column kz' >= 1
// holds c(kx, ky, kz'); column 0 packs the planes kz = 0 and N/2 and needs
// the partner mode (-kx, -ky), which another workgroup transforms, so its
// lines go to `side` ([kx][ky]) for k_plane_accumulate.  With mesh2, a
// second harmonic h2 of the same ell is transformed in the same workgroup
// and added too, so that F is read and written once for both (its packed
// column goes to side2).
template <typename T, int N>
__global__ void __launch_bounds__((XCfg<T, N>::THREADS))
    k_fft_x_accumulate(const cpx<T>* __restrict__ mesh, const cpx<T>* __restrict__ mesh2,
                       cpx<T>* __restrict__ f, cpx<T>* __restrict__ side,
                       cpx<T>* __restrict__ side2, const cpx<T>* __restrict__ tw, Harmonic h1,
                       Harmonic h2, double coef, const T* __restrict__ sinv, int first) {
  using Cf = XCfg<T, N>;
  using YL = YLayout<T, N>;
  using Ix = typename YL::Ix;
  static_assert(YL::CX == Cf::C, "y-pass layout built for this tile width");
  constexpr int E = Cf::E, TPL = Cf::TPL, C = Cf::C;
  __shared__ cpx<T> lds[Cf::LDS_ELEMS];
  __shared__ cpx<T> tws[stage_table_size<N, E>() + 1];
  build_stage_table<T, N, E>(tws, TwGlobal<T>{tw, 1});
  const TwStage<T, N, E> tw1{tws};
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const int tile = xcd_group_tile<YL::G>(blockIdx.x, N * Cf::CHUNKS);
  const int ky = tile / Cf::CHUNKS, col = (tile % Cf::CHUNKS) * C + c;
  // kx = t + TPL e: with TPL a multiple of BX the offsets of a thread's
  // points differ by a constant
  constexpr bool REG = TPL % YL::BX == 0;
  constexpr Ix kstep = REG ? (Ix)(TPL / YL::BX) * ((Ix)N * YL::BX * YL::W) : 0;
  auto at = [&](int e) -> Ix {
    if constexpr (REG) return YL::at(t, ky, col) + (Ix)e * kstep;
    return YL::at(t + TPL * e, ky, col);
  };
  // the running F is loaded with the lines, so its latency overlaps the FFT
  const bool two = mesh2 != nullptr;
  cpx<T> v[E], v2[E], old[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = mesh[at(e)];
  if (two) {
#pragma unroll
    for (int e = 0; e < E; ++e) v2[e] = mesh2[at(e)];
  }
  if (!first && col != 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) old[e] = f[at(e)];
  }
  LdsCols<T, C> lc{lds, c};
  stockham<T, N, E, 1>(v, t, tw1, lc);
  if (two) stockham<T, N, E, 1>(v2, t, tw1, lc);
  const int ny = signed_wave(ky, N);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int kx = t + TPL * e;
    if (col == 0) {
      side[(size_t)kx * N + ky] = v[e];
      if (two) side2[(size_t)kx * N + ky] = v2[e];
      continue;
    }
    const int nx = signed_wave(kx, N);
    const T g =
        mode_factor<T>(nx, ny, col, kx, ky, h1.ell, h1.am, h1.sine, h1.knorm, coef, sinv);
    cpx<T> o = {g * v[e].x, g * v[e].y};
    if (two) {
      const T g2 =
          mode_factor<T>(nx, ny, col, kx, ky, h2.ell, h2.am, h2.sine, h2.knorm, coef, sinv);
      o.x += g2 * v2[e].x;
      o.y += g2 * v2[e].y;
    }
    if (!first) {
      o.x += old[e].x;
      o.y += old[e].y;
    }
    f[at(e)] = o;
  }
}

// The packed column of the harmonic (`side`, after the x-pass): its kz = 0
// value (Z + conj Z(-k)) / 2 is accumulated into the plane buffer of F
// ([kx][ky]).  F is Hermitian on that plane (A_lm is the transform of a real
// field and Y_lm(-k^) = Y_lm(k^) for even ell), so the plane read as a
// packed column is the packed form of a spectrum whose kz = N/2 plane is
// zero -- those modes have |n| >= N/2 and are never binned.
template <typename T>
__global__ void __launch_bounds__(256)
    k_plane_accumulate(int N, const cpx<T>* __restrict__ side, cpx<T>* __restrict__ plane,
                       int ell, int am, int sine, double knorm, double coef,
                       const T* __restrict__ sinv, int first) {
  const int mask = N - 1;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N * N;
       idx += gridDim.x * blockDim.x) {
    const int kx = idx / N, ky = idx % N;
    const cpx<T> z = side[idx], zp = side[((N - kx) & mask) * N + ((N - ky) & mask)];
    const cpx<T> v = {T(0.5) * (z.x + zp.x), T(0.5) * (z.y - zp.y)};
    const T g = mode_factor<T>(signed_wave(kx, N), signed_wave(ky, N), 0, kx, ky, ell, am, sine,
                               knorm, coef, sinv);
    cpx<T> o = {g * v.x, g * v.y};
    if (!first) {
      const cpx<T> old = plane[idx];
      o.x += old.x;
      o.y += old.y;
    }
    plane[idx] = o;
  }
}

unsigned grid_for(size_t work, size_t cap) {
  size_t g = (work + 255) / 256;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

size_t survey_sum_partials() { return (size_t)kSumGroups * 4; }

hipError_t launch_survey_sums(int dtype, const void* wd, int64_t nd, const void* wr, int64_t nr,
                              double* partials, double* sums, hipStream_t s) {
  const unsigned g = grid_for((size_t)(nd > nr ? nd : nr), kSumGroups);
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_survey_sums<float>, dim3(g), dim3(256), 0, s,
                       static_cast<const float*>(wd), nd, static_cast<const float*>(wr), nr,
                       partials);
  else
    hipLaunchKernelGGL(k_survey_sums<double>, dim3(g), dim3(256), 0, s,
                       static_cast<const double*>(wd), nd, static_cast<const double*>(wr), nr,
                       partials);
  hipLaunchKernelGGL(k_survey_sums_final, dim3(1), dim3(256), 0, s, partials, (int)g, sums);
  return hipGetLastError();
}

hipError_t launch_ylm_value(int dtype, const void* pos, const void* wd, int64_t nd, const void* wr,
                            int64_t nr, const double* observer, const Harmonic& h,
                            const double* sums, void* value, hipStream_t s) {
  const unsigned g = grid_for((size_t)(nd + nr), 8192);
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_ylm_value<float>, dim3(g), dim3(256), 0, s,
                       static_cast<const float*>(pos), static_cast<const float*>(wd), nd,
                       static_cast<const float*>(wr), nr, observer[0], observer[1], observer[2],
                       h.ell, h.am, h.sine, h.knorm, sums, static_cast<float*>(value));
  else
    hipLaunchKernelGGL(k_ylm_value<double>, dim3(g), dim3(256), 0, s,
                       static_cast<const double*>(pos), static_cast<const double*>(wd), nd,
                       static_cast<const double*>(wr), nr, observer[0], observer[1], observer[2],
                       h.ell, h.am, h.sine, h.knorm, sums, static_cast<double*>(value));
  return hipGetLastError();
}

hipError_t launch_ylm_records(int dtype, int nmesh, double boxsize, const void* rec,
                              const void* base, const void* bucket_ws, const double* observer,
                              const HarmonicSet& hs, size_t stride, void* amount,
                              hipStream_t s) {
  if (hs.n < 1 || hs.n > kMaxHarmonics) return hipErrorInvalidValue;
  YlmSlots ys;
  for (int q = 0; q < kMaxHarmonics; ++q) {
    ys.slot[q] = -1;
    ys.knorm[q] = 0.0;
  }
  for (int k = 0; k < hs.n; ++k) {
    const Harmonic& hm = hs.h[k];
    if (hm.ell > 4 || hm.am > hm.ell) return hipErrorInvalidValue;
    const int q = hm.ell * (hm.ell + 1) + (hm.sine ? -hm.am : hm.am);
    ys.slot[q] = k;
    ys.knorm[q] = hm.knorm;
  }
  // the column offsets follow the N^2 column counts at the start of the
  // bucketing workspace
  const int* offsets = static_cast<const int*>(bucket_ws) + (size_t)nmesh * nmesh;
  const unsigned g = (unsigned)(((size_t)nmesh * nmesh + 3) / 4);
  const double h = boxsize / nmesh;
  if (dtype == PK_F32)
    hipLaunchKernelGGL((k_ylm_records<float, float4>), dim3(g), dim3(256), 0, s,
                       static_cast<const float4*>(rec), static_cast<const float*>(base), offsets,
                       nmesh, h, observer[0], observer[1], observer[2], ys, stride,
                       static_cast<float*>(amount));
  else
    hipLaunchKernelGGL((k_ylm_records<double, double4>), dim3(g), dim3(256), 0, s,
                       static_cast<const double4*>(rec), static_cast<const double*>(base), offsets,
                       nmesh, h, observer[0], observer[1], observer[2], ys, stride,
                       static_cast<double*>(amount));
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t x_accumulate_t(const void* ymesh, const void* ymesh2, void* field, void* plane,
                                 void* side, void* side2, const void* tw, const Harmonic& h,
                                 const Harmonic& h2, double coef, const T* sinv, int first,
                                 hipStream_t s) {
  using Cf = XCfg<T, N>;
  hipLaunchKernelGGL((k_fft_x_accumulate<T, N>), dim3((unsigned)(N * Cf::CHUNKS)),
                     dim3(Cf::THREADS), 0, s, static_cast<const cpx<T>*>(ymesh),
                     static_cast<const cpx<T>*>(ymesh2), static_cast<cpx<T>*>(field),
                     static_cast<cpx<T>*>(side), static_cast<cpx<T>*>(side2),
                     static_cast<const cpx<T>*>(tw), h, h2, coef, sinv, first);
  hipLaunchKernelGGL(k_plane_accumulate<T>, dim3(grid_for((size_t)N * N, 4096)), dim3(256), 0,
                     s, N, static_cast<const cpx<T>*>(side), static_cast<cpx<T>*>(plane), h.ell,
                     h.am, h.sine, h.knorm, coef, sinv, first);
  if (ymesh2)
    hipLaunchKernelGGL(k_plane_accumulate<T>, dim3(grid_for((size_t)N * N, 4096)), dim3(256), 0,
                       s, N, static_cast<const cpx<T>*>(side2), static_cast<cpx<T>*>(plane),
                       h2.ell, h2.am, h2.sine, h2.knorm, coef, sinv, 0);
  return hipGetLastError();
}

template <typename T>
static hipError_t x_accumulate_n(int nmesh, const void* ymesh, const void* ymesh2, void* field,
                                 void* plane, void* side, void* side2, const void* tw,
                                 const Harmonic& h, const Harmonic& h2, double coef,
                                 const T* sinv, int first, hipStream_t s) {
  switch (nmesh) {
#define PK_XA(NN)                                                                          \
  case NN:                                                                                 \
    return x_accumulate_t<T, NN>(ymesh, ymesh2, field, plane, side, side2, tw, h, h2, coef, \
                                 sinv, first, s);
    PK_XA(8) PK_XA(16) PK_XA(32) PK_XA(64) PK_XA(128) PK_XA(256) PK_XA(512) PK_XA(1024)
    PK_XA(2048)
#undef PK_XA
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_x_accumulate(int dtype, int nmesh, const void* ymesh, const void* ymesh2,
                               void* field, void* plane, void* side, void* side2,
                               const Harmonic& h, const Harmonic& h2, double coef,
                               const MeshTables& t, int order, int compensated, int first,
                               hipStream_t s) {
  if (ymesh2 && (!side2 || h2.ell != h.ell)) return hipErrorInvalidValue;
  if (dtype == PK_F32) {
    const float* sinv =
        compensated ? static_cast<const float*>(t.sinc_inv) + (size_t)(order - 2) * nmesh : nullptr;
    return x_accumulate_n<float>(nmesh, ymesh, ymesh2, field, plane, side, side2, t.tw, h, h2,
                                 coef, sinv, first, s);
  }
  const double* sinv =
      compensated ? static_cast<const double*>(t.sinc_inv) + (size_t)(order - 2) * nmesh : nullptr;
  return x_accumulate_n<double>(nmesh, ymesh, ymesh2, field, plane, side, side2, t.tw, h, h2,
                                coef, sinv, first, s);
}

}  // namespace pk
