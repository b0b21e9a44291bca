// FFTPower binning (Sec. 3.4.1) with interlacing and window compensation
// (Sec. 3.3.2, Eq. 2) fused in.
//
// k_xpass_bin  last FFT pass (along x) of both meshes in LDS, read from the
//              y-pass output layout (YLayout), then for every mode of the
//              tile: interlace, compensate, |c|^2, k / mu bin and Legendre
//              weights, accumulated in float64 LDS bins.  Persistent grid:
//              each workgroup walks many (ky, column-chunk) tiles and writes
//              one row of partial sums at the end.
// k_plane_bin  the two self-conjugate planes kz = 0 and kz = N/2, which the
//              packed layout keeps in one complex column; unpacked with the
//              partner mode (-kx, -ky).
// k_reduce     sums the partial rows in a fixed order (deterministic given
//              the partials).
// k_mode_tables  plan-time counts, sum h|n| and sum h|mu| per bin.
#include <type_traits>

#include "fft_config.h"
#include "internal.h"

namespace pk {

// Exact integer square root of 0 <= v < 2^24 (v converts to float exactly;
// the hardware float root, within an ulp, is at most one unit off the
// answer and is corrected).
__device__ __forceinline__ int isqrt_exact(int v) {
  int s = (int)__builtin_amdgcn_sqrtf((float)v);
  if (s * s > v) --s;
  if ((s + 1) * (s + 1) <= v) ++s;
  return s;
}

// Largest b with e_b^2 <= n^2 among the nk bins, -1 for the DC mode and for
// modes outside [e_0, e_nk).  Whole-number edges use the integer root; other
// edges correct a float estimate with exact comparisons of the integer n^2
// against the float64 table e2.
__device__ __forceinline__ int kbin_of(int n2, const BinSpec& b) {
  if (n2 == 0) return -1;
  if (b.int_edges) {
    const int s = isqrt_exact(n2) - b.kmin_i;
    if (s < 0) return -1;
    const int k = b.dk_i == 1 ? s : s / b.dk_i;
    return k < b.nk ? k : -1;
  }
  const double x = (double)n2;
  const double* __restrict__ e2 = b.e2;
  if (x < e2[0] || x >= e2[b.nk]) return -1;
  int k = (int)((sqrtf((float)n2) - (float)b.kmin_f) / (float)b.dk_f);
  k = k < 0 ? 0 : (k > b.nk - 1 ? b.nk - 1 : k);
  while (k + 1 < b.nk && x >= e2[k + 1]) ++k;
  while (k > 0 && x < e2[k]) --k;
  return k;
}

// Largest j in [0, nmu] with j^2 n^2 <= nmu^2 n_los^2, clipped to nmu - 1.
// The float estimate nmu |mu| is within a few 1e-7 of its exact value (a
// few ulp of hardware reciprocal and root, nmu <= 64), so its floor is at
// most one off; one exact 64-bit integer check each way corrects it.
__device__ __forceinline__ int mubin_of(int nlos2, int n2, int nmu) {
  const unsigned long long rhs = (unsigned long long)(nmu * nmu) * (unsigned)nlos2;
  int j = (int)((float)nmu *
                __builtin_amdgcn_sqrtf((float)nlos2 * __builtin_amdgcn_rcpf((float)n2)));
  j = j < 0 ? 0 : (j > nmu ? nmu : j);
  if (j < nmu && (unsigned long long)((j + 1) * (j + 1)) * (unsigned)n2 <= rhs) ++j;
  if (j > 0 && (unsigned long long)(j * j) * (unsigned)n2 > rhs) --j;
  return j < nmu ? j : nmu - 1;
}

template <typename T>
__device__ __forceinline__ T legendre(int ell, T mu2) {
  if (ell == 2) return (T(3) * mu2 - T(1)) * T(0.5);
  if (ell == 4) return ((T(35) * mu2 - T(30)) * mu2 + T(3)) * T(0.125);
  return (((T(231) * mu2 - T(315)) * mu2 + T(105)) * mu2 - T(5)) * T(0.0625);
}

// mu^2 = n_los^2 / n^2 in the path's precision (float: fast reciprocal,
// ~1 ulp; double: correctly rounded division).
template <typename T>
__device__ __forceinline__ T ratio(int a, int b) {
  if constexpr (sizeof(T) == 4) {
    return __fdividef((float)a, (float)b);
  } else {
    return (double)a / (double)b;
  }
}

// ---- exact bin sums: fixed point
//
// Every bin sum is accumulated as an integer in units of 2^-S: each term is
// rounded to that grid once (towards minus infinity), and integer addition is
// associative, so the sums do not depend on the order in which lanes, waves
// or workgroups add their terms -- a result is the same bit for bit on every
// run, whatever the number of workgroups.  S is chosen from a bound B on
// every partial sum, so nothing overflows.  A slot is two 64-bit LDS words,
// in one of two splits (BinSpec::fix_hb):
//  * 64: a 128-bit two's complement integer (low, high), |sum| < 2^126; the
//    carry of the low word's addition is read from the returning atomic and
//    added to the high word with the rest of the term, which keeps
//    concurrent additions exact.  Float64 spectra: a typical term keeps more
//    than 53 significant bits.
//  * 32: the low 32 bits of the term in the first word (an unsigned count
//    that cannot overflow before 2^32 additions) and the rest, signed, in the
//    second, |sum| < 2^95; both added without return (no wait on the LDS).
//    Float32 spectra: a typical term keeps more than 30 significant bits,
//    far below the float32 path's own rounding.

__device__ __forceinline__ int fix_shift(const BinSpec& b) {
  double bound = b.bound_scale;
  if (b.bound_dev) {
    const double v = *b.bound_dev;
    bound *= b.bound_sq ? v * v : v;
  }
  if (!(bound > 0.0)) return 0;  // every term is zero
  int e;
  (void)frexp(bound, &e);  // bound < 2^e
  return (b.fix_hb == 32 ? 94 : 126) - e;
}

// trunc(v 2^S) as (lo, hi) words of a 128-bit two's complement integer,
// from the bits of v: the 53-bit significand shifted into place.
__host__ __device__ __forceinline__ void fix_split(double v, int S, unsigned long long& lo,
                                                   unsigned long long& hi) {
  const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
  const int e = (int)((bits >> 52) & 0x7ff);
  const unsigned long long mant = bits & 0xfffffffffffffull;
  const unsigned long long m = e ? (mant | (1ull << 52)) : mant;
  const int sh = (e ? e : 1) - 1075 + S;  // v = m 2^(sh - S)
  if (sh >= 64) {
    lo = 0;
    hi = m << (sh - 64);
  } else if (sh >= 0) {
    lo = m << sh;
    hi = sh > 11 ? m >> (64 - sh) : 0;
  } else {
    lo = sh > -64 ? m >> (-sh) : 0;
    hi = 0;
  }
  if (bits >> 63) {  // negate: two's complement of (hi, lo)
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0 ? 1ull : 0ull);
  }
}

// floor(v 2^S) = hi 2^32 + lo with 0 <= lo < 2^32 and hi signed, for
// |v 2^S| < 2^95: doubles split exactly by floors of power-of-two scalings.
__host__ __device__ __forceinline__ void fix_split32(double v, int S, unsigned long long& lo,
                                                     unsigned long long& hi) {
  const double y = ldexp(v, S);
  const double hd = floor(ldexp(y, -32));
  const double ld = y - ldexp(hd, 32);  // exact, in [0, 2^32)
  const double hh = floor(ldexp(hd, -32));
  const double hl = hd - ldexp(hh, 32);  // exact, in [0, 2^32)
  lo = (unsigned long long)(unsigned)ld;
  hi = (unsigned long long)((long long)(int)hh * 4294967296ll + (long long)(unsigned)hl);
}

// Adds a finite term: the 32-bit split for float32 spectra, the 128-bit one
// for float64 (fixed by the element type, as BinSpec::fix_hb is).
template <typename T>
__device__ __forceinline__ void fix_add(unsigned long long* acc, int nlds, int slot, double v,
                                        int S) {
  unsigned long long lo, hi;
  if constexpr (sizeof(T) == 4) {
    fix_split32(v, S, lo, hi);
    atomicAdd(&acc[slot], lo);
    atomicAdd(&acc[nlds + slot], hi);
  } else {
    fix_split(v, S, lo, hi);
    if ((lo | hi) == 0) return;
    const unsigned long long old = atomicAdd(&acc[slot], lo);
    const unsigned long long carry = old + lo < old ? 1ull : 0ull;
    if (hi + carry) atomicAdd(&acc[nlds + slot], hi + carry);
  }
}

// The value of a slot's words, (hi 2^hb + lo) 2^-S, rounded to double the
// same way every time (hi signed, lo unsigned).
__host__ __device__ __forceinline__ double fix_words_value(unsigned long long lo,
                                                           unsigned long long hi, int S,
                                                           int hb = 64) {
  if (hb == 32) {
    // the unique form hi 2^32 + lo with lo < 2^32, so that equal integers
    // round to the same double whatever their split
    hi += lo >> 32;
    lo &= 0xffffffffull;
  }
  const double v = ldexp((double)(long long)hi, hb) + (double)lo;
  return ldexp(v, -S);
}

__device__ __forceinline__ double fix_value(const unsigned long long* acc, const BinSpec& b,
                                            int slot, int S) {
  return fix_words_value(acc[slot], acc[b.nlds + slot], S, b.fix_hb);
}

// Adds one mode of (Hermitian-weighted) power hp to the LDS bins.  The
// per-mode products hp L_ell are formed in the path's precision; every sum
// is exact (fixed point, see above).
template <typename T>
__device__ __forceinline__ void accumulate(unsigned long long* sb, const BinSpec& b, int S, int n2,
                                           int nlos2, T hp) {
  const int k = kbin_of(n2, b);
  if (k < 0) return;
  if (!isfinite(hp)) {  // flagged: the workgroup's sums become NaN
    atomicOr(&sb[2 * b.nlds], 1ull);
    return;
  }
  if (!b.power_from_2d) fix_add<T>(sb, b.nlds, k, (double)hp, S);
  if (b.npl > 0) {
    const T mu2 = ratio<T>(nlos2, n2);
    // at most 4 poles: unrolled, so that the pole tables are read with
    // constant indices (scalar registers) instead of a runtime loop
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < b.npl)
        fix_add<T>(sb, b.nlds, b.pole_lds[i] + k, (double)(hp * legendre<T>(b.pole_ell[i], mu2)),
                   S);
  }
  if (b.off2d_lds >= 0)
    fix_add<T>(sb, b.nlds, b.off2d_lds + k * b.nmu + mubin_of(nlos2, n2, b.nmu), (double)hp,
               S);
}

__device__ __forceinline__ int signed_index(int i, int n) { return i < n / 2 ? i : i - n; }

// float64 accumulators (survey cross sums, projected power, plan-time tables)
__device__ __forceinline__ void zero_bins(double* sb, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) sb[i] = 0.0;
}

__device__ __forceinline__ void flush_bins(const double* sb, int n, double* out) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = sb[i];
}

__device__ __forceinline__ void zero_bins(unsigned long long* sb, const BinSpec& b) {
  for (int i = threadIdx.x; i <= 2 * b.nlds; i += blockDim.x) sb[i] = 0;
}

// Marker of a sum that met a non-finite term (never a valid sum: those stay
// below 2^126 in magnitude).
constexpr unsigned long long kFixNanHi = 0x8000000000000000ull, kFixNanLo = ~0ull;

// One partial row in the result's slot order (the slots of ell = 0 poles are
// zero: they alias the power sum).  Exact rows hold the 128-bit sums (low
// words [0, nsum), high words [nsum, 2 nsum)); otherwise float64 values.
__device__ __forceinline__ void flush_bins(const unsigned long long* sb, const BinSpec& b, int S,
                                           double* row) {
  const bool bad = sb[2 * b.nlds] != 0;
  unsigned long long* words = reinterpret_cast<unsigned long long*>(row);
  for (int r = threadIdx.x; r < b.nsum; r += blockDim.x) {
    int slot = -1;
    if (r < b.nk && b.power_from_2d) {
      // the exact sum of the k-bin's mu-bin sums (both splits add with carry)
      unsigned long long lo = 0, hi = 0;
      for (int j = 0; j < b.nmu; ++j) {
        const int q = b.off2d_lds + r * b.nmu + j;
        if (b.fix_hb == 32) {
          lo += sb[q] & 0xffffffffull;
          hi += sb[b.nlds + q] + (sb[q] >> 32);
        } else {
          const unsigned long long old = lo;
          lo += sb[q];
          hi += sb[b.nlds + q] + (lo < old ? 1ull : 0ull);
        }
      }
      if (b.exact) {
        words[r] = bad ? kFixNanLo : lo;
        words[b.nsum + r] = bad ? kFixNanHi : hi;
      } else {
        row[r] = bad ? __longlong_as_double(0x7ff8000000000000ll)
                     : fix_words_value(lo, hi, S, b.fix_hb);
      }
      continue;
    }
    if (r < b.nk) {
      slot = r;
    } else if (r < b.nk * (1 + b.npoles)) {
      const int pi = r / b.nk - 1;
      if (!((b.zero_mask >> pi) & 1)) {
        // the accumulated poles keep the order of b.poles
        int rank = 0;
        for (int j = 0; j < pi; ++j) rank += ((b.zero_mask >> j) & 1) ? 0 : 1;
        slot = b.pole_lds[rank] + r % b.nk;
      }
    } else {
      slot = b.off2d_lds + (r - b.off2d);
    }
    if (b.exact) {
      words[r] = bad ? kFixNanLo : (slot >= 0 ? sb[slot] : 0ull);
      words[b.nsum + r] = bad ? kFixNanHi : (slot >= 0 ? sb[b.nlds + slot] : 0ull);
    } else {
      row[r] = bad ? __longlong_as_double(0x7ff8000000000000ll)
                   : (slot >= 0 ? fix_value(sb, b, slot, S) : 0.0);
    }
  }
}

// Binning pass layout of the x-pass: the power of a tile's C x N modes is
// staged in LDS as pw[col][kx + kx / S] and re-read so that the 64 lanes of a
// wave see one column at kx spaced S = N / 64 apart: distinct |n| bins, hence
// few same-address collisions of the LDS atomics.  Rows of the C columns
// start 64 / C banks apart (N + N / S is a multiple of 64 words), so that the
// staging writes of a wave (C columns x 64 / C consecutive kx) fall in
// distinct banks.
template <typename T, int N, int C>
struct XStage {
  static constexpr int S = N >= 64 ? N / 64 : 1;
  static constexpr int WPE = (int)(sizeof(T) / 4);  // 4-byte words per staged value
  static constexpr int RPAD = 64 / (C * WPE) > 1 ? 64 / (C * WPE) : 1;
  static constexpr int PROW = N >= 64 ? N + N / S + RPAD : N;
  static constexpr long BYTES = (long)C * PROW * sizeof(T);
  __device__ __forceinline__ static int idx(int cc, int kx) {
    return cc * PROW + (N >= 64 ? kx + kx / S : kx);
  }
  // idx(cc, t + TPL e) - idx(cc, t) for t < TPL, when TPL is a multiple of
  // S: the points of a thread sit at constant offsets from its first
  template <int TPL>
  __host__ __device__ static constexpr int step() {
    static_assert(N < 64 || TPL % S == 0, "x-pass points per thread a multiple of S apart");
    return N >= 64 ? TPL + TPL / S : TPL;
  }
};

// Bins the staged power of one tile (row ky, packed columns col0 .. col0 +
// C - 1).  The modes n_x and -n_x of a column share |n|^2 and n_los^2 (for
// any line of sight), hence every bin, so work item j < N/2 bins the sum of
// the powers at kx = j and N - j; item 0 bins n_x = 0 and n_x = -N/2
// separately.  With 64-lane waves, item m = 64 * slot + lane covers column
// slot / S2 and j = lane * S2 + slot % S2 (distinct |n| bins across a wave:
// few same-address collisions of the LDS atomics); small workgroups take
// column m / IC and j = m % IC.
template <typename T, int N, int C, int THREADS>
__device__ __forceinline__ void bin_tile(const T* pws, unsigned long long* sbx, const BinSpec& b,
                                         int fs, int ky, int col0) {
  using XS = XStage<T, N, C>;
  constexpr int IC = N / 2;
  constexpr bool WAVEWISE = IC >= 64 && THREADS % 64 == 0;
  constexpr int S2 = IC >= 64 ? IC / 64 : 1;
  const int los = b.los;
  const int ny = signed_index(ky, N);
  const int ny2 = ny * ny;
  for (int m = threadIdx.x; m < C * IC; m += THREADS) {
    int cc_, j;
    if constexpr (WAVEWISE) {
      const int slot = (m >> 6);
      cc_ = slot / S2;
      j = (m & 63) * S2 + slot % S2;
    } else {
      cc_ = m / IC;
      j = m % IC;
    }
    const int nz = col0 + cc_;
    if (nz == 0) continue;
    const int nyz2 = ny2 + nz * nz;
    const int nl2_yz = los == 1 ? ny2 : nz * nz;
    if (j == 0) {
      constexpr int H = N / 2;
      accumulate<T>(sbx, b, fs, nyz2, los == 0 ? 0 : nl2_yz, T(2) * pws[XS::idx(cc_, 0)]);
      accumulate<T>(sbx, b, fs, H * H + nyz2, los == 0 ? H * H : nl2_yz,
                    T(2) * pws[XS::idx(cc_, H)]);
    } else {
      const T pw = pws[XS::idx(cc_, j)] + pws[XS::idx(cc_, N - j)];
      accumulate<T>(sbx, b, fs, j * j + nyz2, los == 0 ? j * j : nl2_yz, T(2) * pw);
    }
  }
}

// At least 4 waves per SIMD (at most 128 VGPRs): two 512-thread workgroups
// or one 1024-thread workgroup per CU.
template <typename T, int N>
__global__ void __launch_bounds__((XCfg<T, N>::THREADS)) __attribute__((amdgpu_waves_per_eu(4)))
    k_xpass_bin(const cpx<T>* __restrict__ mesh_a, const cpx<T>* __restrict__ mesh_b,
                const cpx<T>* __restrict__ tw, const cpx<T>* __restrict__ phase,
                const T* __restrict__ sinv, BinSpec b, double* __restrict__ partials,
                cpx<T>* __restrict__ side_a, cpx<T>* __restrict__ side_b) {
  using Cf = XCfg<T, N>;
  constexpr int E = Cf::E, TPL = Cf::TPL, C = Cf::C, CHUNKS = Cf::CHUNKS;
  __shared__ cpx<T> lds[Cf::LDS_ELEMS];
  __shared__ cpx<T> tws[stage_table_size<N, E>() + 1];
  // per-index factors, read for every mode: the interlacing phase
  // exp(i pi n / N) of the signed index n of i, and the compensation 1 / sinc^p
  __shared__ cpx<T> phx[N];
  __shared__ T sxs[N];
  extern __shared__ unsigned long long sbx[];
  zero_bins(sbx, b);
  const int fs = fix_shift(b);
  const cpx<T>* __restrict__ ph1 = phase + 3 * (N / 2);  // ph1[n] = exp(i pi n / N)
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    phx[i] = ph1[signed_index(i, N)];
    sxs[i] = sinv ? sinv[i] : T(1);
  }
  build_stage_table<T, N, E>(tws, TwGlobal<T>{tw, 1});  // ends with a barrier
  const TwStage<T, N, E> tw1{tws};
  const int c = threadIdx.x % C, t = threadIdx.x / C;
  const bool two = mesh_b != nullptr;
  LdsCols<T, C> lc{lds, c};
  using XS = XStage<T, N, C>;
  T* pws = reinterpret_cast<T*>(lds);
  static_assert(XS::BYTES <= (long)Cf::LDS_ELEMS * sizeof(cpx<T>), "staging");
  const int ntiles = N * CHUNKS;
  // The meshes arrive in the y-pass output layout (YLayout).  The lines of a
  // tile are loaded into registers one tile ahead: the loads of the next
  // tile are issued once the current tile's power is staged in LDS, so their
  // latency overlaps the binning of the current tile.
  using YL = YLayout<T, N>;
  static_assert(YL::CX == C, "y-pass layout built for this tile width");
  cpx<T> va[E], vb[E];
  // kx = t + TPL e: with TPL a multiple of BX the offsets of a thread's
  // points differ by a constant
  using Ix = typename YL::Ix;
  constexpr bool REG = TPL % YL::BX == 0;
  constexpr Ix kstep = REG ? (Ix)(TPL / YL::BX) * ((Ix)N * YL::BX * YL::W) : 0;
  auto issue_loads = [&](int tile_id) {
    const int tile = xcd_group_tile<YLayout<T, N>::G>(tile_id, ntiles);
    const int ky = tile / CHUNKS, cl = (tile % CHUNKS) * C + c;
    if constexpr (REG) {
      const Ix base = YL::at(t, ky, cl);
#pragma unroll
      for (int e = 0; e < E; ++e) va[e] = mesh_a[base + (Ix)e * kstep];
      if (two) {
#pragma unroll
        for (int e = 0; e < E; ++e) vb[e] = mesh_b[base + (Ix)e * kstep];
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) va[e] = mesh_a[YL::at(t + TPL * e, ky, cl)];
      if (two) {
#pragma unroll
        for (int e = 0; e < E; ++e) vb[e] = mesh_b[YL::at(t + TPL * e, ky, cl)];
      }
    }
  };
  if ((int)blockIdx.x < ntiles) issue_loads(blockIdx.x);
  for (int tile_id = blockIdx.x; tile_id < ntiles; tile_id += gridDim.x) {
    const int tile = xcd_group_tile<YLayout<T, N>::G>(tile_id, ntiles);
    const int ky = tile / CHUNKS;
    const int col0 = (tile % CHUNKS) * C;
    const int col = col0 + c;
    const cpx<T> phy = phx[ky], phz = phx[col];
    const T s_yz = sxs[ky] * sxs[col];
    stockham<T, N, E, 1>(va, t, tw1, lc);
    if (two) stockham<T, N, E, 1>(vb, t, tw1, lc);
    const cpx<T> phyz = two ? cmul(phy, phz) : cpx<T>{T(1), T(0)};
    const int pbase = XS::idx(c, t);
    __syncthreads();  // every wave is done with the FFT exchanges
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kx = t + TPL * e;
      if (col == 0) {
        // packed kz = 0 / N/2 column: handed to k_plane_bin
        side_a[(size_t)kx * N + ky] = va[e];
        if (two) side_b[(size_t)kx * N + ky] = vb[e];
        continue;
      }
      cpx<T> cc = va[e];
      if (two) {
        const cpx<T> bb = cmul(cmul(phx[kx], phyz), vb[e]);
        cc = {T(0.5) * (cc.x + bb.x), T(0.5) * (cc.y + bb.y)};
      }
      T pw = cc.x * cc.x + cc.y * cc.y;
      if (sinv) {
        const T s = sxs[kx] * s_yz;
        pw *= s * s;
      }
      pws[pbase + e * XS::template step<TPL>()] = pw;
    }
    __syncthreads();
    if (tile_id + (int)gridDim.x < ntiles) issue_loads(tile_id + (int)gridDim.x);
    bin_tile<T, N, C, Cf::THREADS>(pws, sbx, b, fs, ky, col0);
    __syncthreads();  // the staged power is read before the next tile's FFT reuses the LDS
  }
  flush_bins(sbx, b, fs, partials + (size_t)blockIdx.x * 2 * b.nsum);
}

// One thread per (kx, ky): modes (kx, ky, 0) and (kx, ky, N/2), weight h = 1.
// With zb: cross = 0 combines the interlaced pair, cross = 1 bins the cross
// power Re(a conj(b)) of two spectra.
template <typename T>
__global__ void __launch_bounds__(256)
    k_plane_bin(int N, const cpx<T>* __restrict__ za, const cpx<T>* __restrict__ zb, size_t zs,
                const cpx<T>* __restrict__ phase, const T* __restrict__ sinv, BinSpec b,
                double* __restrict__ partials, int cross) {
  extern __shared__ unsigned long long sbx[];
  zero_bins(sbx, b);
  const int fs = fix_shift(b);
  __syncthreads();
  const int mask = N - 1;
  const int los = b.los;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < N * N;
       idx += gridDim.x * blockDim.x) {
    const int kx = idx / N, ky = idx % N;
    const int px = (N - kx) & mask, py = (N - ky) & mask;
    const int nx = signed_index(kx, N), ny = signed_index(ky, N);
    cpx<T> pa[2], pb[2];
    {
      const cpx<T> z = za[((size_t)kx * N + ky) * zs];
      const cpx<T> zp = cconj(za[((size_t)px * N + py) * zs]);
      const cpx<T> s = cadd(z, zp), d = csub(z, zp);
      pa[0] = {T(0.5) * s.x, T(0.5) * s.y};   // (Z + conj Z') / 2
      pa[1] = {T(0.5) * d.y, -T(0.5) * d.x};  // (Z - conj Z') / (2i)
    }
    if (zb) {
      const cpx<T> z = zb[((size_t)kx * N + ky) * zs];
      const cpx<T> zp = cconj(zb[((size_t)px * N + py) * zs]);
      const cpx<T> s = cadd(z, zp), d = csub(z, zp);
      pb[0] = {T(0.5) * s.x, T(0.5) * s.y};
      pb[1] = {T(0.5) * d.y, -T(0.5) * d.x};
    }
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
      const int nz = pl == 0 ? 0 : N / 2;
      cpx<T> cc = pa[pl];
      T pw;
      if (zb && cross) {
        pw = cc.x * pb[pl].x + cc.y * pb[pl].y;
      } else {
        if (zb) {
          const cpx<T> bb = cmul(phase[nx + ny + nz + 3 * (N / 2)], pb[pl]);
          cc = {T(0.5) * (cc.x + bb.x), T(0.5) * (cc.y + bb.y)};
        }
        pw = cc.x * cc.x + cc.y * cc.y;
      }
      if (sinv) {
        const T s = sinv[kx] * sinv[ky] * sinv[nz];
        pw *= s * s;
      }
      const int n2 = nx * nx + ny * ny + nz * nz;
      const int nl = los == 0 ? nx : (los == 1 ? ny : nz);
      accumulate<T>(sbx, b, fs, n2, nl * nl, pw);
    }
  }
  __syncthreads();
  flush_bins(sbx, b, fs, partials + (size_t)blockIdx.x * 2 * b.nsum);
}

// Stand-alone binning of a packed spectrum, columns kz' >= 1 (h = 2): |c|^2,
// or Re(c conj(c2)) when a second spectrum is given (cross power).  lw < 0:
// the plain packed layout; otherwise the y-pass output layout with groups of
// 2^lw columns and x blocks of 2^lbx (YLayout), walked in its storage order:
// the linear index holds, from the lowest bits up, col % W, kx % BX, ky,
// kx / BX and col / W.
template <typename T>
__global__ void __launch_bounds__(256)
    k_bin_packed(int N, const cpx<T>* __restrict__ cm, const cpx<T>* __restrict__ cm2, BinSpec b,
                 double* __restrict__ partials, int lw, int lbx) {
  extern __shared__ unsigned long long sbx[];
  zero_bins(sbx, b);
  const int fs = fix_shift(b);
  __syncthreads();
  const int NC = N / 2;
  const size_t total = (size_t)N * N * NC;
  const int los = b.los;
  const int ln = __ffs(N) - 1;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    int col, kx, ky;
    if (lw < 0) {
      col = (int)(idx % NC);
      const size_t rest = idx / NC;
      ky = (int)(rest % N);
      kx = (int)(rest / N);
    } else {
      col = (int)(((idx >> (lw + 2 * ln)) << lw) | (idx & ((1u << lw) - 1)));
      ky = (int)((idx >> (lw + lbx)) & (size_t)(N - 1));
      kx = (int)((((idx >> (lw + lbx + ln)) & (size_t)((N >> lbx) - 1)) << lbx) |
                 ((idx >> lw) & ((1u << lbx) - 1)));
    }
    if (col == 0) continue;
    const int nx = signed_index(kx, N), ny = signed_index(ky, N), nz = col;
    const cpx<T> cc = cm[idx];
    const cpx<T> dd = cm2 ? cm2[idx] : cc;
    const T pw = cc.x * dd.x + cc.y * dd.y;
    const int n2 = nx * nx + ny * ny + nz * nz;
    const int nl = los == 0 ? nx : (los == 1 ? ny : nz);
    accumulate<T>(sbx, b, fs, n2, nl * nl, T(2) * pw);
  }
  __syncthreads();
  flush_bins(sbx, b, fs, partials + (size_t)blockIdx.x * 2 * b.nsum);
}

// Cross sums of one field with up to four others in one pass: for each
// mode of the (packed or y-layout, as k_bin_packed) spectra, column kz' >= 1,
// h = 2, the k-bin sums of Re(c conj(d_i)), d_i = others.p[i] or c itself
// when NULL.  Field i's block sums go to partials + i * pstride.  The binning
// is plain k bins (no mu bins, no poles).
struct OtherFields {
  const void* p[4];
};

template <typename T>
__global__ void __launch_bounds__(256)
    k_bin_fields(int N, const cpx<T>* __restrict__ cm, OtherFields others, int nf, BinSpec b,
                 double* __restrict__ partials, size_t pstride, int lw, int lbx) {
  extern __shared__ double sb[];
  zero_bins(sb, nf * b.nsum);
  __syncthreads();
  const int NC = N / 2;
  const size_t total = (size_t)N * N * NC;
  const int ln = __ffs(N) - 1;
  const cpx<T>* __restrict__ d[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) d[i] = static_cast<const cpx<T>*>(others.p[i]);
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    int col, kx, ky;
    if (lw < 0) {
      col = (int)(idx % NC);
      const size_t rest = idx / NC;
      ky = (int)(rest % N);
      kx = (int)(rest / N);
    } else {
      col = (int)(((idx >> (lw + 2 * ln)) << lw) | (idx & ((1u << lw) - 1)));
      ky = (int)((idx >> (lw + lbx)) & (size_t)(N - 1));
      kx = (int)((((idx >> (lw + lbx + ln)) & (size_t)((N >> lbx) - 1)) << lbx) |
                 ((idx >> lw) & ((1u << lbx) - 1)));
    }
    if (col == 0) continue;
    const int nx = signed_index(kx, N), ny = signed_index(ky, N);
    const int k = kbin_of(nx * nx + ny * ny + col * col, b);
    if (k < 0) continue;
    const cpx<T> c = cm[idx];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i < nf) {
        const cpx<T> e = d[i] ? d[i][idx] : c;
        atomicAdd(&sb[i * b.nsum + k], (double)(T(2) * (c.x * e.x + c.y * e.y)));
      }
    }
  }
  __syncthreads();
  for (int i = 0; i < nf; ++i)
    flush_bins(sb + i * b.nsum, b.nsum,
               partials + i * pstride + (size_t)blockIdx.x * 2 * b.nsum);
}

// result[s] = sum_g partials[g][src(s)]; the slots of an ell = 0 pole take
// the sum of the plain power slots.  64 slots per workgroup, 16 lanes per
// slot: lane l sums the rows g = l, l + 16, ... in increasing g, then the 16
// lane sums are added in lane order -- a fixed order, so the result depends
// only on the partial rows.
__global__ void __launch_bounds__(1024)
    k_reduce(const double* __restrict__ partials, int ngroups, BinSpec b,
             double* __restrict__ result) {
  // rows of 2 nsum words; exact rows are 128-bit integers, added exactly (the
  // order does not matter), float64 rows are added in a fixed order
  __shared__ unsigned long long part_lo[16][64], part_hi[16][64];
  __shared__ int part_bad[16][64];
  const int slot_in = threadIdx.x & 63, lane = threadIdx.x >> 6;
  const int s = blockIdx.x * 64 + slot_in;
  const size_t stride = 2 * (size_t)b.nsum;
  int src = s;
  if (s < b.nsum && s >= b.nk && s < b.nk * (1 + b.npoles)) {
    const int pi = s / b.nk - 1;
    if ((b.zero_mask >> pi) & 1) src = s % b.nk;
  }
  constexpr int AHEAD = 8;
  if (b.exact) {
    const unsigned long long* w = reinterpret_cast<const unsigned long long*>(partials);
    unsigned long long lo = 0, hi = 0;
    int bad = 0;
    if (s < b.nsum) {
      for (int g0 = lane; g0 < ngroups; g0 += 16 * AHEAD) {
        unsigned long long vl[AHEAD], vh[AHEAD];
#pragma unroll
        for (int k = 0; k < AHEAD; ++k) {
          const int g = g0 + 16 * k;
          vl[k] = g < ngroups ? w[(size_t)g * stride + src] : 0ull;
          vh[k] = g < ngroups ? w[(size_t)g * stride + b.nsum + src] : 0ull;
        }
#pragma unroll
        for (int k = 0; k < AHEAD; ++k) {
          if (vh[k] == kFixNanHi && vl[k] == kFixNanLo) bad = 1;
          if (b.fix_hb == 32) {
            // low words count below 2^64; move their upper half to the high word
            lo += vl[k] & 0xffffffffull;
            hi += vh[k] + (vl[k] >> 32);
          } else {
            const unsigned long long old = lo;
            lo += vl[k];
            hi += vh[k] + (lo < old ? 1ull : 0ull);
          }
        }
      }
    }
    part_lo[lane][slot_in] = lo;
    part_hi[lane][slot_in] = hi;
    part_bad[lane][slot_in] = bad;
    __syncthreads();
    if (lane == 0 && s < b.nsum) {
      unsigned long long tl = 0, th = 0;
      int tb = 0;
#pragma unroll
      for (int l = 0; l < 16; ++l) {
        if (b.fix_hb == 32) {
          tl += part_lo[l][slot_in] & 0xffffffffull;
          th += part_hi[l][slot_in] + (part_lo[l][slot_in] >> 32);
        } else {
          const unsigned long long old = tl;
          tl += part_lo[l][slot_in];
          th += part_hi[l][slot_in] + (tl < old ? 1ull : 0ull);
        }
        tb |= part_bad[l][slot_in];
      }
      result[s] = tb ? __longlong_as_double(0x7ff8000000000000ll)
                     : fix_words_value(tl, th, fix_shift(b), b.fix_hb);
    }
    return;
  }
  double acc = 0.0;
  if (s < b.nsum) {
    // eight rows' loads in flight, then added in the same order (g = lane,
    // lane + 16, ...); a row past the end adds an exact zero
    for (int g0 = lane; g0 < ngroups; g0 += 16 * AHEAD) {
      double v[AHEAD];
#pragma unroll
      for (int k = 0; k < AHEAD; ++k) {
        const int g = g0 + 16 * k;
        v[k] = g < ngroups ? partials[(size_t)g * stride + src] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < AHEAD; ++k) acc += v[k];
    }
  }
  double* part = reinterpret_cast<double*>(&part_lo[0][0]);
  part[lane * 64 + slot_in] = acc;
  __syncthreads();
  if (lane == 0 && s < b.nsum) {
    double tot = 0.0;
#pragma unroll
    for (int l = 0; l < 16; ++l) tot += part[l * 64 + slot_in];
    result[s] = tot;
  }
}

// Plan time: per-bin counts (integers), sum h|n| and, for (k, mu) bins, counts,
// sum h|n| and sum h|mu|, over the r2c half grid with its Hermitian weights.
__global__ void __launch_bounds__(256)
    k_mode_tables(int N, BinSpec b, unsigned long long* __restrict__ partials) {
  // every slot is a 128-bit integer: low words [0, nslots), high words
  // [nslots, 2 nslots); counts use the low word only, the sums are fixed
  // point with kModeSumShift fraction bits (exact: a term h|n| < 2^13 has no
  // bits below 2^-40), so the tables do not depend on the order of the adds
  extern __shared__ unsigned long long sbw[];
  const int nslots = mode_table_slots(b.nk, b.nmu);
  for (int i = threadIdx.x; i < 2 * nslots; i += blockDim.x) sbw[i] = 0;
  __syncthreads();
  const int NH = N / 2 + 1;
  const size_t total = (size_t)N * N * NH;
  const int nk = b.nk, nmu = b.nmu, los = b.los;
  unsigned long long* cnt = sbw;
  constexpr int S = kModeSumShift;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int kz = (int)(idx % NH);
    const size_t rest = idx / NH;
    const int ky = (int)(rest % N), kx = (int)(rest / N);
    const int nx = signed_index(kx, N), ny = signed_index(ky, N), nz = kz;
    const int n2 = nx * nx + ny * ny + nz * nz;
    const int k = kbin_of(n2, b);
    if (k < 0) continue;
    const int h = (kz == 0 || kz == N / 2) ? 1 : 2;
    const double kn = sqrt((double)n2);
    atomicAdd(&cnt[k], (unsigned long long)h);
    fix_add<double>(sbw, nslots, nk + k, h * kn, S);
    if (nmu > 1) {
      const int nl = los == 0 ? nx : (los == 1 ? ny : nz);
      const int f = k * nmu + mubin_of(nl * nl, n2, nmu);
      atomicAdd(&cnt[2 * nk + f], (unsigned long long)h);
      fix_add<double>(sbw, nslots, 2 * nk + nk * nmu + f, h * kn, S);
      fix_add<double>(sbw, nslots, 2 * nk + 2 * nk * nmu + f, h * (double)abs(nl) / kn, S);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * nslots; i += blockDim.x)
    partials[(size_t)blockIdx.x * 2 * nslots + i] = sbw[i];
}

// Mode (nx, ny, nz) of a packed half spectrum, signed indices in
// [-N/2, N/2): columns 1 .. N/2 - 1 directly or through Hermitian symmetry,
// the planes nz = 0 and nz = -N/2 (= N/2) unpacked from column 0 with the
// partner (-nx, -ny).
template <typename T>
__device__ __forceinline__ cpx<T> packed_mode(const cpx<T>* __restrict__ cm, int N, int nx,
                                              int ny, int nz) {
  const int mask = N - 1, NC = N / 2;
  const size_t me = ((size_t)(nx & mask) * N + (ny & mask)) * NC;
  const size_t mirror = ((size_t)((-nx) & mask) * N + ((-ny) & mask)) * NC;
  if (nz > 0) return cm[me + nz];
  if (nz < 0 && nz > -NC) return cconj(cm[mirror - nz]);
  const cpx<T> z = cm[me], zp = cconj(cm[mirror]);
  const cpx<T> s = cadd(z, zp), d = csub(z, zp);
  if (nz == 0) return {T(0.5) * s.x, T(0.5) * s.y};
  return {T(0.5) * d.y, -T(0.5) * d.x};
}

// Projected power (ProjectedFFTPower): the modes whose wave numbers vanish
// on the projected axes, every mode of the full grid of the kept axes once
// (keep: bit a set for a kept axis a; one or two bits).  Sums per k-bin:
// [0, nk) |c|^2, [nk, 2 nk) mode counts, [2 nk, 3 nk) |n|.
template <typename T>
__global__ void __launch_bounds__(256)
    k_bin_projected(int N, const cpx<T>* __restrict__ cm, int keep, BinSpec b,
                    double* __restrict__ partials) {
  extern __shared__ double sb[];
  const int nk = b.nk;
  zero_bins(sb, 3 * nk);
  __syncthreads();
  const int a0 = (keep & 1) ? 0 : ((keep & 2) ? 1 : 2);
  const int rest = keep & ~(1 << a0);
  const int a1 = rest ? ((rest & 2) ? 1 : 2) : -1;
  const int items = a1 >= 0 ? N * N : N;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < items;
       idx += gridDim.x * blockDim.x) {
    int n3[3] = {0, 0, 0};
    n3[a0] = signed_index(idx % N, N);
    if (a1 >= 0) n3[a1] = signed_index(idx / N, N);
    const int n2 = n3[0] * n3[0] + n3[1] * n3[1] + n3[2] * n3[2];
    const int k = kbin_of(n2, b);
    if (k < 0) continue;
    const cpx<T> c = packed_mode(cm, N, n3[0], n3[1], n3[2]);
    atomicAdd(&sb[k], (double)(c.x * c.x + c.y * c.y));
    atomicAdd(&sb[nk + k], 1.0);
    atomicAdd(&sb[2 * nk + k], sqrt((double)n2));
  }
  __syncthreads();
  flush_bins(sb, 3 * nk, partials + (size_t)blockIdx.x * 2 * 3 * nk);  // rows of 2 nsum words
}

// Sums the mode-table partial rows; integer slots are summed as integers.
__global__ void k_reduce_tables(const unsigned long long* __restrict__ partials, int ngroups,
                                int nk, int nmu, double* __restrict__ out) {
  const int nslots = mode_table_slots(nk, nmu);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslots) return;
  const bool integer = s < nk || (nmu > 1 && s >= 2 * nk && s < 2 * nk + nk * nmu);
  unsigned long long lo = 0, hi = 0;
  for (int g = 0; g < ngroups; ++g) {
    const unsigned long long* row = partials + (size_t)g * 2 * nslots;
    const unsigned long long old = lo;
    lo += row[s];
    hi += row[nslots + s] + (lo < old ? 1ull : 0ull);
  }
  if (integer) {
    reinterpret_cast<unsigned long long*>(out)[s] = lo;
  } else {
    out[s] = fix_words_value(lo, hi, kModeSumShift);
  }
}

// Stand-alone interlacing + compensation on packed spectra (in place).
// Columns kz' >= 1 are independent; in column 0 the thread of the smaller
// of (kx, ky) and its partner (-kx, -ky) unpacks both, processes the four
// plane modes and repacks them.
template <typename T>
__device__ __forceinline__ cpx<T> comp_mode(cpx<T> a, const cpx<T>* b, int nx, int ny, int nz,
                                            int kx, int ky, int iz, int N,
                                            const cpx<T>* __restrict__ phase,
                                            const T* __restrict__ sinv) {
  if (b) {
    const cpx<T> bb = cmul(phase[nx + ny + nz + 3 * (N / 2)], *b);
    a = {T(0.5) * (a.x + bb.x), T(0.5) * (a.y + bb.y)};
  }
  if (sinv) a = cscale(a, sinv[kx] * sinv[ky] * sinv[iz]);
  return a;
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_compensate(int N, cpx<T>* __restrict__ cm, const cpx<T>* __restrict__ cb,
                 const cpx<T>* __restrict__ phase, const T* __restrict__ sinv) {
  const int NC = N / 2;
  const size_t total = (size_t)N * N * NC;
  const int mask = N - 1;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(idx % NC);
    const size_t rest = idx / NC;
    const int ky = (int)(rest % N), kx = (int)(rest / N);
    const int nx = signed_index(kx, N), ny = signed_index(ky, N);
    if (col != 0) {
      const cpx<T> bv = cb ? cb[idx] : cpx<T>{T(0), T(0)};
      cm[idx] = comp_mode<T>(cm[idx], cb ? &bv : nullptr, nx, ny, col, kx, ky, col, N, phase, sinv);
      continue;
    }
    const int px = (N - kx) & mask, py = (N - ky) & mask;
    const size_t me = (size_t)kx * N + ky, pa = (size_t)px * N + py;
    if (me > pa) continue;
    const cpx<T> z = cm[me * NC], zp = cm[pa * NC];
    const int pnx = signed_index(px, N), pny = signed_index(py, N);
    // unpack: plane 0 value (Z + conj Z') / 2, plane N/2 value (Z - conj Z') / (2i)
    auto unpack = [](cpx<T> u, cpx<T> w, cpx<T>& p0, cpx<T>& p1) {
      const cpx<T> s = cadd(u, cconj(w)), d = csub(u, cconj(w));
      p0 = {T(0.5) * s.x, T(0.5) * s.y};
      p1 = {T(0.5) * d.y, -T(0.5) * d.x};
    };
    cpx<T> a0, a1, q0, q1;
    unpack(z, zp, a0, a1);
    unpack(zp, z, q0, q1);
    cpx<T> b0, b1, r0, r1;
    if (cb) {
      const cpx<T> w = cb[me * NC], wp = cb[pa * NC];
      unpack(w, wp, b0, b1);
      unpack(wp, w, r0, r1);
    }
    a0 = comp_mode<T>(a0, cb ? &b0 : nullptr, nx, ny, 0, kx, ky, 0, N, phase, sinv);
    a1 = comp_mode<T>(a1, cb ? &b1 : nullptr, nx, ny, N / 2, kx, ky, N / 2, N, phase, sinv);
    q0 = comp_mode<T>(q0, cb ? &r0 : nullptr, pnx, pny, 0, px, py, 0, N, phase, sinv);
    q1 = comp_mode<T>(q1, cb ? &r1 : nullptr, pnx, pny, N / 2, px, py, N / 2, N, phase, sinv);
    // After interlacing the kz = N/2 plane is no longer Hermitian (its phase
    // uses n_z = +N/2 for a mode and its mirror), so it cannot share the packed
    // column; it is set to zero (all its modes have |n| >= N/2, outside every
    // binning allowed for interlaced meshes).
    if (cb) {
      a1 = {T(0), T(0)};
      q1 = {T(0), T(0)};
    }
    // repack Z = p0 + i p1
    cm[me * NC] = {a0.x - a1.y, a0.y + a1.x};
    if (pa != me) cm[pa * NC] = {q0.x - q1.y, q0.y + q1.x};
  }
}

// ---------------------------------------------------------------- launchers

// Workgroups of the persistent x-pass: as many as the device holds at once
// (a second round would only add a tail and partial rows to reduce), never
// more than the tiles.  Residency per CU from the LDS of a workgroup (static
// + nsum float64 bins) and from the waves (at most 128 VGPRs: 4 waves per
// SIMD, 16 per CU).
template <typename T, int N>
static int xpass_groups_t(size_t bin_bytes) {
  using Cf = XCfg<T, N>;
  const long tiles = (long)N * Cf::CHUNKS;
  const size_t lds = ((size_t)Cf::LDS_ELEMS + stage_table_size<N, Cf::E>() + 1 + N) *
                         sizeof(cpx<T>) + (size_t)N * sizeof(T) + bin_bytes;
  long by_lds = (long)(kLdsBytesPerGroup / (lds > 0 ? lds : 1));
  const long waves = (Cf::THREADS + 63) / 64;
  long by_waves = 16 / (waves > 0 ? waves : 1);
  long per_cu = by_lds < by_waves ? by_lds : by_waves;
  if (per_cu < 1) per_cu = 1;
  const long groups = per_cu * kComputeUnits;
  return (int)(tiles < groups ? tiles : groups);
}

int xpass_bin_groups(int dtype, int nmesh, size_t bin_bytes) {
#define PK_T(NN) \
  case NN: return dtype == PK_F32 ? xpass_groups_t<float, NN>(bin_bytes) : xpass_groups_t<double, NN>(bin_bytes);
  switch (nmesh) {
    PK_T(8) PK_T(16) PK_T(32) PK_T(64) PK_T(128) PK_T(256) PK_T(512) PK_T(1024) PK_T(2048)
    default: return 0;
  }
#undef PK_T
}

template <typename T, int N>
static size_t xpass_static_lds_t() {
  using Cf = XCfg<T, N>;
  return ((size_t)Cf::LDS_ELEMS + stage_table_size<N, Cf::E>() + 1 + N) * sizeof(cpx<T>) +
         (size_t)N * sizeof(T);
}

size_t xpass_static_lds(int dtype, int nmesh) {
#define PK_T(NN) case NN: return dtype == PK_F32 ? xpass_static_lds_t<float, NN>() : xpass_static_lds_t<double, NN>();
  switch (nmesh) {
    PK_T(8) PK_T(16) PK_T(32) PK_T(64) PK_T(128) PK_T(256) PK_T(512) PK_T(1024) PK_T(2048)
    default: return 0;
  }
#undef PK_T
}

int plane_bin_groups(int nmesh) {
  const long threads = (long)nmesh * nmesh;
  const long g = (threads + 255) / 256;
  return (int)(g < 256 ? g : 256);
}

int mode_table_groups(int nmesh) {
  const long total = (long)nmesh * nmesh * (nmesh / 2 + 1);
  const long g = (total + 255) / 256;
  return (int)(g < 1024 ? g : 1024);
}

size_t bin_lds_bytes(const BinSpec& b) { return ((size_t)b.nlds * 2 + 1) * sizeof(unsigned long long); }

template <typename T, int N>
static hipError_t xpass_bin_t(const void* mesh_a, const void* mesh_b, const MeshTables& t,
                              int order, int compensated, const BinSpec& b, double* partials,
                              void* side_a, void* side_b, hipStream_t s, int want) {
  using Cf = XCfg<T, N>;
  int groups = xpass_bin_groups(sizeof(T) == 4 ? PK_F32 : PK_F64, N, bin_lds_bytes(b));
  if (want > 0 && want < groups) groups = want;
  const T* sinv = compensated ? static_cast<const T*>(t.sinc_inv) + (size_t)(order - 2) * N
                              : nullptr;
  hipLaunchKernelGGL((k_xpass_bin<T, N>), dim3(groups), dim3(Cf::THREADS), bin_lds_bytes(b), s,
                     static_cast<const cpx<T>*>(mesh_a), static_cast<const cpx<T>*>(mesh_b),
                     static_cast<const cpx<T>*>(t.tw), static_cast<const cpx<T>*>(t.phase), sinv,
                     b, partials, static_cast<cpx<T>*>(side_a), static_cast<cpx<T>*>(side_b));
  return hipGetLastError();
}

hipError_t launch_xpass_bin(int dtype, int nmesh, const void* mesh_a, const void* mesh_b,
                            const MeshTables& t, int order, int compensated, const BinSpec& b,
                            double* partials, void* side_a, void* side_b, hipStream_t s,
                            int groups) {
#define PK_XB(T)                                                                              \
  switch (nmesh) {                                                                            \
    case 8: return xpass_bin_t<T, 8>(mesh_a, mesh_b, t, order, compensated, b, partials, side_a, side_b, s, groups); \
    case 16: return xpass_bin_t<T, 16>(mesh_a, mesh_b, t, order, compensated, b, partials, side_a, side_b, s, groups); \
    case 32: return xpass_bin_t<T, 32>(mesh_a, mesh_b, t, order, compensated, b, partials, side_a, side_b, s, groups); \
    case 64: return xpass_bin_t<T, 64>(mesh_a, mesh_b, t, order, compensated, b, partials, side_a, side_b, s, groups); \
    case 128: return xpass_bin_t<T, 128>(mesh_a, mesh_b, t, order, compensated, b, partials, side_a, side_b, s, groups); \
    case 256: return xpass_bin_t<T, 256>(mesh_a, mesh_b, t, order, compensated, b, partials, side_a, side_b, s, groups); \
    case 512: return xpass_bin_t<T, 512>(mesh_a, mesh_b, t, order, compensated, b, partials, side_a, side_b, s, groups); \
    case 1024: return xpass_bin_t<T, 1024>(mesh_a, mesh_b, t, order, compensated, b, partials, side_a, side_b, s, groups); \
    case 2048: return xpass_bin_t<T, 2048>(mesh_a, mesh_b, t, order, compensated, b, partials, side_a, side_b, s, groups); \
    default: return hipErrorInvalidValue;                                                    \
  }
  if (dtype == PK_F32) {
    PK_XB(float)
  } else {
    PK_XB(double)
  }
#undef PK_XB
}

// log2 of the column group width W and of the x block BX of YLayout<T, N>.
template <typename T>
static bool ylayout_bits(int nmesh, int* lw, int* lbx) {
  switch (nmesh) {
#define PK_YB(NN)                             \
  case NN:                                    \
    *lw = ilog2(YLayout<T, NN>::W);           \
    *lbx = ilog2(YLayout<T, NN>::BX);         \
    return true;
    PK_YB(8) PK_YB(16) PK_YB(32) PK_YB(64) PK_YB(128) PK_YB(256) PK_YB(512) PK_YB(1024)
    PK_YB(2048)
#undef PK_YB
    default: return false;
  }
}

int bin_packed_groups(int nmesh) {
  const size_t total = (size_t)nmesh * nmesh * (nmesh / 2);
  const size_t g = (total + 255) / 256;
  return (int)(g > 1024 ? 1024 : g);
}

hipError_t launch_bin_packed(int dtype, int nmesh, const void* cmesh, const void* cmesh2,
                             const BinSpec& b, double* partials, hipStream_t s, int ylayout,
                             int max_groups) {
  size_t g = (size_t)bin_packed_groups(nmesh);
  if (max_groups > 0 && g > (size_t)max_groups) g = (size_t)max_groups;
  int lw = -1, lbx = 0;
  if (ylayout) {
    const bool ok = dtype == PK_F32 ? ylayout_bits<float>(nmesh, &lw, &lbx)
                                    : ylayout_bits<double>(nmesh, &lw, &lbx);
    if (!ok) return hipErrorInvalidValue;
  }
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_bin_packed<float>, dim3((unsigned)g), dim3(256), bin_lds_bytes(b), s,
                       nmesh, static_cast<const cpx<float>*>(cmesh),
                       static_cast<const cpx<float>*>(cmesh2), b, partials, lw, lbx);
  else
    hipLaunchKernelGGL(k_bin_packed<double>, dim3((unsigned)g), dim3(256), bin_lds_bytes(b), s,
                       nmesh, static_cast<const cpx<double>*>(cmesh),
                       static_cast<const cpx<double>*>(cmesh2), b, partials, lw, lbx);
  return hipGetLastError();
}

hipError_t launch_bin_fields(int dtype, int nmesh, const void* cmesh, const void* const* others,
                             int nf, const BinSpec& b, double* partials, size_t pstride,
                             hipStream_t s, int ylayout) {
  if (nf < 1 || nf > 4) return hipErrorInvalidValue;
  const size_t total = (size_t)nmesh * nmesh * (nmesh / 2);
  size_t g = (total + 255) / 256;
  if (g > 1024) g = 1024;
  int lw = -1, lbx = 0;
  if (ylayout) {
    const bool ok = dtype == PK_F32 ? ylayout_bits<float>(nmesh, &lw, &lbx)
                                    : ylayout_bits<double>(nmesh, &lw, &lbx);
    if (!ok) return hipErrorInvalidValue;
  }
  OtherFields of{};
  for (int i = 0; i < nf; ++i) of.p[i] = others[i];
  const size_t lds = (size_t)nf * b.nsum * sizeof(double);
  if (lds > kLdsBytesPerGroup) return hipErrorInvalidValue;
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_bin_fields<float>, dim3((unsigned)g), dim3(256), lds, s, nmesh,
                       static_cast<const cpx<float>*>(cmesh), of, nf, b, partials, pstride, lw,
                       lbx);
  else
    hipLaunchKernelGGL(k_bin_fields<double>, dim3((unsigned)g), dim3(256), lds, s, nmesh,
                       static_cast<const cpx<double>*>(cmesh), of, nf, b, partials, pstride, lw,
                       lbx);
  return hipGetLastError();
}

hipError_t launch_plane_bin(int dtype, int nmesh, const void* za, const void* zb, size_t zstride,
                            const MeshTables& t, int order, int compensated, const BinSpec& b,
                            double* partials, hipStream_t s, int cross, int groups) {
  const int g = groups > 0 ? groups : plane_bin_groups(nmesh);
  if (dtype == PK_F32) {
    const float* sinv = compensated ? static_cast<const float*>(t.sinc_inv) + (size_t)(order - 2) * nmesh : nullptr;
    hipLaunchKernelGGL(k_plane_bin<float>, dim3(g), dim3(256), bin_lds_bytes(b), s, nmesh,
                       static_cast<const cpx<float>*>(za), static_cast<const cpx<float>*>(zb),
                       zstride, static_cast<const cpx<float>*>(t.phase), sinv, b, partials, cross);
  } else {
    const double* sinv = compensated ? static_cast<const double*>(t.sinc_inv) + (size_t)(order - 2) * nmesh : nullptr;
    hipLaunchKernelGGL(k_plane_bin<double>, dim3(g), dim3(256), bin_lds_bytes(b), s, nmesh,
                       static_cast<const cpx<double>*>(za), static_cast<const cpx<double>*>(zb),
                       zstride, static_cast<const cpx<double>*>(t.phase), sinv, b, partials, cross);
  }
  return hipGetLastError();
}

int projected_groups(int nmesh, int keep) {
  const long items = (keep & (keep - 1)) ? (long)nmesh * nmesh : nmesh;
  const long g = (items + 255) / 256;
  return (int)(g < 64 ? g : 64);
}

hipError_t launch_bin_projected(int dtype, int nmesh, const void* cmesh, int keep,
                                const BinSpec& b, double* partials, hipStream_t s) {
  const int g = projected_groups(nmesh, keep);
  const size_t lds = (size_t)3 * b.nk * sizeof(double);
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_bin_projected<float>, dim3(g), dim3(256), lds, s, nmesh,
                       static_cast<const cpx<float>*>(cmesh), keep, b, partials);
  else
    hipLaunchKernelGGL(k_bin_projected<double>, dim3(g), dim3(256), lds, s, nmesh,
                       static_cast<const cpx<double>*>(cmesh), keep, b, partials);
  return hipGetLastError();
}

// The largest |component| of one or two arrays of reals (count each): the
// bound of the terms that a binning of spectra without weight sums adds
// (|c|^2 <= 2 max^2).  out: one float64 (as its bits; non-negative doubles
// order like their bit patterns), zeroed beforehand.  NaN components are
// skipped here; the binning flags them.
template <typename T>
__global__ void __launch_bounds__(256)
    k_absmax(const T* __restrict__ a, const T* __restrict__ b, size_t count,
             unsigned long long* __restrict__ out) {
  double mx = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256) {
    mx = fmax(mx, fabs((double)a[i]));
    if (b) mx = fmax(mx, fabs((double)b[i]));
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(mx));
}

hipError_t launch_absmax(int dtype, const void* a, const void* b, size_t count, double* out,
                         hipStream_t s) {
  hipError_t e = launch_fill_zero(out, sizeof(double), s);
  if (e != hipSuccess) return e;
  size_t g = (count + 255) / 256;
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  auto* o = reinterpret_cast<unsigned long long*>(out);
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_absmax<float>, dim3((unsigned)g), dim3(256), 0, s,
                       static_cast<const float*>(a), static_cast<const float*>(b), count, o);
  else
    hipLaunchKernelGGL(k_absmax<double>, dim3((unsigned)g), dim3(256), 0, s,
                       static_cast<const double*>(a), static_cast<const double*>(b), count, o);
  return hipGetLastError();
}

// Squared bin edges on the device, with contraction off so that the product
// and the sum are rounded separately, as in the host table.
__global__ void __launch_bounds__(256)
    k_edges_squared(double kmin, double dk, int nk, double* __restrict__ e2) {
#pragma clang fp contract(off)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= nk; i += gridDim.x * blockDim.x) {
    const double e = kmin + (double)i * dk;
    e2[i] = e * e;
  }
}

hipError_t launch_edges_squared(double kmin, double dk, int nk, double* e2, hipStream_t s) {
  const int blocks = (nk + 1 + 255) / 256;
  hipLaunchKernelGGL(k_edges_squared, dim3(blocks), dim3(256), 0, s, kmin, dk, nk, e2);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int ngroups, const BinSpec& b, double* result,
                         hipStream_t s) {
  const int blocks = (b.nsum + 63) / 64;
  hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(1024), 0, s, partials, ngroups, b, result);
  return hipGetLastError();
}

hipError_t launch_mode_tables(int nmesh, const BinSpec& b, double* partials, int ngroups,
                              double* out, hipStream_t s) {
  const int nslots = mode_table_slots(b.nk, b.nmu);
  unsigned long long* words = reinterpret_cast<unsigned long long*>(partials);
  hipLaunchKernelGGL(k_mode_tables, dim3(ngroups), dim3(256),
                     (size_t)2 * nslots * sizeof(unsigned long long), s, nmesh, b, words);
  hipLaunchKernelGGL(k_reduce_tables, dim3((nslots + 255) / 256), dim3(256), 0, s, words,
                     ngroups, b.nk, b.nmu, out);
  return hipGetLastError();
}

hipError_t launch_compensate(int dtype, int nmesh, void* cmesh, const void* cmesh_b,
                             const MeshTables& t, int order, int compensated, hipStream_t s) {
  const size_t total = (size_t)nmesh * nmesh * (nmesh / 2);
  size_t g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  if (dtype == PK_F32) {
    const float* sinv = compensated ? static_cast<const float*>(t.sinc_inv) + (size_t)(order - 2) * nmesh : nullptr;
    hipLaunchKernelGGL(k_compensate<float>, dim3((unsigned)g), dim3(256), 0, s, nmesh,
                       static_cast<cpx<float>*>(cmesh), static_cast<const cpx<float>*>(cmesh_b),
                       static_cast<const cpx<float>*>(t.phase), sinv);
  } else {
    const double* sinv = compensated ? static_cast<const double*>(t.sinc_inv) + (size_t)(order - 2) * nmesh : nullptr;
    hipLaunchKernelGGL(k_compensate<double>, dim3((unsigned)g), dim3(256), 0, s, nmesh,
                       static_cast<cpx<double>*>(cmesh), static_cast<const cpx<double>*>(cmesh_b),
                       static_cast<const cpx<double>*>(t.phase), sinv);
  }
  return hipGetLastError();
}

}  // namespace pk
