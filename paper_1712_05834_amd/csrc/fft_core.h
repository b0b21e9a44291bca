// Device building blocks for the 1-D FFTs that make up the 3-D r2c transform
// (Sec. 3.3.1: RealField -> ComplexField).
//
// Formulation: Stockham autosort (Cochran et al. 1967; Van Loan, "Computational
// Frameworks for the FFT", 1992), radix 2^r stages with r <= 4.  A line of L
// complex points is owned by TPL = L / E threads; thread t holds the E points
// t + TPL * e in registers.  A radix-R stage of span p (the product of the
// radices already applied) takes, for butterfly i, the inputs i + m L / R,
// multiplies input m by W_{pR}^{m k} (k = i mod p), applies an in-register
// DFT_R and sends output m to position (i - k) R + k + m p.  Between stages
// the points are exchanged through LDS; in the last stage the output position
// equals the input position, so the transformed points stay in the same
// registers and the first load / last store can go straight to HBM.
#pragma once

#include <hip/hip_runtime.h>

namespace pk {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

// cos(2 pi j / 16) for j = 0 .. 15.
__host__ __device__ constexpr double cos16(int j) {
  switch (j & 15) {
    case 0: return 1.0;
    case 1: return 0.92387953251128675613;
    case 2: return 0.70710678118654752440;
    case 3: return 0.38268343236508977173;
    case 4: return 0.0;
    case 5: return -0.38268343236508977173;
    case 6: return -0.70710678118654752440;
    case 7: return -0.92387953251128675613;
    case 8: return -1.0;
    case 9: return -0.92387953251128675613;
    case 10: return -0.70710678118654752440;
    case 11: return -0.38268343236508977173;
    case 12: return 0.0;
    case 13: return 0.38268343236508977173;
    case 14: return 0.70710678118654752440;
    default: return 0.92387953251128675613;
  }
}
// sin(2 pi j / 16) = cos(2 pi (j - 4) / 16).
__host__ __device__ constexpr double sin16(int j) { return cos16(j - 4); }

// v * exp(-2 pi i k / R) for R dividing 16; k is a constant after unrolling,
// so the branches and table values fold at compile time.
template <typename T, int R>
__device__ __forceinline__ cpx<T> twiddle_const(int k, cpx<T> v) {
  const int j = (k * (16 / R)) & 15;
  if (j == 0) return v;
  if (j == 4) return {v.y, -v.x};   // * (-i)
  if (j == 8) return {-v.x, -v.y};  // * (-1)
  if (j == 12) return {-v.y, v.x};  // * (+i)
  const T c = static_cast<T>(cos16(j));
  const T s = static_cast<T>(sin16(j));
  return {v.x * c + v.y * s, v.y * c - v.x * s};
}

// In-register forward DFT of size R (R = 1, 2, 4, 8, 16), natural order in
// and out: radix-2 decimation in time, unrolled at compile time.
template <typename T, int R>
__device__ __forceinline__ void dft(cpx<T>* a) {
  if constexpr (R == 2) {
    const cpx<T> t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  } else if constexpr (R > 2) {
    constexpr int H = R / 2;
    cpx<T> ev[H], od[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
      ev[i] = a[2 * i];
      od[i] = a[2 * i + 1];
    }
    dft<T, H>(ev);
    dft<T, H>(od);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const cpx<T> t = twiddle_const<T, R>(k, od[k]);
      a[k] = cadd(ev[k], t);
      a[k + H] = csub(ev[k], t);
    }
  }
}

// Radix of the Stockham stage whose span is P, for a line of L points with
// E points per thread: the first stage takes the remainder 2^(log2 L mod log2 E)
// (or E), every later stage takes E.
template <int L, int E, int P>
__host__ __device__ constexpr int stage_radix() {
  constexpr int n = ilog2(L), e = ilog2(E);
  if constexpr (P == 1) {
    return (n % e) ? (1 << (n % e)) : E;
  } else {
    return E;
  }
}

// LDS view for lines stored column-interleaved: point j of column c at
// base[(j + j / 16) * C + c].  The extra row every 16 points spreads the
// early-stage stride-R writes over the banks.
// put_step / get_step address point j + m S.  (Here the index is formed per
// point: the column passes keep the per-point addresses in registers across
// their tile loop, and constant offsets from one slot -- as LdsLine uses --
// made the 1024^3 x-pass 4% slower.)
template <typename T, int C>
struct LdsCols {
  cpx<T>* base;
  int c;
  __device__ __forceinline__ void put(int j, cpx<T> v) { base[(j + (j >> 4)) * C + c] = v; }
  __device__ __forceinline__ cpx<T> get(int j) const { return base[(j + (j >> 4)) * C + c]; }
  template <int S>
  __device__ __forceinline__ void put_step(int j, int m, cpx<T> v) {
    put(j + m * S, v);
  }
  template <int S>
  __device__ __forceinline__ cpx<T> get_step(int j, int m) const {
    return get(j + m * S);
  }
};

template <int L>
__host__ __device__ constexpr int lds_pad_len() { return L + L / 16 + 1; }

// LDS view for one contiguous line: point j at base[j + j / 16].  Points
// j + m S with S a multiple of 16 sit m (S + S / 16) slots past point j:
// put_step / get_step address them as constant offsets from j's slot.
template <typename T>
struct LdsLine {
  cpx<T>* base;
  __device__ __forceinline__ int slot(int j) const { return j + (j >> 4); }
  __device__ __forceinline__ void put(int j, cpx<T> v) { base[slot(j)] = v; }
  __device__ __forceinline__ cpx<T> get(int j) const { return base[slot(j)]; }
  template <int S>
  __device__ __forceinline__ void put_step(int j, int m, cpx<T> v) {
    if constexpr (S % 16 == 0) {
      base[slot(j) + m * (S + S / 16)] = v;
    } else {
      put(j + m * S, v);
    }
  }
  template <int S>
  __device__ __forceinline__ cpx<T> get_step(int j, int m) const {
    if constexpr (S % 16 == 0) {
      return base[slot(j) + m * (S + S / 16)];
    } else {
      return get(j + m * S);
    }
  }
};

// Twiddle sources: W_Nt^j for the table length Nt (a power of two >= 4).
//  TwGlobal   the full table tw[j * s] in global memory;
//  TwQuarter  the first quarter q[r] = W_Nt^r, r < Nt / 4, kept in LDS; the
//             other quadrants follow from W^(r + a Nt/4) = (-i)^a W^r.
template <typename T>
struct TwGlobal {
  const cpx<T>* __restrict__ p;
  int s;
  __device__ __forceinline__ cpx<T> operator()(int j) const { return p[j * s]; }
  // twiddle m of butterfly k in the radix-R stage of span P of an L-point FFT
  template <int L, int P, int R>
  __device__ __forceinline__ cpx<T> stage(int k, int m) const {
    return (*this)(m * k * (L / (P * R)));
  }
};

template <typename T>
struct TwQuarter {
  const cpx<T>* q;
  int s;          // index stride (2 when an Nt/2-point FFT reads the Nt table)
  int log2q;      // log2(Nt / 4)
  __device__ __forceinline__ cpx<T> operator()(int j) const {
    const int jj = j * s;
    const int a = (jj >> log2q) & 3;
    const cpx<T> w = q[jj & ((1 << log2q) - 1)];
    if (a == 0) return w;
    if (a == 1) return {w.y, -w.x};
    if (a == 2) return {-w.x, -w.y};
    return {-w.y, w.x};
  }
  template <int L, int P, int R>
  __device__ __forceinline__ cpx<T> stage(int k, int m) const {
    return (*this)(m * k * (L / (P * R)));
  }
};

// Per-stage twiddle table in LDS: for the stage of span P and radix R the
// entries W_L^{m k L / (P R)}, k < P, m = 1 .. R-1, stored [k][m-1], built
// once per workgroup.  A butterfly then reads its R-1 twiddles from
// consecutive LDS words, with no index arithmetic and no quadrant selects.
template <int L, int E, int P>
__host__ __device__ constexpr int stage_table_offset() {
  if constexpr (P <= 1) {
    return 0;
  } else {
    // offset of span P = offset of the previous span + its entries
    constexpr int R0 = stage_radix<L, E, 1>();
    int off = 0, p = R0;  // the first stage (span 1) has no twiddles
    while (p < P) {
      off += p * (E - 1);
      p *= E;
    }
    return off;
  }
}

template <int L, int E>
__host__ __device__ constexpr int stage_table_size() {
  constexpr int R0 = stage_radix<L, E, 1>();
  int off = 0, p = R0;
  while (p < L) {
    off += p * (E - 1);
    p *= E;
  }
  return off;
}

template <typename T, int L, int E>
struct TwStage {
  const cpx<T>* t;
  template <int LL, int P, int R>
  __device__ __forceinline__ cpx<T> stage(int k, int m) const {
    static_assert(LL == L && R == E, "table built for this plan");
    return t[stage_table_offset<L, E, P>() + k * (R - 1) + (m - 1)];
  }
};

// Fills a TwStage table (size stage_table_size<L, E>()) from any twiddle
// source; all threads call it; it ends with a barrier.
// Index j of the source twiddle W_L^j of entry i of the stage table, for
// i < stage_table_size<L, E>(): entry i lies in the last stage whose offset
// is at most i (the stages are a compile-time list, so the search is a few
// compares and selects of constants, not a loop).
template <int L, int E>
__host__ __device__ inline int stage_table_source(int i) {
  constexpr int R0 = stage_radix<L, E, 1>();
  int base = 0, step = L / (R0 * E);  // the stage's offset and L / (p E)
  int off = 0;
#pragma unroll
  for (int p = R0; p < L; p *= E) {
    if (i >= off) {
      base = off;
      step = L / (p * E);
    }
    off += p * (E - 1);
  }
  const int r = i - base;
  const int k = r / (E - 1), m = r % (E - 1) + 1;
  return m * k * step;
}

template <typename T, int L, int E, typename Src>
__device__ __forceinline__ void build_stage_table(cpx<T>* dst, const Src& src) {
  for (int i = threadIdx.x; i < stage_table_size<L, E>(); i += blockDim.x)
    dst[i] = src(stage_table_source<L, E>(i));
  __syncthreads();
}

// Loads the first quarter of the global table W_Nt^j into LDS (all threads
// call it; it ends with a barrier).
template <typename T>
__device__ __forceinline__ void load_quarter(cpx<T>* dst, const cpx<T>* __restrict__ tw, int nt) {
  for (int i = threadIdx.x; i < nt / 4; i += blockDim.x) dst[i] = tw[i];
  __syncthreads();
}

// Forward DFT of one line of L points, in place in registers: on entry
// v[e] = x[t + TPL e], on exit v[e] = X[t + TPL e], X_k = sum_j x_j W_L^{jk},
// W_L = exp(-2 pi i / L).  tw(j) must return W_L^j.  Every thread of the
// workgroup must call this with the same template arguments (it contains
// barriers); threads with active = false only take part in the barriers.
template <typename T, int L, int E, int P, typename Lds, typename Tw>
__device__ __forceinline__ void stockham(cpx<T>* v, int t, const Tw& tw, Lds& lds,
                                         bool active = true) {
  if constexpr (P < L) {
    constexpr int R = stage_radix<L, E, P>();
    constexpr int TPL = L / E;
    constexpr int Q = E / R;
    constexpr bool LAST = (P * R == L);
    if constexpr (!LAST) __syncthreads();  // earlier readers of the LDS are done
    if (active) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int i = t + TPL * q;
        const int k = i & (P - 1);
        cpx<T> a[R];
#pragma unroll
        for (int m = 0; m < R; ++m) a[m] = v[q + m * Q];
        if constexpr (P > 1) {
#pragma unroll
          for (int m = 1; m < R; ++m) a[m] = cmul(a[m], tw.template stage<L, P, R>(k, m));
        }
        dft<T, R>(a);
        if constexpr (LAST) {
#pragma unroll
          for (int m = 0; m < R; ++m) v[q + m * Q] = a[m];
        } else {
          const int j = (i - k) * R + k;
#pragma unroll
          for (int m = 0; m < R; ++m) lds.template put_step<P>(j, m, a[m]);
        }
      }
    }
    if constexpr (!LAST) {
      __syncthreads();
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = lds.template get_step<TPL>(t, e);
      }
      stockham<T, L, E, P * R>(v, t, tw, lds, active);
    }
  }
}

}  // namespace pk
