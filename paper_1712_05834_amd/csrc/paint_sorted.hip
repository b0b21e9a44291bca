// Painting fused with the first FFT pass (Sec. 3.3.1 Eq. 1, Sec. 3.3.2
// windows and interlacing; r2c along z).
//
// 1. k_bucket_count   per particle: its column (ix, iy) = floor(u_x, u_y); runs
//                     of equal columns in a wavefront are added to a block-local
//                     LDS table, which reaches the global column counts with one
//                     atomic per column and block; sum w and sum w^2 in float64.
// 2. k_scan_*         exclusive prefix sum of the N^2 column counts.
// 3. k_bucket_scatter per particle: a 16-byte record {t_x, t_y, t_z, iy<<16|iz}
//                     (fractional offsets from the cell, split off in float64)
//                     written to its column's segment; the slots of a step are
//                     reserved with one atomic per column through the same kind
//                     of LDS table.
// Catalogs that are not in column order (random order: no runs) take a
// second route instead, chosen on the device by k_order_probe from sampled
// neighbouring particles, without a round trip to the host (the workgroups
// of k_bucket_count and k_bucket_scatter run the route chosen):
// 1'. counting        per block of the catalog, LDS counts of the x-slabs
//                     ix, stored as [block][slab] and added into per-slab
//                     totals (one atomic per slab and block).
// 3'. scattering      each block scans the slab totals in LDS (slab starts),
//                     reserves its range in every slab (one atomic per slab
//                     and block) and writes its records (and amounts) slab
//                     by slab into scratch memory, places ranked by LDS
//                     atomics.  (The scan kernels of the run route then scan
//                     zero counts; k_slab_columns writes the offsets.)
// 3''. k_slab_columns one workgroup per slab: LDS counts of its columns,
//                     their offsets, then the records moved into column order
//                     (LDS atomics only).
// 4. k_paint_z        one workgroup owns a TX x TY block of full z-columns of
//                     both meshes: it reads the records of the columns whose
//                     windows reach the block, adds the window weights into
//                     64-bit LDS rows (exact fixed point, ds_add_u64, for
//                     float32 meshes; float64, ds_add_f64, otherwise), then
//                     runs the r2c FFT of every column in LDS and writes the
//                     packed rows once.  No mesh clear, no atomics to HBM, no
//                     separate z-pass.
#include "fft_config.h"
#include "internal.h"
#include "window.h"

namespace pk {

// 1.5 * 2^52 and its bits: adding it to a double of magnitude below 2^51
// rounds that double to an integer and leaves it, two's complement, in the
// low bits.
constexpr double kFixMagic = 6755399441055744.0;
constexpr unsigned long long kFixMagicBits = 0x4338000000000000ull;
// slots of the exact painting's grid in the bucketing workspace
constexpr int kFixScale = 0, kFixInv = 1, kFixState = 2, kFixMeanQ = 3;

template <typename T>
struct Rec;
template <>
struct Rec<float> {
  using type = float4;
};
template <>
struct Rec<double> {
  using type = double4;
};

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Runs of equal keys among consecutive lanes of a wavefront: the head lane
// of each run gets the run length; every lane gets its run's head and its
// offset in the run.  Lanes with key < 0 belong to no run.
struct WaveRun {
  bool head;
  int len;      // run length (head lanes)
  int my_head;  // lane of the head of my run
  int offset;   // my position in the run, -1 for key < 0
};

__device__ __forceinline__ WaveRun wave_run(int key) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  const bool valid = key >= 0;
  const bool head = valid && (lane == 0 || prev != key);
  const unsigned long long heads = __ballot(head);
  const unsigned long long valids = __ballot(valid);
  // head lane of my run: highest head at or below me
  const unsigned long long below = heads & ((2ull << lane) - 1ull);
  WaveRun r;
  r.head = head;
  r.my_head = below ? 63 - __clzll(below) : lane;
  r.offset = valid ? lane - r.my_head : -1;
  r.len = 0;
  if (head) {
    // up to the next head or the first invalid lane
    const unsigned long long above = (heads | ~valids) & ~((2ull << lane) - 1ull);
    const int next = above ? __ffsll(above) - 1 : 64;
    r.len = next - lane;
  }
  return r;
}

// Route of a bucketing launch, chosen on the device by k_order_probe: mode
// holds kProbeGroups counts of sampled neighbouring pairs that share a
// column, out of kProbeSamples; with at least a quarter the catalog is taken
// to be in column order (run route), else the slab route runs.  The kernels
// of the other route return at once.  mode NULL: the run route alone.
constexpr int kRouteRuns = 0, kRouteSlabs = 1;
constexpr int kProbeGroups = 16, kProbeSamples = kProbeGroups * 256;
__device__ __forceinline__ int route_of(const int* mode) {
  if (mode == nullptr) return kRouteRuns;
  int same = 0;
#pragma unroll
  for (int g = 0; g < kProbeGroups; ++g) same += mode[g];
  return 4 * same >= kProbeSamples ? kRouteRuns : kRouteSlabs;
}
__device__ __forceinline__ bool off_route(const int* mode, int route) {
  return route_of(mode) != route;
}

// Block-local table of column counts in LDS: runs of the same column from
// the block's particles are added here and reach the global counters with one
// atomic per column and block.  Global atomics (performed beyond the XCD's L2)
// were the cost of the bucketing.  Open addressing with a few probes; a key
// that finds no entry goes straight to the global counter.
constexpr int kHashSize = 1024;
constexpr int kHashProbes = 4;

__device__ __forceinline__ int hash_insert(int* keys, int* cnts, int key, int len, int& rank) {
  const unsigned h = ((unsigned)key * 2654435761u) >> (32 - 10);
#pragma unroll
  for (int probe = 0; probe < kHashProbes; ++probe) {
    const int e = (int)((h + probe) & (kHashSize - 1));
    int t = keys[e];
    if (t == -1) {
      t = atomicCAS(&keys[e], -1, key);
      if (t == -1) t = key;
    }
    if (t == key) {
      rank = atomicAdd(&cnts[e], len);
      return e;
    }
  }
  return -1;
}

__device__ __forceinline__ void hash_clear(int* keys, int* cnts) {
  for (int e = threadIdx.x; e < kHashSize; e += blockDim.x) {
    keys[e] = -1;
    cnts[e] = 0;
  }
}

// Particles per thread per step of the bucketing kernels (256 threads): the
// loads of a step are issued together.  Each block takes a contiguous chunk
// of the catalog (a multiple of 256 * kBucketUnroll particles), so that
// ordered catalogs give it few distinct columns.
constexpr int kBucketUnroll = 4;
constexpr int kBucketStep = 256 * kBucketUnroll;

constexpr int kSlabBlocks = 1024;      // catalog blocks of the slab route (at most)
constexpr int kMaxSlabs = 2048;        // x-slabs = N, N <= 2048
constexpr int64_t kSlabMinParticles = 1 << 14;  // smaller catalogs: run route

template <typename T>
__device__ __forceinline__ int column_key(const T* __restrict__ pos, int64_t i, int nmesh,
                                          double boxsize, double inv_box, double cpl) {
  const int mask = nmesh - 1;
  const double ux = cell_coordinate_rcp((double)pos[3 * i], boxsize, inv_box, cpl);
  const double uy = cell_coordinate_rcp((double)pos[3 * i + 1], boxsize, inv_box, cpl);
  return (((int)floor(ux)) & mask) * nmesh + (((int)floor(uy)) & mask);
}

// Arguments of the slab route's parts of k_bucket_count and
// k_bucket_scatter: catalog blocks of chunk particles (nblocks of them), the
// [block][slab] counts, the slab totals and cursors, the scratch records and
// amounts (amounts NULL without weights or values).
struct SlabArgs {
  int64_t chunk;
  int nblocks;
  int* hist;    // [block][slab] counts
  int* total;   // per-slab totals (zeroed by k_order_probe)
  int* cursor;  // per-slab ranges reserved so far (zeroed by k_order_probe)
  void* trec;
  void* twrec;
};

// Slab route, counting (run by the workgroups of k_bucket_count): block
// blk of the catalog (particles blk chunk .. blk chunk + chunk - 1, nblocks
// blocks): counts of its particles per x-slab in LDS, stored to
// hist[blk][slab] and added into the slab totals; weight sums of the block
// to wpart as in the run route.
template <typename T>
__device__ void slab_count_block(const T* __restrict__ pos, const T* __restrict__ weight,
                                 const T* __restrict__ value, int64_t n, int nmesh,
                                 double boxsize, double inv_box, double cells_per_len,
                                 const SlabArgs& sa, int blk, double* __restrict__ wpart) {
  __shared__ int lh[kMaxSlabs];
  __shared__ double part[2][4];
  const int mask = nmesh - 1;
  constexpr int U = kBucketUnroll;
  const int64_t chunk = sa.chunk;
  int* __restrict__ hist = sa.hist;
  {
    for (int b = threadIdx.x; b < nmesh; b += blockDim.x) lh[b] = 0;
    __syncthreads();
    double ws = 0.0, ws2 = 0.0;
    const int64_t begin = (int64_t)blk * chunk;
    const int64_t end = begin + chunk < n ? begin + chunk : n;
    for (int64_t i0 = begin + threadIdx.x; i0 < end; i0 += kBucketStep) {
      int slab[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + u * 256;
        slab[u] = -1;
        if (i < end) {
          const double ux =
              cell_coordinate_rcp((double)pos[3 * i], boxsize, inv_box, cells_per_len);
          slab[u] = ((int)floor(ux)) & mask;
          const double wp = weight ? (double)weight[i] : 1.0;
          const double wv = value ? wp * (double)value[i] : wp;
          ws += wp;
          // a non-finite coordinate makes sum (w V)^2 NaN, and with it the
          // painted cells and the shot noise
          const double pc = (double)pos[3 * i] + (double)pos[3 * i + 1] + (double)pos[3 * i + 2];
          ws2 += isfinite(pc) ? wv * wv : __longlong_as_double(0x7ff8000000000000ll);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (slab[u] >= 0) atomicAdd(&lh[slab[u]], 1);
    }
    ws = wave_sum_d(ws);
    ws2 = wave_sum_d(ws2);
    if ((threadIdx.x & 63) == 0) {
      part[0][threadIdx.x >> 6] = ws;
      part[1][threadIdx.x >> 6] = ws2;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nmesh; b += blockDim.x) {
      const int c = lh[b];
      hist[(size_t)blk * nmesh + b] = c;
      if (c) atomicAdd(&sa.total[b], c);
    }
    if (threadIdx.x == 0) {
      wpart[2 * blk] = ((part[0][0] + part[0][1]) + part[0][2]) + part[0][3];
      wpart[2 * blk + 1] = ((part[1][0] + part[1][1]) + part[1][2]) + part[1][3];
    }
  }
}

// Exclusive prefix sums of the slab totals (nmesh <= 2048 of them) into
// start[] by a 256-thread workgroup: eight per thread, then a scan of the
// thread sums over the four waves.
__device__ __forceinline__ void slab_starts_256(const int* __restrict__ total, int nmesh,
                                                int* start, int* sh) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int v[8], s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int b = t * 8 + k;
    v[k] = b < nmesh ? total[b] : 0;
    s += v[k];
  }
  int x = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  int ex = x - s;
  for (int w = 0; w < wave; ++w) ex += sh[w];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int b = t * 8 + k;
    if (b < nmesh) start[b] = ex;
    ex += v[k];
  }
  __syncthreads();
}

// Slab route, scattering (run by the workgroups of k_bucket_scatter): the
// records of block blk (same blocks as the counting) written into the slabs
// of the scratch arrays: the block reserves its range in every slab it has
// particles in (slab start from the totals + one atomic on the slab's
// cursor); places within it are taken in LDS.  Record and amount as in the
// run route.
template <typename T>
__device__ void slab_scatter_block(const T* __restrict__ pos, const T* __restrict__ weight,
                                   const T* __restrict__ value, int64_t n, int nmesh,
                                   double boxsize, double inv_box, double cells_per_len,
                                   const SlabArgs& sa, int blk) {
  using RecT = typename Rec<T>::type;
  __shared__ int cur[kMaxSlabs];
  const int mask = nmesh - 1;
  constexpr int U = kBucketUnroll;
  __shared__ int sh[4];
  const int64_t chunk = sa.chunk;
  RecT* __restrict__ trec = static_cast<RecT*>(sa.trec);
  T* __restrict__ twrec = static_cast<T*>(sa.twrec);
  {
  slab_starts_256(sa.total, nmesh, cur, sh);  // ends with a barrier
  for (int b = threadIdx.x; b < nmesh; b += blockDim.x) {
    const int c = sa.hist[(size_t)blk * nmesh + b];
    if (c) cur[b] += atomicAdd(&sa.cursor[b], c);
  }
  __syncthreads();
  const int64_t begin = (int64_t)blk * chunk;
  const int64_t end = begin + chunk < n ? begin + chunk : n;
  for (int64_t i0 = begin + threadIdx.x; i0 < end; i0 += kBucketStep) {
    RecT r[U];
    int slab[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * 256;
      slab[u] = -1;
      r[u] = RecT{};
      if (i < end) {
        double uu[3], f[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          uu[d] = cell_coordinate_rcp((double)pos[3 * i + d], boxsize, inv_box, cells_per_len);
          f[d] = floor(uu[d]);
        }
        slab[u] = ((int)f[0]) & mask;
        const unsigned iy = ((unsigned)(int)f[1]) & mask, iz = ((unsigned)(int)f[2]) & mask;
        r[u].x = static_cast<T>(uu[0] - f[0]);
        r[u].y = static_cast<T>(uu[1] - f[1]);
        r[u].z = static_cast<T>(uu[2] - f[2]);
        if constexpr (sizeof(T) == 4) {
          r[u].w = __uint_as_float((iy << 16) | iz);
        } else {
          r[u].w = (double)((iy << 16) | iz);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * 256;
      if (slab[u] >= 0) {
        const int slot = atomicAdd(&cur[slab[u]], 1);
        trec[slot] = r[u];
        if (twrec) twrec[slot] = weight ? (value ? weight[i] * value[i] : weight[i]) : value[i];
      }
    }
  }
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_bucket_count(const T* __restrict__ pos, const T* __restrict__ weight,
                   const T* __restrict__ value, int64_t n, int64_t chunk, int nmesh,
                   double boxsize, double inv_box, double cells_per_len,
                   int* __restrict__ count, double* __restrict__ wpart,
                   const int* __restrict__ mode, SlabArgs sa) {
  if (route_of(mode) == kRouteSlabs) {
    if ((int)blockIdx.x < sa.nblocks)
      slab_count_block<T>(pos, weight, value, n, nmesh, boxsize, inv_box, cells_per_len, sa,
                          blockIdx.x, wpart);
    return;
  }
  __shared__ int hkeys[kHashSize], hcnts[kHashSize];
  hash_clear(hkeys, hcnts);
  __syncthreads();
  const int mask = nmesh - 1;
  constexpr int U = kBucketUnroll;
  double ws = 0.0, ws2 = 0.0;
  const int64_t begin = (int64_t)blockIdx.x * chunk;
  for (int64_t i0 = begin + threadIdx.x; i0 < begin + chunk; i0 += kBucketStep) {
    int key[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * 256;
      key[u] = -1;
      if (i < n) {
        const double ux = cell_coordinate_rcp((double)pos[3 * i], boxsize, inv_box, cells_per_len);
        const double uy =
            cell_coordinate_rcp((double)pos[3 * i + 1], boxsize, inv_box, cells_per_len);
        key[u] = (((int)floor(ux)) & mask) * nmesh + (((int)floor(uy)) & mask);
        // normalisation: sum w; shot noise: sum (w V)^2 (V = 1 without values)
        const double wp = weight ? (double)weight[i] : 1.0;
        const double wv = value ? wp * (double)value[i] : wp;
        ws += wp;
        // a non-finite coordinate makes sum (w V)^2 NaN, and with it the
        // painted cells and the shot noise
        const double pc = (double)pos[3 * i] + (double)pos[3 * i + 1] + (double)pos[3 * i + 2];
        ws2 += isfinite(pc) ? wv * wv : __longlong_as_double(0x7ff8000000000000ll);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const WaveRun r = wave_run(key[u]);
      if (r.head) {
        int rank;
        if (hash_insert(hkeys, hcnts, key[u], r.len, rank) < 0) atomicAdd(&count[key[u]], r.len);
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kHashSize; e += blockDim.x)
    if (hkeys[e] >= 0) atomicAdd(&count[hkeys[e]], hcnts[e]);
  // per-block partial sums (reduced in a fixed order by k_weight_sums)
  __shared__ double part[2][4];
  ws = wave_sum_d(ws);
  ws2 = wave_sum_d(ws2);
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = ws;
    part[1][threadIdx.x >> 6] = ws2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    wpart[2 * blockIdx.x] = ((part[0][0] + part[0][1]) + part[0][2]) + part[0][3];
    wpart[2 * blockIdx.x + 1] = ((part[1][0] + part[1][1]) + part[1][2]) + part[1][3];
  }
}

// sum w and sum (w V)^2 from the per-block partials of the route taken, in
// block order; then the grid 2^-S of the exact painting from n and
// sum (w V)^2 (see k_paint_z): fix[kFixScale] = 2^S, fix[kFixInv] = 2^-S,
// fix[kFixState] = 0 (exact), 1 (non-finite amounts or coordinates: NaN
// cells) or 2 (S out of range: float64 sums), and fix[kFixMeanQ] the bits
// of the int64 round(2^S sum w / N^3), the mean on the integer grid (0
// unless exact).
__global__ void __launch_bounds__(1024)
    k_weight_sums(const double* __restrict__ wpart, int nblocks_runs, int nblocks_slabs,
                  double* __restrict__ wsums, const int* __restrict__ mode, int64_t n,
                  int nmesh, double* __restrict__ fix) {
  const int nblocks = route_of(mode) == kRouteSlabs ? nblocks_slabs : nblocks_runs;
  __shared__ double sh[2][1024];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += 1024) {
    a += wpart[2 * i];
    b += wpart[2 * i + 1];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int half = 512; half >= 1; half >>= 1) {
    if ((int)threadIdx.x < half) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + half];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + half];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    wsums[0] = sh[0][0];
    wsums[1] = sh[1][0];
    const double w2 = sh[1][0], nt = (double)n;
    double scale = 1.0, state = 0.0;
    if (!isfinite(w2)) {
      state = 1.0;
    } else if (nt > 0.0 && w2 > 0.0) {
      const int e1 = ilogb(sqrt(nt * w2)) + 1, e2 = ilogb(sqrt(w2)) + 1;
      int S = 62 - e1 < 50 - e2 ? 62 - e1 : 50 - e2;
      if (S > 120) S = 120;  // tiny amounts: a coarser grid still holds them
      if (S < -90) state = 2.0;
      scale = ldexp(1.0, S);
    }
    long long mean_q = 0;
    if (state == 0.0) {
      const double mean = sh[0][0] / ((double)nmesh * nmesh * nmesh);
      mean_q = __double2ll_rn(mean * scale);
    }
    fix[kFixScale] = scale;
    fix[kFixInv] = 1.0 / scale;  // exact: a power of two
    fix[kFixState] = state;
    fix[kFixMeanQ] = __longlong_as_double(mean_q);
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_bucket_scatter(const T* __restrict__ pos, const T* __restrict__ weight,
                     const T* __restrict__ value, int64_t n, int64_t chunk, int nmesh,
                     double boxsize, double inv_box, double cells_per_len,
                     int* __restrict__ cursor,
                     typename Rec<T>::type* __restrict__ rec, T* __restrict__ wrec,
                     const int* __restrict__ mode, SlabArgs sa) {
  if (route_of(mode) == kRouteSlabs) {
    if ((int)blockIdx.x < sa.nblocks)
      slab_scatter_block<T>(pos, weight, value, n, nmesh, boxsize, inv_box, cells_per_len, sa,
                            blockIdx.x);
    return;
  }
  // per step: the runs of each column in the step are ranked in the LDS
  // table, one global atomic per column reserves the step's slots, then every
  // particle writes its record at base + rank
  __shared__ int hkeys[kHashSize], hcnts[kHashSize], hbase[kHashSize];
  const int mask = nmesh - 1;
  constexpr int U = kBucketUnroll;
  using RecT = typename Rec<T>::type;
  const int64_t begin = (int64_t)blockIdx.x * chunk;
  for (int64_t i0 = begin + threadIdx.x; i0 < begin + chunk; i0 += kBucketStep) {
    hash_clear(hkeys, hcnts);
    __syncthreads();
    int ent[U], rk[U];
    RecT r[U];
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      const int64_t i = i0 + uu * 256;
      int key = -1;
      r[uu] = RecT{};
      if (i < n) {
        double u[3], f[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          u[d] = cell_coordinate_rcp((double)pos[3 * i + d], boxsize, inv_box, cells_per_len);
          f[d] = floor(u[d]);
        }
        key = (((int)f[0]) & mask) * nmesh + (((int)f[1]) & mask);
        const unsigned iy = ((unsigned)(int)f[1]) & mask, iz = ((unsigned)(int)f[2]) & mask;
        r[uu].x = static_cast<T>(u[0] - f[0]);
        r[uu].y = static_cast<T>(u[1] - f[1]);
        r[uu].z = static_cast<T>(u[2] - f[2]);
        if constexpr (sizeof(T) == 4) {
          r[uu].w = __uint_as_float((iy << 16) | iz);
        } else {
          r[uu].w = (double)((iy << 16) | iz);
        }
      }
      const WaveRun run = wave_run(key);
      int e = -1, rank = 0;
      if (run.head) {
        e = hash_insert(hkeys, hcnts, key, run.len, rank);
        if (e < 0) rank = atomicAdd(&cursor[key], run.len);  // no entry: a direct slot
      }
      ent[uu] = __shfl(e, run.my_head, 64);
      rk[uu] = run.offset >= 0 ? __shfl(rank, run.my_head, 64) + run.offset : -1;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kHashSize; e += blockDim.x)
      if (hkeys[e] >= 0) hbase[e] = atomicAdd(&cursor[hkeys[e]], hcnts[e]);
    __syncthreads();
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      const int64_t i = i0 + uu * 256;
      if (i < n) {
        const int slot = (ent[uu] >= 0 ? hbase[ent[uu]] : 0) + rk[uu];
        rec[slot] = r[uu];
        // the painted amount of the particle: w V
        if (wrec) wrec[slot] = weight ? (value ? weight[i] * value[i] : weight[i]) : value[i];
      }
    }
    __syncthreads();  // the table is read before the next step clears it
  }
}

// ---- exclusive scan of the column counts (3 phases, 4096 entries per block)

__device__ __forceinline__ int block_scan_excl(int v, int* sh, int& total) {
  // 1024 threads; inclusive wave scan, then scan of the 16 wave totals
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < 16; ++w) {
      const int t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    sh[16] = acc;
  }
  __syncthreads();
  total = sh[16];
  const int r = sh[wave] + x - v;
  __syncthreads();
  return r;
}

// Exclusive scan of the run route's column counts into offsets (n + 1
// entries) and cursor.  On the slab route the counts are all zero (the run
// route's counting returned at once) and k_slab_columns writes the offsets
// afterwards, so these kernels need not know the route.
__global__ void __launch_bounds__(1024)
    k_scan_blocks(const int* __restrict__ count, int n, int* __restrict__ block_sums) {
  __shared__ int sh[17];
  const int base = blockIdx.x * 4096 + threadIdx.x * 4;
  int s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) s += (base + j < n) ? count[base + j] : 0;
  int total;
  (void)block_scan_excl(s, sh, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024) k_scan_sums(int* __restrict__ block_sums, int nb) {
  __shared__ int sh[17];
  int carry = 0;
  for (int start = 0; start < nb; start += 1024) {
    const int i = start + threadIdx.x;
    const int v = i < nb ? block_sums[i] : 0;
    int total;
    const int ex = block_scan_excl(v, sh, total);
    if (i < nb) block_sums[i] = carry + ex;
    carry += total;
  }
}

__global__ void __launch_bounds__(1024)
    k_scan_final(const int* __restrict__ count, int n, const int* __restrict__ block_sums,
                 int* __restrict__ offsets, int* __restrict__ cursor) {
  __shared__ int sh[17];
  const int base = blockIdx.x * 4096 + threadIdx.x * 4;
  int v[4];
  int s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[j] = (base + j < n) ? count[base + j] : 0;
    s += v[j];
  }
  int total;
  int ex = block_scan_excl(s, sh, total) + block_sums[blockIdx.x];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) {
      offsets[base + j] = ex;
      cursor[base + j] = ex;
    }
    ex += v[j];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1) offsets[n] = ex;
}

// ---- the slab route (catalogs not in column order)

// The route's sample: kProbeSamples pairs (i, i + 1) spread over the catalog
// (n >= 2), one per thread of kProbeGroups workgroups; each workgroup stores
// how many of its pairs share a column.  It also clears the slab route's
// counters.
template <typename T>
__global__ void __launch_bounds__(256)
    k_order_probe(const T* __restrict__ pos, int64_t n, int nmesh, double boxsize,
                  double inv_box, double cpl, int* __restrict__ mode,
                  int* __restrict__ slab_counters) {
  const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  // the slab totals and cursors (2 nmesh <= kProbeSamples ints) start at zero
  if (j < 2 * nmesh) slab_counters[j] = 0;
  // i <= n - 2, so i + 1 is a particle
  const int64_t i = (int64_t)((double)j * (double)(n - 2) / (double)(kProbeSamples - 1));
  int same = column_key(pos, i, nmesh, boxsize, inv_box, cpl) ==
                     column_key(pos, i + 1, nmesh, boxsize, inv_box, cpl)
                 ? 1
                 : 0;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) same += __shfl_xor(same, off, 64);
  __shared__ int sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = same;
  __syncthreads();
  if (threadIdx.x == 0) mode[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__device__ __forceinline__ int record_iy(float4 r) { return (int)(__float_as_uint(r.w) >> 16); }
__device__ __forceinline__ int record_iy(double4 r) { return (int)((unsigned)r.w >> 16); }

// One workgroup (1024 threads) per x-slab (slabs taken in turn): LDS counts
// of the slab's columns iy, their exclusive prefix sums from the slab start
// give the column offsets (offsets[ix N + iy]; the last slab also writes
// offsets[N^2] = n).  The records then go to their columns in steps of S:
// each step is sorted by column in LDS (counting sort) and written out in
// that order, so that the records of one column leave as one contiguous run
// rather than as single 16-byte stores scattered over all N columns.
template <typename T>
struct ColStage {
  static constexpr int S = sizeof(T) == 4 ? 4096 : 2048;  // records per step
  static constexpr int U = S / 1024;                        // per thread
};

template <typename T>
__global__ void __launch_bounds__(1024)
    k_slab_columns(int nmesh, const int* __restrict__ mode, const int* __restrict__ total,
                   const typename Rec<T>::type* __restrict__ trec,
                   const T* __restrict__ twrec, int* __restrict__ offsets,
                   typename Rec<T>::type* __restrict__ rec, T* __restrict__ wrec) {
  if (off_route(mode, kRouteSlabs)) return;
  using RecT = typename Rec<T>::type;
  constexpr int S = ColStage<T>::S, U = ColStage<T>::U;
  __shared__ int cnt[kMaxSlabs];     // running place of each column
  __shared__ int lb[kMaxSlabs + 1];  // step counts, then their prefix sums
  __shared__ RecT srec[S];
  __shared__ T samt[S];
  __shared__ unsigned short scol[S];
  __shared__ int sh[17];
  const int b0 = 2 * threadIdx.x, b1 = b0 + 1;  // two columns per thread (N <= 2048)
  for (int ix = blockIdx.x; ix < nmesh; ix += gridDim.x) {
    // the slab's start: the totals of the slabs before it
    int s0;
    {
      const int v = (b0 < ix ? total[b0] : 0) + (b1 < ix ? total[b1] : 0);
      (void)block_scan_excl(v, sh, s0);
    }
    const int s1 = s0 + total[ix];
    for (int b = threadIdx.x; b < nmesh; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    for (int64_t j = s0 + (int64_t)threadIdx.x; j < s1; j += blockDim.x)
      atomicAdd(&cnt[record_iy(trec[j])], 1);
    __syncthreads();
    {
      const int c0 = b0 < nmesh ? cnt[b0] : 0, c1 = b1 < nmesh ? cnt[b1] : 0;
      int total;
      const int ex = s0 + block_scan_excl(c0 + c1, sh, total);  // barriers: counts read first
      if (b0 < nmesh) {
        cnt[b0] = ex;
        offsets[(size_t)ix * nmesh + b0] = ex;
      }
      if (b1 < nmesh) {
        cnt[b1] = ex + c0;
        offsets[(size_t)ix * nmesh + b1] = ex + c0;
      }
      if (ix == nmesh - 1 && threadIdx.x == 0) offsets[(size_t)nmesh * nmesh] = s1;
    }
    for (int64_t base = s0; base < s1; base += S) {
      for (int b = threadIdx.x; b < nmesh; b += blockDim.x) lb[b] = 0;
      __syncthreads();  // also orders the cursors written above before their use
      RecT r[U];
      T am[U];
      int col[U], rk[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t j = base + threadIdx.x + u * 1024;
        col[u] = -1;
        rk[u] = 0;
        if (j < s1) {
          r[u] = trec[j];
          am[u] = wrec ? twrec[j] : T(0);
          col[u] = record_iy(r[u]);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (col[u] >= 0) rk[u] = atomicAdd(&lb[col[u]], 1);
      __syncthreads();
      const int c0 = b0 < nmesh ? lb[b0] : 0, c1 = b1 < nmesh ? lb[b1] : 0;
      int m;
      const int ex = block_scan_excl(c0 + c1, sh, m);  // barriers: counts read first
      if (b0 < nmesh) lb[b0] = ex;
      if (b1 < nmesh) lb[b1] = ex + c0;
      if (threadIdx.x == 0) lb[nmesh] = m;
      __syncthreads();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (col[u] >= 0) {
          const int p = lb[col[u]] + rk[u];
          srec[p] = r[u];
          samt[p] = am[u];
          scol[p] = (unsigned short)col[u];
        }
      }
      __syncthreads();
      for (int e = threadIdx.x; e < m; e += blockDim.x) {
        const int c = scol[e];
        const int g = cnt[c] + (e - lb[c]);
        rec[g] = srec[e];
        if (wrec) wrec[g] = samt[e];
      }
      __syncthreads();
      for (int c = threadIdx.x; c < nmesh; c += blockDim.x) cnt[c] += lb[c + 1] - lb[c];
      __syncthreads();  // lb is read before the next step clears it
    }
    __syncthreads();  // the cursors are done with before the next slab clears them
  }
}

// ---- fused paint + r2c z-pass

// Columns per workgroup (TX x TY) and halo of source columns per mesh size.
// The window weights are accumulated in float64 LDS rows with ds_add_f64: on
// gfx950 it runs about 20x faster than ds_add_f32, and the accumulation is
// more precise than the mesh.  (Integer fixed point with ds_add_u32 is faster
// still, but a 32-bit range cannot hold a dense workgroup's cells at float
// precision.)  After the gather a row is reused in place as the padded complex
// line of the r2c.
constexpr int kPaintLdsBudgetKB = 76;  // two workgroups per CU

// Meshes a paint launch produces: kPaintA the plain mesh, kPaintB the mesh
// shifted by half a cell (interlacing), kPaintAB both in one pass.
constexpr int kPaintA = 0, kPaintB = 1, kPaintAB = 2;
// Interlaced meshes are painted by one two-mesh launch by default: each
// record is read once for both meshes (Zel'dovich 1024^3 CIC: 4.82 against
// 4.92 ms for two single-mesh launches, whose record reads from L2 misses
// come to 6.0 GB against 4.4 GB).  For TSC two launches, with tiles twice
// as wide, are within the noise of one (log-normal 512^3: 0.664 against
// 0.674 ms) but fetch 1.36x the algorithmic bytes against 1.15x.  The tuner
// can choose two launches per input.
constexpr bool split_interlaced(int) { return false; }


// A store of output that no later kernel reads while it is still cached (the
// painted meshes, 1-9 GB): nontemporal, so that it does not displace the
// records the next workgroups gather (Zel'dovich 1024^3 paint: 5.18 ->
// 5.02 ms).
template <typename T>
__device__ __forceinline__ void store_stream(cpx<T>* p, cpx<T> v) {
  if constexpr (sizeof(T) == 4) {
    const unsigned long long bits =
        ((unsigned long long)__float_as_uint(v.y) << 32) | __float_as_uint(v.x);
    __builtin_nontemporal_store(bits, reinterpret_cast<unsigned long long*>(p));
  } else {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
  }
}

template <typename T, int N, int P, int MODE>
struct PaintCfg {
  using Acc = double;
  static constexpr int M = N / 2;
  static constexpr int LP = lds_pad_len<M>();           // complex per FFT line
  static constexpr int NM = MODE == kPaintAB ? 2 : 1;
  // accumulator row: cell z at word z + 1 for z in [-1, N + 2], the cells
  // one window can reach from a particle of the column without wrapping (the
  // pad words are folded into their periodic images before the z-FFT), so
  // that the P cells of a stencil are P consecutive words
  static constexpr int ZPAD_LO = 1, ZPAD_HI = 3;
  static constexpr long ACC_BYTES = (long)(N + ZPAD_LO + ZPAD_HI) * sizeof(Acc);
  static constexpr long FFT_BYTES = (long)LP * 2 * sizeof(T);
  // row stride: the row rounded to 16 bytes plus 16 bytes, so that
  // consecutive rows start 4 banks apart
  static constexpr long ROW_BYTES =
      ((ACC_BYTES > FFT_BYTES ? ACC_BYTES : FFT_BYTES) + 15) / 16 * 16 + 16;
  static constexpr int ROWA = (int)(ROW_BYTES / sizeof(Acc));  // row stride in Acc units
  static constexpr int EMIN = M < 2 ? M : 2;
  static constexpr int EMAX = M < e_max<T>() ? M : e_max<T>();
  // LDS budget per workgroup: two workgroups per CU
  static constexpr int pick_cols() {
    int cols = 64;
    while (cols > 1 && (long)cols * NM * ROW_BYTES > kPaintLdsBudgetKB * 1024) cols /= 2;
    while (cols > 1 && (long)cols * NM * (M / EMAX) > 1024) cols /= 2;
    return cols;
  }
  static constexpr int COLS = pick_cols();
  static constexpr int TX0 = COLS >= 16 ? 4 : (COLS >= 4 ? 2 : 1);
  static constexpr int TX = COLS / TX0 > N ? COLS / N : TX0;
  static constexpr int TY = COLS / TX;
  static_assert(TX <= N && TY <= N && TX * TY == COLS, "column block must fit the mesh");
  static constexpr int ROWS = NM * TX * TY;
  // points per thread of the column FFTs: as few as keep the workgroup at
  // most 1024 threads, so that the gather phase runs with many waves
  static constexpr int pick_e() {
    int e = EMIN;
    while (e < EMAX && (long)ROWS * (M / e) > 1024) e *= 2;
    return e;
  }
  static constexpr int E = pick_e();
  static constexpr int TPL = M / E;
  static constexpr int THREADS = ROWS * TPL;
  // points per thread of the z-FFT itself: radix 8 (radix 4 in float64),
  // run by the first ROWS * M / FE threads while the others wait at its
  // barriers -- fewer stages and less address arithmetic than the E of the
  // gather, and the kernel is bound by VALU issue
  static constexpr int FE0 = M < (sizeof(T) == 4 ? 8 : 4) ? M : (sizeof(T) == 4 ? 8 : 4);
  static constexpr int FE = FE0 > E ? FE0 : E;
  static constexpr int FTPL = M / FE;
  static constexpr int FTHREADS = ROWS * FTPL;
  // source columns that can reach an owned column: [X - HLO, X + HHI].  A
  // particle in column i touches cells i .. i+1 (CIC), i-1 .. i+2 (TSC, PCS)
  // of the plain mesh and i .. i+2 (CIC, TSC), i-1 .. i+3 (PCS) of the
  // shifted one.
  static constexpr int HLO_A = P == 2 ? 1 : 2, HHI_A = P == 2 ? 0 : 1;
  static constexpr int HLO_B = P == 4 ? 3 : 2, HHI_B = P == 4 ? 1 : 0;
  static constexpr int HLO = MODE == kPaintA ? HLO_A : (MODE == kPaintB ? HLO_B : (HLO_A > HLO_B ? HLO_A : HLO_B));
  static constexpr int HHI = MODE == kPaintA ? HHI_A : (MODE == kPaintB ? HHI_B : (HHI_A > HHI_B ? HHI_A : HHI_B));
};

template <typename T, int N, int P, int MODE>
__global__ void __launch_bounds__((PaintCfg<T, N, P, MODE>::THREADS))
    k_paint_z(const typename Rec<T>::type* __restrict__ rec, const T* __restrict__ wrec,
              const int* __restrict__ offsets, const double* __restrict__ wsums,
              const double* __restrict__ fix, const cpx<T>* __restrict__ tw,
              T* __restrict__ mesh_a, T* __restrict__ mesh_b, int exact_in) {
  using Cf = PaintCfg<T, N, P, MODE>;
  using Acc = double;
  constexpr int M = Cf::M, TX = Cf::TX, TY = Cf::TY;
  constexpr int ROWS = Cf::ROWS, ROWA = Cf::ROWA;
  constexpr int mask = N - 1;
  __shared__ __align__(16) Acc acc[ROWS * ROWA];
  __shared__ cpx<T> twm[M];  // W_N^k, k < M, for the r2c split
  __shared__ cpx<T> tws[stage_table_size<M, Cf::FE>() + 1];
  __shared__ int seg_start[2 * (TX + 4)], seg_cum[2 * (TX + 4) + 1], seg_row[2 * (TX + 4)];
  static_assert(TX + 4 >= (TX + Cf::HLO + Cf::HHI < N ? TX + Cf::HLO + Cf::HHI : N), "segments");

  const int tiles_y = N / TY;
  const int X0 = (blockIdx.x / tiles_y) * TX, Y0 = (blockIdx.x % tiles_y) * TY;

  // The global loads of the prologue are issued first and consumed late: the
  // segment offsets after the LDS rows are cleared, the twiddles (only the
  // z-FFT needs them) after the gather, so their latency is hidden.
  // segments of the sorted records: for each source row bx, the contiguous
  // column range [by0, by0 + wy) (split in two where it wraps around N); one
  // thread per source row reads its offsets; their prefix sums follow below
  constexpr int HW = Cf::HLO + Cf::HHI;
  constexpr int WX = (TX + HW) >= N ? N : TX + HW;
  constexpr int WY = (TY + HW) >= N ? N : TY + HW;
  const bool seg_thread = (int)threadIdx.x < WX;
  int o0 = 0, o1 = 0, o2 = 0, o3 = 0, bx = 0;
  const int run0 = (N - ((TY + HW) >= N ? 0 : ((Y0 - Cf::HLO) & mask))) < WY
                       ? (N - ((TY + HW) >= N ? 0 : ((Y0 - Cf::HLO) & mask)))
                       : WY;
  const int run1 = WY - run0;  // wrapped part, starting at column 0
  if (seg_thread) {
    const int bx0 = (TX + HW) >= N ? 0 : X0 - Cf::HLO;
    const int by0 = (TY + HW) >= N ? 0 : ((Y0 - Cf::HLO) & mask);
    bx = (bx0 + (int)threadIdx.x) & mask;
    const int b0 = bx * N + by0;
    o0 = offsets[b0];
    o1 = offsets[b0 + run0];
    if (run1 > 0) {
      o2 = offsets[bx * N];
      o3 = offsets[bx * N + run1];
    }
  }
  const double wsum = wsums[0];  // for the mean subtracted before the z-FFT
  // Exact painting: each product is rounded once to a multiple of 2^-S and
  // added as a 64-bit integer, so that a cell's sum is the same whatever the
  // order of its adds (and whatever the tiling).  S is one scale for the
  // whole mesh, from bounds that hold a priori: a cell's sum is at most
  // sum |a| <= sqrt(n sum a^2) (amounts a = w V, n records; the window
  // weights are at most 1), so 2^S sqrt(n sum a^2) < 2^62 keeps every sum in
  // range; one term is at most max |a| <= sqrt(sum a^2), and 2^S sqrt(sum a^2)
  // < 2^50 keeps each term below 2^51, where adding 1.5 * 2^52 rounds it to
  // an integer held in the low mantissa bits.  With unit weights S = 38 for
  // 10^7 particles and 35 for 1.3 x 10^8 (2.9e-11 per term, far below the
  // float32 rounding of a cell; float64 meshes take the float64 sums).  A
  // non-finite amount or coordinate (the bucketing makes the sum of squares
  // NaN then) makes every cell NaN, as float64 sums would.
  // (Amounts so large that 2^-S would leave the float32 range, |a| beyond
  // ~10^27, take the float64 sums.)  The bucketing's k_weight_sums sets the
  // scale once.
  double fix_scale = 1.0, fix_inv = 1.0;
  long long fix_mean = 0;
  bool fix_bad = false, exact = exact_in != 0;
  if (exact) {
    const double state = fix[kFixState];
    fix_bad = state == 1.0;
    if (state == 2.0) exact = false;
    fix_scale = fix[kFixScale];
    fix_inv = fix[kFixInv];
    fix_mean = __double_as_longlong(fix[kFixMeanQ]);
  }

  constexpr int STS = stage_table_size<M, Cf::FE>();
  constexpr bool EARLY_TW = M <= Cf::THREADS && STS <= Cf::THREADS;
  cpx<T> tw_m{}, tw_s{};
  if constexpr (EARLY_TW) {
    if ((int)threadIdx.x < M) tw_m = tw[threadIdx.x];
    if ((int)threadIdx.x < STS) tw_s = tw[2 * stage_table_source<M, Cf::FE>(threadIdx.x)];
  }

  // The mean density, subtracted before the z-FFT.  Exact painting subtracts
  // it on the integer grid (it only moves the DC mode): every word starts at
  // -round(mean 2^S) instead of 0, so that the cells need no subtraction when
  // they are read back (the pad words carry the same start; the fold below
  // adds one mean back with each of them).
  // (the bucketing computed round(mean 2^S) along with S)
  const bool nan_cells = fix_bad;
  const long long mean_q = exact && !nan_cells ? fix_mean : 0ll;
  // cleared 16 bytes at a time (half the stores and loop steps of 8)
  static_assert((ROWS * ROWA) % 2 == 0, "the rows hold whole pairs of words");
  {
    const double f = __longlong_as_double(-mean_q);  // 0.0 unless exact
    for (int i = threadIdx.x; i < ROWS * ROWA / 2; i += blockDim.x)
      reinterpret_cast<double2*>(acc)[i] = double2{f, f};
  }
  // prefix sums of the segment lengths: a scan across the first wavefront
  // (the segment threads are its first WX lanes; the other lanes add 0)
  static_assert(WX <= 64, "segment threads within one wavefront");
  if (threadIdx.x < 64) {
    const int l0 = o1 - o0, l1 = o3 - o2;
    int inc = l0 + l1;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(inc, off, 64);
      if ((int)threadIdx.x >= off) inc += v;
    }
    const int exc = inc - l0 - l1;
    if (seg_thread) {
      seg_start[2 * threadIdx.x] = o0;
      seg_cum[2 * threadIdx.x] = exc;
      seg_row[2 * threadIdx.x] = bx;
      seg_start[2 * threadIdx.x + 1] = o2;
      seg_cum[2 * threadIdx.x + 1] = exc + l0;
      seg_row[2 * threadIdx.x + 1] = bx;
      if ((int)threadIdx.x == WX - 1) seg_cum[2 * WX] = inc;
    }
  }
  __syncthreads();

  // Work item q is the q-th gathered record: the 64 lanes of a wave take
  // consecutive records, which mostly come from one source column, so the
  // window cells that fall outside the block are outside for the whole wave
  // and their branches are skipped.
  constexpr int nseg = 2 * WX;
  static_assert(nseg <= 32, "segment bounds in scalar registers");
  // the segment bounds are the same for every lane: kept in scalar
  // registers, so that finding an item's segment takes no LDS reads
  int scum[nseg + 1];
#pragma unroll
  for (int j = 0; j <= nseg; ++j) scum[j] = __builtin_amdgcn_readfirstlane(seg_cum[j]);
  const int total = scum[nseg];
  // record index of work item q (-1 past the end), and its segment in `seg`:
  // the number of segment starts at or below q (independent compares, not a
  // walk from segment to segment: a step of the loop moves q past several
  // segments).  The next record is loaded before the current one is
  // processed, so its latency overlaps the work.
  // Unless the block's y window wraps around the mesh (two of every N / TY
  // blocks), the second segment of every source row is empty, and only the
  // first segments' starts need comparing.
  const bool y_wraps = run1 > 0;
  auto locate = [&](int q, int& seg) -> int {
    if (q >= total) return -1;
    int s = 0;
    if (y_wraps) {
#pragma unroll
      for (int j = 1; j < nseg; ++j) s += scum[j] <= q ? 1 : 0;
    } else {
#pragma unroll
      for (int j = 2; j < nseg; j += 2) s += scum[j] <= q ? 2 : 0;
    }
    seg = s;
    return seg_start[s] + (q - seg_cum[s]);
  };
  using RecT = typename Rec<T>::type;
  int seg_cur = 0;
  int idx_cur = locate(threadIdx.x, seg_cur);
  RecT r_cur{};
  T w_cur = T(1);
  if (idx_cur >= 0) {
    r_cur = rec[idx_cur];
    if (wrec) w_cur = wrec[idx_cur];
  }
  // The gather loop is instantiated once per summation mode (EX: exact
  // fixed-point sums), so that the mode costs no per-cell selects or
  // branches; the workgroup takes one of them.
  // 2^S in the mesh precision (exact: -90 <= S <= 120)
  const T scale_t = static_cast<T>(fix_scale);
  auto gather = [&](auto ex_tag) {
    constexpr bool EX = decltype(ex_tag)::value;
    for (int q = threadIdx.x; q < total; q += blockDim.x) {
      // inside the loop idx_cur is a valid record; past the end the next load
      // repeats it, so that the load is unconditional and the wait for the
      // current record does not have to drain it
      int seg_nxt = seg_cur;
      const int idx_nxt = locate(q + (int)blockDim.x, seg_nxt);
      const int idx_ld = idx_nxt >= 0 ? idx_nxt : idx_cur;
      const RecT r_nxt = rec[idx_ld];
      T w_nxt = T(1);
      if (wrec) w_nxt = wrec[idx_ld];
      {
        const RecT r = r_cur;
        // exact painting: the amount carries the grid scale 2^S (a power of
        // two, within float range, so the float products below are the
        // unscaled ones times 2^S exactly)
        const T wp = EX ? w_cur * scale_t : w_cur;
        unsigned packed;
        if constexpr (sizeof(T) == 4) {
          packed = __float_as_uint(r.w);
        } else {
          packed = (unsigned)r.w;
        }
        const int ix = seg_row[seg_cur], iy = (int)(packed >> 16), iz = (int)(packed & 0xffff);
        const T t3[3] = {r.x, r.y, r.z};
        const int i3[3] = {ix, iy, iz};
#pragma unroll
        for (int mesh = 0; mesh < Cf::NM; ++mesh) {
          int first[3];
          T w[3][P];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            // window of u = i + t (+ 1/2 for the interlaced mesh)
            T tt = t3[d];
            int base = i3[d];
            if (MODE == kPaintB || (MODE == kPaintAB && mesh == 1)) {
              if (tt >= T(0.5)) {
                tt -= T(0.5);  // exact
                base += 1;
              } else {
                tt += T(0.5);
              }
            }
            window_frac<T, P>(tt, base, first[d], w[d]);
          }
          // the P z cells are P consecutive words from first[2] + ZPAD_LO (the
          // address is computed once per row, the cells are immediate
          // offsets); products in float64 from the z weights converted once
          const int zb = first[2] + Cf::ZPAD_LO;
          double wz[P];
#pragma unroll
          for (int c = 0; c < P; ++c) wz[c] = (double)w[2][c];
          // validity and row offsets (in bytes) of the P x and P y cells,
          // once per mesh (each block then takes only its lane mask and one
          // address add)
          bool vx[P], vy[P];
          int rx[P], ry[P];
#pragma unroll
          for (int a = 0; a < P; ++a) {
            const int lx = (first[0] + a - X0) & mask;
            vx[a] = lx < TX;
            rx[a] = ((mesh * TX + lx) * TY * ROWA + zb) * (int)sizeof(Acc);
            const int ly = (first[1] + a - Y0) & mask;
            vy[a] = ly < TY;
            ry[a] = ly * ROWA * (int)sizeof(Acc);
          }
#pragma unroll
          for (int a = 0; a < P; ++a) {
            if (!vx[a]) continue;
            const T wa = wp * w[0][a];
#pragma unroll
            for (int b2 = 0; b2 < P; ++b2) {
              if (!vy[b2]) continue;
              const double wab = (double)(wa * w[1][b2]);
              Acc* row = reinterpret_cast<Acc*>(reinterpret_cast<char*>(acc) + rx[a] + ry[b2]);
              if constexpr (EX) {
                // the bits of 1.5 * 2^52 + v minus those of 1.5 * 2^52: v
                // rounded to an integer, two's complement (|v| < 2^51)
                unsigned long long* irow = reinterpret_cast<unsigned long long*>(row);
#pragma unroll
                for (int c = 0; c < P; ++c) {
                  const double y = __builtin_fma(wab, wz[c], kFixMagic);
                  atomicAdd(&irow[c], (unsigned long long)__double_as_longlong(y) - kFixMagicBits);
                }
              } else {
#pragma unroll
                for (int c = 0; c < P; ++c) atomicAdd(&row[c], wab * wz[c]);
              }
            }
          }
        }
      }
      idx_cur = idx_nxt;
      seg_cur = seg_nxt;
      r_cur = r_nxt;
      w_cur = w_nxt;
    }
  };
  if constexpr (sizeof(T) == 4) {
    if (exact)
      gather(std::true_type{});
    else
      gather(std::false_type{});
  } else {
    gather(std::false_type{});  // float64 meshes take the float64 sums
  }
  __syncthreads();

  // periodic images: the front pad word (cell -1) into cell N - 1, the back
  // pad words (cells N .. N + 2) into cells 0 .. 2 -- four distinct cells per
  // row, one thread each
  static_assert(N >= 4, "the images of the pad cells must be distinct");
  for (int i = threadIdx.x; i < ROWS * 4; i += blockDim.x) {
    Acc* row = acc + (i >> 2) * ROWA;
    unsigned long long* irow = reinterpret_cast<unsigned long long*>(row);
    const int j = i & 3;
    // cell -1 (word 0) into cell N - 1 (word N); cell N + j - 1 into cell
    // j - 1 (word j)
    const int dst = j == 0 ? N : j, src = j == 0 ? 0 : N + j;
    if (exact) {
      irow[dst] += irow[src] + (unsigned long long)mean_q;
    } else {
      row[dst] += row[src];
    }
  }
  __syncthreads();

  // the twiddle tables of the z-FFT (written after the gather's barrier; the
  // next barrier orders them before their first use)
  if constexpr (EARLY_TW) {
    if ((int)threadIdx.x < M) twm[threadIdx.x] = tw_m;
    if ((int)threadIdx.x < STS) tws[threadIdx.x] = tw_s;
  } else {
    for (int i = threadIdx.x; i < M; i += blockDim.x) twm[i] = tw[i];
    build_stage_table<T, M, Cf::FE>(tws, TwGlobal<T>{tw, 2});  // ends with a barrier
  }

  // r2c along z of every owned column, mean subtracted before the rounding to
  // T (only the DC mode changes; it keeps the rounding relative to the
  // fluctuations): in float64 here, or already on the integer grid (exact
  // painting), where the cell d = hi 2^32 + lo goes to float32 as
  // hi 2^(32-S) + lo 2^-S in float32 arithmetic (no float64 operations per
  // cell; within 1.5 ulp of the rounded value).  The row becomes the padded
  // complex line.
  // (NaN cells: NaN scales, so that every converted cell is NaN)
  const float f_nan = __int_as_float(0x7fc00000);
  const float f_lo = nan_cells ? f_nan : (float)fix_inv;
  const float f_hi = nan_cells ? f_nan : (float)(fix_inv * 4294967296.0);
  constexpr int FE = Cf::FE, FTPL = Cf::FTPL;
  const bool fa = (int)threadIdx.x < Cf::FTHREADS;
  const int r = fa ? (int)threadIdx.x / FTPL : 0, t = (int)threadIdx.x % FTPL;
  Acc* arow = acc + r * ROWA;
  LdsLine<T> line{reinterpret_cast<cpx<T>*>(arow)};
  cpx<T> v[FE];
  if (fa) {
#pragma unroll
    for (int e = 0; e < FE; ++e) {
      const int wj = 2 * (t + FTPL * e) + Cf::ZPAD_LO;  // cells 2j, 2j + 1
      if (exact) {
        const long long* irow = reinterpret_cast<const long long*>(arow);
        const long long d0 = irow[wj], d1 = irow[wj + 1];
        v[e] = {static_cast<T>(fmaf((float)(int)(d0 >> 32), f_hi, (float)(unsigned)d0 * f_lo)),
                static_cast<T>(fmaf((float)(int)(d1 >> 32), f_hi, (float)(unsigned)d1 * f_lo))};
      } else {
        const double mean = nan_cells ? __longlong_as_double(0x7ff8000000000000ll)
                                      : wsum / ((double)N * N * N);
        v[e] = {static_cast<T>(arow[wj] - mean), static_cast<T>(arow[wj + 1] - mean)};
      }
    }
  }
  __syncthreads();  // all cells read before the row is reused
  const TwStage<T, M, FE> tw2{tws};
  stockham<T, M, FE, 1>(v, t, tw2, line, fa);
  __syncthreads();
  if (fa) {
#pragma unroll
    for (int e = 0; e < FE; ++e) line.template put_step<FTPL>(t, e, v[e]);
  }
  __syncthreads();
  if (!fa) return;
  const int mesh = r / (TX * TY), lx = (r / TY) % TX, ly = r % TY;
  T* out = mesh == 0 ? mesh_a : mesh_b;
  cpx<T>* rowp = reinterpret_cast<cpx<T>*>(out + ((size_t)(X0 + lx) * N + (Y0 + ly)) * N);
#pragma unroll
  for (int e = 0; e < FE; ++e) {
    const int k = t + FTPL * e;
    cpx<T> o;
    if (k == 0) {
      o = {v[e].x + v[e].y, v[e].x - v[e].y};
    } else {
      const cpx<T> zc = cconj(line.template get_step<FTPL>(FTPL - t, FE - 1 - e));  // Z_{M-k}
      const cpx<T> s = cadd(v[e], zc);
      const cpx<T> w = cmul(twm[k], csub(v[e], zc));
      o = {T(0.5) * (s.x + w.y), T(0.5) * (s.y - w.x)};
    }
    store_stream(rowp + k, o);
  }
}

// ---------------------------------------------------------------- launchers

constexpr int kCountBlocks = 8192;

static size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

// Bucketing workspace: count, offsets (+1), cursor, scan block sums (ints);
// float64 weight partials; then the route flag and, for the slab route, the
// [block][slab] counts and the slab totals and cursors.
struct BucketWs {
  size_t count, offsets, cursor, bsums, wpart, fix, mode, hist, slabc, total;
  int nb;
  explicit BucketWs(int nmesh) {
    const size_t n2 = (size_t)nmesh * nmesh;
    nb = (int)((n2 + 4095) / 4096);
    count = 0;
    offsets = count + n2 * sizeof(int);
    cursor = offsets + (n2 + 1) * sizeof(int);
    bsums = cursor + n2 * sizeof(int);
    wpart = round256(bsums + (size_t)(nb + 1) * sizeof(int));
    fix = round256(wpart + 2 * kCountBlocks * sizeof(double));  // kFix* slots
    mode = round256(fix + 4 * sizeof(double));
    const size_t nh = (size_t)nmesh * kSlabBlocks;
    hist = mode + 256;
    slabc = round256(hist + nh * sizeof(int));
    total = round256(slabc + 2 * (size_t)nmesh * sizeof(int));
  }
};

size_t bucket_bytes(int nmesh) { return BucketWs(nmesh).total; }

hipError_t launch_bucket(int dtype, int nmesh, double boxsize, const void* pos, const void* weight,
                         const void* value, int64_t n, void* bucket_ws, void* rec, void* wrec,
                         double* wsums, hipStream_t s, void* scratch, size_t scratch_bytes) {
  const int n2 = nmesh * nmesh;
  const double inv_box = 1.0 / boxsize, cpl = nmesh / boxsize;
  const BucketWs L(nmesh);
  char* bw = static_cast<char*>(bucket_ws);
  int* count = reinterpret_cast<int*>(bw + L.count);
  int* offsets = reinterpret_cast<int*>(bw + L.offsets);
  int* cursor = reinterpret_cast<int*>(bw + L.cursor);
  int* bsums = reinterpret_cast<int*>(bw + L.bsums);
  double* wpart = reinterpret_cast<double*>(bw + L.wpart);
  const int nb = L.nb;
  const bool amounts = weight || value;
  // the slab route needs scratch for the records (and amounts) in slab order
  const size_t es = dtype == PK_F32 ? 4 : 8;
  const size_t trec_bytes = round256((size_t)(n > 0 ? n : 0) * 4 * es);
  const size_t twrec_bytes = amounts ? round256((size_t)(n > 0 ? n : 0) * es) : 0;
  const bool slabs = scratch != nullptr && n >= kSlabMinParticles && nmesh <= kMaxSlabs &&
                     scratch_bytes >= trec_bytes + twrec_bytes;
  int* mode = slabs ? reinterpret_cast<int*>(bw + L.mode) : nullptr;
  int* slabc = reinterpret_cast<int*>(bw + L.slabc);  // totals [N], then cursors [N]
  hipError_t e = launch_fill_zero(count, (size_t)n2 * sizeof(int), s);
  if (e != hipSuccess) return e;
  if (slabs) {
    if (dtype == PK_F32)
      hipLaunchKernelGGL(k_order_probe<float>, dim3(kProbeGroups), dim3(256), 0, s,
                         static_cast<const float*>(pos), n, nmesh, boxsize, inv_box, cpl, mode,
                         slabc);
    else
      hipLaunchKernelGGL(k_order_probe<double>, dim3(kProbeGroups), dim3(256), 0, s,
                         static_cast<const double*>(pos), n, nmesh, boxsize, inv_box, cpl, mode,
                         slabc);
  }
  // run route: contiguous chunks of whole steps, at most kCountBlocks blocks
  int64_t steps = (n + kBucketStep - 1) / kBucketStep;
  if (steps < 1) steps = 1;
  int64_t blocks = steps < kCountBlocks ? steps : kCountBlocks;
  const int64_t chunk = (steps + blocks - 1) / blocks * kBucketStep;
  blocks = (n + chunk - 1) / chunk;
  if (blocks < 1) blocks = 1;
  // slab route: at most min(kSlabBlocks, max(256, N)) contiguous blocks of
  // whole steps (each block costs one atomic per slab twice; 256 keep the
  // CUs busy at small N)
  const int64_t scap = nmesh > 256 ? (nmesh < kSlabBlocks ? nmesh : kSlabBlocks) : 256;
  int64_t sblocks = steps < scap ? steps : scap;
  const int64_t schunk = (steps + sblocks - 1) / sblocks * kBucketStep;
  sblocks = (n + schunk - 1) / schunk;
  if (sblocks < 1) sblocks = 1;
  char* sc = static_cast<char*>(scratch);
  SlabArgs sa{schunk, slabs ? (int)sblocks : 0, reinterpret_cast<int*>(bw + L.hist), slabc,
              slabc + nmesh, sc, slabs && amounts ? sc + trec_bytes : nullptr};
  // counts (the workgroups run the route the probe chose)
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_bucket_count<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const float*>(pos), static_cast<const float*>(weight),
                       static_cast<const float*>(value), n, chunk, nmesh, boxsize, inv_box, cpl, count,
                       wpart, mode, sa);
  else
    hipLaunchKernelGGL(k_bucket_count<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const double*>(pos), static_cast<const double*>(weight),
                       static_cast<const double*>(value), n, chunk, nmesh, boxsize, inv_box, cpl, count,
                       wpart, mode, sa);
  hipLaunchKernelGGL(k_weight_sums, dim3(1), dim3(1024), 0, s, wpart, (int)blocks, (int)sblocks,
                     wsums, mode, n, nmesh, reinterpret_cast<double*>(bw + L.fix));
  // the run route's scan (zero counts on the slab route)
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(1024), 0, s, count, n2, bsums);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, bsums, nb);
  hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(1024), 0, s, count, n2, bsums, offsets, cursor);
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_bucket_scatter<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const float*>(pos), static_cast<const float*>(weight),
                       static_cast<const float*>(value), n, chunk, nmesh, boxsize, inv_box, cpl, cursor,
                       static_cast<float4*>(rec), amounts ? static_cast<float*>(wrec) : nullptr,
                       mode, sa);
  else
    hipLaunchKernelGGL(k_bucket_scatter<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const double*>(pos), static_cast<const double*>(weight),
                       static_cast<const double*>(value), n, chunk, nmesh, boxsize, inv_box, cpl, cursor,
                       static_cast<double4*>(rec), amounts ? static_cast<double*>(wrec) : nullptr,
                       mode, sa);
  if (!slabs) return hipGetLastError();
  // slab route: the slabs into column order
  if (dtype == PK_F32)
    hipLaunchKernelGGL(k_slab_columns<float>, dim3((unsigned)nmesh), dim3(1024), 0, s, nmesh,
                       mode, sa.total, static_cast<const float4*>(sa.trec),
                       static_cast<const float*>(sa.twrec), offsets, static_cast<float4*>(rec),
                       amounts ? static_cast<float*>(wrec) : nullptr);
  else
    hipLaunchKernelGGL(k_slab_columns<double>, dim3((unsigned)nmesh), dim3(1024), 0, s, nmesh,
                       mode, sa.total, static_cast<const double4*>(sa.trec),
                       static_cast<const double*>(sa.twrec), offsets, static_cast<double4*>(rec),
                       amounts ? static_cast<double*>(wrec) : nullptr);
  return hipGetLastError();
}

template <typename T, int N, int P, int MODE>
static hipError_t paint_z_t(const void* rec, const void* wrec, const int* offsets,
                            const double* wsums, const double* fix, const void* tw,
                            void* mesh_a, void* mesh_b, bool exact, hipStream_t s) {
  using Cf = PaintCfg<T, N, P, MODE>;
  const unsigned blocks = (unsigned)((N / Cf::TX) * (N / Cf::TY));
  hipLaunchKernelGGL((k_paint_z<T, N, P, MODE>), dim3(blocks), dim3(Cf::THREADS), 0, s,
                     static_cast<const typename Rec<T>::type*>(rec),
                     static_cast<const T*>(wrec), offsets, wsums, fix,
                     static_cast<const cpx<T>*>(tw), static_cast<T*>(mesh_a),
                     static_cast<T*>(mesh_b), exact ? 1 : 0);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t paint_z_n(int order, bool inter, const void* rec, const void* wrec,
                            const int* offsets, const double* wsums, const double* fix,
                            const void* tw, void* mesh_a, void* mesh_b, int split, bool exact,
                            hipStream_t s) {
#define PK_PZ(P, MODE, A) \
  paint_z_t<T, N, P, MODE>(rec, wrec, offsets, wsums, fix, tw, A, mesh_b, exact, s)
#define PK_PZ_ORDER(MODE, A)                                            \
  (order == 2 ? PK_PZ(2, MODE, A) : (order == 3 ? PK_PZ(3, MODE, A) : PK_PZ(4, MODE, A)))
  if (!inter) return PK_PZ_ORDER(kPaintA, mesh_a);
  if (!(split < 0 ? split_interlaced(order) : split != 0)) return PK_PZ_ORDER(kPaintAB, mesh_a);
  hipError_t e = PK_PZ_ORDER(kPaintA, mesh_a);
  if (e != hipSuccess) return e;
  return PK_PZ_ORDER(kPaintB, mesh_b);
#undef PK_PZ_ORDER
#undef PK_PZ
}

hipError_t launch_paint_z(int dtype, int nmesh, int order, bool inter, const void* rec,
                          const void* wrec, const void* bucket_ws, const double* wsums,
                          const void* tw, void* mesh_a, void* mesh_b, hipStream_t s, int split,
                          bool exact) {
  const int* offsets = static_cast<const int*>(bucket_ws) + (size_t)nmesh * nmesh;
  const double* fix = reinterpret_cast<const double*>(static_cast<const char*>(bucket_ws) +
                                                      BucketWs(nmesh).fix);
  // float64 meshes keep float64 sums: one 64-bit fixed-point scale cannot
  // span both the a-priori range of a cell and float64 precision within it
  if (dtype != PK_F32) exact = false;
#define PK_PN(T)                                                                           \
  switch (nmesh) {                                                                         \
    case 8: return paint_z_n<T, 8>(order, inter, rec, wrec, offsets, wsums, fix, tw, mesh_a, mesh_b, split, exact, s); \
    case 16: return paint_z_n<T, 16>(order, inter, rec, wrec, offsets, wsums, fix, tw, mesh_a, mesh_b, split, exact, s); \
    case 32: return paint_z_n<T, 32>(order, inter, rec, wrec, offsets, wsums, fix, tw, mesh_a, mesh_b, split, exact, s); \
    case 64: return paint_z_n<T, 64>(order, inter, rec, wrec, offsets, wsums, fix, tw, mesh_a, mesh_b, split, exact, s); \
    case 128: return paint_z_n<T, 128>(order, inter, rec, wrec, offsets, wsums, fix, tw, mesh_a, mesh_b, split, exact, s); \
    case 256: return paint_z_n<T, 256>(order, inter, rec, wrec, offsets, wsums, fix, tw, mesh_a, mesh_b, split, exact, s); \
    case 512: return paint_z_n<T, 512>(order, inter, rec, wrec, offsets, wsums, fix, tw, mesh_a, mesh_b, split, exact, s); \
    case 1024: return paint_z_n<T, 1024>(order, inter, rec, wrec, offsets, wsums, fix, tw, mesh_a, mesh_b, split, exact, s); \
    case 2048: return paint_z_n<T, 2048>(order, inter, rec, wrec, offsets, wsums, fix, tw, mesh_a, mesh_b, split, exact, s); \
    default: return hipErrorInvalidValue;                                                  \
  }
  if (dtype == PK_F32) {
    PK_PN(float)
  } else {
    PK_PN(double)
  }
#undef PK_PN
}

}  // namespace pk
