// Internal declarations shared by the translation units of libpk.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pk.h"

namespace pk {

// Per (mesh size, precision) device tables, one allocation:
//   tw[N]            W_N^j = exp(-2 pi i j / N)                 (complex T)
//   phase[3N + 1]    exp(i pi s / N), s = -3N/2 .. 3N/2         (complex T)
//   sinc_inv[3][N]   sinc(pi n_i / N)^-p, p = 2, 3, 4, index i  (real T)
// All values are computed on the host in float64 and rounded once.
struct MeshTables {
  void* dev = nullptr;
  size_t bytes = 0;
  const void* tw = nullptr;
  const void* phase = nullptr;
  const void* sinc_inv = nullptr;  // row p - 2
};

// Per binning: device squared edges plus host copies of the field-independent
// sums (mode counts, sum of h |n|, sum of h |mu|).
struct BinTables {
  double* e2_dev = nullptr;  // nk + 1
  std::vector<int64_t> modes;
  std::vector<double> sum_n;  // sum over modes of h |n| (units of k_f)
  std::vector<int64_t> modes2d;
  std::vector<double> sum_n2d;
  std::vector<double> sum_mu2d;
};

// Everything a binning kernel needs to place one mode.
struct BinSpec {
  int nmesh = 0;
  int nk = 0;
  int nmu = 0;
  int los = 2;
  int npoles = 0;       // all requested poles (slot order of the result)
  int zero_mask = 0;    // bit i set: poles[i] == 0 (aliases the plain power)
  int npl = 0;          // poles with ell > 0 that are accumulated
  int pole_ell[4] = {0, 0, 0, 0};
  int pole_slot[4] = {0, 0, 0, 0};
  int off2d = -1;       // first (k, mu) slot, -1 if none
  int nsum = 0;         // number of sum slots (weight slots excluded)
  // LDS accumulators: the sums that are accumulated (power, poles with
  // ell > 0, (k, mu) bins) in 128-bit fixed point, two 64-bit words each.
  int nlds = 0;
  int pole_lds[4] = {0, 0, 0, 0};  // first LDS slot of accumulated pole i
  int off2d_lds = -1;
  // With (k, mu) bins the power sum of a k-bin is the exact sum of its mu-bin
  // sums: it is formed when the partial row is written, not accumulated.
  int power_from_2d = 0;
  // Fixed-point scale: every sum and every term is bounded in magnitude by
  // B = bound_scale * (bound_dev ? *bound_dev (squared if bound_sq) : 1),
  // read on the device; units of 2^-S with B 2^S < 2^126.
  double bound_scale = 0.0;
  const double* bound_dev = nullptr;
  int bound_sq = 0;
  // Word split of the fixed point: 64 = a 128-bit two's complement integer
  // (low word, high word; the carry of the low word taken from a returning
  // atomic), 32 = low 32 bits in the first word and the rest (signed) in the
  // second, both added without return, for sums below 2^95.
  int fix_hb = 64;
  // Partial rows (one per workgroup, 2 nsum 64-bit words each) hold the exact
  // sums as 128-bit integers (low words, then high words) when set, else
  // float64 values in the first nsum words; k_reduce reads them accordingly.
  int exact = 1;
  double kmin_f = 0.0;
  double dk_f = 1.0;
  const double* e2 = nullptr;  // device, nk + 1
  int int_edges = 0;    // kmin_f and dk_f are whole numbers: exact integer rule
  int kmin_i = 0;
  int dk_i = 1;
};

// Mode-table accumulator layout (plan time):
//   [0, nk) counts (as uint64 bits), [nk, 2nk) sum h|n|,
//   then, if nmu > 1: counts2d, sum h|n| 2d, sum h|mu| 2d (nk * nmu each).
__host__ __device__ inline int mode_table_slots(int nk, int nmu) { return 2 * nk + (nmu > 1 ? 3 * nk * nmu : 0); }
// Fraction bits of the fixed-point mode-table sums (sum h|n| < 2 N^4 <= 2^45
// for N <= 2048, held in 128 bits with room to spare).
constexpr int kModeSumShift = 80;

// LDS available to one workgroup on gfx950, and its compute units.
constexpr size_t kLdsBytesPerGroup = 160 * 1024;
constexpr long kComputeUnits = 256;

// ---- launchers (each defined in the translation unit of its kernels) ----
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_paint_atomic(int dtype, int order, int nmesh, double boxsize, const void* pos,
                               const void* weight, int64_t n, double shift_a, void* mesh_a,
                               double shift_b, void* mesh_b, double* wsums, hipStream_t s);

// Sorted painting fused with the z-pass (paint_sorted.hip).
size_t bucket_bytes(int nmesh);
// value: per-particle field values V or NULL; records carry w V, the sums
// are {sum w, sum (w V)^2}.  scratch: device memory free during the
// bucketing (n 4-vector records and n amounts, each rounded up to 256 bytes);
// without it, or for catalogs under 2^14 particles, only the route for
// catalogs in column order is taken.
hipError_t launch_bucket(int dtype, int nmesh, double boxsize, const void* pos, const void* weight,
                         const void* value, int64_t n, void* bucket_ws, void* rec, void* wrec,
                         double* wsums, hipStream_t s, void* scratch = nullptr,
                         size_t scratch_bytes = 0);
// split: interlaced meshes painted by two single-mesh launches (1), one
// two-mesh launch (0), or the default for the window (-1).  exact: float32
// meshes take cell sums in 64-bit fixed point with a scale from wsums[1]
// (sum of squared amounts) and the record count, independent of the order
// of the adds; otherwise (float64 meshes, callers whose wsums do not bound
// the amounts) float64 sums.
hipError_t launch_paint_z(int dtype, int nmesh, int order, bool inter, const void* rec,
                          const void* wrec, const void* bucket_ws, const double* wsums,
                          const void* tw, void* mesh_a, void* mesh_b, hipStream_t s,
                          int split = -1, bool exact = true);

hipError_t launch_fft_z(int dtype, int nmesh, void* mesh, int nmeshes, size_t mesh_stride_bytes,
                        const void* tw, const double* wsum_for_mean, hipStream_t s);
// inverse = 1: the unnormalised backward transform along the axis.
hipError_t launch_fft_cols(int dtype, int nmesh, void* mesh, int nmeshes,
                           size_t mesh_stride_bytes, const void* tw, int axis, hipStream_t s,
                           int inverse = 0);
// Inverse z-pass: packed half-spectrum rows back to real rows (c2r).
hipError_t launch_ifft_z(int dtype, int nmesh, void* mesh, const void* tw, hipStream_t s);
// y-pass of one z-transformed mesh, out of place into the layout read by the
// fused x-pass (YLayout in fft_config.h).
hipError_t launch_fft_y_relayout(int dtype, int nmesh, const void* src, void* dst, const void* tw,
                                 hipStream_t s);

// Workgroup count of the persistent binning kernels for a mesh size.
int xpass_bin_groups(int dtype, int nmesh, size_t bin_bytes);
int plane_bin_groups(int nmesh);
size_t bin_lds_bytes(const BinSpec& b);
// Static LDS bytes of the fused x-pass + binning kernel (0: unsupported size).
size_t xpass_static_lds(int dtype, int nmesh);
// groups > 0: that many workgroups (at most xpass_bin_groups) instead of
// as many as the device holds.
hipError_t launch_xpass_bin(int dtype, int nmesh, const void* mesh_a, const void* mesh_b,
                            const MeshTables& t, int order, int compensated, const BinSpec& b,
                            double* partials, void* side_a, void* side_b, hipStream_t s,
                            int groups = 0);
// cmesh2 != NULL: cross power Re(c conj(c2)) instead of |c|^2.  ylayout = 1:
// both spectra are in the y-pass output layout instead of the packed one.
// max_groups > 0 caps the grid (and so the partial rows written); the
// default grid is bin_packed_groups(nmesh).
int bin_packed_groups(int nmesh);
hipError_t launch_bin_packed(int dtype, int nmesh, const void* cmesh, const void* cmesh2,
                             const BinSpec& b, double* partials, hipStream_t s, int ylayout = 0,
                             int max_groups = 0);
// Plain k-bin sums of Re(c conj(d_i)) for nf <= 4 other spectra d_i (NULL:
// c itself) in one pass; field i's workgroup sums go to partials + i pstride
// (launch_bin_packed's grid and row layout).  ylayout as launch_bin_packed.
hipError_t launch_bin_fields(int dtype, int nmesh, const void* cmesh, const void* const* others,
                             int nf, const BinSpec& b, double* partials, size_t pstride,
                             hipStream_t s, int ylayout);
// cross = 0: za (and the interlaced zb) combined; cross = 1: Re(a conj(b)).
// groups > 0 sets the grid (else plane_bin_groups(nmesh)); t is read only
// for interlacing (zb, cross = 0) and compensation.
hipError_t launch_plane_bin(int dtype, int nmesh, const void* za, const void* zb, size_t zstride,
                            const MeshTables& t, int order, int compensated, const BinSpec& b,
                            double* partials, hipStream_t s, int cross = 0, int groups = 0);
// e2[i] = (kmin + i dk)^2 for i = 0 .. nk, each product and sum rounded on
// its own: the same values as the host-built edge table.
hipError_t launch_edges_squared(double kmin, double dk, int nk, double* e2, hipStream_t s);
// *out = max |x| over count reals of a (and of b if not NULL); out is a device
// float64 that the launch zeroes first (a fill kernel, no memset).
hipError_t launch_absmax(int dtype, const void* a, const void* b, size_t count, double* out,
                         hipStream_t s);
hipError_t launch_reduce(const double* partials, int ngroups, const BinSpec& b, double* result,
                         hipStream_t s);
// Projected power: sums [|c|^2, counts, |n|] x nk over the kept axes' grid.
int projected_groups(int nmesh, int keep);
hipError_t launch_bin_projected(int dtype, int nmesh, const void* cmesh, int keep,
                                const BinSpec& b, double* partials, hipStream_t s);
hipError_t launch_mode_tables(int nmesh, const BinSpec& b, double* partials, int ngroups,
                              double* out, hipStream_t s);
int mode_table_groups(int nmesh);
hipError_t launch_compensate(int dtype, int nmesh, void* cmesh, const void* cmesh_b,
                             const MeshTables& t, int order, int compensated, hipStream_t s);

// c(k) *= table[|n|^2] over a packed spectrum (generate.hip); table holds
// 3 (N/2)^2 + 1 float64 values.
hipError_t launch_shape_packed(int dtype, int nmesh, void* cmesh, const double* table,
                               hipStream_t s);

// Survey multipoles (convolved.hip).  One real spherical harmonic Y_lm:
// ell, |m|, sine = (m < 0), knorm its normalisation (host float64).
struct Harmonic {
  int ell = 0;
  int am = 0;
  int sine = 0;
  double knorm = 0.0;
};
// Doubles of the partials buffer of launch_survey_sums.
size_t survey_sum_partials();
// sums[4] = {sum_data w, sum_data w^2, sum_randoms w, sum_randoms w^2}.
hipError_t launch_survey_sums(int dtype, const void* wd, int64_t nd, const void* wr, int64_t nr,
                              double* partials, double* sums, hipStream_t s);
// value[i] = w_i s_i Y_lm(r^_i) over the concatenated catalog (data first).
hipError_t launch_ylm_value(int dtype, const void* pos, const void* wd, int64_t nd, const void* wr,
                            int64_t nr, const double* observer, const Harmonic& h,
                            const double* sums, void* value, hipStream_t s);
// The harmonics of one set of survey multipoles (at most 1 + 3 + 5 + 7 + 9).
constexpr int kMaxHarmonics = 25;
struct HarmonicSet {
  int n = 0;
  Harmonic h[kMaxHarmonics];
};
// amount[k stride + j] = base[j] Y_k(r^_j), for every harmonic k of the set,
// over the sorted records of launch_bucket (one pass over the records).
hipError_t launch_ylm_records(int dtype, int nmesh, double boxsize, const void* rec,
                              const void* base, const void* bucket_ws, const double* observer,
                              const HarmonicSet& hs, size_t stride, void* amount,
                              hipStream_t s);
// x-pass of a y-transformed spectrum in the y-pass output layout (ymesh,
// from launch_fft_y_relayout) fused with field (+)= coef Y_lm(k^) A / W(k);
// field is in the same layout, its kz = 0 plane goes to plane ([kx][ky],
// N^2 complex) instead; side: N^2 complex scratch for the packed column.
// With ymesh2 (and side2), a second harmonic h2 of the same ell is added in
// the same pass.
hipError_t launch_x_accumulate(int dtype, int nmesh, const void* ymesh, const void* ymesh2,
                               void* field, void* plane, void* side, void* side2,
                               const Harmonic& h, const Harmonic& h2, double coef,
                               const MeshTables& t, int order, int compensated, int first,
                               hipStream_t s);

}  // namespace pk

namespace pk {
// Stages of pk_fftpower, in launch order (names returned by pk_stage_name).
enum Stage { kBucket = 0, kPaintZ, kFftY, kXpassBin, kPlaneBin, kReduce, kNumStages };
}  // namespace pk

struct pk_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  size_t table_bytes = 0;
  std::map<std::pair<int, int>, pk::MeshTables> mesh_tables;  // (nmesh, dtype)
  using BinKey = std::tuple<int, double, double, int, int, int>;  // nmesh, kmin, dk, nk, nmu, los
  std::map<BinKey, std::unique_ptr<pk::BinTables>> bin_tables;
  double* scratch = nullptr;  // plan-time scratch for the mode-table kernel
  size_t scratch_bytes = 0;
  bool timing = false;
  bool timed_once = false;
  bool stage_ran[pk::kNumStages] = {};
  hipEvent_t events[pk::kNumStages + 1] = {};
  // asynchronous lanes: one stream and a completion event each
  struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
  };
  std::vector<Lane> lanes;
  hipEvent_t tables_ready = nullptr;  // recorded on the context stream before lane work
  // second stream of the survey multipoles (x-passes beside the painting)
  // and its events: y-pass output ready [2], x-pass done with it [2], all
  // x-passes done
  hipStream_t aux = nullptr;
  hipEvent_t aux_ev[5] = {};
  // pinned host staging of the result sums read back by the *_to_host calls
  // (a copy into pageable memory goes through a bounce buffer); grown on
  // demand, the pageable vector only if pinned memory is refused
  double* host_stage = nullptr;
  size_t host_stage_n = 0;
  std::vector<double> host_fallback;
  // run-time tuning of the launch choices per (mesh size, precision, window,
  // interlacing, catalog density class); see pk_ctx_set_autotune
  int autotune = 0;
  std::map<std::tuple<int, int, int, int, int>, pk_tune_entry> tuned;
  hipEvent_t tune_ev[2] = {};
};
