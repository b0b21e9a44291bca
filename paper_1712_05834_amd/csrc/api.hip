// The C ABI of libpk (declared in include/pk.h): argument validation, the
// per-mesh-size and per-binning tables, and the launch sequences of the
// stages.  No kernel lives here.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "internal.h"

using namespace pk;

// Device memory of pk_bin_power_noalloc: the squared bin edges and the
// per-workgroup partial sums live in this fixed array instead of memory the
// library allocates.  Each GPU holds its own copy (at its own address) from
// the load of the library until the process ends; every call on a GPU shares
// it, so calls that overlap on one GPU race.
constexpr size_t kNoAllocScratchBytes = 8u << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_create_error;

// Device address of `scratch` per device, looked up once per device with that
// device current (pk_ctx_create).  In host code the array's name is only a
// host-side stand-in; kernels and copies take these addresses.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
hipError_t g_scratch_err[kMaxScratchDevices] = {};

void bind_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) {
    g_scratch_ptr[device] = p;
    g_scratch_err[device] = hipSuccess;
  } else {
    g_scratch_err[device] = e == hipSuccess ? hipErrorInvalidSymbol : e;
    (void)hipGetLastError();
  }
}

void* scratch_of(int device, hipError_t* err) {
  if (device < 0 || device >= kMaxScratchDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}

struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      changed = hipSetDevice(dev) == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

pk_status fail(pk_ctx* ctx, pk_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

pk_status dev_fail(pk_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, PK_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

size_t elem_bytes(const pk_mesh_desc* m) { return m->dtype == PK_F32 ? 4 : 8; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// nullptr when the descriptor is valid, else the reason.
const char* check_mesh(const pk_mesh_desc* m) {
  if (!m) return "mesh descriptor is NULL";
  if (!is_pow2(m->nmesh) || m->nmesh < 8 || m->nmesh > 2048)
    return "nmesh must be a power of two in [8, 2048]";
  if (m->window < 2 || m->window > 4) return "window must be 2 (CIC), 3 (TSC) or 4 (PCS)";
  if (m->interlaced != 0 && m->interlaced != 1) return "interlaced must be 0 or 1";
  if (m->compensated != 0 && m->compensated != 1) return "compensated must be 0 or 1";
  if (m->dtype != PK_F32 && m->dtype != PK_F64) return "dtype must be PK_F32 or PK_F64";
  if (m->reserved != 0) return "reserved must be 0";
  if (!std::isfinite(m->boxsize) || !(m->boxsize > 0)) return "boxsize must be finite and > 0";
  return nullptr;
}

int nsum_of(const pk_bin_desc* b) {
  return b->nk * (1 + b->npoles) + (b->nmu > 1 ? b->nk * b->nmu : 0);
}

// Accumulated sums of a binning: the power, the poles with ell > 0 and the
// (k, mu) bins (ell = 0 poles alias the power).
int nlds_of(const pk_bin_desc* b) {
  int npl = 0;
  for (int i = 0; i < b->npoles; ++i) npl += b->poles[i] != 0 ? 1 : 0;
  // the power sum is accumulated only without (k, mu) bins
  return b->nk * (npl + (b->nmu > 1 ? b->nmu : 1));
}

// LDS bytes of the bin accumulators: two 64-bit words per sum, one flag word.
size_t bin_acc_bytes(const pk_bin_desc* b) {
  return ((size_t)nlds_of(b) * 2 + 1) * sizeof(unsigned long long);
}

// Largest compensation factor of one mode, squared: prod_d sinc^-2p(pi n_d / N)
// is largest at |n_d| = N/2, where each factor is (pi / 2)^p.
double comp2_max(const pk_mesh_desc* m) {
  return m->compensated ? std::pow(3.14159265358979323846 / 2.0, 6.0 * m->window) : 1.0;
}

const char* check_bins(const pk_bin_desc* b, const pk_mesh_desc* m) {
  if (!b) return "bin descriptor is NULL";
  if (!std::isfinite(b->kmin_f) || b->kmin_f < 0) return "kmin_f must be finite and >= 0";
  if (!std::isfinite(b->dk_f) || !(b->dk_f > 0)) return "dk_f must be finite and > 0";
  if (b->nk < 1 || b->nk > 4096) return "nk must be in [1, 4096]";
  if (b->nmu < 0 || b->nmu > 64) return "nmu must be in [0, 64]";
  if (b->npoles < 0 || b->npoles > 4) return "npoles must be in [0, 4]";
  for (int i = 0; i < b->npoles; ++i) {
    const int l = b->poles[i];
    if (l != 0 && l != 2 && l != 4 && l != 6) return "poles must be even ell in {0, 2, 4, 6}";
    for (int j = 0; j < i; ++j)
      if (b->poles[j] == l) return "poles must be distinct";
  }
  if (b->los < 0 || b->los > 2) return "los must be an axis 0, 1 or 2";
  const double top = b->kmin_f + b->nk * b->dk_f;
  if (m) {
    const double nmax = std::sqrt(3.0) * (m->nmesh / 2) + 1.0;
    if (top > nmax * 4.0 + 16.0) return "top edge far beyond the largest mode";
    if (m->interlaced && top > m->nmesh / 2)
      return "interlaced meshes: the top edge kmin_f + nk * dk_f may not exceed N/2";
  }
  return nullptr;
}

// Slot limits of the LDS bins (float64).
constexpr int kMaxLdsSlots = 8192;

const char* check_lds(const pk_bin_desc* b, const pk_mesh_desc* m) {
  if (nsum_of(b) > kMaxLdsSlots) return "too many bin slots for the LDS accumulator";
  if (bin_acc_bytes(b) > kLdsBytesPerGroup)
    return "too many bin slots for the LDS accumulator";
  if (m && xpass_static_lds(m->dtype, m->nmesh) + bin_acc_bytes(b) > kLdsBytesPerGroup)
    return "too many bin slots for the LDS accumulator at this mesh size and precision";
  if (mode_table_slots(b->nk, b->nmu > 1 ? b->nmu : 0) > kMaxLdsSlots)
    return "too many (k, mu) bins for the mode-table accumulator";
  return nullptr;
}

template <typename T>
void fill_mesh_tables(int n, unsigned char* buf, size_t off_tw, size_t off_ph, size_t off_si) {
  T* tw = reinterpret_cast<T*>(buf + off_tw);
  T* ph = reinterpret_cast<T*>(buf + off_ph);
  T* si = reinterpret_cast<T*>(buf + off_si);
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < n; ++j) {
    const double a = 2.0 * pi * (double)j / (double)n;
    tw[2 * j] = (T)std::cos(a);
    tw[2 * j + 1] = (T)(-std::sin(a));
  }
  for (int s = -3 * (n / 2); s <= 3 * (n / 2); ++s) {
    const double a = pi * (double)s / (double)n;
    const int i = s + 3 * (n / 2);
    ph[2 * i] = (T)std::cos(a);
    ph[2 * i + 1] = (T)std::sin(a);
  }
  for (int p = 2; p <= 4; ++p) {
    for (int i = 0; i < n; ++i) {
      const int k = i < n / 2 ? i : i - n;
      const double x = pi * (double)k / (double)n;
      const double sc = k == 0 ? 1.0 : std::sin(x) / x;
      si[(size_t)(p - 2) * n + i] = (T)std::pow(sc, -(double)p);
    }
  }
}

pk_status get_mesh_tables(pk_ctx* ctx, int n, int dtype, const MeshTables** out) {
  const auto key = std::make_pair(n, dtype);
  auto it = ctx->mesh_tables.find(key);
  if (it != ctx->mesh_tables.end()) {
    *out = &it->second;
    return PK_OK;
  }
  const size_t es = dtype == PK_F32 ? 4 : 8;
  const size_t off_tw = 0;
  const size_t off_ph = align256(off_tw + (size_t)n * 2 * es);
  const size_t off_si = align256(off_ph + (size_t)(3 * n + 1) * 2 * es);
  const size_t bytes = align256(off_si + (size_t)3 * n * es);
  std::vector<unsigned char> host(bytes, 0);
  if (dtype == PK_F32)
    fill_mesh_tables<float>(n, host.data(), off_tw, off_ph, off_si);
  else
    fill_mesh_tables<double>(n, host.data(), off_tw, off_ph, off_si);
  void* dev = nullptr;
  hipError_t e = hipMalloc(&dev, bytes);
  if (e != hipSuccess) return fail(ctx, PK_ENOMEM, std::string("hipMalloc(tables): ") + hipGetErrorString(e));
  e = hipMemcpyAsync(dev, host.data(), bytes, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(dev);
    return dev_fail(ctx, e, "upload of mesh tables");
  }
  MeshTables t;
  t.dev = dev;
  t.bytes = bytes;
  t.tw = static_cast<unsigned char*>(dev) + off_tw;
  t.phase = static_cast<unsigned char*>(dev) + off_ph;
  t.sinc_inv = static_cast<unsigned char*>(dev) + off_si;
  ctx->table_bytes += bytes;
  auto res = ctx->mesh_tables.emplace(key, t);
  *out = &res.first->second;
  return PK_OK;
}

// Squared bin edges e_b^2 = (kmin + b dk)^2 in float64, without contraction
// into fused multiply-adds, so that each value is the correctly rounded
// result of the three operations in this order.
#pragma clang fp contract(off)
void edges_squared(double kmin, double dk, int nk, std::vector<double>& e2) {
  e2.resize(nk + 1);
  for (int i = 0; i <= nk; ++i) {
    volatile double prod = (double)i * dk;
    volatile double e = kmin + prod;
    e2[i] = e * e;
  }
}
#pragma clang fp contract(on)

BinSpec make_spec(const pk_mesh_desc* m, const pk_bin_desc* b, const double* e2_dev) {
  BinSpec s;
  s.nmesh = m->nmesh;
  s.nk = b->nk;
  s.nmu = b->nmu > 1 ? b->nmu : 0;
  s.los = b->los;
  s.npoles = b->npoles;
  s.zero_mask = 0;
  s.npl = 0;
  for (int i = 0; i < b->npoles; ++i) {
    if (b->poles[i] == 0) {
      s.zero_mask |= 1 << i;
    } else {
      s.pole_ell[s.npl] = b->poles[i];
      s.pole_slot[s.npl] = b->nk * (1 + i);
      ++s.npl;
    }
  }
  s.off2d = b->nmu > 1 ? b->nk * (1 + b->npoles) : -1;
  s.nsum = nsum_of(b);
  s.power_from_2d = b->nmu > 1 ? 1 : 0;
  const int p0 = s.power_from_2d ? 0 : 1;  // LDS slots of the power sum (k-bins)
  for (int i = 0; i < s.npl; ++i) s.pole_lds[i] = b->nk * (p0 + i);
  s.fix_hb = m->dtype == PK_F32 ? 32 : 64;
  s.off2d_lds = b->nmu > 1 ? b->nk * s.npl : -1;
  s.nlds = nlds_of(b);
  s.kmin_f = b->kmin_f;
  s.dk_f = b->dk_f;
  s.e2 = e2_dev;
  // Whole-number edges e_b = kmin + b dk: e_b^2 <= n^2 iff e_b <= isqrt(n^2),
  // so the bin follows from the integer square root alone.
  const double lim = 1 << 20;
  if (b->kmin_f == std::floor(b->kmin_f) && b->dk_f == std::floor(b->dk_f) && b->kmin_f < lim &&
      b->dk_f < lim) {
    s.int_edges = 1;
    s.kmin_i = (int)b->kmin_f;
    s.dk_i = (int)b->dk_f;
  }
  return s;
}

pk_status get_bin_tables(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                         BinTables** out) {
  const int nmu = b->nmu > 1 ? b->nmu : 0;
  const pk_ctx::BinKey key{m->nmesh, b->kmin_f, b->dk_f, b->nk, nmu, b->los};
  auto it = ctx->bin_tables.find(key);
  if (it != ctx->bin_tables.end()) {
    *out = it->second.get();
    return PK_OK;
  }
  std::unique_ptr<BinTables> bt(new (std::nothrow) BinTables());
  if (!bt) return fail(ctx, PK_ENOMEM, "host allocation of bin tables");
  std::vector<double> e2;
  edges_squared(b->kmin_f, b->dk_f, b->nk, e2);
  hipError_t e = hipMalloc(&bt->e2_dev, e2.size() * sizeof(double));
  if (e != hipSuccess) return fail(ctx, PK_ENOMEM, std::string("hipMalloc(edges): ") + hipGetErrorString(e));
  e = hipMemcpyAsync(bt->e2_dev, e2.data(), e2.size() * sizeof(double), hipMemcpyHostToDevice,
                     ctx->stream);
  const BinSpec spec = make_spec(m, b, bt->e2_dev);
  const int groups = mode_table_groups(m->nmesh);
  const int slots = mode_table_slots(b->nk, nmu);
  double* scratch = nullptr;
  // partial rows of two words per slot, then the reduced table
  if (e == hipSuccess) e = hipMalloc(&scratch, ((size_t)2 * groups + 1) * slots * sizeof(double));
  double* table = scratch + (size_t)2 * groups * slots;
  if (e == hipSuccess)
    e = launch_mode_tables(m->nmesh, spec, scratch, groups, table, ctx->stream);
  std::vector<double> host(slots);
  if (e == hipSuccess)
    e = hipMemcpyAsync(host.data(), table, slots * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (scratch) (void)hipFree(scratch);
  if (e != hipSuccess) {
    (void)hipFree(bt->e2_dev);
    return dev_fail(ctx, e, "mode tables");
  }
  const int nk = b->nk;
  bt->modes.resize(nk);
  bt->sum_n.resize(nk);
  for (int k = 0; k < nk; ++k) {
    uint64_t c;
    std::memcpy(&c, &host[k], 8);
    bt->modes[k] = (int64_t)c;
    bt->sum_n[k] = host[nk + k];
  }
  if (nmu > 1) {
    const int n2 = nk * nmu;
    bt->modes2d.resize(n2);
    bt->sum_n2d.resize(n2);
    bt->sum_mu2d.resize(n2);
    for (int f = 0; f < n2; ++f) {
      uint64_t c;
      std::memcpy(&c, &host[2 * nk + f], 8);
      bt->modes2d[f] = (int64_t)c;
      bt->sum_n2d[f] = host[2 * nk + n2 + f];
      bt->sum_mu2d[f] = host[2 * nk + 2 * n2 + f];
    }
  }
  ctx->table_bytes += e2.size() * sizeof(double);
  *out = bt.get();
  ctx->bin_tables.emplace(key, std::move(bt));
  return PK_OK;
}

// Largest (Hermitian-weighted) number of modes in one bin of a binning.
double mode_max(const BinTables* bt) {
  int64_t mx = 1;
  for (int64_t c : bt->modes) mx = c > mx ? c : mx;
  return (double)mx;
}

// Context-owned scratch for the stand-alone binning (partial sums); grown on
// demand and kept until pk_ctx_destroy.
pk_status get_scratch(pk_ctx* ctx, size_t bytes, double** out) {
  if (ctx->scratch_bytes < bytes) {
    if (ctx->scratch) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(ctx->scratch);
      ctx->table_bytes -= ctx->scratch_bytes;
      ctx->scratch = nullptr;
      ctx->scratch_bytes = 0;
    }
    hipError_t e = hipMalloc(&ctx->scratch, bytes);
    if (e != hipSuccess) {
      ctx->scratch = nullptr;
      return fail(ctx, PK_ENOMEM, std::string("hipMalloc(scratch): ") + hipGetErrorString(e));
    }
    ctx->scratch_bytes = bytes;
    ctx->table_bytes += bytes;
  }
  *out = ctx->scratch;
  return PK_OK;
}

// Copies `count` result doubles to the context's host staging (pinned when
// possible) after the work enqueued before it; *h points at them.
pk_status read_result(pk_ctx* ctx, const double* result_dev, size_t count, const double** h,
                      const char* who) {
  double* dst = nullptr;
  if (ctx->host_stage_n < count) {
    if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
    ctx->host_stage = nullptr;
    ctx->host_stage_n = 0;
    void* p = nullptr;
    if (hipHostMalloc(&p, count * sizeof(double), hipHostMallocDefault) == hipSuccess) {
      ctx->host_stage = static_cast<double*>(p);
      ctx->host_stage_n = count;
    } else {
      (void)hipGetLastError();  // refused: read through pageable memory instead
    }
  }
  if (ctx->host_stage_n >= count) {
    dst = ctx->host_stage;
  } else {
    ctx->host_fallback.resize(count);
    dst = ctx->host_fallback.data();
  }
  hipError_t e = hipMemcpyAsync(dst, result_dev, count * sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, who);
  *h = dst;
  return PK_OK;
}

// Records the start event of a stage of pk_fftpower when timing is enabled.
void mark_stage(pk_ctx* ctx, int stage) {
  if (!ctx->timing) return;
  (void)hipEventRecord(ctx->events[stage], ctx->stream);
  ctx->stage_ran[stage] = true;
}

void mark_end(pk_ctx* ctx) {
  if (!ctx->timing) return;
  (void)hipEventRecord(ctx->events[kNumStages], ctx->stream);
  ctx->timed_once = true;
}

const char* const kStageNames[kNumStages] = {"bucket", "paint_z", "fft_y",
                                             "xpass_bin", "plane_bin", "reduce"};

// Workspace layout of pk_fftpower (offsets in bytes, 256-aligned).
struct Layout {
  size_t mesh_a = 0, mesh_b = 0, ytmp = 0, side_a = 0, side_b = 0, partials = 0, bucket = 0,
         rec = 0, wrec = 0, total = 0;
  int gx = 0, gp = 0;
};

Layout layout_of(const pk_mesh_desc* m, const pk_bin_desc* b, int64_t npart) {
  Layout l;
  const size_t n = (size_t)m->nmesh;
  const size_t es = elem_bytes(m);
  const size_t mesh = align256(n * n * n * es);
  const size_t side = align256(n * n * 2 * es);
  const int two = m->interlaced ? 1 : 0;
  const size_t np = npart > 0 ? (size_t)npart : 0;
  l.gx = xpass_bin_groups(m->dtype, m->nmesh, bin_acc_bytes(b));
  l.gp = plane_bin_groups(m->nmesh);
  size_t off = 0;
  l.mesh_a = off;
  off += mesh;
  l.mesh_b = off;
  off += two * mesh;
  l.ytmp = off;  // y-pass output of mesh A (mesh B's goes to mesh A's buffer)
  off += mesh;
  l.side_a = off;
  off += side;
  l.side_b = off;
  off += two * side;
  l.partials = off;
  off += align256((size_t)(l.gx + l.gp) * 2 * nsum_of(b) * sizeof(double));
  l.bucket = off;
  off += align256(bucket_bytes(m->nmesh));
  l.rec = off;
  off += align256(np * 4 * es);  // one 4-vector record per particle
  l.wrec = off;
  off += align256(np * es);
  l.total = off;
  return l;
}

// Binning of one packed spectrum (|c|^2) or of two (Re(c1 conj(c2))).
pk_status bin_packed(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b, const void* c1,
                     const void* c2, double* result_dev, const char* who) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_bins(b, m)) return fail(ctx, PK_EINVAL, why);
  if (!c1 || !result_dev) return fail(ctx, PK_EINVAL, "cmesh or result is NULL");
  if (const char* why = check_lds(b, m)) return fail(ctx, PK_EUNSUPPORTED, why);
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  BinTables* bt = nullptr;
  if (pk_status st = get_bin_tables(ctx, m, b, &bt)) return st;
  const MeshTables* t = nullptr;
  if (pk_status st = get_mesh_tables(ctx, m->nmesh, m->dtype, &t)) return st;
  BinSpec spec = make_spec(m, b, bt->e2_dev);
  const size_t gb = (size_t)bin_packed_groups(m->nmesh);
  const int gp = plane_bin_groups(m->nmesh);
  double* partials = nullptr;
  if (pk_status st = get_scratch(ctx, ((gb + gp) * 2 * spec.nsum + 1) * sizeof(double), &partials))
    return st;
  // the bound of the exact sums: every term is at most 2 max|component|^2
  // per mode, and a bin holds at most all N^3 (weighted) modes of the packed
  // spectrum (a factor 4 to spare); the same scale as pk_bin_power_noalloc,
  // so that the two give the same sums bit for bit
  double* amax = partials + (gb + gp) * 2 * spec.nsum;
  spec.bound_scale = 8.0 * (double)m->nmesh * m->nmesh * m->nmesh;
  spec.bound_dev = amax;
  spec.bound_sq = 1;
  hipError_t e = launch_absmax(m->dtype, c1, c2, (size_t)m->nmesh * m->nmesh * m->nmesh, amax,
                               ctx->stream);
  if (e == hipSuccess)
    e = launch_bin_packed(m->dtype, m->nmesh, c1, c2, spec, partials, ctx->stream);
  if (e == hipSuccess)
    e = launch_plane_bin(m->dtype, m->nmesh, c1, c2, m->nmesh / 2, *t, m->window, 0, spec,
                         partials + gb * 2 * spec.nsum, ctx->stream, c2 ? 1 : 0);
  if (e == hipSuccess) e = launch_reduce(partials, (int)(gb + gp), spec, result_dev, ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, who);
  return PK_OK;
}

}  // namespace

extern "C" {

pk_status pk_ctx_create(pk_ctx** ctx, int device, void* hip_stream) {
  if (!ctx) {
    g_create_error = "ctx is NULL";
    return PK_EINVAL;
  }
  *ctx = nullptr;
  if (device != PK_DEVICE_NONE) {
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) {
      g_create_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(e);
      return PK_EDEVICE;
    }
    if (device < 0 || device >= ndev) {
      g_create_error = "device index out of range";
      return PK_EINVAL;
    }
  }
  pk_ctx* c = new (std::nothrow) pk_ctx();
  if (!c) {
    g_create_error = "host allocation of the context";
    return PK_ENOMEM;
  }
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (device != PK_DEVICE_NONE) {
    DeviceGuard g(device);
    bind_scratch(device);  // a failure is reported by pk_bin_power_noalloc
  }
  *ctx = c;
  return PK_OK;
}

void pk_ctx_destroy(pk_ctx* ctx) {
  if (!ctx) return;
  if (ctx->device == PK_DEVICE_NONE) {
    delete ctx;
    return;
  }
  DeviceGuard g(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t ev : ctx->tune_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& kv : ctx->mesh_tables) (void)hipFree(kv.second.dev);
  for (auto& kv : ctx->bin_tables) (void)hipFree(kv.second->e2_dev);
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  for (auto& ev : ctx->events)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& ln : ctx->lanes) {
    (void)hipStreamSynchronize(ln.stream);
    (void)hipEventDestroy(ln.done);
    (void)hipStreamDestroy(ln.stream);
  }
  if (ctx->tables_ready) (void)hipEventDestroy(ctx->tables_ready);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  for (auto& ev : ctx->aux_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
  delete ctx;
}

const char* pk_last_error(const pk_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

size_t pk_mesh_bytes(const pk_mesh_desc* m) {
  if (check_mesh(m)) return 0;
  const size_t n = (size_t)m->nmesh;
  return n * n * n * elem_bytes(m);
}

size_t pk_result_doubles(const pk_bin_desc* b) {
  if (check_bins(b, nullptr)) return 0;
  return (size_t)nsum_of(b) + 2;
}

int32_t pk_num_kbins(double kmin_f, double dk_f, double kmax_f) {
  if (!std::isfinite(kmin_f) || !std::isfinite(dk_f) || !std::isfinite(kmax_f)) return PK_EINVAL;
  if (kmin_f < 0 || !(dk_f > 0) || !(kmax_f > kmin_f)) return PK_EINVAL;
  const double nk = std::floor((kmax_f - kmin_f) / dk_f + 1e-9);
  if (nk > 4096.0) return PK_EUNSUPPORTED;
  return (int32_t)nk;
}

size_t pk_workspace_bytes(const pk_mesh_desc* m, const pk_bin_desc* b, int64_t npart) {
  (void)npart;
  if (check_mesh(m) || check_bins(b, m)) return 0;
  if (npart < 0) return 0;
  return layout_of(m, b, npart).total;
}

size_t pk_ctx_table_bytes(const pk_ctx* ctx) { return ctx ? ctx->table_bytes : 0; }

pk_status pk_paint(pk_ctx* ctx, const pk_mesh_desc* m, const void* pos, const void* weight,
                   int64_t n, double shift_cells, void* mesh, double* wsums) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (n < 0) return fail(ctx, PK_EINVAL, "n must be >= 0");
  if (n > 0 && !pos) return fail(ctx, PK_EINVAL, "pos is NULL with n > 0");
  if (!mesh) return fail(ctx, PK_EINVAL, "mesh is NULL");
  if (!std::isfinite(shift_cells)) return fail(ctx, PK_EINVAL, "shift_cells must be finite");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_fill_zero(mesh, pk_mesh_bytes(m), ctx->stream);
  if (e == hipSuccess && wsums) e = launch_fill_zero(wsums, 2 * sizeof(double), ctx->stream);
  if (e == hipSuccess && n > 0)
    e = launch_paint_atomic(m->dtype, m->window, m->nmesh, m->boxsize, pos, weight, n, shift_cells,
                            mesh, 0.0, nullptr, wsums, ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_paint");
  return PK_OK;
}

pk_status pk_fft_r2c(pk_ctx* ctx, const pk_mesh_desc* m, void* mesh_inout) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (!mesh_inout) return fail(ctx, PK_EINVAL, "mesh is NULL");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  const MeshTables* t = nullptr;
  if (pk_status st = get_mesh_tables(ctx, m->nmesh, m->dtype, &t)) return st;
  const size_t bytes = pk_mesh_bytes(m);
  hipError_t e = launch_fft_z(m->dtype, m->nmesh, mesh_inout, 1, bytes, t->tw, nullptr, ctx->stream);
  if (e == hipSuccess) e = launch_fft_cols(m->dtype, m->nmesh, mesh_inout, 1, bytes, t->tw, 1, ctx->stream);
  if (e == hipSuccess) e = launch_fft_cols(m->dtype, m->nmesh, mesh_inout, 1, bytes, t->tw, 0, ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_fft_r2c");
  return PK_OK;
}

pk_status pk_fft_c2r(pk_ctx* ctx, const pk_mesh_desc* m, void* mesh_inout) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (!mesh_inout) return fail(ctx, PK_EINVAL, "mesh is NULL");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  const MeshTables* t = nullptr;
  if (pk_status st = get_mesh_tables(ctx, m->nmesh, m->dtype, &t)) return st;
  const size_t bytes = pk_mesh_bytes(m);
  hipError_t e = launch_fft_cols(m->dtype, m->nmesh, mesh_inout, 1, bytes, t->tw, 0, ctx->stream, 1);
  if (e == hipSuccess)
    e = launch_fft_cols(m->dtype, m->nmesh, mesh_inout, 1, bytes, t->tw, 1, ctx->stream, 1);
  if (e == hipSuccess) e = launch_ifft_z(m->dtype, m->nmesh, mesh_inout, t->tw, ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_fft_c2r");
  return PK_OK;
}

int64_t pk_shape_table_len(const pk_mesh_desc* m) {
  if (check_mesh(m)) return 0;
  const int64_t h = m->nmesh / 2;
  return 3 * h * h + 1;
}

pk_status pk_shape_spectrum(pk_ctx* ctx, const pk_mesh_desc* m, void* cmesh_inout,
                            const double* table_dev, int64_t table_len) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (!cmesh_inout || !table_dev) return fail(ctx, PK_EINVAL, "cmesh or table is NULL");
  if (table_len < pk_shape_table_len(m)) return fail(ctx, PK_EINVAL, "table shorter than 3 (N/2)^2 + 1");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  hipError_t e = launch_shape_packed(m->dtype, m->nmesh, cmesh_inout, table_dev, ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_shape_spectrum");
  return PK_OK;
}

pk_status pk_compensate(pk_ctx* ctx, const pk_mesh_desc* m, void* cmesh_inout,
                        const void* cmesh_b) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (!cmesh_inout) return fail(ctx, PK_EINVAL, "cmesh is NULL");
  if (cmesh_b == cmesh_inout) return fail(ctx, PK_EINVAL, "cmesh_b aliases cmesh");
  if (!cmesh_b && !m->compensated) return PK_OK;
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  const MeshTables* t = nullptr;
  if (pk_status st = get_mesh_tables(ctx, m->nmesh, m->dtype, &t)) return st;
  hipError_t e = launch_compensate(m->dtype, m->nmesh, cmesh_inout, cmesh_b, *t, m->window,
                                   m->compensated, ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_compensate");
  return PK_OK;
}

pk_status pk_bin_power(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                       const void* cmesh, double* result_dev) {
  return bin_packed(ctx, m, b, cmesh, nullptr, result_dev, "pk_bin_power");
}

pk_status pk_bin_power_noalloc(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                               const void* cmesh, double* result_dev) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_bins(b, m)) return fail(ctx, PK_EINVAL, why);
  if (!cmesh || !result_dev) return fail(ctx, PK_EINVAL, "cmesh or result is NULL");
  if (const char* why = check_lds(b, m)) return fail(ctx, PK_EUNSUPPORTED, why);
  // scratch: the nk + 1 squared edges, then one row of nsum partial sums per
  // workgroup of the two binning kernels; the grids shrink to the rows that fit
  const size_t edges = align256(((size_t)b->nk + 1) * sizeof(double)) + 256;  // + the max
  const size_t row = (size_t)nsum_of(b) * 2 * sizeof(double);
  const size_t rows = edges < kNoAllocScratchBytes ? (kNoAllocScratchBytes - edges) / row : 0;
  if (rows < 2)
    return fail(ctx, PK_EUNSUPPORTED,
                "pk_bin_power_noalloc: the bin sums need more than its " +
                    std::to_string(kNoAllocScratchBytes >> 20) + " MiB of fixed device memory");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  hipError_t e = hipSuccess;
  unsigned char* base = static_cast<unsigned char*>(scratch_of(ctx->device, &e));
  if (!base)
    return fail(ctx, PK_EDEVICE, std::string("pk_bin_power_noalloc: no address of the fixed "
                                             "scratch on this device: ") + hipGetErrorString(e));
  DeviceGuard g(ctx->device);
  const int gp = (int)std::min<size_t>(std::min(plane_bin_groups(m->nmesh), 64), rows / 2);
  const int gb = (int)std::min<size_t>(bin_packed_groups(m->nmesh), rows - gp);
  double* e2 = reinterpret_cast<double*>(base);
  double* amax = reinterpret_cast<double*>(base + edges - 256);
  double* partials = reinterpret_cast<double*>(base + edges);
  BinSpec spec = make_spec(m, b, e2);
  // bound of the exact sums as in pk_bin_power, with every mode of the
  // packed spectrum (N^3 counted with their weights) as the count
  const double nmodes = (double)m->nmesh * m->nmesh * m->nmesh;
  spec.bound_scale = 8.0 * nmodes;
  spec.bound_dev = amax;
  spec.bound_sq = 1;
  e = launch_edges_squared(b->kmin_f, b->dk_f, b->nk, e2, ctx->stream);
  if (e == hipSuccess)
    e = launch_absmax(m->dtype, cmesh, nullptr, (size_t)m->nmesh * m->nmesh * m->nmesh, amax,
                      ctx->stream);
  if (e == hipSuccess)
    e = launch_bin_packed(m->dtype, m->nmesh, cmesh, nullptr, spec, partials, ctx->stream, 0, gb);
  if (e == hipSuccess)
    e = launch_plane_bin(m->dtype, m->nmesh, cmesh, nullptr, m->nmesh / 2, MeshTables{}, m->window,
                         0, spec, partials + (size_t)gb * 2 * spec.nsum, ctx->stream, 0, gp);
  if (e == hipSuccess) e = launch_reduce(partials, gb + gp, spec, result_dev, ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_bin_power_noalloc");
  return PK_OK;
}

size_t pk_projected_doubles(const pk_bin_desc* b) {
  if (!b || b->nk < 1 || b->nk > 4096) return 0;
  return (size_t)3 * b->nk + 2;
}

namespace {
const char* check_projected(const pk_bin_desc* b, int keep) {
  if (keep <= 0 || keep > 7 || keep == 7) return "keep must name one or two axes (bits 1, 2, 4)";
  if (b->nmu > 1 || b->npoles != 0) return "the projected power has no mu bins or multipoles";
  if (3 * b->nk > kMaxLdsSlots) return "too many bins for the LDS accumulator";
  return nullptr;
}
}  // namespace

pk_status pk_bin_projected(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b, int keep,
                           const void* cmesh, double* result_dev) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_bins(b, m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_projected(b, keep)) return fail(ctx, PK_EINVAL, why);
  if (!cmesh || !result_dev) return fail(ctx, PK_EINVAL, "cmesh or result is NULL");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  BinTables* bt = nullptr;
  if (pk_status st = get_bin_tables(ctx, m, b, &bt)) return st;
  BinSpec spec = make_spec(m, b, bt->e2_dev);
  spec.nsum = 3 * b->nk;  // the reduce sums these slots plainly
  spec.npoles = 0;
  spec.npl = 0;
  spec.zero_mask = 0;
  spec.off2d = -1;
  spec.exact = 0;  // float64 partial rows
  const int gp = projected_groups(m->nmesh, keep);
  double* partials = nullptr;
  if (pk_status st = get_scratch(ctx, (size_t)gp * 2 * spec.nsum * sizeof(double), &partials))
    return st;
  hipError_t e = launch_bin_projected(m->dtype, m->nmesh, cmesh, keep, spec, partials, ctx->stream);
  if (e == hipSuccess) e = launch_reduce(partials, gp, spec, result_dev, ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_bin_projected");
  return PK_OK;
}

pk_status pk_projected_to_host(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                               int keep, const double* result_dev, pk_result* out) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_bins(b, m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_projected(b, keep)) return fail(ctx, PK_EINVAL, why);
  if (!result_dev || !out || !out->k || !out->power || !out->modes)
    return fail(ctx, PK_EINVAL, "result, out or one of its 1-D arrays is NULL");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  const int nk = b->nk;
  const double* h = nullptr;
  if (pk_status st = read_result(ctx, result_dev, 3 * (size_t)nk + 2, &h, "pk_projected_to_host"))
    return st;
  const int d = (keep & 1) + ((keep >> 1) & 1) + ((keep >> 2) & 1);
  const double L = m->boxsize;
  const double area = d == 1 ? L : L * L;
  const double kf = 2.0 * 3.14159265358979323846 / L;
  const double wsum = h[3 * (size_t)nk], w2sum = h[3 * (size_t)nk + 1];
  const double norm = area / (wsum * wsum);
  const double nan = std::nan("");
  for (int k = 0; k < nk; ++k) {
    const int64_t nb = (int64_t)std::llround(h[(size_t)nk + k]);
    out->modes[k] = nb;
    out->k[k] = nb ? kf * h[2 * (size_t)nk + k] / (double)nb : nan;
    out->power[k] = nb ? norm * h[k] / (double)nb : nan;
  }
  out->shotnoise = area * w2sum / (wsum * wsum);
  out->wsum = wsum;
  out->w2sum = w2sum;
  return PK_OK;
}

pk_status pk_bin_cross(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                       const void* cmesh1, const void* cmesh2, double* result_dev) {
  if (ctx && !cmesh2) return fail(ctx, PK_EINVAL, "cmesh2 is NULL");
  return bin_packed(ctx, m, b, cmesh1, cmesh2, result_dev, "pk_bin_cross");
}

}  // extern "C"

namespace {

// The sorted painting indexes its records with 32-bit offsets.
constexpr int64_t kMaxSortedParticles = 2147483647;

// Argument checks shared by the synchronous and the lane entry points.
pk_status check_fftpower(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                         const void* pos, int64_t n, const void* workspace,
                         size_t workspace_bytes, const double* result_dev) {
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_bins(b, m)) return fail(ctx, PK_EINVAL, why);
  if (n < 0) return fail(ctx, PK_EINVAL, "n must be >= 0");
  if (n > kMaxSortedParticles)
    return fail(ctx, PK_EUNSUPPORTED, "more than 2^31 - 1 particles (32-bit record offsets)");
  if (n > 0 && !pos) return fail(ctx, PK_EINVAL, "pos is NULL with n > 0");
  if (!workspace || !result_dev) return fail(ctx, PK_EINVAL, "workspace or result is NULL");
  const Layout l = layout_of(m, b, n);
  if (workspace_bytes < l.total) return fail(ctx, PK_EINVAL, "workspace too small");
  if (const char* why = check_lds(b, m)) return fail(ctx, PK_EUNSUPPORTED, why);
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  return PK_OK;
}

// Enqueues the whole path on stream s (tables must exist); stage events are
// recorded only for the context stream.
// Key of the tuning table: mesh size, precision, window, interlacing and
// the density class round(log2(n / N^3)).
std::tuple<int, int, int, int, int> tune_key(const pk_mesh_desc* m, int64_t n) {
  const double cells = (double)m->nmesh * m->nmesh * m->nmesh;
  const int dens = n > 0 ? (int)std::lround(std::log2((double)n / cells)) : -64;
  return std::make_tuple(m->nmesh, m->dtype, m->window, m->interlaced, dens);
}

pk_tune_entry default_choice(const pk_mesh_desc* m, int64_t n) {
  pk_tune_entry c{};
  std::tie(c.nmesh, c.dtype, c.window, c.interlaced, c.density) = tune_key(m, n);
  c.split = -1;  // the window's default
  c.xpass_per_cu = 0;
  c.ms = 0.0;
  return c;
}

pk_tune_entry choice_for(const pk_ctx* ctx, const pk_mesh_desc* m, int64_t n) {
  auto it = ctx->tuned.find(tune_key(m, n));
  return it != ctx->tuned.end() ? it->second : default_choice(m, n);
}

hipError_t enqueue_fftpower(pk_ctx* ctx, hipStream_t s, const pk_mesh_desc* m,
                            const BinSpec& spec, const MeshTables* t, const void* pos,
                            const void* weight, const void* value, int64_t n, void* workspace,
                            const Layout& l, double* result_dev, const pk_tune_entry& ch) {
  const bool timed = s == ctx->stream;
  auto stage = [&](int st) {
    if (timed) mark_stage(ctx, st);
  };
  char* ws = static_cast<char*>(workspace);
  void* mesh_a = ws + l.mesh_a;
  void* mesh_b = m->interlaced ? ws + l.mesh_b : nullptr;
  void* side_a = ws + l.side_a;
  void* side_b = m->interlaced ? ws + l.side_b : nullptr;
  double* partials = reinterpret_cast<double*>(ws + l.partials);
  double* wsums = result_dev + spec.nsum;
  // bound of the exact bin sums: |c(k)| <= sum |w| <= sqrt(n sum w^2) for a
  // painted field (window weights are positive and sum to one), times the
  // compensation and the number of modes per bin (prepare_tables), the
  // Hermitian weight and the pair of modes binned together (a factor 8)
  BinSpec bs = spec;
  bs.bound_scale = spec.bound_scale * (double)(n > 0 ? n : 1);
  bs.bound_dev = wsums + 1;
  bs.bound_sq = 0;
  if (timed)
    for (bool& r : ctx->stage_ran) r = false;
  void* rec = ws + l.rec;
  void* wrec = (weight || value) ? ws + l.wrec : nullptr;
  stage(kBucket);
  // the meshes are free until the painting: scratch of the bucketing
  hipError_t e = launch_bucket(m->dtype, m->nmesh, m->boxsize, pos, weight, value, n,
                               ws + l.bucket, rec, wrec, wsums, s, ws + l.mesh_a,
                               l.side_a - l.mesh_a);
  stage(kPaintZ);
  if (e == hipSuccess)
    e = launch_paint_z(m->dtype, m->nmesh, m->window, m->interlaced != 0, rec, wrec,
                       ws + l.bucket, wsums, t->tw, mesh_a, mesh_b, s, ch.split);
  // y-pass out of place into the x-pass layout: A into the spare buffer,
  // then B into A's buffer, which A no longer needs
  stage(kFftY);
  void* ya = ws + l.ytmp;
  void* yb = m->interlaced ? mesh_a : nullptr;
  if (e == hipSuccess) e = launch_fft_y_relayout(m->dtype, m->nmesh, mesh_a, ya, t->tw, s);
  if (e == hipSuccess && yb) e = launch_fft_y_relayout(m->dtype, m->nmesh, mesh_b, yb, t->tw, s);
  stage(kXpassBin);
  // x-pass workgroups: as many as fit (l.gx) or the tuned number per CU
  const int gx = ch.xpass_per_cu > 0
                     ? std::min(l.gx, (int)kComputeUnits * ch.xpass_per_cu) : l.gx;
  if (e == hipSuccess)
    e = launch_xpass_bin(m->dtype, m->nmesh, ya, yb, *t, m->window, m->compensated, bs,
                         partials, side_a, side_b, s, gx);
  stage(kPlaneBin);
  if (e == hipSuccess)
    e = launch_plane_bin(m->dtype, m->nmesh, side_a, side_b, 1, *t, m->window, m->compensated,
                         bs, partials + (size_t)gx * 2 * spec.nsum, s);
  stage(kReduce);
  if (e == hipSuccess) e = launch_reduce(partials, gx + l.gp, bs, result_dev, s);
  if (timed) mark_end(ctx);
  return e;
}

// Builds (on the context stream) whatever tables the request needs and
// returns them with its kernel-side bin description.
pk_status prepare_tables(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                         const MeshTables** t, BinSpec* spec) {
  BinTables* bt = nullptr;
  if (pk_status st = get_bin_tables(ctx, m, b, &bt)) return st;
  if (pk_status st = get_mesh_tables(ctx, m->nmesh, m->dtype, t)) return st;
  *spec = make_spec(m, b, bt->e2_dev);
  spec->bound_scale = 8.0 * comp2_max(m) * mode_max(bt);  // times n sum w^2 at launch
  return PK_OK;
}

// Creates the lane streams and events up to n lanes.
pk_status ensure_lanes(pk_ctx* ctx, int n) {
  while ((int)ctx->lanes.size() < n) {
    pk_ctx::Lane ln;
    hipError_t e = hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ln.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (ln.stream) (void)hipStreamDestroy(ln.stream);
      return dev_fail(ctx, e, "lane creation");
    }
    ctx->lanes.push_back(ln);
  }
  if (!ctx->tables_ready) {
    hipError_t e = hipEventCreateWithFlags(&ctx->tables_ready, hipEventDisableTiming);
    if (e != hipSuccess) return dev_fail(ctx, e, "lane creation");
  }
  return PK_OK;
}

// Enqueues one request on a lane: the tables are prepared on the context
// stream, the lane waits for them, runs the path and records its event.
pk_status submit_on_lane(pk_ctx* ctx, int lane, const pk_mesh_desc* m, const pk_bin_desc* b,
                         const void* pos, const void* weight, int64_t n, void* workspace,
                         double* result_dev) {
  const MeshTables* t = nullptr;
  BinSpec spec;
  if (pk_status st = prepare_tables(ctx, m, b, &t, &spec)) return st;
  pk_ctx::Lane& ln = ctx->lanes[lane];
  hipError_t e = hipEventRecord(ctx->tables_ready, ctx->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(ln.stream, ctx->tables_ready, 0);
  if (e == hipSuccess)
    e = enqueue_fftpower(ctx, ln.stream, m, spec, t, pos, weight, nullptr, n, workspace,
                         layout_of(m, b, n), result_dev, choice_for(ctx, m, n));
  if (e == hipSuccess) e = hipEventRecord(ln.done, ln.stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "lane submission");
  return PK_OK;
}

// The tuner: every candidate setting runs the whole path twice (warm-up,
// then timed with events on the context stream); the fastest is kept.
pk_status tune_fftpower(pk_ctx* ctx, const pk_mesh_desc* m, const BinSpec& spec,
                        const MeshTables* t, const void* pos, const void* weight,
                        const void* value, int64_t n, void* workspace, const Layout& l,
                        double* result_dev) {
  for (hipEvent_t& ev : ctx->tune_ev) {
    if (!ev) {
      const hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return dev_fail(ctx, e, "tuner events");
    }
  }
  std::vector<pk_tune_entry> cands;
  const pk_tune_entry base = default_choice(m, n);
  const int splits[2] = {0, 1};
  for (int si = 0; si < (m->interlaced ? 2 : 1); ++si)
    for (int xpc = 0; xpc < (l.gx > (int)kComputeUnits ? 2 : 1); ++xpc) {
      pk_tune_entry c = base;
      c.split = m->interlaced ? splits[si] : 0;
      c.xpass_per_cu = xpc;
      cands.push_back(c);
    }
  pk_tune_entry best = base;
  float best_ms = 1e30f;
  for (pk_tune_entry& c : cands) {
    hipError_t e = enqueue_fftpower(ctx, ctx->stream, m, spec, t, pos, weight, value, n,
                                    workspace, l, result_dev, c);
    if (e == hipSuccess) e = hipEventRecord(ctx->tune_ev[0], ctx->stream);
    if (e == hipSuccess)
      e = enqueue_fftpower(ctx, ctx->stream, m, spec, t, pos, weight, value, n, workspace, l,
                           result_dev, c);
    if (e == hipSuccess) e = hipEventRecord(ctx->tune_ev[1], ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ctx->tune_ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->tune_ev[0], ctx->tune_ev[1]);
    if (e != hipSuccess) return dev_fail(ctx, e, "tuning");
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  best.ms = best_ms;
  ctx->tuned[tune_key(m, n)] = best;
  return PK_OK;
}

}  // namespace

extern "C" {

pk_status pk_ctx_set_autotune(pk_ctx* ctx, int mode) {
  if (!ctx) return PK_EINVAL;
  if (mode != 0 && mode != 1) return fail(ctx, PK_EINVAL, "mode must be 0 or 1");
  ctx->autotune = mode;
  return PK_OK;
}

int pk_tune_count(const pk_ctx* ctx) { return ctx ? (int)ctx->tuned.size() : 0; }

pk_status pk_tune_get(const pk_ctx* ctx, int i, pk_tune_entry* out) {
  if (!ctx || !out || i < 0 || i >= (int)ctx->tuned.size()) return PK_EINVAL;
  auto it = ctx->tuned.begin();
  std::advance(it, i);
  *out = it->second;
  return PK_OK;
}

pk_status pk_tune_put(pk_ctx* ctx, const pk_tune_entry* entry) {
  if (!ctx) return PK_EINVAL;
  if (!entry) return fail(ctx, PK_EINVAL, "entry is NULL");
  pk_mesh_desc m{};
  m.nmesh = entry->nmesh;
  m.window = entry->window;
  m.interlaced = entry->interlaced;
  m.compensated = 1;
  m.dtype = entry->dtype;
  m.boxsize = 1.0;
  if (const char* why = check_mesh(&m)) return fail(ctx, PK_EINVAL, why);
  if ((entry->split != 0 && entry->split != 1) || entry->xpass_per_cu < 0 ||
      entry->xpass_per_cu > 2)
    return fail(ctx, PK_EINVAL, "split must be 0 or 1, xpass_per_cu 0, 1 or 2");
  ctx->tuned[std::make_tuple(entry->nmesh, entry->dtype, entry->window, entry->interlaced,
                             entry->density)] = *entry;
  return PK_OK;
}

pk_status pk_fftpower_v(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                        const void* pos, const void* weight, const void* value, int64_t n,
                        void* workspace, size_t workspace_bytes, double* result_dev) {
  if (!ctx) return PK_EINVAL;
  if (pk_status st = check_fftpower(ctx, m, b, pos, n, workspace, workspace_bytes, result_dev))
    return st;
  DeviceGuard g(ctx->device);
  const MeshTables* t = nullptr;
  BinSpec spec;
  if (pk_status st = prepare_tables(ctx, m, b, &t, &spec)) return st;
  const Layout l = layout_of(m, b, n);
  if (ctx->autotune && !ctx->tuned.count(tune_key(m, n)) && !ctx->timing) {
    if (pk_status st = tune_fftpower(ctx, m, spec, t, pos, weight, value, n, workspace, l,
                                     result_dev))
      return st;
  }
  hipError_t e = enqueue_fftpower(ctx, ctx->stream, m, spec, t, pos, weight, value, n, workspace,
                                  l, result_dev, choice_for(ctx, m, n));
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_fftpower");
  return PK_OK;
}

pk_status pk_fftpower(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b, const void* pos,
                      const void* weight, int64_t n, void* workspace, size_t workspace_bytes,
                      double* result_dev) {
  return pk_fftpower_v(ctx, m, b, pos, weight, nullptr, n, workspace, workspace_bytes,
                       result_dev);
}

pk_status pk_ctx_set_lanes(pk_ctx* ctx, int nlanes) {
  if (!ctx) return PK_EINVAL;
  if (nlanes < 1 || nlanes > PK_MAX_LANES) return fail(ctx, PK_EINVAL, "nlanes out of range");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  return ensure_lanes(ctx, nlanes);
}

int pk_ctx_lanes(const pk_ctx* ctx) { return ctx ? (int)ctx->lanes.size() : 0; }

pk_status pk_fftpower_async(pk_ctx* ctx, int lane, const pk_mesh_desc* m, const pk_bin_desc* b,
                            const void* pos, const void* weight, int64_t n, void* workspace,
                            size_t workspace_bytes, double* result_dev) {
  if (!ctx) return PK_EINVAL;
  if (lane < 0 || lane >= (int)ctx->lanes.size()) return fail(ctx, PK_EINVAL, "no such lane");
  if (pk_status st = check_fftpower(ctx, m, b, pos, n, workspace, workspace_bytes, result_dev))
    return st;
  DeviceGuard g(ctx->device);
  return submit_on_lane(ctx, lane, m, b, pos, weight, n, workspace, result_dev);
}

int pk_lane_query(pk_ctx* ctx, int lane) {
  if (!ctx) return PK_EINVAL;
  if (lane < 0 || lane >= (int)ctx->lanes.size()) return fail(ctx, PK_EINVAL, "no such lane");
  DeviceGuard g(ctx->device);
  const hipError_t e = hipEventQuery(ctx->lanes[lane].done);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return dev_fail(ctx, e, "pk_lane_query");
}

pk_status pk_lane_wait(pk_ctx* ctx, int lane) {
  if (!ctx) return PK_EINVAL;
  if (lane < 0 || lane >= (int)ctx->lanes.size()) return fail(ctx, PK_EINVAL, "no such lane");
  DeviceGuard g(ctx->device);
  const hipError_t e = hipEventSynchronize(ctx->lanes[lane].done);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_lane_wait");
  return PK_OK;
}

}  // extern "C"

namespace {

// Validation and plan-time tables of a batch (before any work is enqueued).
pk_status prepare_batch(pk_ctx* ctx, int count, const pk_mesh_desc* m, const pk_bin_desc* b,
                        const void* const* pos, const int64_t* n, void* const* lane_workspace,
                        size_t lane_workspace_bytes, double* const* result_dev, int nworkspaces) {
  if (count < 0) return fail(ctx, PK_EINVAL, "count must be >= 0");
  if (count > 0 && (!m || !b || !pos || !n || !result_dev))
    return fail(ctx, PK_EINVAL, "request arrays are NULL");
  if (!lane_workspace) return fail(ctx, PK_EINVAL, "lane_workspace is NULL");
  for (int i = 0; i < nworkspaces; ++i)
    if (!lane_workspace[i]) return fail(ctx, PK_EINVAL, "a lane workspace is NULL");
  for (int i = 0; i < count; ++i)
    if (pk_status st = check_fftpower(ctx, &m[i], &b[i], pos[i], n[i], lane_workspace[0],
                                      lane_workspace_bytes, result_dev[i]))
      return st;
  // every table first, so that no lane waits behind a table build later (and
  // nothing is allocated while a graph is captured)
  for (int i = 0; i < count; ++i) {
    const MeshTables* t = nullptr;
    BinSpec spec;
    if (pk_status st = prepare_tables(ctx, &m[i], &b[i], &t, &spec)) return st;
  }
  return PK_OK;
}

// Enqueues a prepared batch: with lanes, largest requests first, each to the
// lane with the least queued work (estimated as the mesh cells plus the
// particles it has to process), and the context stream waits for every lane;
// without lanes, one after another on the context stream in one workspace.
pk_status schedule_batch(pk_ctx* ctx, int count, const pk_mesh_desc* m, const pk_bin_desc* b,
                         const void* const* pos, const void* const* weight, const int64_t* n,
                         void* const* lane_workspace, double* const* result_dev) {
  const int nl = (int)ctx->lanes.size();
  if (nl == 0) {
    for (int i = 0; i < count; ++i) {
      const MeshTables* t = nullptr;
      BinSpec spec;
      if (pk_status st = prepare_tables(ctx, &m[i], &b[i], &t, &spec)) return st;
      const hipError_t e =
          enqueue_fftpower(ctx, ctx->stream, &m[i], spec, t, pos[i], weight ? weight[i] : nullptr,
                           nullptr, n[i], lane_workspace[0], layout_of(&m[i], &b[i], n[i]),
                           result_dev[i], choice_for(ctx, &m[i], n[i]));
      if (e != hipSuccess) return dev_fail(ctx, e, "batch");
    }
    return PK_OK;
  }
  std::vector<int> order(count);
  std::vector<double> cost(count);
  for (int i = 0; i < count; ++i) {
    const double nm = (double)m[i].nmesh;
    order[i] = i;
    cost[i] = (m[i].interlaced ? 2.0 : 1.0) * nm * nm * nm + 4.0 * (double)n[i];
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
  std::vector<double> queued(nl, 0.0);
  for (int i : order) {
    const int lane = (int)(std::min_element(queued.begin(), queued.end()) - queued.begin());
    queued[lane] += cost[i];
    if (pk_status st = submit_on_lane(ctx, lane, &m[i], &b[i], pos[i], weight ? weight[i] : nullptr,
                                      n[i], lane_workspace[lane], result_dev[i]))
      return st;
  }
  // the context stream continues after every lane
  for (int i = 0; i < nl; ++i) {
    const hipError_t e = hipStreamWaitEvent(ctx->stream, ctx->lanes[i].done, 0);
    if (e != hipSuccess) return dev_fail(ctx, e, "batch");
  }
  return PK_OK;
}

}  // namespace

struct pk_graph {
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  size_t nodes = 0;
};

extern "C" {

pk_status pk_fftpower_batch(pk_ctx* ctx, int count, const pk_mesh_desc* m, const pk_bin_desc* b,
                            const void* const* pos, const void* const* weight, const int64_t* n,
                            void* const* lane_workspace, size_t lane_workspace_bytes,
                            double* const* result_dev) {
  if (!ctx) return PK_EINVAL;
  const int nl = (int)ctx->lanes.size();
  if (nl < 1) return fail(ctx, PK_EINVAL, "no lanes: call pk_ctx_set_lanes first");
  if (pk_status st = prepare_batch(ctx, count, m, b, pos, n, lane_workspace, lane_workspace_bytes,
                                   result_dev, nl))
    return st;
  if (count == 0) return PK_OK;
  DeviceGuard g(ctx->device);
  return schedule_batch(ctx, count, m, b, pos, weight, n, lane_workspace, result_dev);
}

pk_status pk_fftpower_batch_graph(pk_ctx* ctx, int count, const pk_mesh_desc* m,
                                  const pk_bin_desc* b, const void* const* pos,
                                  const void* const* weight, const int64_t* n,
                                  void* const* lane_workspace, size_t lane_workspace_bytes,
                                  double* const* result_dev, pk_graph** out) {
  if (!ctx) return PK_EINVAL;
  if (!out) return fail(ctx, PK_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1) return fail(ctx, PK_EINVAL, "a graph needs at least one request");
  if (ctx->timing) return fail(ctx, PK_EINVAL, "stage timing records events: disable it first");
  const int nl = (int)ctx->lanes.size();
  if (pk_status st = prepare_batch(ctx, count, m, b, pos, n, lane_workspace, lane_workspace_bytes,
                                   result_dev, nl > 0 ? nl : 1))
    return st;
  DeviceGuard g(ctx->device);
  // the tables were uploaded on the context stream: done before the capture
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_fftpower_batch_graph");
  std::unique_ptr<pk_graph> gr(new (std::nothrow) pk_graph());
  if (!gr) return fail(ctx, PK_ENOMEM, "host allocation of the graph");
  gr->device = ctx->device;
  e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return dev_fail(ctx, e, "hipStreamBeginCapture");
  const pk_status st = schedule_batch(ctx, count, m, b, pos, weight, n, lane_workspace, result_dev);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(ctx->stream, &graph);
  if (st != PK_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return dev_fail(ctx, e, "hipStreamEndCapture");
  gr->graph = graph;
  e = hipGraphGetNodes(graph, nullptr, &gr->nodes);
  if (e == hipSuccess) e = hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return dev_fail(ctx, e, "hipGraphInstantiate");
  }
  *out = gr.release();
  return PK_OK;
}

pk_status pk_graph_launch(pk_ctx* ctx, pk_graph* graph) {
  if (!ctx) return PK_EINVAL;
  if (!graph || !graph->exec) return fail(ctx, PK_EINVAL, "graph is NULL");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  if (graph->device != ctx->device) return fail(ctx, PK_EINVAL, "graph of another device");
  DeviceGuard g(ctx->device);
  const hipError_t e = hipGraphLaunch(graph->exec, ctx->stream);
  if (e != hipSuccess) return dev_fail(ctx, e, "hipGraphLaunch");
  return PK_OK;
}

size_t pk_graph_nodes(const pk_graph* graph) { return graph ? graph->nodes : 0; }

void pk_graph_destroy(pk_graph* graph) {
  if (!graph) return;
  DeviceGuard g(graph->device);
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  delete graph;
}

pk_status pk_result_to_host(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                            const double* result_dev, pk_result* out) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_bins(b, m)) return fail(ctx, PK_EINVAL, why);
  if (!result_dev || !out || !out->k || !out->power || !out->modes)
    return fail(ctx, PK_EINVAL, "result, out or one of its 1-D arrays is NULL");
  if (b->npoles > 0 && !out->poles) return fail(ctx, PK_EINVAL, "out->poles is NULL");
  if (const char* why = check_lds(b, m)) return fail(ctx, PK_EUNSUPPORTED, why);
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  BinTables* bt = nullptr;
  if (pk_status st = get_bin_tables(ctx, m, b, &bt)) return st;
  const int nsum = nsum_of(b);
  const double* h = nullptr;
  if (pk_status st = read_result(ctx, result_dev, (size_t)nsum + 2, &h, "pk_result_to_host"))
    return st;
  const double L = m->boxsize;
  const double volume = L * L * L;
  const double kf = 2.0 * 3.14159265358979323846 / L;
  const double wsum = h[nsum], w2sum = h[nsum + 1];
  const double norm = volume / (wsum * wsum);
  const double nan = std::nan("");
  const int nk = b->nk;
  for (int k = 0; k < nk; ++k) {
    const int64_t nb = bt->modes[k];
    out->modes[k] = nb;
    out->k[k] = nb ? kf * bt->sum_n[k] / (double)nb : nan;
    out->power[k] = nb ? norm * h[k] / (double)nb : nan;
    for (int i = 0; i < b->npoles; ++i) {
      const int ell = b->poles[i];
      out->poles[(size_t)i * nk + k] =
          nb ? (2 * ell + 1) * norm * h[(size_t)nk * (1 + i) + k] / (double)nb : nan;
    }
  }
  if (b->nmu > 1) {
    const int off = nk * (1 + b->npoles);
    for (int f = 0; f < nk * b->nmu; ++f) {
      const int64_t nb = bt->modes2d[f];
      if (out->modes2d) out->modes2d[f] = nb;
      if (out->k2d) out->k2d[f] = nb ? kf * bt->sum_n2d[f] / (double)nb : nan;
      if (out->mu2d) out->mu2d[f] = nb ? bt->sum_mu2d[f] / (double)nb : nan;
      if (out->power2d) out->power2d[f] = nb ? norm * h[off + f] / (double)nb : nan;
    }
  }
  out->wsum = wsum;
  out->w2sum = w2sum;
  out->shotnoise = volume * w2sum / (wsum * wsum);
  return PK_OK;
}

pk_status pk_ctx_set_timing(pk_ctx* ctx, int enable) {
  if (!ctx) return PK_EINVAL;
  if (enable && ctx->device == PK_DEVICE_NONE)
    return fail(ctx, PK_EDEVICE, "validation-only context");
  if (enable && !ctx->events[0]) {
    DeviceGuard g(ctx->device);
    for (auto& ev : ctx->events) {
      const hipError_t e = hipEventCreate(&ev);
      if (e != hipSuccess) return dev_fail(ctx, e, "hipEventCreate");
    }
  }
  ctx->timing = enable != 0;
  return PK_OK;
}

int pk_stage_count(void) { return kNumStages; }

const char* pk_stage_name(int stage) {
  return (stage >= 0 && stage < kNumStages) ? kStageNames[stage] : nullptr;
}

pk_status pk_ctx_stage_times(pk_ctx* ctx, double* ms) {
  if (!ctx || !ms) return PK_EINVAL;
  if (!ctx->timed_once) return fail(ctx, PK_EINVAL, "no timed pk_fftpower call yet");
  DeviceGuard g(ctx->device);
  hipError_t e = hipEventSynchronize(ctx->events[kNumStages]);
  if (e != hipSuccess) return dev_fail(ctx, e, "hipEventSynchronize");
  for (int i = 0; i < kNumStages; ++i) {
    ms[i] = 0.0;
    if (!ctx->stage_ran[i]) continue;
    int j = i + 1;
    while (j < kNumStages && !ctx->stage_ran[j]) ++j;
    float t = 0.f;
    e = hipEventElapsedTime(&t, ctx->events[i], ctx->events[j]);
    if (e != hipSuccess) return dev_fail(ctx, e, "hipEventElapsedTime");
    ms[i] = t;
  }
  return PK_OK;
}

}  // extern "C"

// ---- Survey multipoles (ConvolvedFFTPower) ---------------------------------

namespace {

// Survey binning: 1-D k bins, poles among 0, 2, 4, top edge <= N/2.
const char* check_survey_bins(const pk_bin_desc* b, const pk_mesh_desc* m) {
  if (const char* why = check_bins(b, m)) return why;
  if (b->nmu > 1) return "the survey multipoles have no mu bins (nmu must be 0 or 1)";
  if (b->npoles < 1) return "at least one multipole must be requested";
  for (int i = 0; i < b->npoles; ++i)
    if (b->poles[i] > 4) return "survey multipoles: ell must be 0, 2 or 4";
  if (b->kmin_f + b->nk * b->dk_f > m->nmesh / 2)
    return "survey multipoles: the top edge kmin_f + nk * dk_f may not exceed N/2";
  return nullptr;
}

// The plain k binning the cross sums of the fields use.
pk_bin_desc survey_plain_bins(const pk_bin_desc* b) {
  pk_bin_desc p = *b;
  p.nmu = 0;
  p.npoles = 0;
  p.los = 2;
  return p;
}

// Fields F_ell kept: F_0 always, then every requested ell > 0.
int survey_fields(const pk_bin_desc* b, int* ells) {
  int nf = 0;
  ells[nf++] = 0;
  for (int i = 0; i < b->npoles; ++i)
    if (b->poles[i] != 0) ells[nf++] = b->poles[i];
  return nf;
}

struct SurveyLayout {
  size_t pos = 0, value = 0, sums = 0, zero = 0, bsums = 0, sumpart = 0, bucket = 0, rec = 0,
         wbase = 0, amounts = 0, mesh = 0, ymesh = 0, ymesh2 = 0, ymesh3 = 0, ymesh4 = 0,
         side = 0, side2 = 0,
         fields = 0, planes = 0,
         bpart = 0, amax = 0, total = 0;
  size_t field_bytes = 0, plane_bytes = 0, amount_bytes = 0;
  int gb = 0, gp = 0, nh = 0;
};

SurveyLayout survey_layout(const pk_mesh_desc* m, const pk_bin_desc* b, int64_t nd, int64_t nr) {
  SurveyLayout l;
  const size_t n = (size_t)m->nmesh;
  const size_t es = elem_bytes(m);
  const size_t np = (size_t)(nd > 0 ? nd : 0) + (size_t)(nr > 0 ? nr : 0);
  int ells[4];
  const int nf = survey_fields(b, ells);
  for (int f = 0; f < nf; ++f) l.nh += 2 * ells[f] + 1;
  l.field_bytes = align256(n * n * n * es);
  l.plane_bytes = align256(n * n * 2 * es);
  l.amount_bytes = align256(np * es);
  const size_t total_modes = n * n * (n / 2);
  size_t gb = (total_modes + 255) / 256;
  if (gb > 1024) gb = 1024;
  l.gb = (int)gb;
  l.gp = plane_bin_groups(m->nmesh);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return at;
  };
  l.pos = take(np * 3 * es);
  l.value = take(np * es);
  l.sums = take(4 * sizeof(double));
  l.zero = take(2 * sizeof(double));
  l.bsums = take(2 * sizeof(double));
  l.sumpart = take(survey_sum_partials() * sizeof(double));
  l.bucket = take(bucket_bytes(m->nmesh));
  l.rec = take(np * 4 * es);
  l.wbase = take(np * es);
  l.amounts = take((size_t)l.nh * l.amount_bytes);
  l.mesh = take(l.field_bytes);
  l.ymesh = take(l.field_bytes);
  l.ymesh2 = take(l.field_bytes);
  l.ymesh3 = take(l.field_bytes);
  l.ymesh4 = take(l.field_bytes);
  l.side = take(n * n * 2 * es);
  l.side2 = take(n * n * 2 * es);
  l.fields = take((size_t)nf * l.field_bytes);
  l.planes = take((size_t)nf * l.plane_bytes);
  l.bpart = take((size_t)b->npoles * (l.gb + l.gp) * 2 * b->nk * sizeof(double));
  l.amax = take(sizeof(double));
  l.total = off;
  return l;
}

// Normalisation of the real harmonic Y_lm: sqrt((2l+1)/4pi (l-|m|)!/(l+|m|)!),
// times sqrt(2) for m != 0.
Harmonic harmonic_of(int ell, int m) {
  Harmonic h;
  h.ell = ell;
  h.am = m < 0 ? -m : m;
  h.sine = m < 0 ? 1 : 0;
  double ratio = 1.0;  // (l - |m|)! / (l + |m|)!
  for (int i = ell - h.am + 1; i <= ell + h.am; ++i) ratio /= (double)i;
  const double pi = 3.14159265358979323846;
  h.knorm = std::sqrt((2.0 * ell + 1.0) / (4.0 * pi) * ratio) * (h.am ? std::sqrt(2.0) : 1.0);
  return h;
}

}  // namespace

extern "C" {

size_t pk_convolved_doubles(const pk_bin_desc* b) {
  if (!b || b->nk < 1 || b->nk > 4096 || b->npoles < 1 || b->npoles > 4) return 0;
  return (size_t)b->npoles * b->nk + 4;
}

size_t pk_convolved_workspace_bytes(const pk_mesh_desc* m, const pk_bin_desc* b, int64_t n_data,
                                    int64_t n_rand) {
  if (check_mesh(m) || !b || check_survey_bins(b, m) || n_data < 0 || n_rand < 0) return 0;
  return survey_layout(m, b, n_data, n_rand).total;
}

pk_status pk_convolved_power(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                             const double* observer, const void* data_pos,
                             const void* data_weight, int64_t n_data, const void* rand_pos,
                             const void* rand_weight, int64_t n_rand, void* workspace,
                             size_t workspace_bytes, double* result_dev) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_survey_bins(b, m)) return fail(ctx, PK_EINVAL, why);
  if (m->interlaced) return fail(ctx, PK_EUNSUPPORTED, "survey multipoles: interlacing is not implemented");
  if (!observer || !std::isfinite(observer[0]) || !std::isfinite(observer[1]) ||
      !std::isfinite(observer[2]))
    return fail(ctx, PK_EINVAL, "observer must be 3 finite host doubles");
  if (n_data < 1 || n_rand < 1) return fail(ctx, PK_EINVAL, "n_data and n_rand must be >= 1");
  if (n_data > kMaxSortedParticles - n_rand)
    return fail(ctx, PK_EUNSUPPORTED, "more than 2^31 - 1 particles (32-bit record offsets)");
  if (!data_pos || !rand_pos) return fail(ctx, PK_EINVAL, "data_pos or rand_pos is NULL");
  if (!workspace || !result_dev) return fail(ctx, PK_EINVAL, "workspace or result is NULL");
  const SurveyLayout l = survey_layout(m, b, n_data, n_rand);
  if (workspace_bytes < l.total) return fail(ctx, PK_EINVAL, "workspace too small");
  const pk_bin_desc pb = survey_plain_bins(b);
  if (const char* why = check_lds(&pb, m)) return fail(ctx, PK_EUNSUPPORTED, why);
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  const MeshTables* t = nullptr;
  BinSpec spec;
  if (pk_status st = prepare_tables(ctx, m, &pb, &t, &spec)) return st;
  hipStream_t s = ctx->stream;
  char* ws = static_cast<char*>(workspace);
  const size_t es = elem_bytes(m);
  const int64_t n = n_data + n_rand;
  void* pos = ws + l.pos;
  void* value = ws + l.value;
  double* sums = reinterpret_cast<double*>(ws + l.sums);
  double* zero = reinterpret_cast<double*>(ws + l.zero);
  double* bsums = reinterpret_cast<double*>(ws + l.bsums);
  void* mesh = ws + l.mesh;
  int ells[4];
  const int nf = survey_fields(b, ells);
  auto field = [&](int i) -> void* { return ws + l.fields + (size_t)i * l.field_bytes; };
  // one catalog, data first, so that one painting covers both
  hipError_t e = hipMemcpyAsync(pos, data_pos, (size_t)n_data * 3 * es, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(static_cast<char*>(pos) + (size_t)n_data * 3 * es, rand_pos,
                       (size_t)n_rand * 3 * es, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_fill_zero(zero, 2 * sizeof(double), s);
  if (e == hipSuccess)
    e = launch_survey_sums(m->dtype, data_weight, n_data, rand_weight, n_rand,
                           reinterpret_cast<double*>(ws + l.sumpart), sums, s);
  // the amounts w s (s = 1 for data, -alpha for randoms), bucketed once
  Harmonic unit;
  unit.knorm = 1.0;
  if (e == hipSuccess)
    e = launch_ylm_value(m->dtype, pos, data_weight, n_data, rand_weight, n_rand, observer, unit,
                         sums, value, s);
  if (e == hipSuccess)
    e = launch_bucket(m->dtype, m->nmesh, m->boxsize, pos, nullptr, value, n, ws + l.bucket,
                      ws + l.rec, ws + l.wbase, bsums, s, ws + l.mesh, l.bpart - l.mesh);
  void* rec = ws + l.rec;
  void* base = ws + l.wbase;
  void* ymesh = ws + l.ymesh;
  auto plane = [&](int i) -> void* { return ws + l.planes + (size_t)i * l.plane_bytes; };
  auto amount = [&](int k) -> void* { return ws + l.amounts + (size_t)k * l.amount_bytes; };
  // the sorted amounts times Y_lm(r^), every harmonic in one pass
  HarmonicSet hs;
  int field_of[kMaxHarmonics], first_of[kMaxHarmonics];
  for (int f = 0; f < nf; ++f)
    for (int mm = -ells[f]; mm <= ells[f]; ++mm) {
      field_of[hs.n] = f;
      first_of[hs.n] = mm == -ells[f] ? 1 : 0;
      hs.h[hs.n++] = harmonic_of(ells[f], mm);
    }
  if (e == hipSuccess)
    e = launch_ylm_records(m->dtype, m->nmesh, m->boxsize, rec, base, ws + l.bucket, observer, hs,
                           l.amount_bytes / es, ws + l.amounts, s);
  // the harmonics of each ell two at a time: each painted with the z-pass and
  // taken through the y-pass into the x-pass layout (a set of two buffers),
  // then one x-pass adds both into F_ell.  The x-passes run on a second
  // stream, beside the painting of the next harmonics (the painting is bound
  // by LDS atomics, the x-pass by memory and FFT work); the buffer sets
  // alternate, and events order each set's y-passes before its x-pass and
  // that x-pass before the set is written again.  The painted field has mean
  // ~0: nothing is subtracted before the z-FFT.
  if (e == hipSuccess && !ctx->aux) {
    // created together; kept only if all of them could be
    hipStream_t st = nullptr;
    hipEvent_t ev[5] = {};
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    for (int i = 0; i < 5 && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
      if (st) (void)hipStreamDestroy(st);
      return dev_fail(ctx, e, "survey stream");
    }
    ctx->aux = st;
    for (int i = 0; i < 5; ++i) ctx->aux_ev[i] = ev[i];
  }
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_convolved_power");
  hipStream_t sx = ctx->aux;
  hipEvent_t* ydone = ctx->aux_ev;      // [2]
  hipEvent_t* xdone = ctx->aux_ev + 2;  // [2]
  const double pi = 3.14159265358979323846;
  void* ysets[2][2] = {{ymesh, ws + l.ymesh2}, {ws + l.ymesh3, ws + l.ymesh4}};
  for (int k = 0, pass = 0; k < hs.n && e == hipSuccess; ++pass) {
    const int f = field_of[k], set = pass & 1;
    const int np2 = (k + 1 < hs.n && field_of[k + 1] == f) ? 2 : 1;
    if (pass >= 2) e = hipStreamWaitEvent(s, xdone[set], 0);  // x-pass pass - 2 is done with it
    for (int j = 0; j < np2 && e == hipSuccess; ++j) {
      e = launch_paint_z(m->dtype, m->nmesh, m->window, false, rec, amount(k + j), ws + l.bucket,
                         zero, t->tw, mesh, nullptr, s, -1, /*exact=*/false);
      if (e == hipSuccess)
        e = launch_fft_y_relayout(m->dtype, m->nmesh, mesh, ysets[set][j], t->tw, s);
    }
    if (e == hipSuccess) e = hipEventRecord(ydone[set], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(sx, ydone[set], 0);
    if (e == hipSuccess)
      e = launch_x_accumulate(m->dtype, m->nmesh, ysets[set][0],
                              np2 == 2 ? ysets[set][1] : nullptr, field(f), plane(f),
                              ws + l.side, np2 == 2 ? ws + l.side2 : nullptr, hs.h[k],
                              hs.h[k + np2 - 1], 4.0 * pi / (2 * ells[f] + 1), *t, m->window,
                              m->compensated, first_of[k], sx);
    if (e == hipSuccess) e = hipEventRecord(xdone[set], sx);
    k += np2;
  }
  // the binning (on the context stream) after the last x-pass
  if (e == hipSuccess) e = hipEventRecord(ctx->aux_ev[4], sx);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->aux_ev[4], 0);
  // sums of Re F_0 conj F_ell per k bin: one pass over the fields (in the
  // y-pass output layout) for every pole, then each pole's kz = 0 plane and
  // its reduction; then the weight sums
  double* part = reinterpret_cast<double*>(ws + l.bpart);
  const size_t pstride = (size_t)(l.gb + l.gp) * 2 * spec.nsum;
  spec.exact = 0;  // the cross sums of the fields are float64 rows
  const void* others[4] = {nullptr, nullptr, nullptr, nullptr};
  int fof[4] = {0, 0, 0, 0};
  for (int i = 0; i < b->npoles; ++i) {
    while (ells[fof[i]] != b->poles[i]) ++fof[i];
    others[i] = fof[i] == 0 ? nullptr : field(fof[i]);
  }
  if (e == hipSuccess)
    e = launch_bin_fields(m->dtype, m->nmesh, field(0), others, b->npoles, spec, part, pstride, s,
                          1);
  for (int i = 0; i < b->npoles && e == hipSuccess; ++i) {
    const int f = fof[i];
    double* pole_part = part + (size_t)i * pstride;
    // the exact sums' bound from the largest component of the two planes
    BinSpec ps = spec;
    double* amax = reinterpret_cast<double*>(ws + l.amax);
    ps.bound_scale = 8.0 * (double)m->nmesh * m->nmesh;
    ps.bound_dev = amax;
    ps.bound_sq = 1;
    e = launch_absmax(m->dtype, plane(0), f == 0 ? nullptr : plane(f),
                      (size_t)m->nmesh * m->nmesh * 2, amax, s);
    if (e == hipSuccess)
      e = launch_plane_bin(m->dtype, m->nmesh, plane(0), f == 0 ? nullptr : plane(f), 1, *t,
                           m->window, 0, ps, pole_part + (size_t)l.gb * 2 * spec.nsum, s,
                           f == 0 ? 0 : 1);
    if (e == hipSuccess)
      e = launch_reduce(pole_part, l.gb + l.gp, spec, result_dev + (size_t)i * b->nk, s);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(result_dev + (size_t)b->npoles * b->nk, sums, 4 * sizeof(double),
                       hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return dev_fail(ctx, e, "pk_convolved_power");
  return PK_OK;
}

pk_status pk_convolved_to_host(pk_ctx* ctx, const pk_mesh_desc* m, const pk_bin_desc* b,
                               double norm, const double* result_dev, pk_result* out) {
  if (!ctx) return PK_EINVAL;
  if (const char* why = check_mesh(m)) return fail(ctx, PK_EINVAL, why);
  if (const char* why = check_survey_bins(b, m)) return fail(ctx, PK_EINVAL, why);
  if (!std::isfinite(norm) || !(norm > 0)) return fail(ctx, PK_EINVAL, "norm must be finite and > 0");
  if (!result_dev || !out || !out->k || !out->modes || !out->poles)
    return fail(ctx, PK_EINVAL, "result, out or one of out->k, modes, poles is NULL");
  if (ctx->device == PK_DEVICE_NONE) return fail(ctx, PK_EDEVICE, "validation-only context");
  DeviceGuard g(ctx->device);
  const pk_bin_desc pb = survey_plain_bins(b);
  BinTables* bt = nullptr;
  if (pk_status st = get_bin_tables(ctx, m, &pb, &bt)) return st;
  const int nk = b->nk;
  const double* h = nullptr;
  if (pk_status st = read_result(ctx, result_dev, pk_convolved_doubles(b), &h,
                                 "pk_convolved_to_host"))
    return st;
  const double kf = 2.0 * 3.14159265358979323846 / m->boxsize;
  const double nan = std::nan("");
  for (int k = 0; k < nk; ++k) {
    const int64_t nb = bt->modes[k];
    out->modes[k] = nb;
    out->k[k] = nb ? kf * bt->sum_n[k] / (double)nb : nan;
    for (int i = 0; i < b->npoles; ++i)
      out->poles[(size_t)i * nk + k] =
          nb ? (2 * b->poles[i] + 1) * h[(size_t)i * nk + k] / (norm * (double)nb) : nan;
  }
  const double* ws = h + (size_t)b->npoles * nk;
  const double alpha = ws[0] / ws[2];
  out->wsum = ws[0];
  out->w2sum = ws[1];
  out->shotnoise = (ws[1] + alpha * alpha * ws[3]) / norm;
  return PK_OK;
}

}  // extern "C"
