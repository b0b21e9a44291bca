/*
 * pk.h -- C ABI of libpk, the FFT power-spectrum hot path of nbodykit
 * (Hand, Feng et al. 2018) for AMD MI355X (gfx950).
 *
 * The library paints a particle catalog onto a periodic mesh with the CIC,
 * TSC or PCS window (optionally interlaced), takes the 3D real-to-complex FFT,
 * divides out the window and bins |delta(k)|^2 into P(k), P(k, mu) and
 * Legendre multipoles P_ell(k).  Paper passages:
 *   painting, Eq. (1) ......................... Sec. 3.3.1 "Painting a Mesh"
 *   windows, interlacing, compensation Eq. (2)  Sec. 3.3.2 "From Catalog to Mesh"
 *   r2c between RealField and ComplexField .... Sec. 3.3.1
 *   FFTPower: P(k), P(k, mu), P_ell(k) ........ Sec. 3.4.1 "Power Spectra"
 *   survey multipoles (ConvolvedFFTPower) ..... Sec. 3.4.1, named there
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.  Every buffer argument is a DEVICE pointer unless its comment
 *   says "host".  Device buffers are owned by the caller (typically PyTorch
 *   allocations); the library never frees them.  The library owns only the
 *   context, its FFT twiddle tables and the per-binning mode tables, which it
 *   allocates on first use of a mesh size / binning and frees in
 *   pk_ctx_destroy.
 * Streams.  All device work is enqueued on the stream given to
 *   pk_ctx_create and is asynchronous, except pk_result_to_host, which
 *   synchronises that stream.
 * Errors.  Every call returns a pk_status; negative values are failures and
 *   pk_last_error() holds a message.  Argument errors (PK_EINVAL) are
 *   detected before any device work, leave outputs untouched and need no GPU.
 *   PK_EDEVICE carries the HIP error string.  No C++ exception crosses the
 *   ABI.  A context must not be used from two host threads at once.
 * Real mesh layout.  N^3 values of the mesh precision, row-major [x][y][z]
 *   (z fastest); mesh node (i, j, l) sits at position (i, j, l) * L / N.
 * Spectrum layout ("packed half spectrum", produced in place over the real
 *   mesh by pk_fft_r2c).  N * N * (N/2) complex values (re, im interleaved),
 *   row-major [kx][ky][kz'], kz' = 0 .. N/2 - 1.  For kz' >= 1 the element is
 *   the DFT c(kx, ky, kz') = sum_x F(x) exp(-2 pi i k.x / N) (unnormalised).
 *   Element kz' = 0 packs the two self-conjugate planes kz = 0 and kz = N/2:
 *   Z(kx, ky) = c(kx, ky, 0) + i c(kx, ky, N/2), so that
 *     c(kx, ky, 0)   = [Z(kx, ky) + conj Z(-kx, -ky)] / 2,
 *     c(kx, ky, N/2) = [Z(kx, ky) - conj Z(-kx, -ky)] / (2 i),
 *   indices taken mod N.  Array index i maps to the signed wave number
 *   n = i for i < N/2, else i - N (numpy fftfreq order).
 */
#ifndef PK_H
#define PK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PK_ABI_VERSION 1

typedef enum {
  PK_OK = 0,
  PK_EINVAL = -1,       /* bad argument; nothing was launched            */
  PK_ENOMEM = -2,       /* the library could not allocate its own tables */
  PK_EDEVICE = -3,      /* a HIP call failed                             */
  PK_EUNSUPPORTED = -4  /* valid request outside the implemented range   */
} pk_status;

typedef enum { PK_F32 = 0, PK_F64 = 1 } pk_dtype;

/* The value is the order p of the window in Eq. (2): sinc^p. */
typedef enum { PK_CIC = 2, PK_TSC = 3, PK_PCS = 4 } pk_window;

/* Mesh description (Sec. 3.3.2, Catalog.to_mesh). */
typedef struct {
  int32_t nmesh;       /* N, cells per side: a power of two, 8 .. 2048      */
  int32_t window;      /* pk_window: 2 = CIC, 3 = TSC, 4 = PCS               */
  int32_t interlaced;  /* 0 or 1: paint a second mesh shifted by half a cell */
  int32_t compensated; /* 0 or 1: divide by prod_i sinc^p(pi k_i / 2 k_N)    */
  int32_t dtype;       /* pk_dtype: precision of positions, weights, meshes  */
  int32_t reserved;    /* must be 0                                          */
  double boxsize;      /* L > 0, same units as the positions                 */
} pk_mesh_desc;

/* Binning description (Sec. 3.4.1, FFTPower).  Wave numbers are in units of
 * the fundamental k_f = 2 pi / L.  k-bin b covers [e_b, e_{b+1}) with
 * e_b = kmin_f + b * dk_f, decided on the integer n^2 against e_b^2
 * (float64); the DC mode is never binned and the top edge is exclusive.
 * |mu| = |n_los| / |n| is split into nmu equal bins; bin j holds
 * j / nmu <= |mu| < (j + 1) / nmu, decided in exact integers, and |mu| = 1
 * belongs to the last bin. */
typedef struct {
  double kmin_f;      /* >= 0                                                */
  double dk_f;        /* > 0                                                 */
  int32_t nk;         /* number of k bins, >= 1                              */
  int32_t nmu;        /* 0 or 1: no P(k, mu) output; else 2 .. 64            */
  int32_t npoles;     /* 0 .. 4                                              */
  int32_t poles[4];   /* even ell in {0, 2, 4, 6}, distinct                  */
  int32_t los;        /* line-of-sight axis 0, 1 or 2                        */
} pk_bin_desc;

/* Host-side result of pk_result_to_host.  The caller allocates every array
 * (host memory) with the sizes given; 2-D arrays are row-major [nk][nmu] and
 * may be NULL when nmu <= 1.  Empty bins hold NaN and a zero count. */
typedef struct {
  double *k;          /* [nk]  mean |k| of the modes in the bin              */
  double *power;      /* [nk]  P(k) = mean of V |delta(k)|^2                  */
  int64_t *modes;     /* [nk]  number of modes (full-grid count)             */
  double *poles;      /* [npoles][nk]  P_ell = (2 ell + 1) mean(P L_ell(mu))  */
  double *k2d;        /* [nk][nmu] mean |k|                                  */
  double *mu2d;       /* [nk][nmu] mean |mu|                                 */
  double *power2d;    /* [nk][nmu] P(k, mu)                                  */
  int64_t *modes2d;   /* [nk][nmu]                                           */
  double shotnoise;   /* V sum(w^2) / sum(w)^2, reported, not subtracted     */
  double wsum;        /* sum of weights                                      */
  double w2sum;       /* sum of squared weights                              */
} pk_result;

typedef struct pk_ctx pk_ctx;

/* Device index of a validation-only context: it checks every argument of
 * every call exactly as a device context does, but any call that would touch
 * a device returns PK_EDEVICE.  It needs no GPU (front ends, CPU tests). */
#define PK_DEVICE_NONE (-1)

/* Creates a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL means the legacy default stream), or a
 * validation-only context for device == PK_DEVICE_NONE.  *ctx receives the
 * handle (host).  Errors: PK_EINVAL for a NULL ctx or a bad device,
 * PK_ENOMEM, PK_EDEVICE. */
pk_status pk_ctx_create(pk_ctx **ctx, int device, void *hip_stream);

/* Frees the context and every device table it owns.  NULL is a no-op. */
void pk_ctx_destroy(pk_ctx *ctx);

/* Message of the last failed call on this context (static storage inside
 * the context, valid until the next call).  ctx may be NULL: then the message
 * of the last failed pk_ctx_create. */
const char *pk_last_error(const pk_ctx *ctx);

/* Bytes of one real mesh (N^3 values of the mesh precision); the packed
 * spectrum occupies the same bytes.  0 for an invalid descriptor. */
size_t pk_mesh_bytes(const pk_mesh_desc *m);

/* Number of float64 slots of the device result buffer used by
 * pk_bin_power / pk_fftpower:
 *   [0, nk)                          sum h P over k-bin
 *   [nk * (1 + i), nk * (2 + i))     sum h P L_ell over k-bin, ell = poles[i]
 *   next nk * nmu (only if nmu > 1)  sum h P over (k, mu)-bin
 *   last 2                           sum w, sum w^2
 * P here is the unnormalised |c|^2 after interlacing and compensation;
 * pk_result_to_host applies V / (sum w)^2.  0 for an invalid descriptor. */
size_t pk_result_doubles(const pk_bin_desc *b);

/* Sizing query for FFTPower k-bins (Sec. 3.4.1: bins of width dk from kmin
 * up to kmax, wave numbers in units of k_f = 2 pi / L): the number of whole
 * bins [kmin_f + b dk_f, kmin_f + (b + 1) dk_f) whose top edge does not
 * exceed kmax_f, i.e. the largest nk with kmin_f + nk dk_f <= kmax_f (an
 * edge within 1e-9 dk_f of kmax_f counts as equal, so exact multiples are
 * kept).  kmax_f = N/2 gives the bins up to the Nyquist index, the largest
 * binning allowed for interlaced meshes.  Pure host arithmetic, no context.
 * Returns PK_EINVAL (negative) for non-finite arguments, kmin_f < 0,
 * dk_f <= 0 or kmax_f <= kmin_f; 0 when no whole bin fits; at most 4096 (the
 * largest nk a pk_bin_desc accepts), else PK_EUNSUPPORTED. */
int32_t pk_num_kbins(double kmin_f, double dk_f, double kmax_f);

/* Device workspace that pk_fftpower needs for this request (bytes). */
size_t pk_workspace_bytes(const pk_mesh_desc *m, const pk_bin_desc *b, int64_t npart);

/* Device memory the context currently owns for tables (bytes). */
size_t pk_ctx_table_bytes(const pk_ctx *ctx);

/* Painting, Eq. (1) with V = 1 (Sec. 3.3.1 / 3.3.2).
 * mesh[j] = sum_p w_p prod_d M_p(u_{p,d} + shift_cells - j_d), periodic,
 * u = (x mod L) N / L, M_p the order-p B-spline of the window.
 *   pos        device, n x 3 positions (x, y, z), dtype of the mesh
 *   weight     device, n weights, or NULL for unit weights
 *   n          number of particles, >= 0
 *   shift_cells  0 for the plain mesh, 0.5 for the interlaced mesh
 *   mesh       device, pk_mesh_bytes(m); overwritten (zeroed, then painted)
 *   wsums      device, 2 float64 {sum w, sum w^2} overwritten, or NULL
 * Accumulation order is not fixed (atomics), so results are reproducible to
 * rounding only.  Errors: PK_EINVAL (bad descriptor, NULL pos with n > 0,
 * NULL mesh, non-finite shift), PK_EDEVICE. */
pk_status pk_paint(pk_ctx *ctx, const pk_mesh_desc *m, const void *pos,
                   const void *weight, int64_t n, double shift_cells, void *mesh,
                   double *wsums);

/* Forward 3D real-to-complex FFT in place (Sec. 3.3.1, r2c): exp(-i k.x),
 * unnormalised; mesh_inout holds the real mesh on entry and the packed half
 * spectrum (layout above) on exit.  Deterministic.
 * Errors: PK_EINVAL, PK_EDEVICE. */
pk_status pk_fft_r2c(pk_ctx *ctx, const pk_mesh_desc *m, void *mesh_inout);

/* Backward 3D complex-to-real FFT in place (Sec. 3.3.1, ComplexField to
 * RealField, c2r): exp(+i k.x), unnormalised, so that
 * pk_fft_c2r(pk_fft_r2c(F)) = N^3 F.  mesh_inout holds a packed half spectrum
 * (layout above) on entry and the real mesh on exit.  The spectrum is taken
 * as that of a real field: the kz = 0 and N/2 planes are read through the
 * packed column (their Hermitian parts), and m->window, interlaced and
 * compensated are ignored.  Deterministic.  Errors: PK_EINVAL, PK_EDEVICE. */
pk_status pk_fft_c2r(pk_ctx *ctx, const pk_mesh_desc *m, void *mesh_inout);

/* Isotropic scaling of a packed spectrum in place, c(k) *= table[|n|^2]
 * (n the signed integer mode, |n|^2 = n_x^2 + n_y^2 + n_z^2), for device-side
 * field generation (Sec. 3.2, catalogs from Gaussian fields): white noise,
 * pk_fft_r2c, pk_shape_spectrum with sqrt(N^3 P(k) / V) / N^3, pk_fft_c2r
 * gives a Gaussian field of spectrum P.  The spectrum is taken as that of a
 * real field (the kz = 0 and N/2 planes through the packed column, each pair
 * of partner modes updated together), so the result stays one.
 *   table_dev  device, table_len float64, table_len >= pk_shape_table_len(m)
 * Errors: PK_EINVAL (also a short table), PK_EDEVICE. */
int64_t pk_shape_table_len(const pk_mesh_desc *m); /* 3 (N/2)^2 + 1, 0 if invalid */
pk_status pk_shape_spectrum(pk_ctx *ctx, const pk_mesh_desc *m, void *cmesh_inout,
                            const double *table_dev, int64_t table_len);

/* Interlacing and window compensation on packed spectra (Sec. 3.3.2, Eq. 2),
 * in place on cmesh_inout:
 *   if cmesh_b != NULL: c <- [c + exp(i pi (n_x + n_y + n_z) / N) c_b] / 2
 *   if m->compensated:  c <- c / prod_d sinc^p(pi n_d / N)
 * cmesh_b is the spectrum of the mesh painted with shift_cells = 0.5 and is
 * left unchanged.  The result is a packed spectrum again.  After interlacing
 * the kz = N/2 plane is not Hermitian and cannot be packed: it is set to zero,
 * and plane-0 modes on a Nyquist index (|n_x| or |n_y| = N/2) are left
 * unspecified.  All these modes have |n| >= N/2 and lie outside every binning
 * allowed for interlaced meshes.
 * Errors: PK_EINVAL, PK_EDEVICE. */
pk_status pk_compensate(pk_ctx *ctx, const pk_mesh_desc *m, void *cmesh_inout,
                        const void *cmesh_b);

/* Binning of a packed spectrum as it is (no interlacing or compensation is
 * applied here) into the sums described at pk_result_doubles (Sec. 3.4.1).
 * The sums are unnormalised: the factor V / (sum w)^2 of P = V |delta(k)|^2
 * is applied by pk_result_to_host, which reads sum w from the same result
 * buffer, so that no call needs a host round trip between painting and
 * binning.
 * result_dev: device, pk_result_doubles(b) float64; every sum slot is
 * overwritten, the two weight slots are left unchanged.
 * Errors: PK_EINVAL (also for an interlaced m with a top edge above N/2),
 * PK_EUNSUPPORTED (too many bins for one workgroup's LDS), PK_EDEVICE. */
pk_status pk_bin_power(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b,
                       const void *cmesh, double *result_dev);

/* pk_bin_power for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same binning and the same result slots, but the squared bin edges and
 * the per-workgroup partial sums are kept in a fixed 8 MiB array of device
 * memory that the library holds on each GPU from its load until the process
 * ends (its address is looked up by pk_ctx_create).  The call allocates
 * nothing: no hipMalloc, no hipFree, no table of the context (the counts and
 * mean |k| that pk_result_to_host adds are built there, on first use of a
 * binning).  Its grids shrink to the partial rows that fit the array, so
 * every binning pk_bin_power accepts fits; larger ones are refused with
 * PK_EUNSUPPORTED and a message.  All calls on one GPU share the array:
 * calls that overlap on one GPU (other streams, other contexts, other host
 * threads) race and must not be issued.  The sums equal pk_bin_power's up to
 * the order of float64 additions.
 * Errors: as pk_bin_power; PK_EDEVICE if the array's address could not be
 * obtained on this device. */
pk_status pk_bin_power_noalloc(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b,
                               const void *cmesh, double *result_dev);

/* Cross power of two fields on the same mesh (the two-field form of the
 * FFTPower estimator, Sec. 3.4.1): as pk_bin_power with |c|^2 replaced by
 * Re(c1 conj(c2)) mode by mode, for packed spectra prepared the same way
 * (pk_paint, pk_fft_r2c, pk_compensate).  pk_result_to_host normalises by the
 * first weight slot squared: store sqrt(W1 W2) there (W = sum of the weights
 * of each catalog) and 0 in the second, the shot noise of two distinct
 * catalogs.  Errors: as pk_bin_power, PK_EINVAL for a NULL cmesh2. */
pk_status pk_bin_cross(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b,
                       const void *cmesh1, const void *cmesh2, double *result_dev);

/* Projected power (ProjectedFFTPower, Sec. 3.4.1): the power of the field
 * summed along the axes not kept, P = L^d |c|^2 / (sum w)^2 over the d kept
 * axes.  The d-dimensional transform of the projected field is the 3-D
 * spectrum on the plane (or line) where the projected wave numbers vanish,
 * so it is read from a packed spectrum prepared as for pk_bin_power
 * (pk_paint, pk_fft_r2c, pk_compensate); every mode of the full kept grid
 * counts once.  keep: bit 1 = x, 2 = y, 4 = z kept, one or two bits.  b: k-bins
 * in units of k_f over the kept axes, nmu <= 1 and no poles.  result_dev:
 * device, pk_projected_doubles(b) float64: [3 nk] sums overwritten (|c|^2,
 * counts, |n|), then {sum w, sum w^2} left for the caller to fill, as for
 * pk_bin_power.  Errors: PK_EINVAL, PK_EDEVICE. */
size_t pk_projected_doubles(const pk_bin_desc *b);
pk_status pk_bin_projected(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b, int keep,
                           const void *cmesh, double *result_dev);
/* Finalises a projected power: out->k, power, modes (the other arrays are
 * not touched), shotnoise = L^d sum w^2 / (sum w)^2, wsum, w2sum. */
pk_status pk_projected_to_host(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b,
                               int keep, const double *result_dev, pk_result *out);

/* The whole FFTPower hot path for one catalog (Sec. 3.3.1 painting, Eq. 1;
 * Sec. 3.3.2 windows, interlacing and compensation, Eq. 2; Sec. 3.4.1
 * binning into P(k), P(k, mu) and P_ell): paint (both meshes if
 * interlaced), r2c, interlace, compensate, bin.  n <= 2^31 - 1 (the sorted
 * records are indexed with 32-bit offsets; PK_EUNSUPPORTED beyond; pk_paint
 * has no such limit).  workspace: device,
 * >= pk_workspace_bytes(m, b, n) bytes, caller-owned scratch (content on
 * entry ignored).  result_dev as in pk_bin_power, all slots overwritten
 * including sum w and sum w^2.  Nothing is allocated when the context
 * already holds the tables for this mesh size and binning.  The particles
 * are grouped by mesh column on the device, by one of two routes chosen there
 * from the catalog's order (no host round trip); the order of the float64
 * sums within a column is not fixed, so results are reproducible to rounding
 * only.
 * Errors: PK_EINVAL (also a too small workspace), PK_EUNSUPPORTED,
 * PK_EDEVICE. */
pk_status pk_fftpower(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b,
                      const void *pos, const void *weight, int64_t n,
                      void *workspace, size_t workspace_bytes, double *result_dev);

/* ---- Lanes: concurrent requests on one device (batching and serving).
 * A lane is a HIP stream of its own (default priority) with a completion
 * event.  Requests on different lanes run concurrently; each needs its own
 * workspace while it runs.  Small meshes do not fill the 256 CUs, so several
 * lanes keep the device busy.  The context is not thread-safe: one host
 * thread submits and polls. */
#define PK_MAX_LANES 64

/* Creates lanes until the context has nlanes (1 .. PK_MAX_LANES); existing
 * lanes are kept.  Errors: PK_EINVAL, PK_EDEVICE. */
pk_status pk_ctx_set_lanes(pk_ctx *ctx, int nlanes);
int pk_ctx_lanes(const pk_ctx *ctx);

/* pk_fftpower enqueued on a lane, returning once enqueued.  The tables the
 * request needs are built first on the context stream (plan time, only the
 * first time a mesh size or binning is seen) and the lane waits for them.
 * workspace and result_dev must stay untouched until the lane has finished
 * (pk_lane_query / pk_lane_wait); then pk_result_to_host reads the result.
 * Errors: as pk_fftpower, PK_EINVAL for a lane that does not exist. */
pk_status pk_fftpower_async(pk_ctx *ctx, int lane, const pk_mesh_desc *m,
                            const pk_bin_desc *b, const void *pos, const void *weight,
                            int64_t n, void *workspace, size_t workspace_bytes,
                            double *result_dev);

/* 1 when the lane's last submitted request has finished, 0 while it runs,
 * a negative pk_status on error. */
int pk_lane_query(pk_ctx *ctx, int lane);
/* Blocks until the lane's last submitted request has finished. */
pk_status pk_lane_wait(pk_ctx *ctx, int lane);

/* A batch of independent requests (Sec. 6: many mocks analysed one after
 * another) spread over the context's lanes: request i has mesh m[i], bins
 * b[i], positions pos[i], weights weight[i] (weight may be NULL for all unit
 * weights, or hold NULL entries), n[i] particles and result_dev[i].  Lane l
 * works in lane_workspace[l] (lane_workspace_bytes each, enough for every
 * request).  Requests are taken largest first, each to the lane with the
 * least queued work; the context stream waits for all lanes, so a
 * synchronisation of the context stream (pk_result_to_host) sees every
 * result.  All requests are validated before any work is enqueued.
 * Errors: PK_EINVAL (also no lanes), PK_EUNSUPPORTED, PK_EDEVICE. */
pk_status pk_fftpower_batch(pk_ctx *ctx, int count, const pk_mesh_desc *m,
                            const pk_bin_desc *b, const void *const *pos,
                            const void *const *weight, const int64_t *n,
                            void *const *lane_workspace, size_t lane_workspace_bytes,
                            double *const *result_dev);

/* ---- Run-time tuning of the launch choices of pk_fftpower.
 * Two choices have no winner that holds for every input: painting an
 * interlaced pair of meshes in one two-mesh launch or in two single-mesh
 * launches (the halos of the two meshes differ by window), and the number
 * of persistent workgroups per CU of the fused x-pass + binning (one or two
 * where the LDS allows two).  With autotuning on, the first
 * synchronous pk_fftpower call for a key (N, dtype, window, interlaced and
 * the density class round(log2(n / N^3))) runs the whole path once per
 * candidate (a warm-up run and a timed run each, with HIP events on the
 * context stream, synchronising it) and keeps the fastest in the context;
 * that call's result is the last run's, with the chosen settings.  Later
 * calls with the key (pk_fftpower, pk_fftpower_v, lanes, batches, graphs
 * built afterwards) use the choice.  Without a choice the defaults are:
 * one two-mesh paint launch; as many x-pass workgroups as the device
 * holds.  The table can be read and stored by the
 * caller and loaded into another context, so the tuning runs once per
 * machine. */
typedef struct {
  int32_t nmesh, dtype, window, interlaced, density;  /* the key            */
  int32_t split;         /* interlaced: 1 two single-mesh launches, 0 one  */
  int32_t xpass_per_cu;  /* x-pass workgroups per CU, 0 = as many as fit   */
  double ms;             /* timed run of the chosen settings (diagnostic)  */
} pk_tune_entry;
/* mode 1: tune on first use; 0: use the table as it is (defaults for keys
 * without an entry).  Errors: PK_EINVAL. */
pk_status pk_ctx_set_autotune(pk_ctx *ctx, int mode);
int pk_tune_count(const pk_ctx *ctx);
/* Entry i (0 .. pk_tune_count - 1) into *out (host).  Errors: PK_EINVAL. */
pk_status pk_tune_get(const pk_ctx *ctx, int i, pk_tune_entry *out);
/* Sets (or replaces) the entry of its key; the choice fields must be valid
 * (split in {0, 1}, xpass_per_cu in {0, 1, 2}).  Errors: PK_EINVAL. */
pk_status pk_tune_put(pk_ctx *ctx, const pk_tune_entry *entry);

/* ---- Graph-captured batches (repeated analyses, Sec. 6: the same batch
 * of mocks run many times).  pk_fftpower_batch_graph records the whole
 * launch sequence of a batch -- bucketing, fused paint + z-FFT, y-pass,
 * fused x-pass + binning, reduce for every request, spread over the lanes as
 * pk_fftpower_batch spreads them (or one after another on the context stream
 * in lane_workspace[0] when the context has no lanes) -- into one HIP graph,
 * instantiated once; pk_graph_launch replays it on the context stream with
 * one host call.  The graph keeps the addresses it was built with: pos,
 * weight, n, the workspaces and result_dev must stay allocated, and a replay
 * reads the positions as they are at that time and overwrites the results.
 * Every table the batch needs is built (and synchronised) before the
 * capture; nothing is allocated while capturing or replaying.  The context
 * stream must be a stream created by the caller (not the legacy default
 * stream) and stage timing must be off.  A replay is ordered on the context
 * stream like any call; pk_result_to_host reads the results afterwards.
 * Errors: as pk_fftpower_batch (count >= 1), PK_EINVAL if timing is on,
 * PK_EDEVICE (capture refused, e.g. on the legacy default stream). */
typedef struct pk_graph pk_graph;
pk_status pk_fftpower_batch_graph(pk_ctx *ctx, int count, const pk_mesh_desc *m,
                                  const pk_bin_desc *b, const void *const *pos,
                                  const void *const *weight, const int64_t *n,
                                  void *const *lane_workspace, size_t lane_workspace_bytes,
                                  double *const *result_dev, pk_graph **graph);
pk_status pk_graph_launch(pk_ctx *ctx, pk_graph *graph);
size_t pk_graph_nodes(const pk_graph *graph); /* kernel and dependency nodes; 0 for NULL */
void pk_graph_destroy(pk_graph *graph);         /* NULL is a no-op */

/* pk_fftpower with per-particle field values (Sec. 3.3.1: the painted field
 * is [1 + delta'] V, delta' the weighted overdensity): each particle paints
 * w V; the normalisation stays sum w, and the second weight slot holds
 * sum (w V)^2, so that the reported shot noise is V_box sum (w V)^2 /
 * (sum w)^2.  value: device, n values of the mesh dtype, or NULL (then this
 * is pk_fftpower).  Errors: as pk_fftpower. */
pk_status pk_fftpower_v(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b,
                        const void *pos, const void *weight, const void *value, int64_t n,
                        void *workspace, size_t workspace_bytes, double *result_dev);

/* ---- Survey multipoles with a varying line of sight (ConvolvedFFTPower,
 * named in Sec. 3.4.1; the paper cites the FFT estimator of Hand et al. 2017
 * without writing it out, so the standard form is implemented):
 *   F(x)     = sum_data w delta_D(x - x_i) - alpha sum_randoms w delta_D(x - x_j),
 *              alpha = sum_data w / sum_randoms w,
 *   A_lm(k)  = FFT of F painted with the factor Y_lm(r^), r^ the unit vector
 *              from the observer to the particle (z^ where they coincide),
 *              divided by the window when m->compensated (Eq. 2),
 *   F_ell(k) = 4 pi / (2 ell + 1) sum_m Y_lm(k^) A_lm(k), Y_lm real and
 *              orthonormal,
 *   P_ell(k) = (2 ell + 1) / I  <Re F_0(k) conj F_ell(k)>  over the k-bin,
 * I the survey normalisation (an input of pk_convolved_to_host).  Shot noise
 * (sum_data w^2 + alpha^2 sum_randoms w^2) / I is reported, not subtracted.
 * Every multipole ell takes 2 ell + 1 paintings and FFTs (F_0 is always
 * formed).
 *
 * Positions are box coordinates (painted periodically, like pk_fftpower);
 * the line of sight uses them as given.  m: interlaced must be 0
 * (PK_EUNSUPPORTED otherwise).  b: 1-D k-bins (nmu 0 or 1), 1 .. 4 poles
 * among 0, 2, 4, top edge kmin_f + nk dk_f <= N/2 (the kz = N/2 plane is not
 * formed); los is ignored.
 *
 * Result (device, pk_convolved_doubles(b) float64): [npoles][nk] sums of
 * h Re(F_0 conj F_ell) per k-bin in the order of b->poles, then
 * {sum_data w, sum_data w^2, sum_randoms w, sum_randoms w^2}.  */
size_t pk_convolved_doubles(const pk_bin_desc *b);
/* Device workspace of pk_convolved_power (bytes), 0 for invalid arguments:
 * the concatenated catalog, its records, the painted amounts of every
 * harmonic Y_lm (sum over the fields of 2 ell + 1 values per particle), five
 * meshes and one spectrum per field F_ell kept. */
size_t pk_convolved_workspace_bytes(const pk_mesh_desc *m, const pk_bin_desc *b, int64_t n_data,
                                    int64_t n_rand);
/*   observer    host, 3 doubles, box coordinates
 *   data_pos    device, n_data x 3 positions of the mesh dtype (n_data >= 1,
 *               n_data + n_rand <= 2^31 - 1, else PK_EUNSUPPORTED)
 *   data_weight device, n_data weights, or NULL for unit weights
 *   rand_pos    device, n_rand x 3 positions (n_rand >= 1)
 *   rand_weight device, n_rand weights, or NULL
 *   workspace   device, >= pk_convolved_workspace_bytes, caller-owned
 *   result_dev  device, pk_convolved_doubles(b) float64, overwritten
 * Enqueued on the context stream: part of the work runs on a second stream
 * that the context owns (created on first use), joined back to the context
 * stream before the result is written, so the call is ordered on the
 * context stream like the others.  A zero sum of random weights gives NaN
 * results.  Errors: PK_EINVAL, PK_EUNSUPPORTED, PK_EDEVICE. */
pk_status pk_convolved_power(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b,
                             const double *observer, const void *data_pos,
                             const void *data_weight, int64_t n_data, const void *rand_pos,
                             const void *rand_weight, int64_t n_rand, void *workspace,
                             size_t workspace_bytes, double *result_dev);
/* Synchronises the context stream and finalises: out->k, out->modes and
 * out->poles ([npoles][nk], P_ell as above) are written, out->power is not
 * touched; out->wsum / w2sum are the data sums and out->shotnoise the shot
 * noise above.  norm: I > 0.  Errors: PK_EINVAL, PK_EDEVICE. */
pk_status pk_convolved_to_host(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b,
                               double norm, const double *result_dev, pk_result *out);

/* FFTPower finalisation (Sec. 3.4.1: P(k) and P(k, mu) as mode averages of
 * V |delta(k)|^2 with delta = DFT(F) / sum w, the painted field being 1 + delta
 * of Sec. 3.3.1; P_ell the Legendre moments; shot noise reported, not
 * subtracted).  Synchronises the context stream, copies the sums back and
 * finalises them with the mode tables (counts, mean |k|, mean |mu|):
 *   P = V sum(h P) / (sum w)^2 / N_b,
 *   P_ell = (2 ell + 1) V sum(h P L_ell) / (sum w)^2 / N_b,
 *   P(k, mu) likewise per (k, mu)-bin; empty bins give NaN and count 0.
 * out: host struct with caller-allocated arrays (see pk_result).
 * Errors: PK_EINVAL, PK_EDEVICE. */
pk_status pk_result_to_host(pk_ctx *ctx, const pk_mesh_desc *m, const pk_bin_desc *b,
                            const double *result_dev, pk_result *out);

/* Stage timing (diagnostics, Sec. 6 of the paper reports per-step wall
 * clock).  While enabled, pk_fftpower records a HIP event on the context
 * stream before each of its stages and one after the last; the events cost a
 * few microseconds per call.  pk_ctx_stage_times synchronises on the last
 * event and writes the milliseconds of every stage of the last timed call
 * (host array of pk_stage_count() doubles, 0 for stages that did not run).
 * Errors: PK_EINVAL (NULL arguments, no timed call yet), PK_EDEVICE. */
pk_status pk_ctx_set_timing(pk_ctx *ctx, int enable);
int pk_stage_count(void);
const char *pk_stage_name(int stage); /* NULL outside [0, pk_stage_count()) */
pk_status pk_ctx_stage_times(pk_ctx *ctx, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* PK_H */
