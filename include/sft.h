/*
 * sft.h -- C ABI of libsft.so: short-Fourier-transform (SFT) inner products of
 * long-duration compact-binary gravitational-wave templates on one AMD MI355X
 * (gfx950).  Method: Tenorio & Gerosa, arXiv:2502.11823.
 *
 * The library evaluates, for every template of a bank, the SFT approximation of
 * the inner product <x,h> = 4 Re int x~* h~ / S_n df (Sec. I, Eq. fd_product):
 *
 *   ([d,h]) = sum_a A_a Lambda_a exp(i phi_a) C_a                (Sec. III.E, Eq. efficient)
 *   C_a     = sum_{k = k0-K}^{k0+K} conj(d~'_a[k]) F(kappa_a - k, beta_a)   (Eq. with_f_1)
 *
 * with the waveform quantities {A_a, phi_a, f_a, fdot_a} taken at the midpoint of
 * each SFT, kappa_a = f_a T_SFT, beta_a = fdot_a T_SFT^2, d~_a = 2 x~_a / S_a the
 * per-SFT whitened data (Sec. III.B), d~'_a[k] = (-1)^k d~_a[k] (midpoint reference)
 * and F the Fresnel kernel (Sec. III.C) or, when |beta| <= beta_switch, its
 * Dirichlet limit sinc(x) (App. B).  Lambda_a = F+_a A+ Re + Fx_a Ax Im is the
 * projector of Sec. II.A.  Per template the library returns
 *
 *   z+ = sum_a F+_a A_a exp(i phi_a) C_a,  zx = sum_a Fx_a A_a exp(i phi_a) C_a,
 *   ([d,h]) = A+ Re z+ + Ax Im zx,
 *   hh+ = sum_a F+_a^2 A_a^2 T / S_a(f_a),  hhx likewise (the narrow-band <h,h>),
 *   rho = |A+ z+ - i Ax zx| / sqrt(A+^2 hh+ + Ax^2 hhx)   (phase-maximised SNR,
 *         Sec. II.B, Eq. det_short).
 *
 * Every call returns sft_status: SFT_OK (0) or a negative error code; on error
 * sft_last_error() returns a thread-local message.  Problems of one template
 * never fail a call: they set bits of that template's flags word.
 */
#ifndef SFT_H
#define SFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sft_status;
enum {
  SFT_OK = 0,
  SFT_E_INVALID = -1,     /* null pointer, bad size or descriptor field */
  SFT_E_NOMEM = -2,       /* device or host allocation failed */
  SFT_E_DEVICE = -3,      /* a HIP runtime call or kernel launch failed */
  SFT_E_RANGE = -4,       /* a size or option outside the supported range */
  SFT_E_UNSUPPORTED = -5  /* an option combination the library does not implement */
};

/* device storage of the whitened SFT bins */
enum { SFT_STORE_F64 = 0, SFT_STORE_F32 = 1, SFT_STORE_BF16 = 2 };
/* kernel choice (Sec. III.C, App. B) */
enum { SFT_KERNEL_DIRICHLET = 0, SFT_KERNEL_FRESNEL = 1, SFT_KERNEL_AUTO = 2 };
/* arithmetic of the bin contraction and of the sums over SFTs; the waveform
 * phase, its reduction mod 2 pi and the bin split are FP64 in every mode.  FP64 forms the
 * Fresnel weights from FP64 Fresnel integrals (power series, continued fraction of erfcx;
 * ~1e-15) bin by bin: a reference mode, much slower than the FP32 modes with Fresnel. */
enum { SFT_PREC_FP64 = 0, SFT_PREC_FP32_KAHAN = 1, SFT_PREC_FP32_NAIVE = 2 };
/* waveform model: leading-order (Newtonian) chirp, the 3.5PN closed-form inspiral, or
 * the learned surrogate (opts.surrogate) with the 3.5PN waveform as judge and fallback.
 * PN35 and SURROGATE need F32 or F64 storage and read the bank's mass ratio q >= 1
 * (NULL => q = 1). */
enum { SFT_WF_NEWTON = 0, SFT_WF_PN35 = 1, SFT_WF_SURROGATE = 2 };

/* per-template flag bits */
enum {
  SFT_FLAG_OUT_OF_BAND = 1u,      /* a window bin, or a PSD bin of the norm, lies outside the stored band,
                                     or a window centre lies below DC or above Nyquist (that SFT
                                     then contributes nothing) */
  SFT_FLAG_TAU_NONPOSITIVE = 2u,  /* an SFT of the template's range starts its midpoint at or after t_c; skipped */
  SFT_FLAG_TAYLOR_INVALID = 4u,   /* fddot T^3 / 8 > delta_max in some SFT (Eq. max_tsft, midpoint lever arm) */
  SFT_FLAG_NONFINITE = 8u,        /* an output is not finite */
  SFT_FLAG_SURROGATE_FALLBACK = 32u, /* surrogate judged worse than the tolerance: 3.5PN waveform used */
  SFT_FLAG_EMPTY = 64u,           /* no SFT contributed to the norm; rho is set to 0 */
  SFT_FLAG_FSTAT_DEGENERATE = 128u /* F-statistic form only: the weighted response vectors (F+_a) and
                                     (Fx_a) are within ~5.7 degrees of parallel (det < 1e-2 hh+ hhx);
                                     2F keeps the dominant pattern only (see sft_out.twoF) */
};

/* Largest window half-width K supported by the scan. */
#define SFT_K_MAX 64

typedef struct sft_data sft_data; /* opaque; owns every device buffer it refers to */

typedef struct {
  int32_t n_sft;      /* SFT rows (all detectors); a data gap is an absent row */
  int32_t n_samples;  /* samples per SFT, n (even); dt = t_sft / n */
  double t_sft;       /* SFT duration T [s]; bin k has frequency k / T */
  int32_t k_lo;       /* first stored bin, 0 <= k_lo <= n/2 */
  int32_t n_bins;     /* stored bins k_lo .. k_lo + n_bins - 1, all <= n/2 */
  int32_t storage;    /* SFT_STORE_* */
  int32_t reserved;   /* must be 0 */
} sft_data_desc;

/*
 * sft_load_data -- whiten and stage SFTs on the device (Sec. III.B per-SFT
 * whitening, Eq. d_SFT normalisation).
 *   desc     : sizes and storage precision.
 *   t_start  : host [n_sft] start time of each SFT [s].
 *   x_bins   : host [n_sft][n_bins][2] raw SFT bins (re, im), x~_a[k] = dt sum_j x_j e^{-2 pi i jk/n}.
 *   psd      : host [n_sft][n_bins] one-sided noise PSD S_a(f_k); a bin whose PSD is not
 *              positive and finite is masked (contributes zero).
 *   fplus, fcross : host [n_sft] antenna patterns, or NULL for F+ = 1, Fx = 0.
 *   hip_stream: hipStream_t (NULL = default stream) for the uploads and the load kernel;
 *              the call returns after the data are ready on the device.
 *   out      : receives the handle; release it with sft_free_data.
 * Host arrays are only read during the call.  Bins of the stored band are
 * mirrored through d~[-k] = conj(d~[k]) and d~[n-k] = conj(d~[k]) (footnote of
 * Sec. III.C) when the band reaches DC or Nyquist.  Errors: SFT_E_INVALID (null
 * pointer, n_sft < 1, odd n, band outside [0, n/2]), SFT_E_NOMEM, SFT_E_DEVICE.
 */
sft_status sft_load_data(const sft_data_desc* desc, const double* t_start, const double* x_bins,
                         const double* psd, const double* fplus, const double* fcross,
                         void* hip_stream, sft_data** out);

/* Release a handle and its device memory (NULL is a no-op). */
void sft_free_data(sft_data* data);

/*
 * SFTs from raw strain on the device (Sec. III.B segmentation, Eq. d_SFT), with the per-SFT
 * noise PSD estimated from the SFT itself: the running median of the periodogram
 * P[k] = |x~[k]|^2 over blocks of 2w+1 bins centred on k (shifted at the ends of [0, n/2]),
 * divided by B = sum_{i=0}^{w} 1/(2w+1-i) (the mean of the middle order statistic of 2w+1
 * unit exponentials) and scaled by 2/T (E|x~|^2 = T S / 2 for stationary Gaussian noise).
 * Each detector's series is cut into consecutive segments of n samples, segment a covering
 * samples [a n, (a+1) n) and starting at t0 + a n dt; a segment holding a non-finite sample is
 * a data gap (missing SFT).  n a power of two: an FFT per segment; other even n (the SFT
 * lengths of Sec. IV, e.g. 106 s at 40 Hz) with a known white PSD: the band bins by their
 * defining sum.
 */
typedef struct {
  int32_t n_det;        /* detector series */
  int32_t n_samples;    /* samples per SFT, n: a power of two in [16, 16384] */
  int64_t n_total;      /* samples per series; n_seg = n_total / n segments (a remainder is unused) */
  double dt;            /* sampling interval [s]; T = n dt */
  double t0;            /* time of sample 0 of every series [s] */
  int32_t k_lo;         /* first stored bin */
  int32_t n_bins;       /* stored bins k_lo .. k_lo + n_bins - 1, all <= n/2 */
  int32_t psd_w;        /* running-median half width w; 2w + 1 <= n/2 + 1 */
  int32_t storage;      /* SFT_STORE_* of the handle made by sft_load_strain */
  double s_white;       /* > 0: a known white one-sided PSD, used for every bin (no estimate, psd_w
                           ignored); 0: the running-median estimate (needs n a power of two) */
} sft_strain_desc;

/*
 * sft_make_sfts -- the SFTs and PSDs of every segment, asynchronously on hip_stream (returns
 * once the launch is enqueued; a device's first call for a segment length also builds that
 * length's twiddle tables, tens of KB, and keeps them on the device until the process ends).
 *   x    : DEVICE [n_det][n_total] strain series (FP64), read only.
 *   bins : DEVICE out [n_det][n_seg][n_bins][2] x~ = dt sum_j x_j e^{-2 pi i j k / n} of the band.
 *   psd  : DEVICE out [n_det][n_seg][n_bins] the estimated one-sided PSD.
 *   keep : DEVICE out [n_det][n_seg] 1, or 0 for a gap (whose bins and PSD are written as 0).
 * Errors: SFT_E_INVALID (null, bad descriptor, band or block outside [0, n/2]),
 * SFT_E_UNSUPPORTED (n odd or outside [16, 16384], or not a power of two without s_white),
 * SFT_E_RANGE, SFT_E_DEVICE.
 */
sft_status sft_make_sfts(const sft_strain_desc* desc, const double* x, double* bins, double* psd, int32_t* keep,
                         void* hip_stream);

/*
 * sft_load_strain -- sft_make_sfts followed by sft_load_data on the device: the segments that
 * are not gaps become the handle's SFT rows (detector by detector, in time order), whitened by
 * their own PSD estimates.
 *   fplus, fcross : host [n_det][n_seg] antenna patterns per segment, or NULL (F+ = 1, Fx = 0).
 *   n_rows        : host out (may be NULL), the number of SFT rows kept.
 * Synchronous on hip_stream.  Errors: those of sft_make_sfts and sft_load_data; SFT_E_INVALID
 * when every segment is a gap.
 */
sft_status sft_load_strain(const sft_strain_desc* desc, const double* x, const double* fplus, const double* fcross,
                           void* hip_stream, sft_data** out, int32_t* n_rows);

/*
 * Time-domain companions, for accuracy studies of the SFT inner product (Sec. IV.A: the
 * relative error r = 1 - sqrt(([d,h]) / <d,h>) against the direct integral).
 *
 * sft_waveform_series -- the strain of one template at the samples t_j = t0 + j dt, j < n:
 *   h_j = A(t_j) [F+_j A+ cos phi(t_j) + Fx_j Ax sin phi(t_j)]   (the projector of Sec. II.A),
 * with the waveform of the scans (SFT_WF_NEWTON or SFT_WF_PN35, mass ratio q for the latter),
 * zero where tau = t_c - t_j <= 0.  fplus, fcross: DEVICE [n] per-sample antenna patterns, or
 * NULL (1 and 0).  h: DEVICE out [n].  quantities: DEVICE out [n][5] (A, phi, f, fdot, fddot at
 * each sample) or NULL.  Asynchronous on hip_stream.  Errors: SFT_E_INVALID, SFT_E_UNSUPPORTED
 * (other waveforms), SFT_E_RANGE, SFT_E_DEVICE.
 */
sft_status sft_waveform_series(int32_t waveform, double mc, double q, double t_c, double phi_c, double tsun,
                               double t0, double dt, int64_t n, const double* fplus, const double* fcross,
                               double a_plus, double a_cross, double* h, double* quantities, void* hip_stream);

/*
 * sft_td_product -- <x, y> = 4 Re int x~* y~ / S df = (2 / S) dt sum_j x_j y_j for a white
 * one-sided PSD S (Eqs. fd_product, td_product, whitened_data), x, y DEVICE [n].  FP64,
 * compensated, in a fixed order (bitwise reproducible).  Synchronous on hip_stream; the result
 * goes to the host *out.  Errors: SFT_E_INVALID, SFT_E_DEVICE.
 */
sft_status sft_td_product(const double* x, const double* y, int64_t n, double dt, double psd, void* hip_stream,
                          double* out);

/*
 * sft_set_ephemeris -- detector motion for the Doppler form of the scan (Sec. III.B: the
 * phase as a function of the emission time t_s(t; n), the frequency
 * (1/2 pi)(dphi/dt_s)(dt_s/dt)).
 *   eph : host [n_sft][9], for each SFT row at its midpoint: the detector's position r/c [s],
 *         velocity v/c and acceleration a/c [1/s] relative to the solar-system barycentre,
 *         in any fixed frame (the bank's sky vectors use the same frame).  Only the Roemer
 *         delay r.n/c is modelled (the relativistic delays are left out).
 * Rows that share a start time no longer share a waveform: afterwards every row is its own
 * timestamp group (time order kept), for every scan of the handle.  The call returns after
 * the upload on hip_stream.  Errors: SFT_E_INVALID (null, non-finite entry), SFT_E_NOMEM,
 * SFT_E_DEVICE.
 */
sft_status sft_set_ephemeris(sft_data* data, const double* eph, void* hip_stream);

/* Reference time of each SFT's Taylor expansion (Sec. III.B): the midpoint (default) or the
 * start, as the paper writes it.  With SFT_REF_START the waveform is evaluated at t_a, the
 * window is centred on the start frequency, k0 = floor(f_a T + 1/2), the kernel is
 * int_0^1 exp(i (2 pi x s + pi beta s^2)) ds on the data without the (-1)^k of the midpoint
 * form, the norm uses A_a and S_a(f_a) at the start, and the validity flag f_ddot T^3 / 2. */
enum { SFT_REF_MID = 0, SFT_REF_START = 1 };

typedef struct {
  int32_t K;            /* window half-width: bins k0-K .. k0+K, 0 <= K <= SFT_K_MAX (Sec. III.C truncation) */
  int32_t kernel;       /* SFT_KERNEL_* */
  int32_t precision;    /* SFT_PREC_*: FP64 needs SFT_STORE_F64 data, the FP32 modes need F32 or BF16 data */
  int32_t waveform;     /* SFT_WF_* */
  int32_t t_ref;        /* SFT_REF_MID or SFT_REF_START (the start needs the Newtonian or 3.5PN waveform
                           and no ephemeris) */
  double beta_switch;   /* AUTO kernel: Dirichlet when |fdot T^2| <= beta_switch (bins) */
  double a_plus;        /* A+ of the projector, used for rho */
  double a_cross;       /* Ax of the projector, used for rho */
  double tsun;          /* G M_sun / c^3 [s]; M = Mc * tsun */
  double delta_max;     /* Taylor-validity threshold in bins (Eq. max_tsft); <= 0 disables the flag */
  const struct sft_surrogate* surrogate;  /* network of SFT_WF_SURROGATE; NULL otherwise */
} sft_opts;

/* Fill *opts with K = 8, AUTO kernel, FP32_KAHAN, Newtonian waveform, midpoint reference,
 * beta_switch = 1e-7, A+ = 1, Ax = 0, tsun = 4.925490947641267e-6 s, delta_max = 0,
 * surrogate = NULL. */
void sft_default_opts(sft_opts* opts);

/* Template bank, structure of arrays in DEVICE memory owned by the caller.
 * Leading-order chirp (Newtonian) with chirp mass mc [Msun], coalescence time
 * t_c [s] and phase phi_c [rad]: f = (5M/tau)^{3/8}/(8 pi M), phi = phi_c - 2 (tau/5M)^{5/8},
 * A = (pi M f)^{2/3}, tau = t_c - t, M = mc * tsun.  The 3.5PN waveform uses in addition
 * the mass ratio q (nu = q/(1+q)^2, total mass mc nu^(-3/5)); its phase and frequency are
 * the post-Newtonian series in Theta = nu tau / (5 M_total) and its amplitude the
 * dominant-mode amplitude through 2PN.  Template m uses SFT rows a_first[m]..a_last[m]
 * (inclusive, clamped to the data).  q (mass ratio) is read only by waveforms that
 * depend on it and may be NULL otherwise; phi_c, a_first, a_last may be NULL
 * (0, 0, n_sft - 1).
 * sky [n][3] (may be NULL): unit vectors toward the sources, in the frame of the data's
 * ephemeris (sft_set_ephemeris).  Given, the scan runs its Doppler form (Sec. III.B): the
 * phase is taken at the emission time t_s = t + r(t).n / c of each SFT row's detector, and
 * f = f_s (1 + v.n/c), fdot = fdot_s (1 + v.n/c)^2 + f_s a.n/c at the SFT midpoint, with
 * f_s, fdot_s the source-frame chirp at t_s (t_c is then the coalescence time at the source,
 * up to the constant light travel time); fddot for the validity flag is fddot_s (1 + v.n/c)^3.
 * The Doppler form exists for the Newtonian waveform with FP32-Kahan sums on F32 data or
 * FP64 sums on F64 data (SFT_E_UNSUPPORTED otherwise). */
typedef struct {
  const double* mc;
  const double* q;
  const double* t_c;
  const double* phi_c;
  const int32_t* a_first;
  const int32_t* a_last;
  const double* sky;
} sft_bank;

/* Outputs, DEVICE memory owned by the caller: zp, zx are [n][2] (re, im);
 * hhp, hhx, rho are [n]; flags is [n].  mismatch [n] may be NULL; with the surrogate
 * waveform it receives each template's judge mismatch (see SFT_WF_SURROGATE below),
 * other waveforms leave it untouched.
 *
 * F-statistic (Sec. II.B, Eq. det_long and the maximisation over the four amplitudes c_nu):
 * when twoF [n] is not NULL the scan runs its F-statistic form, which reads the antenna
 * patterns F+_a, Fx_a of each SFT row as the functions a(t), b(t) of Eq. det_long and writes
 *   hhpx = sum_a F+_a Fx_a A_a^2 T / S_a(f_a)       (when hhpx [n] is not NULL),
 *   2F   = x.M^{-1}.x,  x = (Re z+, Re zx, Im z+, Im zx) = <x, h_nu> for
 *          h_nu = A (a cos phi, b cos phi, a sin phi, b sin phi),
 *          M = [[N, 0], [0, N]], N = [[hh+, hh+x], [hh+x, hhx]] (cos-sin products vanish
 *          under the narrow-band norm), i.e. twice the maximum over c of c.x - c.M.c/2.
 * When det N < 1e-2 hh+ hhx (patterns nearly parallel, e.g. one detector over much less than
 * a day) only the dominant eigenvector u of N (eigenvalue lambda) is kept:
 * 2F = ((u.x_cos)^2 + (u.x_sin)^2) / lambda, flagged SFT_FLAG_FSTAT_DEGENERATE.  In noise 2F
 * follows chi^2 with 4 degrees of freedom.  The F-statistic form keeps the three norm sums in
 * FP64 and exists for the Newtonian waveform with FP32-Kahan sums on F32 data or FP64 sums
 * on F64 data (otherwise SFT_E_UNSUPPORTED); z+, zx are bitwise those of the plain scan. */
typedef struct {
  double* zp;
  double* zx;
  double* hhp;
  double* hhx;
  double* rho;
  uint32_t* flags;
  double* mismatch;
  double* hhpx;
  double* twoF;
  int32_t* n_used;  /* [n] or NULL: SFT rows that entered the template's sum (rows of its range
                       whose reference time precedes t_c) */
} sft_out;

/*
 * sft_template_bank_scan -- SFT inner products of n_templates templates against
 * one data handle (Sec. V.B two-step evaluation, batched over the bank).
 * Asynchronous on hip_stream (NULL = default stream): inputs must stay valid and
 * outputs must not be read until the stream reaches this point.  A workspace of
 * about 56 bytes per template and SFT chunk is taken from the stream-ordered
 * allocator and returned on the same stream.  Results are bitwise deterministic
 * for a given bank, data and options.  n_templates == 0 is a no-op.
 * With SFT_WF_SURROGATE the scan runs in template batches of about
 * 2^23 / (timestamp groups) templates, each with a workspace of about 1 GiB (network
 * inputs and outputs, the chirp table) on the same stream; the network must not be
 * trained or freed while such a scan is in flight.
 * Errors: SFT_E_INVALID (null pointers), SFT_E_RANGE (K), SFT_E_UNSUPPORTED
 * (precision/storage or kernel combinations), SFT_E_NOMEM, SFT_E_DEVICE.
 */
sft_status sft_template_bank_scan(const sft_data* data, const sft_bank* bank, int64_t n_templates,
                                  const sft_opts* opts, sft_out* out, void* hip_stream);

/* Size of the library-owned device array that is the workspace of
 * sft_template_bank_scan_noalloc, on every GPU the library runs on. */
#define SFT_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

/*
 * sft_template_bank_scan_noalloc -- the bank scan for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same kernels and arguments as sft_template_bank_scan; the
 * workspace (partial sums per template and chunk of timestamp groups, flags, the
 * work-queue counter) lives in a file-scope device array of SFT_NOALLOC_SCRATCH_BYTES
 * instead of the stream-ordered allocator.  The call makes no hipMalloc, hipFree or
 * allocating library call.  Its device address is resolved once per GPU, on the first
 * call made with that GPU current; every GPU that runs the library holds its own copy
 * until the process ends.
 * Launch shape: the handle's tuning, with fewer (larger) chunks when its workspace
 * would not fit; results then agree with sft_template_bank_scan to rounding (the FP64
 * combination of the partial sums runs over other chunks), not bitwise.
 * All calls on one GPU share the array, which keeps the last call's contents: calls
 * that overlap in time on one GPU (different streams or host threads) race and must be
 * serialised by the caller; calls on one stream are ordered.  Must be called with the
 * data's device current.
 * Errors: those of sft_template_bank_scan; SFT_E_INVALID (data on another device);
 * SFT_E_RANGE when a single chunk's partial sums (52 bytes per template, 60 in the
 * F-statistic form) do not fit the array (more than about 1.29e6 templates, 1.12e6 in
 * the F-statistic form); SFT_E_UNSUPPORTED for
 * SFT_WF_SURROGATE (its template batches need about 1 GiB of workspace);
 * SFT_E_DEVICE when the array's address cannot be resolved or a launch fails.
 */
sft_status sft_template_bank_scan_noalloc(const sft_data* data, const sft_bank* bank, int64_t n_templates,
                                          const sft_opts* opts, sft_out* out, void* hip_stream);

/* Order in which a scan visits the bank (sft_tuning.order). */
enum { SFT_ORDER_GIVEN = 0, SFT_ORDER_TRACK = 1 };

/*
 * Launch shape of the bank scan, kept per data handle (fields equal to 0 select the
 * automatic choice).  block: templates per workgroup, 64, 128 or 256 (default 256).
 * chunk_groups: timestamp groups (SFT rows sharing a start time, one per detector) per
 * work item; a work item is (template tile, chunk), and partial sums are combined in
 * chunk order (default: chunks of about 1 MiB of bins and at least four work items per
 * resident workgroup).  persistent: 1 launches one workgroup per resident slot, each
 * pulling work items from a device counter until the queue is empty; 0 launches one
 * workgroup per item.  An all-zero tuning selects the automatic chunks with the
 * persistent grid.
 * order: SFT_ORDER_GIVEN scans the bank in the caller's order, which is fast when
 * neighbouring templates have nearly equal frequency tracks (a bank sorted by chirp mass at
 * one coalescence time, say).  SFT_ORDER_TRACK first sorts the bank on the device by (first
 * SFT row, leading-order frequency at the middle of the template's SFT range), scans it in
 * that order and writes every result back to its template's given position: a bank in any
 * order then runs at the speed of a sorted one.  The sort takes about 60 bytes per template
 * of extra stream-ordered workspace.  A graph plan computes the order once, when it is
 * created, and gathers the bank into it at every launch (contents changed later still give
 * correct results); the allocation-free scan and the surrogate waveform always use the
 * given order.
 * Results are bitwise identical for a given tuning and bank order; different tunings change
 * the order of the FP64 combination of partial sums, and a different bank order can change
 * which series of the kernel a template's wavefront evaluates (rounding-level differences).
 */
typedef struct {
  int32_t block;
  int32_t chunk_groups;
  int32_t persistent;
  int32_t order;       /* SFT_ORDER_GIVEN (default) or SFT_ORDER_TRACK */
} sft_tuning;

/* Read or replace the tuning of a handle.  Errors: SFT_E_INVALID, SFT_E_RANGE. */
sft_status sft_get_tuning(const sft_data* data, sft_tuning* tuning);
sft_status sft_set_tuning(sft_data* data, const sft_tuning* tuning);

/*
 * sft_autotune -- time candidate tunings (block 64/128/256, 1..64 chunks, plain and
 * persistent grids) on the given bank in its given order with HIP events on hip_stream,
 * reps timed runs each after one warm-up; time the candidates within 2% of the fastest twice
 * more, in turn, and take the best of those repeated times; then time the fastest with
 * SFT_ORDER_TRACK (sort included) and keep that order when it is faster.  Store the result in the handle and
 * return it (best, best_ms may be NULL).  Writes the outputs like a scan.  Synchronises
 * hip_stream.
 * Errors: those of sft_template_bank_scan, SFT_E_RANGE (reps outside [1, 100]).
 */
sft_status sft_autotune(sft_data* data, const sft_bank* bank, int64_t n_templates, const sft_opts* opts,
                        sft_out* out, void* hip_stream, int32_t reps, sft_tuning* best, float* best_ms);

/*
 * Graph plans: a bank scan captured once into a HIP graph with its own workspace
 * (about 56 bytes per template and chunk, allocated at creation), replayed by
 * sft_plan_launch on any stream.  The plan keeps the device pointers of bank and out
 * and the handle's tuning at creation: their contents may change between launches,
 * the pointers may not, and data must outlive the plan.  Launches of one plan must not
 * overlap (they share the workspace).  Errors: those of sft_template_bank_scan,
 * SFT_E_NOMEM, SFT_E_DEVICE (capture or instantiation failed).
 */
typedef struct sft_plan sft_plan;
sft_status sft_plan_create(const sft_data* data, const sft_bank* bank, int64_t n_templates,
                           const sft_opts* opts, sft_out* out, sft_plan** plan);
sft_status sft_plan_launch(sft_plan* plan, void* hip_stream);
void sft_plan_destroy(sft_plan* plan);

/*
 * Learned surrogate waveform (an MLP correction to the leading-order chirp; the method
 * evaluates any waveform model at the SFT midpoints, Sec. III.A, and the 3.5PN model
 * serves to train it and to judge it).
 *
 * Network: u = (u_mc, u_q, u_tau) -> `layers` hidden layers of width `hidden` with SiLU
 * -> (y1, y2), inputs mapped to [-1, 1]: u_mc = 2 (mc - mc_lo) / (mc_hi - mc_lo) - 1,
 * u_q likewise, u_tau = 2 (ln tau - lt_lo) / (lt_hi - lt_lo) - 1.  Parameters are FP32,
 * packed layer by layer: W [n_in][n_out] (input-major), then b [n_out].
 * Waveform at tau = t_c - t, with M = mc tsun, Theta_N = tau / (5 M) and p = 1/8 when
 * head = 1, 3/8 when head = 0:
 *   phi  = phi_Newton + head * phi_head + c_phi Theta_N^p y1,
 *   A    = A_Newton exp(c_amp y2),
 *   f    = f_Newton - (d/dtau)(head * phi_head + c_phi Theta_N^p y1) / (2 pi)
 *          (dy1/dtau by forward-mode differentiation through the network),
 *   fdot = fdot_Newton (f / f_Newton)^(11/3),  fddot = (11/3) fdot^2 / f,
 * phi_head = the 1PN and 1.5PN terms of the 3.5PN phase series.  Trained on targets
 * y1 = (phi_3.5PN - phi_Newton - head * phi_head) / (c_phi Theta_N^p),
 * y2 = ln(A_3.5PN / A_Newton) / c_amp.
 * Judge: per template, over the SFT rows it uses, the match of the surrogate against
 * the 3.5PN waveform in the SFT picture, mismatch = 1 - |sum_a w_a exp(i dphi_a)
 * sinc(T df_a)| / sum_a w_a with w_a = A_3.5PN,a^2 T / S_a(f_3.5PN,a) (the row's share of
 * <h,h>, S_a interpolated like the norm; a row whose PSD is masked or outside the stored band
 * there has no weight), dphi and df the surrogate minus 3.5PN phase and frequency at the SFT
 * midpoint.  With F32 storage the weights use the stored FP32 PSD (mismatch within ~1e-7 of
 * the FP64 value).  A template whose mismatch is not
 * <= judge_tol is evaluated with the 3.5PN waveform and flagged
 * SFT_FLAG_SURROGATE_FALLBACK.  The judge itself is always FP64.
 * Inference arithmetic of the network (sft_surrogate_desc.inference):
 *   SFT_INFER_FP64       FP64 evaluation of the FP32 parameters (FP64 matrix cores when
 *                        hidden is a multiple of 16 up to 128);
 *   SFT_INFER_FP64_BF16W FP64 evaluation of the parameters rounded to BF16;
 *   SFT_INFER_BF16X3     BF16 matrix cores with FP32 accumulation and FP32 activations, every
 *                        operand split into two BF16 numbers (16 significant bits) and each
 *                        product taken as three BF16 products: network outputs within ~1e-5 of
 *                        FP64;
 *   SFT_INFER_BF16       BF16 matrix cores, operands rounded to BF16 (8 significant bits),
 *                        FP32 accumulation: outputs within ~1e-2, for speed studies; the judge
 *                        rejects what this costs in phase.
 * The BF16 modes need hidden = 32, 64, 96 or 128 (SFT_E_UNSUPPORTED otherwise).
 */
enum { SFT_INFER_FP64 = 0, SFT_INFER_FP64_BF16W = 1, SFT_INFER_BF16X3 = 2, SFT_INFER_BF16 = 3 };

typedef struct {
  int32_t hidden;        /* hidden width, 8 .. 256 */
  int32_t layers;        /* hidden layers, 1 .. 8 */
  int32_t head;          /* 1: analytic 1PN + 1.5PN phase head; 0: the network carries it */
  int32_t inference;     /* SFT_INFER_* */
  double mc_lo, mc_hi;   /* input ranges of the normalisation */
  double q_lo, q_hi;
  double lt_lo, lt_hi;   /* range of ln(tau / s) */
  double c_phi;          /* phase scale [rad] */
  double c_amp;          /* log-amplitude scale */
  double judge_tol;      /* mismatch tolerance of the judge (e.g. 1e-4) */
} sft_surrogate_desc;

typedef struct sft_surrogate sft_surrogate;  /* opaque; owns its device buffers */

/* Parameter count of a network (0 for hidden < 1 or layers < 1). */
int64_t sft_surrogate_param_count(int32_t hidden, int32_t layers);

/* Create a network on the current device from host FP32 parameters
 * [sft_surrogate_param_count] (copied).  Errors: SFT_E_INVALID (null pointer, empty
 * ranges, zero scales), SFT_E_RANGE (hidden, layers), SFT_E_NOMEM, SFT_E_DEVICE. */
sft_status sft_surrogate_create(const sft_surrogate_desc* desc, const float* params, sft_surrogate** out);
/* Release a network (NULL is a no-op).  Calls on one network are not thread-safe, and a
 * network must outlive the scans and training calls enqueued with it. */
void sft_surrogate_free(sft_surrogate* s);
/* Copy the current FP32 parameters to host memory (synchronous). */
sft_status sft_surrogate_get_params(const sft_surrogate* s, float* params);

/*
 * sft_surrogate_targets -- training pairs from the library's own Newtonian and 3.5PN
 * waveforms: device mc, q, tau [n] (FP64) -> device u [n][3] and y [n][2] (FP32, the
 * network inputs and targets defined above).  Asynchronous on hip_stream.
 * Errors: SFT_E_INVALID (null pointers, n < 0), SFT_E_DEVICE.
 */
sft_status sft_surrogate_targets(const sft_surrogate* s, const double* mc, const double* q, const double* tau,
                                 int64_t n, double tsun, float* u, float* y, void* hip_stream);

/*
 * sft_surrogate_loss_grad -- loss L = (1/n) sum_i |net(u_i) - y_i|^2 of the FP32 network
 * on device u [n][3], y [n][2], and its gradient: *loss (device, one float) and grad
 * (device [P] floats, may be NULL; the network keeps it too).  Asynchronous on
 * hip_stream.  Errors: SFT_E_INVALID, SFT_E_RANGE (n outside [1, 2^21]), SFT_E_NOMEM,
 * SFT_E_DEVICE.
 */
sft_status sft_surrogate_loss_grad(sft_surrogate* s, const float* u, const float* y, int64_t n, float* loss,
                                   float* grad, void* hip_stream);

/*
 * sft_surrogate_adam -- one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected)
 * with learning rate lr on the gradient of the last sft_surrogate_loss_grad call.
 * Asynchronous on hip_stream.  Errors: SFT_E_INVALID, SFT_E_DEVICE.
 */
sft_status sft_surrogate_adam(sft_surrogate* s, float lr, void* hip_stream);

/*
 * sft_surrogate_train -- epochs of mini-batch Adam over device u [n][3], y [n][2], the rows
 * shuffled afresh every epoch: epoch e visits the rows in the order of a keyed bijection of
 * [0, n) (a four-round Feistel network on the indices with cycle walking, keyed by e and the
 * network's Adam step count; deterministic), in batches of `batch` rows, n mod batch rows left
 * out per epoch; learning rate on a cosine schedule from lr to lr_min over the call.  The
 * GEMMs of the forward and backward passes run on the FP32 matrix cores.
 * epoch_loss (host [epochs], may be NULL) receives the mean batch loss of each epoch.
 * Synchronises hip_stream; refreshes the inference copy of the parameters.
 * Errors: SFT_E_INVALID, SFT_E_RANGE (batch outside [16, min(n, 2^20)], epochs < 1,
 * n > 2^31), SFT_E_NOMEM, SFT_E_DEVICE.
 */
sft_status sft_surrogate_train(sft_surrogate* s, const float* u, const float* y, int64_t n, int32_t batch,
                               int32_t epochs, float lr, float lr_min, void* hip_stream, float* epoch_loss);

/*
 * sft_surrogate_infer -- the scan's FP64 evaluation of the network: device u [n][3]
 * (FP64) -> y [n][2] and dy [n][2] = dy/du_tau.  Asynchronous on hip_stream.
 * Errors: SFT_E_INVALID, SFT_E_NOMEM, SFT_E_DEVICE.
 */
sft_status sft_surrogate_infer(const sft_surrogate* s, const double* u, int64_t n, double* y, double* dy,
                               void* hip_stream);

/*
 * sft_inner_product -- the SFT inner product of one template (Sec. III.E, Eq. efficient:
 * ([d,h]) = A+ Re z+ + Ax Im zx with z+, zx, the norms and rho as for the bank scan), host
 * arguments and host results: mc, q, t_c, phi_c as one entry of sft_bank, SFT rows
 * a_first..a_last.  Runs the bank scan with n = 1 on the default stream and waits for it;
 * allocates and frees a small device block per call (a convenience for single evaluations,
 * not for throughput).  zp and zx receive (re, im).  Any of the output pointers may be NULL.
 * Same errors as sft_template_bank_scan.
 */
sft_status sft_inner_product(const sft_data* data, double mc, double q, double t_c, double phi_c,
                             int32_t a_first, int32_t a_last, const sft_opts* opts,
                             double zp[2], double zx[2], double* hhp, double* hhx, double* rho,
                             uint32_t* flags);

/*
 * Kernel timing for benchmarks.  sft_kernel_timing(n) with n > 0 makes the next n
 * calls of sft_template_bank_scan (from any thread) record a pair of HIP events on
 * their stream around their scan kernel; n = 0 stops recording and drops the
 * records.  sft_kernel_times waits for the recorded events and copies up to max
 * elapsed times [ms] into ms; it returns the number of recorded scans.  Meant for a
 * single benchmarking thread.  Errors: SFT_E_DEVICE (event creation), SFT_E_RANGE
 * (n > 4096).
 */
sft_status sft_kernel_timing(int32_t n);
int32_t sft_kernel_times(float* ms, int32_t max);

/*
 * Issue-rate probe of the vector ALU, for benchmarks: the scan's roofline counts FP32 slots
 * against the nominal FP32 vector peak, which needs the packed FP32 instructions that this
 * library does not use; the probe measures what plain wave64 instructions sustain on the part.
 * One launch of 2048 workgroups of 256 lanes, each lane 16 independent chains of the chosen
 * instruction for 4096 iterations (SFT_PROBE_FMA_F32_INT32: 8 FP32 FMA chains beside 8 chains
 * of a 32-bit shift and xor), timed with HIP events on hip_stream after one warm-up launch, the
 * best of three.  instr_per_s: host out, VALU wave-instructions per second over the launch.
 * Synchronous on hip_stream; allocates and frees a 2 MiB device buffer.  Errors: SFT_E_INVALID
 * (null, unknown probe), SFT_E_DEVICE.
 */
enum { SFT_PROBE_FMA_F32 = 0, SFT_PROBE_RCP_F32 = 1, SFT_PROBE_FMA_F64 = 2, SFT_PROBE_FMA_F32_INT32 = 3 };
sft_status sft_probe_issue_rate(int32_t op, double* instr_per_s, void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* sft_last_error(void);

/* Library version string. */
const char* sft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SFT_H */
