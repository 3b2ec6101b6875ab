/*
 * mp3.h -- C ABI of the MI355X in-situ multipole 3PCF library.
 *
 * The library evaluates the multipole moments zeta_l(r1, r2) of the isotropic
 * three-point correlation function of a periodic density field with the
 * in-situ multipole algorithm of Ju, Feng, Huang, Sun & Zhu ("An Optimal
 * In-Situ Multipole Algorithm for the Isotropic Three-Point Correlation
 * Function"):
 *
 *   deposit      catalogue -> basis coefficients -> density contrast
 *                (Sec. 2.1, multiresolution reconstruction; Sec. 3, workflow
 *                step 2 and the periodic-box contrast delta = n/nbar - 1)
 *   fields       a_{lm,b}(x) = IFFT[ FFT(delta) K_{lm,b} ],
 *                K_{lm,b}(k) = i^l jbar_{l,b}(|k|) conj(Y_lm(k_hat))
 *                (Sec. 2.2, Eqs. 3PCF-multipole-window and SFC-3PCF-vertex,
 *                with the radial-bin window of the paragraph after Eq. nL-2fold)
 *   zeta         zeta_l[b1,b2] = (4 pi / N^3) sum_x delta_x sum_{m=-l..l}
 *                a_{lm,b1}(x) conj(a_{lm,b2}(x))   (Sec. 2.2,
 *                Eqs. 3PCF-multipole-sum and SFC-3PCF, grid summation with
 *                the connection coefficients lumped onto the primary node)
 *   backward     gradient of J = sum_l <lambda_l, zeta_l> with respect to
 *                the density grid and the particle weights (chain rule of
 *                the above; the paper gives no gradient)
 *
 * Conventions shared by every entry point
 *   - Grid: N^3 periodic nodes at x = l * a, a = box / N, row-major with the
 *     x index slowest: element (ix, iy, iz) at (ix * N + iy) * N + iz.
 *   - DFT: dhat(q) = sum_x delta_x exp(-2 pi i q.x / N); q_d in [-N/2, N/2)
 *     stored at index q_d mod N; k = 2 pi q / box.  The window vanishes on
 *     every Nyquist plane (any q_d = -N/2).
 *   - Precision: a plan is MP3_F32 (fields, FFTs and filter in float32,
 *     tables generated in float64, reductions in float64) or MP3_F64 (the
 *     plain float64 form, same kernels).  "real" below means float for
 *     MP3_F32 and double for MP3_F64; complex values are interleaved
 *     (re, im) pairs of real.
 *   - Bulk buffers are DEVICE pointers owned by the caller; the library never
 *     frees caller memory and never allocates during a call.  It owns only
 *     the plan (tables) allocated by mp3_plan_create.
 *   - Every call is asynchronous on the given stream (a hipStream_t passed as
 *     void*, NULL = default stream).  Argument errors are detected on the
 *     host before any launch and return a negative status; a failed launch
 *     returns MP3_EHIP.  mp3_last_error() gives a message for the last
 *     failure of the calling thread.
 *   - A plan may be used by one stream at a time.
 */
#ifndef MP3_H
#define MP3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mp3_plan_s* mp3_plan_t;

enum mp3_status {
  MP3_OK = 0,
  MP3_EINVAL = -1,        /* bad argument (NULL pointer, size, order, range)       */
  MP3_ENOMEM = -2,        /* device or host allocation failed in mp3_plan_create   */
  MP3_EHIP = -3,          /* a HIP runtime call or kernel launch failed            */
  MP3_EUNSUPPORTED = -4,  /* valid request the library does not implement          */
  MP3_EWORKSPACE = -5,    /* workspace pointer NULL or smaller than required       */
  MP3_ENONFINITE = -6     /* a NaN or infinity in the description, or (with
                             MP3_KF_CHECK_FINITE) in the catalogue or delta       */
};

/* MP3_F32_BF16X3 is MP3_F32 whose contractions on the matrix cores (nodal,
 * grid-Gamma and particle forms with at most 32 bins) take BF16-split inputs:
 * each float32 operand x is carried as hi = bf16(x), lo = bf16(x - hi) and each
 * product as hi*hi + hi*lo + lo*hi, accumulated in float32 (relative error of
 * about 2^-16 per product against 2^-24).  Everything else is as MP3_F32. */
enum mp3_precision { MP3_F32 = 0, MP3_F64 = 1, MP3_F32_BF16X3 = 2 };

enum mp3_summation {
  MP3_SUM_NODAL = 0,      /* grid summation on the nodes (connection coefficients
                             lumped onto the primary node)                          */
  MP3_SUM_GRID_GAMMA = 1, /* grid summation with the B-spline connection
                             coefficients (Eqs. con-coeff, SFC-3PCF)                 */
  MP3_SUM_PARTICLE = 2    /* particle summation: primary vertex on the catalogue    */
};

/* Basis of the density reconstruction (Sec. 2.1, the scaling functions of the
 * multiresolution analysis; Sec. 3, the basis paragraph), in cell units u:
 *   MP3_BASIS_BSPLINE3     the centred cubic B-spline B3(u - l), support 4
 *                          cells per axis (not orthogonal; the deposit is the
 *                          projection coefficient sum_i w_i B3(u_i - l))
 *   MP3_BASIS_DAUBECHIES4  the Daubechies scaling function of genus 4 (four
 *                          orthonormal filter taps, support 3 cells): node l
 *                          carries phi(u - l + 1), phi taken as the linear
 *                          interpolant of its values at the points i / 1024
 *                          of [0, 3] from the cascade algorithm.  Nodal and
 *                          particle summation; with MP3_SUM_GRID_GAMMA
 *                          mp3_plan_create returns MP3_EUNSUPPORTED.
 * The basis sets the deposit, the interpolation at particles (the particle
 * form), the autocorrelation in the particle form's volume mean and the
 * Phi-hat factor of MP3_KF_PHI_HAT. */
enum mp3_basis { MP3_BASIS_BSPLINE3 = 0, MP3_BASIS_DAUBECHIES4 = 1 };

/* Radial window of the two secondary vertices (Sec. 2.2, the paragraph after
 * Eq. nL-2fold: a binning window multiplies the multipole window of
 * Eq. 3PCF-multipole-window at each vertex):
 *   MP3_BIN_SHELL_AVERAGE  jbar_{l,b}(k) = 3/(r_{b+1}^3 - r_b^3) int r^2 j_l(kr) dr
 *                          over the shell [edges[b], edges[b+1])
 *   MP3_BIN_THIN_SHELL     j_l(k r_b) at the shell's mid radius
 *                          r_b = (edges[b] + edges[b+1]) / 2 (the infinitely
 *                          thin shell of Eq. 3PCF-multipole-window) */
enum mp3_binning { MP3_BIN_SHELL_AVERAGE = 0, MP3_BIN_THIN_SHELL = 1 };

/* Option bits of mp3_plan_desc.kflags. */
enum mp3_kflags {
  /* multiply the secondary vertices' window by the power spectrum of the
   * father scaling function, Phi-hat(q) = prod_d |phi-hat(2 pi q_d / N)|^2
   * (sinc^8(pi q_d / N) for the cubic B-spline; the infinite product of the
   * filter's |m0|^2 for Daubechies-4), as in Eq. SFC-3PCF-vertex (default: no
   * such factor) */
  MP3_KF_PHI_HAT = 1u << 0,
  /* validate inputs on the device before using them: mp3_deposit checks the
   * positions and weights, the zeta / backward / value-and-grad calls check
   * delta, and a NaN or infinity returns MP3_ENONFINITE before any other
   * launch.  The check synchronises the stream (the call then blocks). */
  MP3_KF_CHECK_FINITE = 1u << 1
};

typedef struct {
  int32_t n;              /* grid points per side: 16, 32, 64, 128, 256 or 512       */
  double box;             /* periodic box side (length units of the catalogue), > 0  */
  int32_t lmax;           /* multipole truncation L, 0 <= L <= 20                    */
  int32_t nbins;          /* radial bins Nr, 1 <= Nr <= 64                           */
  const double* edges;    /* HOST array of nbins+1 strictly increasing edges >= 0,
                             copied into the plan; bin b is [edges[b], edges[b+1])   */
  int32_t precision;      /* enum mp3_precision                                     */
  int32_t summation;      /* enum mp3_summation                                     */
  int32_t batch;          /* mocks per call, >= 1                                   */
  int32_t basis;          /* enum mp3_basis                                         */
  uint32_t kflags;        /* OR of enum mp3_kflags (0 = none)                       */
  int32_t binning;        /* enum mp3_binning                                       */
  double smoothing;       /* radius R >= 0 of the spherical top-hat window assigned
                             to every vertex (Sec. 3, the triple-sphere binning):
                             W_TH(kR) = 3 j_1(kR) / (kR) multiplies both
                             secondaries' radial window, and the grid forms
                             (nodal, grid-Gamma) take the primary as delta
                             filtered by the same window.  The particle form's
                             primary is the catalogue itself (no window, the
                             paragraph before Eq. DDD-sum-privertex).  0 = none */
} mp3_plan_desc;

/* Build a plan: validates the description, generates the float64 tables (bin-
 * averaged spherical Bessel functions on every |q|^2 of the grid, FFT twiddles)
 * and uploads them.  *out is set only on success.  Blocking (host + device). */
int mp3_plan_create(const mp3_plan_desc* desc, mp3_plan_t* out);

/* Free a plan and its device tables.  NULL is accepted. */
int mp3_plan_destroy(mp3_plan_t plan);

/* Bytes of device workspace a call needs for catalogues of up to np_total
 * particles in total over the batch (0 for field-level calls).  The same size
 * serves every entry point.  The workspace is scratch: its content on entry is
 * ignored and on exit undefined. */
int mp3_workspace_size(mp3_plan_t plan, int64_t np_total, size_t* bytes);

/* Deposit a batch of catalogues (Sec. 2.1, reconstruction on the basis; Sec. 3,
 * density contrast):
 *   eps_l = sum_i w_i prod_d B3(x_{i,d} N / box - l_d),  B3 the centred cubic
 *   B-spline (support 4 cells per axis, periodic wrap),
 *   delta_l = eps_l N^3 / W - 1,  W = sum_i w_i.
 * pos     device float32 [np_total][3], positions in [0, box) (values outside
 *         are wrapped periodically);
 * w       device float32 [np_total] weights, or NULL for unit weights;
 * np_off  HOST int64 [batch+1], strictly increasing prefix offsets with
 *         np_off[0] = 0: mock j owns particles np_off[j] .. np_off[j+1]-1;
 *         an empty mock (W = 0, contrast undefined) returns MP3_EINVAL.
 *         pos, w (and dw of the gradient calls) must hold np_off[batch]
 *         entries: the library reads and writes exactly that many;
 * delta   device real [batch][N^3], written. */
int mp3_deposit(mp3_plan_t plan, const float* pos, const float* w, const int64_t* np_off,
                void* delta, void* workspace, size_t workspace_bytes, void* stream);

/* Fields of one multipole (Eq. SFC-3PCF-vertex with the binning window):
 *   a_{lm,b} = ifftn( fftn(delta) K_{lm,b} ),  0 <= m <= l <= lmax
 * (fields with m < 0 follow from a_{l,-m} = (-1)^m conj(a_{lm}) for real delta).
 * delta  device real [batch][N^3];
 * a_out  device complex [batch][nbins][N^3], written. */
int mp3_multipole_fields(mp3_plan_t plan, const void* delta, int32_t l, int32_t m, void* a_out,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Multipole moments of one batch.
 *
 * MP3_SUM_NODAL (Eqs. 3PCF-multipole-sum and SFC-3PCF, grid summation with the
 * connection coefficients lumped onto the primary node):
 *   zeta_l[b1,b2] = (4 pi / N^3) sum_x delta_x sum_{m=-l}^{l} a_{lm,b1}(x) conj(a_{lm,b2}(x)).
 *   pos, w and np_off are ignored (may be NULL).
 *
 * MP3_SUM_GRID_GAMMA (Eqs. con-coeff, SFC-3PCF, 3PCF-multipole-sum):
 *   zeta_l[b1,b2] = (4 pi / N^3) sum_x delta_x sum_m sum_{s,t} Gamma_{s,t}
 *                   a_{lm,b1}(x+s) conj(a_{lm,b2}(x+t)),
 *   Gamma_{s,t} = prod_d int B3(u) B3(u - s_d) B3(u - t_d) du, evaluated exactly
 *   as the integral of the three B-spline interpolants (5-point Gauss-Legendre
 *   per cell and axis).  pos, w, np_off ignored.
 *
 * MP3_SUM_PARTICLE (Sec. 2.2, the particle sum after Eq. DDD-sum-privertex; the
 * primary vertex is the catalogue's contrast n/nbar - 1):
 *   zeta_l[b1,b2] = 4 pi [ (1/W) sum_i w_i F_l(x_i) - Fbar_l ],
 *   F_l(x) = sum_{m=-l}^{l} atilde_{lm,b1}(x) conj(atilde_{lm,b2}(x)),
 *   atilde the cubic B-spline interpolant of the fields at the particle, Fbar_l
 *   the exact volume mean of F_l:
 *   Fbar_l = (2l+1)/(4 pi N^6) sum_q |dhat(q)|^2 B7hat(q) jbar_{l,b1} jbar_{l,b2},
 *   B7hat the DFT of the B-spline autocorrelation samples.  pos, w (NULL =
 *   unit) and np_off as for mp3_deposit (delta must be their deposit).
 *   At most 2^31 - 1 particles in total.
 *
 * Both forms sum m >= 0 only (m > 0 counted twice).  Result real and symmetric.
 * delta  device real [batch][N^3];
 * zeta   device float64 [batch][lmax+1][nbins][nbins], overwritten. */
int mp3_zeta(mp3_plan_t plan, const void* delta, const float* pos, const float* w, const int64_t* np_off,
             double* zeta, void* workspace, size_t workspace_bytes, void* stream);

/* Gradient of J = sum_{j,l,b1,b2} dzeta[j][l][b1][b2] zeta_l^{(j)}[b1][b2] for
 * every form; the paper gives no gradient, this is the chain rule of mp3_zeta
 * and mp3_deposit.  The grid-Gamma form's adjoint takes the bins in chunks
 * that fit the LDS of its shift stencil.
 * The nodal and particle forms work in the eigenbasis of each symmetrised
 * cotangent (dzeta_l + dzeta_l^T) / 2 = V diag(d) V^T, decomposed per (l,
 * mock) on the device in float64: their fields come from the radial window
 * rotated by V, so the adjoint sources are diagonal in the bins; the
 * gradient is the same to rounding.
 * The fields are recomputed per (l, m); nothing is kept from mp3_zeta.
 *   ddelta = dJ/ddelta                                          (device real [batch][N^3])
 *            For the particle form this is the dependence through the
 *            secondary vertices (the fields and the volume mean), the
 *            primary's weights held fixed.
 *   dw     = dJ/dw_i (device real [np_total]): through delta = eps N^3 / W - 1
 *            of mp3_deposit, (N^3/W) [ sum_l B_i(l) g_l - N^-3 sum_l (1 + delta_l) g_l ]
 *            with g = ddelta, plus for the particle form the primary vertex's
 *            4 pi [ F_J(u_i) / W - sum_j w_j F_J(u_j) / W^2 ],
 *            F_J = sum_{l,m,b1,b2} dzeta_l[b1][b2] atilde_{b1} conj(atilde_{b2}).
 *            Needs pos, w, np_off as given to mp3_deposit.
 * ddelta must not be NULL.  dw may be NULL: then the nodal form ignores pos,
 * w and np_off; the particle form always needs them.
 * dzeta  device float64 [batch][lmax+1][nbins][nbins]. */
int mp3_zeta_backward(mp3_plan_t plan, const void* delta, const double* dzeta,
                      void* ddelta, const float* pos, const float* w, const int64_t* np_off,
                      void* dw, void* workspace, size_t workspace_bytes, void* stream);

/* Value and gradient of J = sum_{j,l,b1,b2} dzeta[j][l][b1][b2] zeta_l^{(j)}[b1][b2]
 * in one sweep over (l, m): J is linear in zeta, so its cotangent dzeta is
 * known before the forward (the paper gives no gradient; this is the chain
 * rule of mp3_zeta, as for mp3_zeta_backward).
 *   zeta   : as mp3_zeta, overwritten;
 *   ddelta, dw : as mp3_zeta_backward for the same dzeta.
 * Arguments, layouts, workspace and error codes are those of the two calls.
 * Nodal form, float32 or float64, at most 32 bins: each (l, m) computes the
 * window, y and x passes once, and one z pass both contracts the fields and
 * forms the adjoint sources, so the fields are neither stored across (l, m)
 * nor computed twice.  Particle form: the per-call steps (tile sort, stencil
 * records, power histogram) run once and each (l, m)'s stored fields feed
 * both the gather contraction and the adjoint sources.  Grid-Gamma form:
 * the adjoint's node values of each (l, m) are also contracted for zeta.
 * BF16-split plans and nodal plans above 32 bins run mp3_zeta and then
 * mp3_zeta_backward.  The nodal and particle forms contract zeta over the
 * fields of the cotangent's eigenbasis (see mp3_zeta_backward) and rotate it
 * back, zeta = V zetabar V^T (exactly symmetric); the particle form then
 * subtracts its volume means.  The results agree with the two separate calls
 * to rounding (per multipole: an entry's rounding follows the largest entry
 * of its multipole; the grid-Gamma contraction visits the nodes in another
 * order). */
int mp3_zeta_value_and_grad(mp3_plan_t plan, const void* delta, const double* dzeta,
                            double* zeta, void* ddelta, const float* pos, const float* w,
                            const int64_t* np_off, void* dw, void* workspace,
                            size_t workspace_bytes, void* stream);

/* Two-point correlation function of delta by the same window machinery
 * (Sec. 2.1, Eqs. pair-counting and window-sphshell): with the plan's
 * top-hat radius R on both vertices (the grid forms' primary filtered as in
 * mp3_zeta; the particle form's plan leaves the primary unfiltered),
 *   xi(r) = N^-6 sum_q |dhat(q)|^2 Wp(|k|) W_TH(|k| R) Phi(q) j_0(|k| r)
 *         = N^-3 sum_x delta_p(x) (W_r o delta)(x),
 * Wp = W_TH(|k| R) for the grid forms with R > 0, else 1; Phi = phi-hat with
 * MP3_KF_PHI_HAT, else 1; W_r the infinitely thin shell of radius r; the
 * Nyquist planes excluded (as for the secondary vertices of mp3_zeta).
 * radii  HOST double [nr], >= 0, 1 <= nr <= 4096;
 * xi     device float64 [batch][nr], overwritten. */
int mp3_xi(mp3_plan_t plan, const void* delta, const double* radii, int32_t nr, double* xi, void* workspace,
           size_t workspace_bytes, void* stream);

/* Line-of-sight multipoles of the two-point function (Sec. 2.1, Eqs.
 * DD-multipole and DD-windowfunction; the line of sight is the grid's z axis,
 * the plane-parallel form of axial symmetry):
 *   xi_ell(r) = N^-6 sum_q |dhat(q)|^2 Wp Ws Phi (2 ell + 1) Re(i^ell) j_ell(|k| r) P_ell(q_z / |q|),
 * windows as mp3_xi, so that the azimuthal average of the pair correlation at
 * separation r and polar angle theta is sum_ell xi_ell(r) P_ell(cos theta);
 * odd ell vanish for real delta.
 * radii  HOST double [nr], >= 0, 1 <= nr <= 4096;  0 <= ell_max <= 16;
 * xi     device float64 [batch][ell_max+1][nr], overwritten. */
int mp3_xi_multipoles(mp3_plan_t plan, const void* delta, const double* radii, int32_t nr, int32_t ell_max,
                      double* xi, void* workspace, size_t workspace_bytes, void* stream);

/* The 3PCF at the bin radii reconstructed from its multipoles, truncated at
 * lt (Sec. 2.2, Eq. triplet-counting; Sec. 3, Eq. Q-factor):
 *   zeta(r_b1, r_b2, theta) = sum_{l=0}^{lt} zeta_l[b1][b2] P_l(cos theta),
 *   Q = zeta / (xi(r1) xi(r2) + xi(r2) xi(r3) + xi(r3) xi(r1)),
 *   r3^2 = r1^2 + r2^2 - 2 r1 r2 cos theta,
 * with r_b the bins' mid radii (edges[b] + edges[b+1]) / 2 and xi as mp3_xi
 * of the same delta.
 * zeta  device float64 [batch][lmax+1][nbins][nbins] (as written by mp3_zeta);
 * lt    0 <= lt <= lmax;
 * mu    HOST double [nth] values of cos theta in [-1, 1], 1 <= nth <= 4096;
 * zeta_theta  device float64 [batch][nbins][nbins][nth], overwritten;
 * q     device float64, same shape, overwritten, or NULL to skip Q (delta
 *       may then be NULL too). */
int mp3_reduced_3pcf(mp3_plan_t plan, const void* delta, const double* zeta, int32_t lt, const double* mu,
                     int32_t nth, double* zeta_theta, double* q, void* workspace, size_t workspace_bytes,
                     void* stream);

/* mp3_zeta_value_and_grad for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation, arguments and results, with the scratch
 * memory taken from a fixed device array inside the library instead of a
 * caller's workspace.  Each GPU the library runs on holds its own copy of
 * that array (mp3_static_scratch_bytes() bytes, 64 MiB) until the process
 * ends.  A call whose mp3_workspace_size exceeds it returns MP3_EWORKSPACE
 * (nothing launched).  The call itself allocates nothing.  Every call on one
 * GPU uses that GPU's one copy, which keeps the last call's contents: calls
 * that overlap on one GPU (two streams, two threads) race and must be
 * serialised by the caller.  The plan's device must be current. */
int mp3_zeta_value_and_grad_static(mp3_plan_t plan, const void* delta, const double* dzeta, double* zeta,
                                   void* ddelta, const float* pos, const float* w, const int64_t* np_off, void* dw,
                                   void* stream);

/* Bytes of the static scratch array of mp3_zeta_value_and_grad_static. */
size_t mp3_static_scratch_bytes(void);

/* Edge-corrected estimator with a random catalogue (Sec. 3, Eq. SSestimator):
 * zeta = (D - R)^3 / R^3, D - R reconstructed from the differences of the
 * two catalogues' basis coefficients.  Three steps, each on the device:
 *   1. mp3_deposit the data and the random catalogue (delta_D, delta_R);
 *      mp3_ss_fields gives f = delta_D - delta_R = n_D/nbar_D - n_R/nbar_R
 *      and r = 1 + delta_R = n_R/nbar_R (device real [batch][N^3] each);
 *   2. mp3_zeta of f and of r with a grid-summation plan (nodal or
 *      grid-Gamma): the multipoles N_l, R_l of the triplet correlations of
 *      (D - R) and of R (the q = 0 mode is kept, so r's mean enters);
 *   3. mp3_ss_multipoles: zeta_l = (2l+1)/2 int N(mu) / R(mu) P_l(mu) dmu,
 *      N and R summed over l <= lt (Eq. triplet-counting), the integral by
 *      nquad-point Gauss-Legendre quadrature.
 * zeta_n, zeta_r  device float64 [batch][lmax+1][nbins][nbins];
 * zeta_ss         device float64 [batch][lt+1][nbins][nbins], overwritten;
 * 0 <= lt <= lmax, 1 <= nquad <= 4096. */
int mp3_ss_fields(mp3_plan_t plan, const void* delta_d, const void* delta_r, void* f, void* r, void* stream);
int mp3_ss_multipoles(mp3_plan_t plan, const double* zeta_n, const double* zeta_r, int32_t lt, int32_t nquad,
                      double* zeta_ss, void* workspace, size_t workspace_bytes, void* stream);

/* Pass identifiers for per-pass timing. */
enum mp3_pass {
  MP3_PASS_DFT = 0,        /* forward 3-D DFT of delta; final DFT of the adjoint accumulator */
  MP3_PASS_FILTER = 1,     /* window K_{lm,b} + y-transform, all bins (one launch per (l, m)) */
  MP3_PASS_X = 2,          /* x-transform of all bins                                          */
  MP3_PASS_Z_NODAL = 3,    /* z-transform + nodal contraction                                  */
  MP3_PASS_Z_ADJOINT = 4,  /* z-transform + adjoint sources + their z-transform                */
  MP3_PASS_ADJOINT = 5,    /* y-transform of the adjoint sources, window, bin sum into G       */
  MP3_PASS_DEPOSIT = 6,    /* B-spline scatter of the catalogue                                */
  MP3_PASS_Z_STORE = 7,    /* z-transform, fields stored bin-interleaved (particle form)       */
  MP3_PASS_GATHER = 8,     /* B-spline gather at the particles + contraction                   */
  MP3_PASS_GAMMA = 9,      /* grid-Gamma quadrature contraction                                */
  MP3_PASS_SCATTER = 10,   /* adjoint sources scattered from the particles onto the grid      */
  MP3_PASS_Z_FUSED = 11,   /* z-transform + contraction + adjoint sources (value and gradient) */
  MP3_NPASS = 12
};

/* Per-pass timing for measurement: with enable != 0 every pass launch of
 * later calls on this plan is bracketed by two HIP events on the call's
 * stream.  Calling it resets the totals.  Diagnostic only; adds two event
 * records per launch. */
int mp3_profile(mp3_plan_t plan, int enable);

/* Total milliseconds and number of launches of one pass since the last
 * mp3_profile call.  Waits for the recorded events (synchronises the
 * stream up to the last profiled launch). */
int mp3_profile_read(mp3_plan_t plan, int pass, double* total_ms, int64_t* launches);

/* Launch-shape knobs of a plan.  They change how the work is cut into
 * workgroups and which FFT radix plan a pass uses, never what is computed
 * (results agree to rounding order).  Defaults are values measured good on
 * MI355X across the benchmark workloads; the autotuner of the Python package
 * searches them per (n, nbins, lmax, form, precision, batch, basis, device)
 * and caches the winners (the package ships those of its benchmark
 * workloads). */
enum mp3_tune_knob {
  MP3_TUNE_ZPASS_WGS = 0,     /* workgroups of the z passes per call, split over the batch;
                                 64 .. 65536, default 4096                                       */
  MP3_TUNE_CONTRACT_WGS = 1,  /* workgroups of the particle gather and the grid-Gamma
                                 contraction per call; 64 .. 65536, default 4096                 */
  MP3_TUNE_FFT_X_PLAN = 2,    /* radix plan of the strided x pass: 0 = largest radix first
                                 (16 at n = 256), 1 = radix-8 stages; default 0                  */
  MP3_TUNE_DEPOSIT_TILE = 3,  /* side of the deposit's LDS tile in cells: 4, 8 or 16;
                                 default 8                                                       */
  MP3_TUNE_DEPOSIT_WGS = 4,   /* workgroups of the persistent deposit; 64 .. 65536, default 2048
                                 (never more than there are tiles)                               */
  MP3_TUNE_FUSED_WAVES = 5,   /* waves per workgroup of the one-sweep (value and gradient) z
                                 pass: 0 = the fewest whole waves that hold one round of every
                                 bin's columns (default; best measured at 128^3, 12 bins),
                                 else 1 .. 8, raised to what n needs (one thread per z point;
                                 4 is best measured at 256^3, 20 bins)                           */
  MP3_TUNE_ITEM_GROUP = 6,    /* (l, m) items per launch of the nodal adjoint passes (window,
                                 x and z passes of mp3_zeta_backward and the one sweep of
                                 mp3_zeta_value_and_grad): 0 = as many as fit 1 GiB of fields
                                 (default), else 1 .. 1024, capped at (lmax+1)(lmax+2)/2     */
  MP3_TUNE_GAMMA_ADJOINT = 7, /* kernel of the grid-Gamma adjoint (B-spline plans): 0 = the
                                 stencil over the shifts of the connection coefficients
                                 (default), 1 = the transposed node quadrature; Daubechies-4
                                 plans always take the stencil                               */
  MP3_NTUNE = 8
};

/* Set a knob.  Out-of-range values return MP3_EINVAL and leave the knob as
 * it was.  The workspace size depends on MP3_TUNE_ZPASS_WGS,
 * MP3_TUNE_CONTRACT_WGS, MP3_TUNE_DEPOSIT_TILE, MP3_TUNE_ITEM_GROUP (the
 * fields of every item of a group are held at once) and MP3_TUNE_GAMMA_ADJOINT:
 * query mp3_workspace_size
 * again after changing them.  Not to be called while work of the plan is in
 * flight on another thread. */
int mp3_tune_set(mp3_plan_t plan, int knob, int32_t value);

/* Read a knob's current value into *value. */
int mp3_tune_get(mp3_plan_t plan, int knob, int32_t* value);

/* Read back the plan's parameters (any out pointer may be NULL). */
int mp3_plan_info(mp3_plan_t plan, int32_t* n, int32_t* lmax, int32_t* nbins,
                  int32_t* precision, int32_t* batch);

/* Host-side float64 routines of plan creation, exported so that they can be
 * checked without a GPU (no device work, no plan needed). */

/* Spherical Bessel functions j_0(x) .. j_lmax(x) into out[0 .. lmax]
 * (the radial functions of the plane-wave expansion, Sec. 2.1,
 * Eq. plane-sph-harmonics): upward recurrence for x > lmax, Miller's downward
 * recurrence below, exact at x = 0.  lmax in [0, 64], x >= 0 and finite. */
int mp3_sph_bessel(int32_t lmax, double x, double* out);

/* The radial window table a plan built from desc uses (Sec. 2.2, the radial
 * part of Eq. 3PCF-multipole-window times the binning window):
 *   out[(l * nq2 + s) * nbins + b] = R_{l,b}(k_s) W_TH(k_s R),
 *   k_s = (2 pi / box) sqrt(s), s = 0 .. nq2 - 1, nq2 = 3 (n/2)^2 + 1,
 * with R_{l,b} the bin-average or thin-shell window of desc->binning and
 * W_TH = 1 when desc->smoothing = 0.  count must be (lmax+1) nq2 nbins.
 * Validates desc as mp3_plan_create does. */
int mp3_window_table(const mp3_plan_desc* desc, double* out, size_t count);

/* Host tables of a basis (Sec. 3, the basis paragraph; Eqs. SFC-3PCF-vertex
 * and con-coeff), computed without a GPU as mp3_plan_create does; any output
 * may be NULL:
 *   table[i] = phi(i / 1024), i = 0 .. 3072 (table_count must be 3073),
 *              Daubechies-4 only (NULL for the B-spline);
 *   acf[s]   = int phi(x) phi(x - s) dx, s = 0 .. 3, of the basis as the
 *              deposit uses it (the autocorrelation of the particle form's
 *              volume mean);
 *   phi_hat[i] = |phi-hat(2 pi q / n)|^2, q = i for i < n/2 else i - n
 *              (n a supported grid size);
 *   gamma[(s + 3) * 7 + t + 3] = int phi phi(. - s) phi(. - t), s, t in
 *              -3 .. 3 (the connection coefficients of one axis; for
 *              Daubechies-4 those of the exact scaling function, zero for
 *              |s| or |t| = 3).
 * Returns MP3_EINVAL for an unknown basis, a wrong count or a table the basis
 * does not have. */
int mp3_basis_tables(int32_t basis, int32_t n, double* table, size_t table_count, double* acf, double* phi_hat,
                     double* gamma);

/* Human-readable name of a status code (static storage). */
const char* mp3_status_string(int status);

/* Message describing the last failure on the calling thread (thread-local,
 * valid until the next library call on that thread). */
const char* mp3_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MP3_H */
