// kernels.hpp -- host entry points of the device kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stddef.h>

namespace mp3 {

// Recurrence of the reduced associated Legendre functions Q_k^m for one
// (l, m), set on the host: Q_m^m = pmm, Q_{m+1}^m = (2m + 1) x pmm and
// Q_k^m = c1[k] x Q_{k-1}^m - c2[k] Q_{k-2}^m for k = m + 2 .. l, with
// c1[k] = (2k - 1) / (k - m), c2[k] = (k + m - 1) / (k - m).
struct YlmRec {
  double pmm;
  double c1[21], c2[21];
};

// One (l, m) work item of a call: everything the window passes need, kept in
// a device table (the workspace) for every item of the call.
// Daubechies-4 table: phi at i / 2^kD4Level, i = 0 .. 3 2^kD4Level
constexpr int kD4Level = 10;
constexpr int kD4TableSize = 3 * (1 << kD4Level) + 1;

// autocorrelation samples A(s) = int phi(x) phi(x - s) dx, s = 0 .. 3, of the basis
struct Acf {
  double a[4];
};

struct ItemRec {
  int l, m;
  double norm;       // Y_lm normalisation
  double wm;         // m weight of the contraction: 1 for m = 0, 2 otherwise
  YlmRec yr;         // Legendre recurrence of (l, m)
};

// Window passes over a group of nitems consecutive items of the table,
// starting at item0: the forward pass writes fields [item][batch][nbins][N^3],
// the adjoint pass sums every item of the group into G.
struct FilterArgs {
  const void* src;   // k_filter_y: dhat [batch][N^3]; k_adjoint_y: sources [item][batch][nbins][N^3]
  void* dst;         // k_filter_y: fields [item][batch][nbins][N^3]; k_adjoint_y: accumulator G [batch][N^3]
  const void* jtab;  // [lmax+1][jmocks][nq2][nbp] radial window, bin axis padded to nbp = 4 ceil(nbins / 4)
  int jmocks = 1;    // tables per l: 1 (the plan's), or batch (rotated into each mock's cotangent eigenbasis)
  const void* tw;    // twiddles exp(-2 pi i t / N)
  int nq2, nbins, nbp, batch;
  const ItemRec* items;   // device item table
  int item0, nitems;
  double scale;      // real factor (1/N^3); the adjoint pass also takes each item's m weight
  const void* phi = nullptr;   // [N] per-axis phi-hat factors (real), or NULL for none
};

struct ZpassArgs {
  const void* fields;   // [batch][nbins][N^3], layout [x][y][qz] (adjoint passes: [item][batch][nbins][N^3])
  const void* delta;    // [batch][N^3]
  double* partials;     // forward: [batch][nwg][nbins^2]; one sweep: [item][batch][nwg][nbins^2]
  const double* dzeta;  // backward: [batch][lmax+1][nbins^2]
  void* direct;         // backward: [batch][N^3] explicit-primary gradient accumulator
  const void* lam;      // backward: eigenvalues of the symmetrised dzeta, [lmax+1][batch][nbins] real
  const void* tw;
  int nbins, nwg, ppw, batch, l, lmax;
  bool split;           // float32 contraction with BF16-split inputs on the matrix cores
  int waves = 0;        // one-sweep z pass: waves per workgroup (0 = default)
  // adjoint passes: the group of items (table, first item, count) and the
  // persistent launch's work counter (device int, zeroed by the launch)
  const ItemRec* items = nullptr;
  int item0 = 0, nitems = 1;
  int* counter = nullptr;
};

struct GatherArgs {
  const void* fields;     // bin-interleaved fields [batch][N^3][nbins]
  const int* tcell;       // stencil records in sorted order (launch_tap_records)
  const void* twt;
  const float* pos;       // [np_total][3]
  const float* w;         // [np_total] or NULL
  const int* perm;        // particle order (tile-sorted), [np_total]
  const long long* off;   // device [batch+1]
  const double* W;        // device [batch] weight sums
  double* partials;       // [batch][nwg][nbins^2]
  int n, nbins, nwg, batch;
  double sc;              // N / box
  bool split;             // float32 contraction with BF16-split inputs on the matrix cores
  // adjoint sources from the same gather (value and gradient in one sweep) when src != NULL:
  // the fields are those of the rotated radial tables, lam the cotangent's eigenvalues
  const void* lam;        // [batch][nbins] eigenvalues of the symmetrised cotangent
  double wm;              // m weight
  double* FJ;             // [np_total] F_J accumulator
  void* src;              // [np_total][nbins] sources in sorted order
};

// The bins a grid-Gamma contraction takes: local bin i < na is stored bin
// a0 + i, the others stored bins c0 + (i - na), of nbt stored bins
// (all bins: {nbt, 0, nbt, 0, 0}).
struct BinPair {
  int nbt, a0, na, c0, nc;
};

// grid summation with connection coefficients (5-point Gauss-Legendre per cell);
// m[s][t] = B3(xi_s + 1 - t), wq[s] node weights on [0, 1]; partials over the
// pair's (na + nc)^2 local bin pairs
hipError_t launch_gamma_contract(int prec, bool split, const void* fields, const void* delta, int n,
                                 const BinPair& bp, const double (*m)[4], const double* wq, double* partials, int nwg,
                                 int batch, hipStream_t st);
// LDS bytes of a contraction tile holding nbins bins
size_t gamma_lds_need(int prec, int nbins);
// zeta += the pair's partials at their stored-bin positions (cross block always,
// diagonal blocks when owned)
hipError_t launch_reduce_partials_map(const double* partials, int nwg, const BinPair& bp, double* zeta, int l,
                                      int lmax, double scale, bool own_a, bool own_c, int batch, hipStream_t st);
// U[x][b] = sum_b' lam_s[b][b'] F[x][b'] over bin-interleaved fields
hipError_t launch_bin_mix(int prec, const void* F, const void* lam_s, void* U, long long n3, int nbins, int batch,
                          hipStream_t st);
// grid-Gamma adjoint of stored bins b0 .. b0 + nbc - 1 from the fields and
// their mix U: sources into cout, wm times the chunk's primary share into direct
hipError_t launch_gamma_adjoint_bins(int prec, const void* fields, const void* U, const void* delta, int n, int nbt,
                                     int b0, int nbc, const double (*m)[4], const double* wq, double wm, int nwg,
                                     int batch, void* cout, void* direct, hipStream_t st);
size_t gamma_adjoint_bins_lds_need(int prec, int nbc);

// grid summation with connection coefficients as a stencil over the shifts
// -halo .. halo per axis (stencil.hip): gamma(s, t) at g[s + 3][t + 3];
// halo 2 (Daubechies-4, support 3) or 3 (cubic B-spline, support 4)
struct StencilGamma {
  double g[7][7];
  int halo;
};
// partials over the pair's local bins, as launch_gamma_contract
hipError_t launch_stencil_contract(int prec, const void* fields, const void* delta, int n, const BinPair& bp,
                                   const StencilGamma& sg, double* partials, int nwg, int batch, hipStream_t st);
size_t stencil_lds_need(int prec, int halo, int nl);
// adjoint of stored bins b0 .. b0 + nbc - 1 from the fields and their mix U: sources
// into cout (per-bin layout), wm times the primary's share into direct
hipError_t launch_stencil_adjoint(int prec, const void* fields, const void* U, const void* delta, int n, int nbt,
                                  int b0, int nbc, const StencilGamma& sg, double wm, int nwg, int batch, void* cout,
                                  void* direct, hipStream_t st);
size_t stencil_adjoint_lds_need(int prec, int halo, int nbc);
hipError_t launch_zpass_store(int n, int prec, const ZpassArgs& a, void* out, hipStream_t st);
// counting sort of the particles by (2^shift)^3-cell tile of their mock; offs
// gets batch * (n >> shift)^3 + 1 exclusive tile offsets
hipError_t launch_tile_sort(const float* pos, const long long* off, int batch, long long np_total, int n, double sc,
                            int shift, int* counts, int* offs, int* cursor, int* perm, hipStream_t st);
// persistent tiled deposit over tiles of side tside (4, 8, 16) with at most
// wgs workgroups; toff from launch_tile_sort with shift log2(tside)
// btab: NULL for the cubic B-spline, else the Daubechies-4 table (kD4TableSize doubles)
hipError_t launch_deposit_tiled(int prec, int tside, const float* pos, const float* w, const int* perm, const int* toff,
                                int ntiles_total, int wgs, int* counter, int n, double sc, void* eps, const double* btab,
                                hipStream_t st);
hipError_t launch_gather_contract(int prec, const GatherArgs& a, hipStream_t st);
// per-|q|^2 histogram of |dhat|^2 Ahat (the basis autocorrelation's transform; times phi-hat^2
// when phi != NULL), Nyquist planes excluded
hipError_t launch_power_hist(int prec, const void* dhat, int n, int nq2, double* P, int batch, const void* phi,
                             const Acf& acf, hipStream_t st);
hipError_t launch_fbar_subtract(int prec, const double* P, const void* jtab, int nq2, int nbp, int nbins, int l, int lmax,
                                double n6, double* zeta, int batch, hipStream_t st);
hipError_t launch_fft3d(int n, int prec, int dir, bool real_in, const void* in, void* out, int nfields, const void* tw,
                        hipStream_t st);
hipError_t launch_fft_x(int n, int prec, int dir, void* buf, int nfields, const void* tw, int variant, hipStream_t st);
hipError_t launch_fft_y(int n, int prec, int dir, void* buf, int nfields, const void* tw, hipStream_t st);
hipError_t launch_fft_z(int n, int prec, int dir, const void* in, void* out, int nfields, const void* tw, hipStream_t st);
hipError_t launch_filter_y(int n, int prec, const FilterArgs& a, hipStream_t st);
hipError_t launch_adjoint_y(int n, int prec, const FilterArgs& a, hipStream_t st);
hipError_t launch_zpass_nodal(int n, int prec, const ZpassArgs& a, hipStream_t st);
hipError_t launch_zpass_adjoint(int n, int prec, const ZpassArgs& a, hipStream_t st);
// adjoint z pass that also writes the forward partials (value and gradient in one sweep), <= 32 bins
hipError_t launch_zpass_fused(int n, int prec, const ZpassArgs& a, hipStream_t st);
size_t zpass_lds_need(int n, int prec, int nbins);
// LDS bytes of the value-and-gradient z pass ((size_t)1 << 40 beyond 32 bins)
size_t zpass_fused_lds_need(int n, int prec, int nbins);
hipError_t launch_fill(int prec, void* p, long long count, double value, hipStream_t st);
hipError_t launch_fill_f64(double* p, long long count, double value, hipStream_t st);
hipError_t launch_fill_i32(int* p, long long count, int value, hipStream_t st);
// lam_s[l][batch][nbins^2] for every l <= lmax
hipError_t launch_lam_sym(int prec, const double* dzeta, void* lam_s, int nbins, int lmax, int batch, hipStream_t st);
// eigen-decomposition of every symmetrised cotangent (float64 Jacobi, nbins <= 64): eigenvalues
// lam_d[l][batch][nbins] at the plan precision, eigenvectors evec[l][batch][nbins][nbins] (columns)
hipError_t launch_lam_eig(int prec, const double* dzeta, void* lam_d, double* evec, int nbins, int lmax, int batch,
                          hipStream_t st);
// jrot[l][batch][nq2][nbp] = jtab[l][nq2][:] rotated by evec[l][batch]
hipError_t launch_rotate_jtab(int prec, const void* jtab, void* jrot, const double* evec, int nq2, int nbins, int nbp,
                              int lmax, int batch, hipStream_t st);
// zeta[batch][l] = evec zeta evec^T for every l (the value of the rotated fields back to the bins)
hipError_t launch_rotate_zeta(double* zeta, const double* evec, int nbins, int lmax, int batch, hipStream_t st);
// partials of a group of items [item][batch][nwg][nb2] into zeta at each item's l (times scale and the item's m weight)
hipError_t launch_reduce_items(const double* partials, int nwg, int nb2, double* zeta, int lmax, double scale,
                               const ItemRec* items, int item0, int nitems, int batch, hipStream_t st);
hipError_t launch_reduce_partials(const double* partials, int nwg, int nb2, double* zeta, int l, int lmax, double scale,
                                  int batch, hipStream_t st);
hipError_t launch_weight_sum(const float* w, const long long* off, int batch, long long np_max, double* W, hipStream_t st);
// out[j] = sum over mock j of w_i f_i (w NULL = unit weights)
hipError_t launch_weighted_sum(const float* w, const double* f, const long long* off, int batch, long long np_max,
                               double* out, hipStream_t st);
// particle-form adjoint: per-particle sources and F_J, their scatter onto the
// grid ([batch][nbins][N^3], every node written), the volume-mean term into G
// and the primary vertex's share of dJ/dw
hipError_t launch_gather_source(int prec, const void* fields, const int* tcell, const void* twt, const float* w,
                                const int* perm, const long long* off, const double* W, const void* lam_d, int n,
                                int nbins, double wm, int nwg, int batch, double* FJ, void* src, hipStream_t st);
hipError_t launch_scatter_source(int prec, const int* tcell, const void* twt, const int* toff, const void* src, int n,
                                 int nbins, int batch, void* out, hipStream_t st);
// per-particle stencil records in sorted order: packed cell (-1 if not
// finite) and 12 tap weights in the working precision
hipError_t launch_tap_records(int prec, const float* pos, const int* perm, long long np_total, int n, double sc,
                              int* tcell, void* twt, const double* btab, hipStream_t st);
hipError_t launch_fbar_adjoint(int prec, const double* dzeta, const void* jtab, int nq2, int nbp, int nbins, int lmax,
                               const void* dhat, int n, double scale, double* h, void* G, int batch, const void* phi,
                               const Acf& acf, hipStream_t st);
// grid-Gamma adjoint for one (l, m): adds the transposed-quadrature sources
// into cout ([batch][nbins][N^3], zeroed by the caller) and wm times the
// primary's share into direct; fields bin-interleaved, at most 20 bins.
// partials != NULL: also writes the forward contraction's partials
// ([batch][nwg][nbins^2], as launch_gamma_contract) from the same node values
hipError_t launch_gamma_adjoint(int prec, const void* fields, const void* delta, const void* lam_s, int n, int nbins,
                                const double (*m)[4], const double* wq, double wm, int nwg, int batch, void* cout,
                                void* direct, double* partials, hipStream_t st);
size_t gamma_adjoint_lds_need(int prec, int nbins);
hipError_t launch_primary_dw(int prec, const long long* off, int batch, long long np_total, const double* FJ,
                             const double* W, const double* SF, void* dw, hipStream_t st);
hipError_t launch_normalise(int prec, void* eps, const double* W, long long n3, int batch, hipStream_t st);
hipError_t launch_grad_combine(int prec, const void* direct, const void* ghat, void* ddelta, long long count, double scale,
                               hipStream_t st);
hipError_t launch_dot_rho_g(int prec, const void* delta, const void* g, long long n3, double* S, int batch, hipStream_t st);
hipError_t launch_gather_dw(int prec, const float* pos, const long long* off, int batch, long long np_total, int n,
                            double sc, const void* g, const double* W, const double* S, void* dw, const double* btab,
                            hipStream_t st);

// stats.hip: input validation, the top-hat filter of the primary vertex, xi and Q
// flag[0] += 1 when any of count values (float or double by prec) is NaN or infinite
hipError_t launch_count_nonfinite(int prec, const void* p, long long count, int* flag, hipStream_t st);
// X *= scale * W_TH(|k| R) in place over [batch][N^3] complex spectra, k = kf q
hipError_t launch_tophat_filter(int prec, void* X, int n, double kf, double R, double scale, int batch, hipStream_t st);
hipError_t launch_real_part(int prec, const void* in, void* out, long long count, hipStream_t st);
// per-|q|^2 histogram of |dhat|^2 (times phi-hat when phi != NULL), Nyquist planes excluded
hipError_t launch_power_plain(int prec, const void* dhat, int n, int nq2, double* P, int batch, const void* phi,
                              hipStream_t st);
// xi[batch][nr] at device radii from the histogram of launch_power_plain
hipError_t launch_xi(const double* P, int nq2, double kf, double R, bool prim_smooth, const double* radii, int nr,
                     double n6, double* xi, int batch, hipStream_t st);
// H[batch][lmx+1][nq2]: per-|q|^2 Legendre moments of |dhat|^2 along z (lmx <= 16)
hipError_t launch_power_multipoles(int prec, const void* dhat, int n, int nq2, int lmx, double* H, int batch,
                                  const void* phi, hipStream_t st);
// out[batch][lmx+1][nr]: line-of-sight multipoles of xi at device radii
hipError_t launch_xi_multipoles(const double* H, int nq2, int lmx, double kf, double R, bool prim_smooth,
                                const double* radii, int nr, double n6, double* out, int batch, hipStream_t st);
// f = delta_D - delta_R, r = 1 + delta_R over count values
hipError_t launch_ss_fields(int prec, const void* dd, const void* dr, void* f, void* r, long long count,
                            hipStream_t st);
// out[batch][lt+1][nbins][nbins]: Gauss-Legendre projection of N(mu) / R(mu) on P_l (lt <= 20)
hipError_t launch_ss_multipoles(const double* zn, const double* zr, int lmax, int lt, int nbins, const double* xq,
                                const double* wq, int nq, double* out, int batch, hipStream_t st);
// zt[batch][nbins][nbins][nth] = sum_{l <= lt} zeta_l P_l(mu) and, when q != NULL, the reduced 3PCF
hipError_t launch_reduced_3pcf(const double* zeta, int lmax, int lt, int nbins, const double* mu, int nth,
                               const double* rb, const double* xib, const double* P, int nq2, double kf, double R,
                               bool prim_smooth, double n6, double* zt, double* q, int batch, hipStream_t st);

}  // namespace mp3
