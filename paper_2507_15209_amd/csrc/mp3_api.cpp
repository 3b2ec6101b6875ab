// mp3_api.cpp -- the C ABI declared in include/mp3.h: plan, validation,
// workspace layout and the per-(l, m) launch sequence.
#include "mp3.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "tables.hpp"

struct mp3_plan_s {
  int n = 0, lmax = 0, nbins = 0, prec = 0, summation = 0, batch = 1;
  bool split = false;    // MP3_F32_BF16X3: float32 with BF16-split contraction inputs
  double box = 0.0;
  std::vector<double> edges;
  int nq2 = 0, nbp = 0;
  void* jtab = nullptr;  // [lmax+1][nq2][nbp] real, bin axis zero-padded to a multiple of 4
  void* tw = nullptr;    // [n] complex
  size_t elt = 4, celt = 8;
  int device = 0;
  double gm[5][4] = {{0}};   // grid-Gamma quadrature: B3 tap weights at the nodes
  double gw[5] = {0};        // and node weights
  int tune[MP3_NTUNE] = {4096, 4096, 0, 8, 2048, 0, 0, 0};   // launch-shape knobs (mp3_tune_knob)
  int basis = 0, binning = 0;
  unsigned kflags = 0;
  double smoothing = 0.0;   // top-hat radius of every vertex (0 = none)
  void* phi = nullptr;      // [n] real per-axis phi-hat factors when MP3_KF_PHI_HAT
  double* btab = nullptr;   // Daubechies-4 basis: phi at the dyadic points (NULL for the B-spline)
  mp3::Acf acf{{2416.0 / 5040.0, 1191.0 / 5040.0, 120.0 / 5040.0, 1.0 / 5040.0}};   // basis autocorrelation
  mp3::StencilGamma sgam{};  // Daubechies-4 connection coefficients (grid summation as a stencil)
  std::vector<mp3::ItemRec> items;   // every (l, m >= 0) of the plan, index l (l + 1) / 2 + m
  mp3::ItemRec* items_dev = nullptr; // the same table on the device
  // optional per-pass HIP event timing
  bool profile = false;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  struct Rec { int pass; hipEvent_t a, b; };
  std::vector<Rec> recs;
  double prof_ms[MP3_NPASS] = {0};
  long long prof_n[MP3_NPASS] = {0};
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(MP3_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define MP3_HIP(call, where)                       \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

constexpr double kFourPi = 12.566370614359172953850573533118011536788677597500;
constexpr size_t kLdsLimit = 160 * 1024;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t dprim, flag, pplain, aux, xib, fields_u, counter;
  size_t evec, jrot;   // nodal gradient: the cotangents' eigenvectors and the rotated radial tables
  int group;   // (l, m) items per launch of the one-sweep nodal passes
  size_t off, W, S, dhat, fields, partials, G, direct, lam, fields_i, perm, counts, offs, cursor, power;
  size_t src, fj, hq, SF, tcell, twt;
  size_t dperm, dcounts, doffs, dcursor, dcounter, total;
  int nwg, ppw;
};

constexpr int kGatherSlice = 256;
constexpr int kMaxAux = 4096;   // radii of mp3_xi, angles of mp3_reduced_3pcf

// workgroups per mock of the particle gather: at least four slices each
int gather_wgs(const mp3_plan_s* p, long long np_max) {
  long long g = (np_max + 4LL * kGatherSlice - 1) / (4LL * kGatherSlice);
  long long cap = p->tune[MP3_TUNE_CONTRACT_WGS] / p->batch;
  if (cap < 1) cap = 1;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

// workgroups per mock of the grid-Gamma contraction and the gather partials
size_t contract_wgs(const mp3_plan_s* p) {
  const int g = p->tune[MP3_TUNE_CONTRACT_WGS] / p->batch;
  return (size_t)(g > 1 ? g : 1);
}

size_t deposit_tiles(const mp3_plan_s* p) {
  const size_t t = (size_t)(p->n / p->tune[MP3_TUNE_DEPOSIT_TILE]);
  return t * t * t * (size_t)p->batch;
}

int tile_shift(int side) { return side == 4 ? 2 : (side == 8 ? 3 : 4); }

// (l, m) items per launch of the one-sweep nodal passes: the knob, or (0)
// as many as fit a 1 GiB field budget, at least one
constexpr double kGroupBudget = 1073741824.0;

int item_group(const mp3_plan_s* p) {
  const int total = (int)p->items.size();
  if (p->summation != MP3_SUM_NODAL) return 1;
  int g = p->tune[MP3_TUNE_ITEM_GROUP];
  if (g <= 0) {
    const double set = (double)p->batch * p->nbins * p->n * (double)p->n * p->n * (double)p->celt;
    g = (int)(kGroupBudget / set);
  }
  if (g < 1) g = 1;
  return g < total ? g : total;
}

// the grid-Gamma adjoint as the shift stencil (Daubechies-4 always; the
// B-spline unless the node-quadrature kernel is selected)
bool gamma_stencil_adjoint(const mp3_plan_s* p) {
  return p->basis == MP3_BASIS_DAUBECHIES4 || p->tune[MP3_TUNE_GAMMA_ADJOINT] == 0;
}

Layout layout(const mp3_plan_s* p, long long np_total = 0) {
  Layout L{};
  L.group = item_group(p);
  const size_t n3 = (size_t)p->n * p->n * p->n;
  const size_t B = (size_t)p->batch;
  const size_t nb2 = (size_t)p->nbins * p->nbins;
  const long long pencils = (long long)p->n * p->n;
  long long nwg = p->tune[MP3_TUNE_ZPASS_WGS] / p->batch;
  if (nwg < 1) nwg = 1;
  if (nwg > pencils) nwg = pencils;
  L.ppw = (int)((pencils + nwg - 1) / nwg);
  L.nwg = (int)((pencils + L.ppw - 1) / L.ppw);
  // partial sums: one per workgroup of the z pass or of the particle gather
  size_t pw = (size_t)L.nwg;
  const size_t gw = contract_wgs(p);
  if (p->summation != MP3_SUM_NODAL && gw > pw) pw = gw;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  L.off = take((B + 1) * sizeof(long long));
  L.W = take(B * sizeof(double));
  L.S = take(B * sizeof(double));
  L.dhat = take(B * n3 * p->celt);
  L.fields = take((size_t)L.group * B * (size_t)p->nbins * n3 * p->celt);
  L.partials = take((size_t)L.group * B * pw * nb2 * sizeof(double));
  L.G = take(B * n3 * p->celt);
  L.direct = take(B * n3 * p->elt);
  L.lam = take((size_t)(p->lmax + 1) * B * nb2 * p->elt);
  L.counter = take(sizeof(int));
  if (p->summation == MP3_SUM_NODAL || p->summation == MP3_SUM_PARTICLE) {
    L.evec = take((size_t)(p->lmax + 1) * B * nb2 * sizeof(double));
    L.jrot = take((size_t)(p->lmax + 1) * B * (size_t)p->nq2 * p->nbp * p->elt);
  }
  // primary vertex filtered by the top-hat window (grid forms with smoothing)
  if (p->smoothing > 0.0 && p->summation != MP3_SUM_PARTICLE) L.dprim = take(B * n3 * p->elt);
  L.flag = take(sizeof(int));
  // plain power histogram, radii / cosines of mp3_xi and mp3_reduced_3pcf, xi at the bins
  L.pplain = take(B * (size_t)mp3::nq2_count(p->n) * sizeof(double));
  L.aux = take((size_t)2 * kMaxAux * sizeof(double));
  L.xib = take(B * (size_t)p->nbins * sizeof(double));
  if (p->summation != MP3_SUM_NODAL) L.fields_i = take(B * (size_t)p->nbins * n3 * p->celt);
  // grid-Gamma adjoint by bin chunks: the bin mix U of the fields
  if (p->summation == MP3_SUM_GRID_GAMMA &&
      (gamma_stencil_adjoint(p) || mp3::gamma_adjoint_lds_need(p->prec, p->nbins) > kLdsLimit))
    L.fields_u = take(B * (size_t)p->nbins * n3 * p->celt);
  if (p->summation == MP3_SUM_PARTICLE) {
    const size_t nt = (size_t)(p->n / 4) * (p->n / 4) * (p->n / 4) * B + 1;
    L.perm = take((size_t)(np_total > 0 ? np_total : 1) * sizeof(int));
    L.counts = take(nt * sizeof(int));
    L.offs = take(nt * sizeof(int));
    L.cursor = take(nt * sizeof(int));
    L.power = take(B * (size_t)mp3::nq2_count(p->n) * sizeof(double));
    // adjoint: per-particle sources (sorted order, all bins), F_J, the
    // volume-mean weights per |q|^2 and sum_i w_i F_J(u_i)
    const size_t npt = (size_t)(np_total > 0 ? np_total : 1);
    L.src = take(npt * (size_t)p->nbins * p->celt);
    L.fj = take(npt * sizeof(double));
    L.hq = take(B * (size_t)mp3::nq2_count(p->n) * sizeof(double));
    L.SF = take(B * sizeof(double));
    L.tcell = take(npt * sizeof(int));
    L.twt = take(npt * 12 * p->elt);
  }
  // tiled deposit, last so that the offsets above do not depend on the
  // number of particles of the nodal and grid forms
  const size_t ntd = deposit_tiles(p) + 1;
  L.dperm = take((size_t)(np_total > 0 ? np_total : 1) * sizeof(int));
  L.dcounts = take(ntd * sizeof(int));
  L.doffs = take(ntd * sizeof(int));
  L.dcursor = take(ntd * sizeof(int));
  L.dcounter = take(sizeof(int));
  L.total = o;
  return L;
}

bool pow2_supported(int n) { return n == 16 || n == 32 || n == 64 || n == 128 || n == 256 || n == 512; }

constexpr unsigned kKnownFlags = MP3_KF_PHI_HAT | MP3_KF_CHECK_FINITE;

// checks shared by mp3_plan_create and mp3_window_table
int validate_desc(const mp3_plan_desc* d) {
  if (!pow2_supported(d->n)) return fail(MP3_EUNSUPPORTED, "n must be one of 16, 32, 64, 128, 256, 512");
  if (!std::isfinite(d->box)) return fail(MP3_ENONFINITE, "box is not finite");
  if (!(d->box > 0.0)) return fail(MP3_EINVAL, "box must be positive");
  if (d->lmax < 0 || d->lmax > 20) return fail(MP3_EINVAL, "lmax must be in [0, 20]");
  if (d->nbins < 1 || d->nbins > 64) return fail(MP3_EINVAL, "nbins must be in [1, 64]");
  if (!d->edges) return fail(MP3_EINVAL, "edges is NULL");
  for (int b = 0; b <= d->nbins; ++b) {
    if (!std::isfinite(d->edges[b])) return fail(MP3_ENONFINITE, "edges must be finite");
    if (d->edges[b] < 0.0) return fail(MP3_EINVAL, "edges must be >= 0");
    if (b > 0 && !(d->edges[b] > d->edges[b - 1])) return fail(MP3_EINVAL, "edges must increase strictly");
  }
  if (d->precision != MP3_F32 && d->precision != MP3_F64 && d->precision != MP3_F32_BF16X3)
    return fail(MP3_EINVAL, "precision must be MP3_F32, MP3_F64 or MP3_F32_BF16X3");
  if (d->summation != MP3_SUM_NODAL && d->summation != MP3_SUM_PARTICLE && d->summation != MP3_SUM_GRID_GAMMA)
    return fail(MP3_EUNSUPPORTED, "summation form not supported");
  if (d->batch < 1) return fail(MP3_EINVAL, "batch must be >= 1");
  if (d->basis != MP3_BASIS_BSPLINE3 && d->basis != MP3_BASIS_DAUBECHIES4)
    return fail(MP3_EINVAL, "basis must be MP3_BASIS_BSPLINE3 or MP3_BASIS_DAUBECHIES4");
  if (d->basis == MP3_BASIS_DAUBECHIES4 && d->summation == MP3_SUM_GRID_GAMMA && d->precision == MP3_F32_BF16X3)
    return fail(MP3_EUNSUPPORTED, "BF16-split inputs: cubic B-spline grid summation only");
  if (d->kflags & ~kKnownFlags) return fail(MP3_EINVAL, "unknown kflags bits");
  if (d->binning != MP3_BIN_SHELL_AVERAGE && d->binning != MP3_BIN_THIN_SHELL)
    return fail(MP3_EINVAL, "binning must be MP3_BIN_SHELL_AVERAGE or MP3_BIN_THIN_SHELL");
  if (!std::isfinite(d->smoothing)) return fail(MP3_ENONFINITE, "smoothing is not finite");
  if (d->smoothing < 0.0) return fail(MP3_EINVAL, "smoothing must be >= 0");
  return MP3_OK;
}

// with MP3_KF_CHECK_FINITE: count non-finite values on the device and wait
// for the answer (the call blocks); ptrs/counts/precisions of up to 3 arrays
int check_finite(const mp3_plan_s* p, void* ws, size_t flag_off, hipStream_t st, const void* a, long long na, int pa,
                 const void* b = nullptr, long long nb = 0, int pb = 0) {
  if (!(p->kflags & MP3_KF_CHECK_FINITE)) return MP3_OK;
  int* flag = reinterpret_cast<int*>(static_cast<char*>(ws) + flag_off);
  MP3_HIP(mp3::launch_fill_i32(flag, 1, 0, st), "zero flag");
  if (a) MP3_HIP(mp3::launch_count_nonfinite(pa, a, na, flag, st), "finite check");
  if (b) MP3_HIP(mp3::launch_count_nonfinite(pb, b, nb, flag, st), "finite check");
  int h = 0;
  MP3_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st), "read flag");
  MP3_HIP(hipStreamSynchronize(st), "wait for the finite check");
  if (h) return fail(MP3_ENONFINITE, "a NaN or infinity in the input");
  return MP3_OK;
}

int check_plan(const mp3_plan_s* p) {
  if (!p) return fail(MP3_EINVAL, "plan is NULL");
  return MP3_OK;
}

int check_ws(const mp3_plan_s* p, void* ws, size_t wsb, size_t need) {
  (void)p;
  if (!ws) return fail(MP3_EWORKSPACE, "workspace is NULL");
  if (wsb < need)
    return fail(MP3_EWORKSPACE, "workspace too small: " + std::to_string(wsb) + " < " + std::to_string(need) + " bytes");
  return MP3_OK;
}

int check_offsets(const mp3_plan_s* p, const int64_t* np_off, long long* np_total, long long* np_max) {
  if (!np_off) return fail(MP3_EINVAL, "np_off is NULL");
  if (np_off[0] != 0) return fail(MP3_EINVAL, "np_off[0] must be 0");
  long long mx = 0;
  for (int j = 0; j < p->batch; ++j) {
    const long long c = np_off[j + 1] - np_off[j];
    if (c <= 0) return fail(MP3_EINVAL, "mock " + std::to_string(j) + " has no particles (np_off must increase strictly)");
    if (c > mx) mx = c;
  }
  *np_total = np_off[p->batch];
  *np_max = mx;
  return MP3_OK;
}

char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

hipEvent_t next_event(mp3_plan_s* p) {
  if (p->pool_used == p->pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->pool.push_back(e);
  }
  return p->pool[p->pool_used++];
}

// Launch f() on stream st; with profiling on, bracket it by two events
// attributed to the given pass.
template <typename Fn>
hipError_t timed(const mp3_plan_s* cp, int pass, hipStream_t st, Fn f) {
  mp3_plan_s* p = const_cast<mp3_plan_s*>(cp);
  if (!p->profile) return f();
  hipEvent_t a = next_event(p), b = next_event(p);
  if (!a || !b) return f();
  hipEventRecord(a, st);
  hipError_t e = f();
  hipEventRecord(b, st);
  p->recs.push_back({pass, a, b});
  return e;
}

void collect_profile(mp3_plan_s* p) {
  for (auto& r : p->recs) {
    hipEventSynchronize(r.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      p->prof_ms[r.pass] += ms;
      p->prof_n[r.pass] += 1;
    }
  }
  p->recs.clear();
  p->pool_used = 0;
}

int upload_offsets(const mp3_plan_s* p, const int64_t* np_off, void* ws, const Layout& L, hipStream_t st) {
  MP3_HIP(hipMemcpyAsync(at(ws, L.off), np_off, (p->batch + 1) * sizeof(long long), hipMemcpyHostToDevice, st),
          "copy np_off");
  return MP3_OK;
}

// delta -> dhat (forward DFT, unnormalised)
int forward_dft(const mp3_plan_s* p, const void* delta, void* ws, const Layout& L, hipStream_t st) {
  MP3_HIP(timed(p, MP3_PASS_DFT, st, [&] { return mp3::launch_fft3d(p->n, p->prec, -1, true, delta, at(ws, L.dhat), p->batch, p->tw, st); }), "forward FFT");
  return MP3_OK;
}

int item_index(int l, int m) { return l * (l + 1) / 2 + m; }

// the symmetrised cotangent of multipole l: [batch][nbins^2] real
void* lam_at(const mp3_plan_s* p, void* ws, const Layout& L, int l) {
  return at(ws, L.lam + (size_t)l * p->batch * p->nbins * p->nbins * p->elt);
}

// the cotangent's eigenvalues of multipole l after lam_eig_all: [batch][nbins] real
void* lam_d_at(const mp3_plan_s* p, void* ws, const Layout& L, int l) {
  return at(ws, L.lam + (size_t)l * p->batch * p->nbins * p->elt);
}

// symmetrised cotangents of every l into the workspace (one launch)
int lam_all(const mp3_plan_s* p, const double* dzeta, void* ws, const Layout& L, hipStream_t st) {
  MP3_HIP(mp3::launch_lam_sym(p->prec, dzeta, at(ws, L.lam), p->nbins, p->lmax, p->batch, st), "lambda");
  return MP3_OK;
}

// The nodal gradient runs in the eigenbasis of each symmetrised cotangent
// lam_s = V diag(d) V^T (per l and mock): the eigenvalues d into the lambda
// slot, V into L.evec, and the radial tables rotated by V into L.jrot.
int lam_eig_all(const mp3_plan_s* p, const double* dzeta, void* ws, const Layout& L, hipStream_t st) {
  double* evec = reinterpret_cast<double*>(at(ws, L.evec));
  MP3_HIP(mp3::launch_lam_eig(p->prec, dzeta, at(ws, L.lam), evec, p->nbins, p->lmax, p->batch, st),
          "cotangent eigenbasis");
  MP3_HIP(mp3::launch_rotate_jtab(p->prec, p->jtab, at(ws, L.jrot), evec, p->nq2, p->nbins, p->nbp, p->lmax,
                                  p->batch, st),
          "rotated radial tables");
  return MP3_OK;
}

// rotated: the radial tables of the cotangents' eigenbasis (lam_eig_all), one per (l, mock)
mp3::FilterArgs filter_args(const mp3_plan_s* p, void* ws, const Layout& L, const void* src, void* dst, int item0,
                            int nitems, bool rotated = false) {
  mp3::FilterArgs a;
  a.src = src;
  a.dst = dst;
  a.jtab = rotated ? at(ws, L.jrot) : p->jtab;
  a.jmocks = rotated ? p->batch : 1;
  a.tw = p->tw;
  a.nq2 = p->nq2;
  a.nbp = p->nbp;
  a.nbins = p->nbins;
  a.batch = p->batch;
  a.items = p->items_dev;
  a.item0 = item0;
  a.nitems = nitems;
  a.scale = 1.0 / ((double)p->n * p->n * p->n);
  a.phi = p->phi;
  return a;
}

// arguments of the adjoint z passes over a group of items
mp3::ZpassArgs adjoint_zargs(const mp3_plan_s* p, void* ws, const Layout& L, void* F, const void* prim,
                             const double* dzeta, void* direct, int item0, int nitems) {
  mp3::ZpassArgs z{};
  z.fields = F;
  z.delta = prim;
  z.dzeta = dzeta;
  z.lam = at(ws, L.lam);
  z.direct = direct;
  z.tw = p->tw;
  z.nbins = p->nbins;
  z.nwg = L.nwg;
  z.ppw = L.ppw;
  z.batch = p->batch;
  z.lmax = p->lmax;
  z.items = p->items_dev;
  z.item0 = item0;
  z.nitems = nitems;
  z.counter = reinterpret_cast<int*>(at(ws, L.counter));
  return z;
}

// fields of a group of items after the y and x passes: layout [item][batch][nbins][x][y][qz]
int fields_xy(const mp3_plan_s* p, void* ws, const Layout& L, void* dst, int item0, int nitems, hipStream_t st,
              bool rotated = false) {
  mp3::FilterArgs a = filter_args(p, ws, L, at(ws, L.dhat), dst, item0, nitems, rotated);
  MP3_HIP(timed(p, MP3_PASS_FILTER, st, [&] { return mp3::launch_filter_y(p->n, p->prec, a, st); }), "window pass");
  MP3_HIP(timed(p, MP3_PASS_X, st, [&] { return mp3::launch_fft_x(p->n, p->prec, +1, dst, nitems * p->batch * p->nbins, p->tw, p->tune[MP3_TUNE_FFT_X_PLAN], st); }), "x pass");
  return MP3_OK;
}

// The grid forms' primary vertex: delta itself, or with a smoothing radius
// delta_p = IFFT[ W_TH(kR) FFT(delta) ] (dhat must be current), stored in the
// workspace; the fields buffer serves as scratch.
const void* primary_field(const mp3_plan_s* p, const void* delta, void* ws, const Layout& L, hipStream_t st,
                          int* status) {
  *status = MP3_OK;
  if (!(p->smoothing > 0.0) || p->summation == MP3_SUM_PARTICLE) return delta;
  const long long n3 = (long long)p->n * p->n * p->n;
  void* tmp = at(ws, L.fields);
  hipError_t e = hipMemcpyAsync(tmp, at(ws, L.dhat), (size_t)p->batch * n3 * p->celt, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = mp3::launch_tophat_filter(p->prec, tmp, p->n, 2.0 * M_PI / p->box, p->smoothing, 1.0 / (double)n3, p->batch, st);
  if (e == hipSuccess) e = mp3::launch_fft3d(p->n, p->prec, +1, false, tmp, tmp, p->batch, p->tw, st);
  if (e == hipSuccess) e = mp3::launch_real_part(p->prec, tmp, at(ws, L.dprim), n3 * p->batch, st);
  if (e != hipSuccess) {
    *status = hip_fail(e, "primary top-hat filter");
    return nullptr;
  }
  return at(ws, L.dprim);
}

// the transpose of primary_field applied to the primary's gradient share
// (the filter is real and even, so it is its own transpose), in place
int filter_direct(const mp3_plan_s* p, void* direct, void* ws, const Layout& L, hipStream_t st) {
  if (!(p->smoothing > 0.0) || p->summation == MP3_SUM_PARTICLE) return MP3_OK;
  const long long n3 = (long long)p->n * p->n * p->n;
  void* tmp = at(ws, L.fields);
  MP3_HIP(mp3::launch_fft3d(p->n, p->prec, -1, true, direct, tmp, p->batch, p->tw, st), "transpose filter: DFT");
  MP3_HIP(mp3::launch_tophat_filter(p->prec, tmp, p->n, 2.0 * M_PI / p->box, p->smoothing, 1.0 / (double)n3, p->batch,
                                    st),
          "transpose filter");
  MP3_HIP(mp3::launch_fft3d(p->n, p->prec, +1, false, tmp, tmp, p->batch, p->tw, st), "transpose filter: inverse DFT");
  MP3_HIP(mp3::launch_real_part(p->prec, tmp, direct, n3 * p->batch, st), "transpose filter: real part");
  return MP3_OK;
}

}  // namespace

namespace mp3 {
// the last-error message of the calling thread, for entry points defined in other sources
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace mp3

extern "C" {

const char* mp3_status_string(int s) {
  switch (s) {
    case MP3_OK: return "MP3_OK";
    case MP3_EINVAL: return "MP3_EINVAL";
    case MP3_ENOMEM: return "MP3_ENOMEM";
    case MP3_EHIP: return "MP3_EHIP";
    case MP3_EUNSUPPORTED: return "MP3_EUNSUPPORTED";
    case MP3_EWORKSPACE: return "MP3_EWORKSPACE";
    case MP3_ENONFINITE: return "MP3_ENONFINITE";
    default: return "MP3_UNKNOWN";
  }
}

const char* mp3_last_error(void) { return g_last_error.c_str(); }

int mp3_plan_create(const mp3_plan_desc* d, mp3_plan_t* out) {
  if (!d || !out) return fail(MP3_EINVAL, "desc and out must not be NULL");
  if (int s = validate_desc(d)) return s;
  const int storage = d->precision == MP3_F64 ? 1 : 0;
  (void)storage;
  // the nodal z passes hold every bin of a pencil in LDS (the other forms'
  // store pass takes the bins in chunks)
  if (d->summation == MP3_SUM_NODAL && mp3::zpass_lds_need(d->n, storage, d->nbins) > kLdsLimit)
    return fail(MP3_EUNSUPPORTED, "n * nbins too large for the nodal z pass's LDS at this precision");

  mp3_plan_s* p = new (std::nothrow) mp3_plan_s;
  if (!p) return fail(MP3_ENOMEM, "host allocation failed");
  p->n = d->n;
  p->box = d->box;
  p->lmax = d->lmax;
  p->nbins = d->nbins;
  p->prec = storage;
  p->split = d->precision == MP3_F32_BF16X3;
  p->summation = d->summation;
  p->batch = d->batch;
  p->basis = d->basis;
  p->binning = d->binning;
  p->kflags = d->kflags;
  p->smoothing = d->smoothing;
  p->edges.assign(d->edges, d->edges + d->nbins + 1);
  p->nq2 = mp3::nq2_count(p->n);
  p->nbp = (p->nbins + 3) / 4 * 4;
  mp3::gamma_quadrature(p->gm, p->gw);
  p->elt = p->prec ? sizeof(double) : sizeof(float);
  p->celt = 2 * p->elt;
  hipGetDevice(&p->device);

  std::vector<double> jt;
  mp3::jbar_table(p->n, p->box, p->lmax, p->edges, jt, p->binning, p->smoothing);
  std::vector<double> twr, twi;
  mp3::twiddles(p->n, twr, twi);
  const size_t rows = (size_t)(p->lmax + 1) * p->nq2;
  std::vector<char> hj(rows * p->nbp * p->elt, 0), ht((size_t)p->n * p->celt);
  for (size_t rw = 0; rw < rows; ++rw) {
    for (int b = 0; b < p->nbins; ++b) {
      const double v = jt[rw * p->nbins + b];
      const size_t i = rw * p->nbp + b;
      if (p->prec) reinterpret_cast<double*>(hj.data())[i] = v;
      else reinterpret_cast<float*>(hj.data())[i] = (float)v;
    }
  }
  for (int i = 0; i < p->n; ++i) {
    if (p->prec) {
      reinterpret_cast<double*>(ht.data())[2 * i] = twr[i];
      reinterpret_cast<double*>(ht.data())[2 * i + 1] = twi[i];
    } else {
      reinterpret_cast<float*>(ht.data())[2 * i] = (float)twr[i];
      reinterpret_cast<float*>(ht.data())[2 * i + 1] = (float)twi[i];
    }
  }
  if (hipMalloc(&p->jtab, hj.size()) != hipSuccess || hipMalloc(&p->tw, ht.size()) != hipSuccess) {
    if (p->jtab) hipFree(p->jtab);
    if (p->tw) hipFree(p->tw);
    delete p;
    (void)hipGetLastError();
    return fail(MP3_ENOMEM, "device allocation of the plan tables failed");
  }
  hipError_t e1 = hipMemcpy(p->jtab, hj.data(), hj.size(), hipMemcpyHostToDevice);
  hipError_t e2 = hipMemcpy(p->tw, ht.data(), ht.size(), hipMemcpyHostToDevice);
  hipError_t e3 = hipSuccess;
  for (int l = 0; l <= p->lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      mp3::ItemRec it{};
      it.l = l;
      it.m = m;
      it.norm = mp3::ylm_norm(l, m);
      it.wm = m == 0 ? 1.0 : 2.0;
      it.yr.pmm = 1.0;
      for (int k = 1; k <= m; ++k) it.yr.pmm *= -(2.0 * k - 1.0);
      for (int k = 0; k < 21; ++k) {
        it.yr.c1[k] = k >= m + 2 ? (2.0 * k - 1.0) / (double)(k - m) : 0.0;
        it.yr.c2[k] = k >= m + 2 ? (k + m - 1.0) / (double)(k - m) : 0.0;
      }
      p->items.push_back(it);
    }
  }
  const size_t ib = p->items.size() * sizeof(mp3::ItemRec);
  if (p->basis == MP3_BASIS_BSPLINE3) {
    mp3::b3_gamma(p->sgam.g);
    p->sgam.halo = 3;
  }
  hipError_t e4 = hipMalloc(&p->items_dev, ib);
  if (e4 == hipSuccess) e4 = hipMemcpy(p->items_dev, p->items.data(), ib, hipMemcpyHostToDevice);
  if (p->basis == MP3_BASIS_DAUBECHIES4 && e4 == hipSuccess) {
    std::vector<double> tab;
    mp3::d4_table(mp3::kD4Level, tab);
    mp3::d4_autocorr(tab, mp3::kD4Level, p->acf.a);
    double g5[5][5];
    mp3::d4_gamma(g5);
    for (int s = 0; s < 5; ++s)
      for (int t = 0; t < 5; ++t) p->sgam.g[s + 1][t + 1] = g5[s][t];
    p->sgam.halo = 2;
    e4 = hipMalloc(&p->btab, tab.size() * sizeof(double));
    if (e4 == hipSuccess) e4 = hipMemcpy(p->btab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
  }
  if (p->kflags & MP3_KF_PHI_HAT) {
    std::vector<double> ph;
    if (p->basis == MP3_BASIS_DAUBECHIES4) mp3::d4_phi_hat_axis(p->n, ph);
    else mp3::phi_hat_axis(p->n, ph);
    std::vector<char> hp((size_t)p->n * p->elt);
    for (int i = 0; i < p->n; ++i) {
      if (p->prec) reinterpret_cast<double*>(hp.data())[i] = ph[i];
      else reinterpret_cast<float*>(hp.data())[i] = (float)ph[i];
    }
    e3 = hipMalloc(&p->phi, hp.size());
    if (e3 == hipSuccess) e3 = hipMemcpy(p->phi, hp.data(), hp.size(), hipMemcpyHostToDevice);
  }
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
    hipFree(p->jtab);
    hipFree(p->tw);
    if (p->phi) hipFree(p->phi);
    if (p->items_dev) hipFree(p->items_dev);
    if (p->btab) hipFree(p->btab);
    delete p;
    const hipError_t e = e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : (e3 != hipSuccess ? e3 : e4));
    return hip_fail(e, "upload plan tables");
  }
  *out = p;
  return MP3_OK;
}

int mp3_profile(mp3_plan_t p, int enable) {
  if (int s = check_plan(p)) return s;
  collect_profile(p);
  for (int i = 0; i < MP3_NPASS; ++i) {
    p->prof_ms[i] = 0.0;
    p->prof_n[i] = 0;
  }
  p->profile = enable != 0;
  return MP3_OK;
}

int mp3_profile_read(mp3_plan_t p, int pass, double* total_ms, int64_t* launches) {
  if (int s = check_plan(p)) return s;
  if (pass < 0 || pass >= MP3_NPASS) return fail(MP3_EINVAL, "pass id out of range");
  collect_profile(p);
  if (total_ms) *total_ms = p->prof_ms[pass];
  if (launches) *launches = p->prof_n[pass];
  return MP3_OK;
}

int mp3_plan_destroy(mp3_plan_t p) {
  if (!p) return MP3_OK;
  collect_profile(p);
  for (hipEvent_t e : p->pool) hipEventDestroy(e);
  if (p->jtab) hipFree(p->jtab);
  if (p->tw) hipFree(p->tw);
  if (p->phi) hipFree(p->phi);
  if (p->items_dev) hipFree(p->items_dev);
  if (p->btab) hipFree(p->btab);
  delete p;
  return MP3_OK;
}

int mp3_tune_set(mp3_plan_t p, int knob, int32_t value) {
  if (int s = check_plan(p)) return s;
  switch (knob) {
    case MP3_TUNE_ZPASS_WGS:
    case MP3_TUNE_CONTRACT_WGS:
    case MP3_TUNE_DEPOSIT_WGS:
      if (value < 64 || value > 65536) return fail(MP3_EINVAL, "workgroup count must lie in 64 .. 65536");
      break;
    case MP3_TUNE_FFT_X_PLAN:
      if (value != 0 && value != 1) return fail(MP3_EINVAL, "x-pass radix plan must be 0 or 1");
      break;
    case MP3_TUNE_DEPOSIT_TILE:
      if (value != 4 && value != 8 && value != 16) return fail(MP3_EINVAL, "deposit tile side must be 4, 8 or 16");
      break;
    case MP3_TUNE_FUSED_WAVES:
      if (value < 0 || value > 8) return fail(MP3_EINVAL, "one-sweep z-pass waves must lie in 0 .. 8");
      break;
    case MP3_TUNE_ITEM_GROUP:
      if (value < 0 || value > 1024) return fail(MP3_EINVAL, "items per nodal adjoint launch must lie in 0 .. 1024");
      break;
    case MP3_TUNE_GAMMA_ADJOINT:
      if (value != 0 && value != 1) return fail(MP3_EINVAL, "grid-Gamma adjoint kernel must be 0 or 1");
      break;
    default:
      return fail(MP3_EINVAL, "unknown tuning knob");
  }
  p->tune[knob] = value;
  return MP3_OK;
}

int mp3_tune_get(mp3_plan_t p, int knob, int32_t* value) {
  if (int s = check_plan(p)) return s;
  if (knob < 0 || knob >= MP3_NTUNE) return fail(MP3_EINVAL, "unknown tuning knob");
  if (!value) return fail(MP3_EINVAL, "value must not be NULL");
  *value = p->tune[knob];
  return MP3_OK;
}

int mp3_plan_info(mp3_plan_t p, int32_t* n, int32_t* lmax, int32_t* nbins, int32_t* precision, int32_t* batch) {
  if (int s = check_plan(p)) return s;
  if (n) *n = p->n;
  if (lmax) *lmax = p->lmax;
  if (nbins) *nbins = p->nbins;
  if (precision) *precision = p->split ? MP3_F32_BF16X3 : p->prec;
  if (batch) *batch = p->batch;
  return MP3_OK;
}

int mp3_workspace_size(mp3_plan_t p, int64_t np_total, size_t* bytes) {
  if (int s = check_plan(p)) return s;
  if (!bytes) return fail(MP3_EINVAL, "bytes is NULL");
  if (np_total < 0) return fail(MP3_EINVAL, "np_total must be >= 0");
  *bytes = layout(p, np_total).total;
  return MP3_OK;
}

int mp3_deposit(mp3_plan_t p, const float* pos, const float* w, const int64_t* np_off, void* delta, void* ws,
                size_t wsb, void* stream) {
  if (int s = check_plan(p)) return s;
  long long np_total = 0, np_max = 0;
  if (int s = check_offsets(p, np_off, &np_total, &np_max)) return s;
  if (!pos) return fail(MP3_EINVAL, "pos is NULL");
  if (!delta) return fail(MP3_EINVAL, "delta is NULL");
  const Layout L = layout(p, np_total);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n3 = (long long)p->n * p->n * p->n;
  if (np_total >= (1LL << 31)) return fail(MP3_EUNSUPPORTED, "more than 2^31 - 1 particles");
  if (int s = check_finite(p, ws, L.flag, st, pos, 3 * np_total, 0, w, w ? np_total : 0, 0)) return s;
  if (int s = upload_offsets(p, np_off, ws, L, st)) return s;
  const long long* off = reinterpret_cast<const long long*>(at(ws, L.off));
  double* W = reinterpret_cast<double*>(at(ws, L.W));
  MP3_HIP(mp3::launch_fill_f64(W, p->batch, 0.0, st), "zero W");
  MP3_HIP(mp3::launch_weight_sum(w, off, p->batch, np_max, W, st), "weight sum");
  MP3_HIP(mp3::launch_fill(p->prec, delta, n3 * p->batch, 0.0, st), "zero grid");
  const double sc = (double)p->n / p->box;
  int* dperm = reinterpret_cast<int*>(at(ws, L.dperm));
  int* doffs = reinterpret_cast<int*>(at(ws, L.doffs));
  const int ntiles = (int)deposit_tiles(p);
  const int tside = p->tune[MP3_TUNE_DEPOSIT_TILE];
  MP3_HIP(timed(p, MP3_PASS_DEPOSIT, st, [&] {
            hipError_t e = mp3::launch_tile_sort(pos, off, p->batch, np_total, p->n, sc, tile_shift(tside),
                                                 reinterpret_cast<int*>(at(ws, L.dcounts)), doffs,
                                                 reinterpret_cast<int*>(at(ws, L.dcursor)), dperm, st);
            if (e != hipSuccess) return e;
            return mp3::launch_deposit_tiled(p->prec, tside, pos, w, dperm, doffs, ntiles, p->tune[MP3_TUNE_DEPOSIT_WGS],
                                             reinterpret_cast<int*>(at(ws, L.dcounter)), p->n, sc, delta, p->btab, st);
          }),
          "deposit");
  MP3_HIP(mp3::launch_normalise(p->prec, delta, W, n3, p->batch, st), "normalise");
  return MP3_OK;
}

int mp3_multipole_fields(mp3_plan_t p, const void* delta, int32_t l, int32_t m, void* a_out, void* ws, size_t wsb,
                         void* stream) {
  if (int s = check_plan(p)) return s;
  if (!delta || !a_out) return fail(MP3_EINVAL, "delta and a_out must not be NULL");
  if (l < 0 || l > p->lmax || m < 0 || m > l) return fail(MP3_EINVAL, "need 0 <= m <= l <= lmax");
  const Layout L = layout(p);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int s = forward_dft(p, delta, ws, L, st)) return s;
  if (int s = fields_xy(p, ws, L, a_out, item_index(l, m), 1, st)) return s;
  MP3_HIP(mp3::launch_fft_z(p->n, p->prec, +1, a_out, a_out, p->batch * p->nbins, p->tw, st), "z pass");
  return MP3_OK;
}

namespace {

// The grid-Gamma contraction's bin pairs: every bin in one tile when the LDS
// holds them, else the bins in chunks and one contraction per pair of
// chunks, each diagonal block owned by exactly one pair.
struct GammaPass {
  mp3::BinPair bp;
  bool own_a, own_c;
};

// LDS bytes of the forward contraction tile holding nl local bins (the basis' kernel)
size_t contract_lds_need(const mp3_plan_s* p, int nl) {
  return p->basis == MP3_BASIS_DAUBECHIES4 ? mp3::stencil_lds_need(p->prec, 2, nl) : mp3::gamma_lds_need(p->prec, nl);
}

std::vector<GammaPass> gamma_passes(const mp3_plan_s* p) {
  const int nb = p->nbins;
  std::vector<GammaPass> out;
  if (contract_lds_need(p, nb) <= kLdsLimit) {
    out.push_back({{nb, 0, nb, 0, 0}, true, true});
    return out;
  }
  int cs = nb / 2;
  while (cs > 1 && contract_lds_need(p, 2 * cs) > kLdsLimit) --cs;
  const int k = (nb + cs - 1) / cs;
  for (int i = 0; i < k; ++i) {
    for (int j = i + 1; j < k; ++j) {
      const int a0 = i * cs, na = std::min(cs, nb - a0), c0 = j * cs, nc = std::min(cs, nb - c0);
      out.push_back({{nb, a0, na, c0, nc}, j == i + 1, i == k - 2 && j == k - 1});
    }
  }
  return out;
}

// bins per chunk of the chunked grid-Gamma adjoint
int gamma_adjoint_chunk(const mp3_plan_s* p) {
  int c = p->nbins;
  if (gamma_stencil_adjoint(p)) {
    while (c > 1 && mp3::stencil_adjoint_lds_need(p->prec, p->sgam.halo, c) > kLdsLimit) --c;
    return c;
  }
  while (c > 1 && mp3::gamma_adjoint_bins_lds_need(p->prec, c) > kLdsLimit) --c;
  return c;
}

// the contraction of the stored bin-interleaved fields of one (l, m), all passes, into zeta
int gamma_contract_all(const mp3_plan_s* p, const void* Fi, const void* prim, double* partials, int gwg, double* zeta,
                       int l, double scale, hipStream_t st) {
  for (const GammaPass& g : gamma_passes(p)) {
    MP3_HIP(timed(p, MP3_PASS_GAMMA, st, [&] {
              if (p->basis == MP3_BASIS_DAUBECHIES4)
                return mp3::launch_stencil_contract(p->prec, Fi, prim, p->n, g.bp, p->sgam, partials, gwg, p->batch,
                                                    st);
              return mp3::launch_gamma_contract(p->prec, p->split, Fi, prim, p->n, g.bp, p->gm, p->gw, partials, gwg,
                                                p->batch, st);
            }),
            "grid-Gamma contraction");
    MP3_HIP(mp3::launch_reduce_partials_map(partials, gwg, g.bp, zeta, l, p->lmax, scale, g.own_a, g.own_c, p->batch,
                                            st),
            "reduce");
  }
  return MP3_OK;
}

int zeta_nodal(mp3_plan_t p, const void* delta, double* zeta, void* ws, const Layout& L, hipStream_t st) {
  const int nb2 = p->nbins * p->nbins;
  const double n3 = (double)p->n * p->n * p->n;
  void* F = at(ws, L.fields);
  double* partials = reinterpret_cast<double*>(at(ws, L.partials));
  for (int l = 0; l <= p->lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      if (int s = fields_xy(p, ws, L, F, item_index(l, m), 1, st)) return s;
      mp3::ZpassArgs z{};
      z.fields = F;
      z.delta = delta;
      z.partials = partials;
      z.tw = p->tw;
      z.nbins = p->nbins;
      z.nwg = L.nwg;
      z.ppw = L.ppw;
      z.batch = p->batch;
      z.l = l;
      z.lmax = p->lmax;
      z.split = p->split;
      MP3_HIP(timed(p, MP3_PASS_Z_NODAL, st, [&] { return mp3::launch_zpass_nodal(p->n, p->prec, z, st); }), "z pass (contraction)");
      const double wm = m == 0 ? 1.0 : 2.0;
      MP3_HIP(mp3::launch_reduce_partials(partials, L.nwg, nb2, zeta, l, p->lmax, wm * kFourPi / n3, p->batch, st),
              "reduce");
    }
  }
  return MP3_OK;
}

// particle summation: zeta_l = 4 pi [ (1/W) sum_i w_i F_l(x_i) - Fbar_l ]
int zeta_particle(mp3_plan_t p, const float* pos, const float* w, const int64_t* np_off, long long np_total,
                  long long np_max, double* zeta, void* ws, const Layout& L, hipStream_t st) {
  const int nb2 = p->nbins * p->nbins;
  const double n3 = (double)p->n * p->n * p->n;
  const double sc = (double)p->n / p->box;
  if (int s = upload_offsets(p, np_off, ws, L, st)) return s;
  const long long* off = reinterpret_cast<const long long*>(at(ws, L.off));
  double* W = reinterpret_cast<double*>(at(ws, L.W));
  MP3_HIP(mp3::launch_fill_f64(W, p->batch, 0.0, st), "zero W");
  MP3_HIP(mp3::launch_weight_sum(w, off, p->batch, np_max, W, st), "weight sum");
  int* perm = reinterpret_cast<int*>(at(ws, L.perm));
  MP3_HIP(mp3::launch_tile_sort(pos, off, p->batch, np_total, p->n, sc, 2, reinterpret_cast<int*>(at(ws, L.counts)),
                                reinterpret_cast<int*>(at(ws, L.offs)), reinterpret_cast<int*>(at(ws, L.cursor)), perm, st),
          "tile sort");
  int* tcell = reinterpret_cast<int*>(at(ws, L.tcell));
  void* twt = at(ws, L.twt);
  MP3_HIP(mp3::launch_tap_records(p->prec, pos, perm, np_total, p->n, sc, tcell, twt, p->btab, st), "stencil records");
  double* P = reinterpret_cast<double*>(at(ws, L.power));
  const int nq2 = mp3::nq2_count(p->n);
  MP3_HIP(mp3::launch_fill_f64(P, (long long)p->batch * nq2, 0.0, st), "zero power");
  MP3_HIP(mp3::launch_power_hist(p->prec, at(ws, L.dhat), p->n, nq2, P, p->batch, p->phi, p->acf, st), "power histogram");
  void* F = at(ws, L.fields);
  void* Fi = at(ws, L.fields_i);
  double* partials = reinterpret_cast<double*>(at(ws, L.partials));
  const int gwg = gather_wgs(p, np_max);
  for (int l = 0; l <= p->lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      if (int s = fields_xy(p, ws, L, F, item_index(l, m), 1, st)) return s;
      mp3::ZpassArgs z{};
      z.fields = F;
      z.tw = p->tw;
      z.nbins = p->nbins;
      z.nwg = L.nwg;
      z.ppw = L.ppw;
      z.batch = p->batch;
      MP3_HIP(timed(p, MP3_PASS_Z_STORE, st, [&] { return mp3::launch_zpass_store(p->n, p->prec, z, Fi, st); }), "z pass (store)");
      mp3::GatherArgs g{};
      g.fields = Fi;
      g.tcell = tcell;
      g.twt = twt;
      g.pos = pos;
      g.w = w;
      g.perm = perm;
      g.off = off;
      g.W = W;
      g.partials = partials;
      g.n = p->n;
      g.nbins = p->nbins;
      g.nwg = gwg;
      g.batch = p->batch;
      g.sc = sc;
      g.split = p->split;
      MP3_HIP(timed(p, MP3_PASS_GATHER, st, [&] { return mp3::launch_gather_contract(p->prec, g, st); }), "gather");
      const double wm = m == 0 ? 1.0 : 2.0;
      MP3_HIP(mp3::launch_reduce_partials(partials, gwg, nb2, zeta, l, p->lmax, wm * kFourPi, p->batch, st), "reduce");
    }
    MP3_HIP(mp3::launch_fbar_subtract(p->prec, P, p->jtab, nq2, p->nbp, p->nbins, l, p->lmax, n3 * n3, zeta, p->batch, st),
            "volume mean");
  }
  return MP3_OK;
}

// grid summation with connection coefficients:
// zeta_l = (4 pi / N^3) int delta_B sum_m atilde_b1 conj(atilde_b2) d^3u
int zeta_gamma(mp3_plan_t p, const void* delta, double* zeta, void* ws, const Layout& L, hipStream_t st) {
  const int nb2 = p->nbins * p->nbins;
  const double n3 = (double)p->n * p->n * p->n;
  void* F = at(ws, L.fields);
  void* Fi = at(ws, L.fields_i);
  double* partials = reinterpret_cast<double*>(at(ws, L.partials));
  const long long tiles = (long long)(p->n / 4) * (p->n / 4) * (p->n / 4);
  long long gwg = (long long)contract_wgs(p);
  if (gwg < 1) gwg = 1;
  if (gwg > tiles) gwg = tiles;
  for (int l = 0; l <= p->lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      if (int s = fields_xy(p, ws, L, F, item_index(l, m), 1, st)) return s;
      mp3::ZpassArgs z{};
      z.fields = F;
      z.tw = p->tw;
      z.nbins = p->nbins;
      z.nwg = L.nwg;
      z.ppw = L.ppw;
      z.batch = p->batch;
      MP3_HIP(timed(p, MP3_PASS_Z_STORE, st, [&] { return mp3::launch_zpass_store(p->n, p->prec, z, Fi, st); }), "z pass (store)");
      const double wm = m == 0 ? 1.0 : 2.0;
      if (int s = gamma_contract_all(p, Fi, delta, partials, (int)gwg, zeta, l, wm * kFourPi / n3, st)) return s;
    }
  }
  return MP3_OK;
}

}  // namespace

int mp3_zeta(mp3_plan_t p, const void* delta, const float* pos, const float* w, const int64_t* np_off, double* zeta,
             void* ws, size_t wsb, void* stream) {
  if (int s = check_plan(p)) return s;
  if (!delta || !zeta) return fail(MP3_EINVAL, "delta and zeta must not be NULL");
  long long np_total = 0, np_max = 0;
  if (p->summation == MP3_SUM_PARTICLE) {
    if (int s = check_offsets(p, np_off, &np_total, &np_max)) return s;
    if (!pos) return fail(MP3_EINVAL, "pos is NULL (particle summation needs the catalogue)");
    if (np_total >= (1LL << 31)) return fail(MP3_EUNSUPPORTED, "more than 2^31 - 1 particles");
  }
  const Layout L = layout(p, np_total);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n3 = (long long)p->n * p->n * p->n;
  if (int s = check_finite(p, ws, L.flag, st, delta, n3 * p->batch, p->prec)) return s;
  if (int s = forward_dft(p, delta, ws, L, st)) return s;
  MP3_HIP(mp3::launch_fill_f64(zeta, (long long)p->batch * (p->lmax + 1) * p->nbins * p->nbins, 0.0, st), "zero zeta");
  if (p->summation == MP3_SUM_PARTICLE) return zeta_particle(p, pos, w, np_off, np_total, np_max, zeta, ws, L, st);
  int ps = MP3_OK;
  const void* prim = primary_field(p, delta, ws, L, st, &ps);
  if (ps) return ps;
  if (p->summation == MP3_SUM_GRID_GAMMA) return zeta_gamma(p, prim, zeta, ws, L, st);
  return zeta_nodal(p, prim, zeta, ws, L, st);
}

namespace {

// end of the nodal adjoint: final transform of the accumulator G, ddelta, and
// dJ/dw through the deposit when dw is requested
int nodal_gradient_tail(mp3_plan_t p, const void* delta, void* ddelta, const float* pos, const float* w,
                        const int64_t* np_off, void* dw, void* ws, const Layout& L, long long np_total,
                        long long np_max, hipStream_t st) {
  const long long n3 = (long long)p->n * p->n * p->n;
  void* G = at(ws, L.G);
  void* direct = at(ws, L.direct);
  MP3_HIP(timed(p, MP3_PASS_DFT, st, [&] { return mp3::launch_fft3d(p->n, p->prec, -1, false, G, G, p->batch, p->tw, st); }), "adjoint final FFT");
  if (int s = filter_direct(p, direct, ws, L, st)) return s;
  MP3_HIP(mp3::launch_grad_combine(p->prec, direct, G, ddelta, n3 * p->batch, kFourPi / (double)n3, st), "combine");
  if (dw) {
    if (int s = upload_offsets(p, np_off, ws, L, st)) return s;
    const long long* off = reinterpret_cast<const long long*>(at(ws, L.off));
    double* W = reinterpret_cast<double*>(at(ws, L.W));
    double* S = reinterpret_cast<double*>(at(ws, L.S));
    MP3_HIP(mp3::launch_fill_f64(W, p->batch, 0.0, st), "zero W");
    MP3_HIP(mp3::launch_fill_f64(S, p->batch, 0.0, st), "zero S");
    MP3_HIP(mp3::launch_weight_sum(w, off, p->batch, np_max, W, st), "weight sum");
    MP3_HIP(mp3::launch_dot_rho_g(p->prec, delta, ddelta, n3, S, p->batch, st), "dot");
    MP3_HIP(mp3::launch_gather_dw(p->prec, pos, off, p->batch, np_total, p->n, (double)p->n / p->box, ddelta, W, S, dw, p->btab, st),
            "gather dw");
  }
  return MP3_OK;
}

// Adjoint of the particle summation (chain rule of zeta_particle):
//   dJ/ddelta = (4 pi / N^3) 2 Re fftn( sum_{l,m,b} wm K_b ifftn(c_b) - H conj(dhat) / (4 pi N^3) ),
//   c_b = N^3 scatter_i[ (w_i / W) sum_b' lam_s[b][b'] conj(atilde_b'(u_i)) ],
//   H(q) = B7hat(q) sum_l (2l+1) sum_{b1,b2} lam_l[b1][b2] jbar_{l,b1} jbar_{l,b2},
// and dJ/dw adds the primary vertex's 4 pi [F_J(u_i) / W - sum_j w_j F_J(u_j) / W^2]
// to the deposit's chain rule.
int backward_particle(mp3_plan_t p, const void* delta, const double* dzeta, void* ddelta, const float* pos,
                      const float* w, const int64_t* np_off, void* dw, void* ws, size_t wsb, void* stream) {
  long long np_total = 0, np_max = 0;
  if (int s = check_offsets(p, np_off, &np_total, &np_max)) return s;
  if (!pos) return fail(MP3_EINVAL, "pos is NULL (the particle form's adjoint needs the catalogue)");
  if (np_total >= (1LL << 31)) return fail(MP3_EUNSUPPORTED, "more than 2^31 - 1 particles");
  const Layout L = layout(p, np_total);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n3 = (long long)p->n * p->n * p->n;
  const double sc = (double)p->n / p->box;
  if (int s = check_finite(p, ws, L.flag, st, delta, n3 * p->batch, p->prec)) return s;
  if (int s = forward_dft(p, delta, ws, L, st)) return s;
  if (int s = lam_eig_all(p, dzeta, ws, L, st)) return s;
  if (int s = upload_offsets(p, np_off, ws, L, st)) return s;
  const long long* off = reinterpret_cast<const long long*>(at(ws, L.off));
  double* W = reinterpret_cast<double*>(at(ws, L.W));
  MP3_HIP(mp3::launch_fill_f64(W, p->batch, 0.0, st), "zero W");
  MP3_HIP(mp3::launch_weight_sum(w, off, p->batch, np_max, W, st), "weight sum");
  int* perm = reinterpret_cast<int*>(at(ws, L.perm));
  const int* toff = reinterpret_cast<const int*>(at(ws, L.offs));
  MP3_HIP(mp3::launch_tile_sort(pos, off, p->batch, np_total, p->n, sc, 2, reinterpret_cast<int*>(at(ws, L.counts)),
                                reinterpret_cast<int*>(at(ws, L.offs)), reinterpret_cast<int*>(at(ws, L.cursor)), perm, st),
          "tile sort");
  int* tcell = reinterpret_cast<int*>(at(ws, L.tcell));
  void* twt = at(ws, L.twt);
  MP3_HIP(mp3::launch_tap_records(p->prec, pos, perm, np_total, p->n, sc, tcell, twt, p->btab, st), "stencil records");
  void* F = at(ws, L.fields);
  void* Fi = at(ws, L.fields_i);
  void* G = at(ws, L.G);
  void* direct = at(ws, L.direct);
  void* src = at(ws, L.src);
  double* FJ = reinterpret_cast<double*>(at(ws, L.fj));
  MP3_HIP(mp3::launch_fill(p->prec, G, 2 * n3 * p->batch, 0.0, st), "zero G");
  MP3_HIP(mp3::launch_fill(p->prec, direct, n3 * p->batch, 0.0, st), "zero direct");
  MP3_HIP(mp3::launch_fill_f64(FJ, np_total, 0.0, st), "zero F_J");
  const int gwg = gather_wgs(p, np_max);
  for (int l = 0; l <= p->lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      const double wm = m == 0 ? 1.0 : 2.0;
      if (int s = fields_xy(p, ws, L, F, item_index(l, m), 1, st, true)) return s;
      mp3::ZpassArgs z{};
      z.fields = F;
      z.tw = p->tw;
      z.nbins = p->nbins;
      z.nwg = L.nwg;
      z.ppw = L.ppw;
      z.batch = p->batch;
      MP3_HIP(timed(p, MP3_PASS_Z_STORE, st, [&] { return mp3::launch_zpass_store(p->n, p->prec, z, Fi, st); }), "z pass (store)");
      MP3_HIP(timed(p, MP3_PASS_GATHER, st, [&] {
                return mp3::launch_gather_source(p->prec, Fi, tcell, twt, w, perm, off, W, lam_d_at(p, ws, L, l), p->n, p->nbins,
                                                 wm, gwg, p->batch, FJ, src, st);
              }),
              "gather (adjoint sources)");
      MP3_HIP(timed(p, MP3_PASS_SCATTER, st, [&] {
                return mp3::launch_scatter_source(p->prec, tcell, twt, toff, src, p->n, p->nbins, p->batch, F, st);
              }),
              "scatter (adjoint sources)");
      MP3_HIP(timed(p, MP3_PASS_Z_ADJOINT, st, [&] { return mp3::launch_fft_z(p->n, p->prec, +1, F, F, p->batch * p->nbins, p->tw, st); }),
              "adjoint z pass");
      MP3_HIP(timed(p, MP3_PASS_X, st, [&] { return mp3::launch_fft_x(p->n, p->prec, +1, F, p->batch * p->nbins, p->tw, p->tune[MP3_TUNE_FFT_X_PLAN], st); }),
              "adjoint x pass");
      mp3::FilterArgs a = filter_args(p, ws, L, F, G, item_index(l, m), 1, true);
      MP3_HIP(timed(p, MP3_PASS_ADJOINT, st, [&] { return mp3::launch_adjoint_y(p->n, p->prec, a, st); }), "adjoint window pass");
    }
  }
  MP3_HIP(mp3::launch_fbar_adjoint(p->prec, dzeta, p->jtab, p->nq2, p->nbp, p->nbins, p->lmax, at(ws, L.dhat), p->n,
                                   -1.0 / (kFourPi * (double)n3), reinterpret_cast<double*>(at(ws, L.hq)), G, p->batch,
                                   p->phi, p->acf, st),
          "volume-mean adjoint");
  MP3_HIP(timed(p, MP3_PASS_DFT, st, [&] { return mp3::launch_fft3d(p->n, p->prec, -1, false, G, G, p->batch, p->tw, st); }), "adjoint final FFT");
  MP3_HIP(mp3::launch_grad_combine(p->prec, direct, G, ddelta, n3 * p->batch, kFourPi / (double)n3, st), "combine");
  if (dw) {
    double* S = reinterpret_cast<double*>(at(ws, L.S));
    double* SF = reinterpret_cast<double*>(at(ws, L.SF));
    MP3_HIP(mp3::launch_fill_f64(S, p->batch, 0.0, st), "zero S");
    MP3_HIP(mp3::launch_fill_f64(SF, p->batch, 0.0, st), "zero SF");
    MP3_HIP(mp3::launch_dot_rho_g(p->prec, delta, ddelta, n3, S, p->batch, st), "dot");
    MP3_HIP(mp3::launch_gather_dw(p->prec, pos, off, p->batch, np_total, p->n, sc, ddelta, W, S, dw, p->btab, st), "gather dw");
    MP3_HIP(mp3::launch_weighted_sum(w, FJ, off, p->batch, np_max, SF, st), "sum w F_J");
    MP3_HIP(mp3::launch_primary_dw(p->prec, off, p->batch, np_total, FJ, W, SF, dw, st), "primary dw");
  }
  return MP3_OK;
}

// Adjoint of the grid summation with connection coefficients: the nodal
// adjoint with the primary's weight delta_x and the pointwise products
// replaced by the quadrature of the B-spline reconstructions (k_gamma_adjoint
// produces c_b and the direct term per (l, m)); the same adjoint transforms
// and deposit chain rule follow.
// One sweep of the particle form: the forward's and the adjoint's per-call
// steps run once, and per (l, m) the stored fields feed both the contraction
// (gather_contract) and the adjoint sources (gather_source).
int value_and_grad_particle(mp3_plan_t p, const void* delta, const double* dzeta, double* zeta, void* ddelta,
                            const float* pos, const float* w, const int64_t* np_off, void* dw, void* ws, size_t wsb,
                            hipStream_t st) {
  long long np_total = 0, np_max = 0;
  if (int s = check_offsets(p, np_off, &np_total, &np_max)) return s;
  if (!pos) return fail(MP3_EINVAL, "pos is NULL (particle summation needs the catalogue)");
  if (np_total >= (1LL << 31)) return fail(MP3_EUNSUPPORTED, "more than 2^31 - 1 particles");
  const Layout L = layout(p, np_total);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  const int nb2 = p->nbins * p->nbins;
  const long long n3 = (long long)p->n * p->n * p->n;
  const double n3d = (double)n3;
  const double sc = (double)p->n / p->box;
  if (int s = check_finite(p, ws, L.flag, st, delta, n3 * p->batch, p->prec)) return s;
  if (int s = forward_dft(p, delta, ws, L, st)) return s;
  if (int s = lam_eig_all(p, dzeta, ws, L, st)) return s;
  MP3_HIP(mp3::launch_fill_f64(zeta, (long long)p->batch * (p->lmax + 1) * nb2, 0.0, st), "zero zeta");
  if (int s = upload_offsets(p, np_off, ws, L, st)) return s;
  const long long* off = reinterpret_cast<const long long*>(at(ws, L.off));
  double* W = reinterpret_cast<double*>(at(ws, L.W));
  MP3_HIP(mp3::launch_fill_f64(W, p->batch, 0.0, st), "zero W");
  MP3_HIP(mp3::launch_weight_sum(w, off, p->batch, np_max, W, st), "weight sum");
  int* perm = reinterpret_cast<int*>(at(ws, L.perm));
  const int* toff = reinterpret_cast<const int*>(at(ws, L.offs));
  MP3_HIP(mp3::launch_tile_sort(pos, off, p->batch, np_total, p->n, sc, 2, reinterpret_cast<int*>(at(ws, L.counts)),
                                reinterpret_cast<int*>(at(ws, L.offs)), reinterpret_cast<int*>(at(ws, L.cursor)), perm, st),
          "tile sort");
  int* tcell = reinterpret_cast<int*>(at(ws, L.tcell));
  void* twt = at(ws, L.twt);
  MP3_HIP(mp3::launch_tap_records(p->prec, pos, perm, np_total, p->n, sc, tcell, twt, p->btab, st), "stencil records");
  double* P = reinterpret_cast<double*>(at(ws, L.power));
  const int nq2 = mp3::nq2_count(p->n);
  MP3_HIP(mp3::launch_fill_f64(P, (long long)p->batch * nq2, 0.0, st), "zero power");
  MP3_HIP(mp3::launch_power_hist(p->prec, at(ws, L.dhat), p->n, nq2, P, p->batch, p->phi, p->acf, st), "power histogram");
  void* F = at(ws, L.fields);
  void* Fi = at(ws, L.fields_i);
  void* G = at(ws, L.G);
  void* direct = at(ws, L.direct);
  void* src = at(ws, L.src);
  double* FJ = reinterpret_cast<double*>(at(ws, L.fj));
  double* partials = reinterpret_cast<double*>(at(ws, L.partials));
  MP3_HIP(mp3::launch_fill(p->prec, G, 2 * n3 * p->batch, 0.0, st), "zero G");
  MP3_HIP(mp3::launch_fill(p->prec, direct, n3 * p->batch, 0.0, st), "zero direct");
  MP3_HIP(mp3::launch_fill_f64(FJ, np_total, 0.0, st), "zero F_J");
  const int gwg = gather_wgs(p, np_max);
  for (int l = 0; l <= p->lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      const double wm = m == 0 ? 1.0 : 2.0;
      if (int s = fields_xy(p, ws, L, F, item_index(l, m), 1, st, true)) return s;
      mp3::ZpassArgs z{};
      z.fields = F;
      z.tw = p->tw;
      z.nbins = p->nbins;
      z.nwg = L.nwg;
      z.ppw = L.ppw;
      z.batch = p->batch;
      MP3_HIP(timed(p, MP3_PASS_Z_STORE, st, [&] { return mp3::launch_zpass_store(p->n, p->prec, z, Fi, st); }), "z pass (store)");
      mp3::GatherArgs g{};
      g.fields = Fi;
      g.tcell = tcell;
      g.twt = twt;
      g.pos = pos;
      g.w = w;
      g.perm = perm;
      g.off = off;
      g.W = W;
      g.partials = partials;
      g.n = p->n;
      g.nbins = p->nbins;
      g.nwg = gwg;
      g.batch = p->batch;
      g.sc = sc;
      g.split = p->split;
      // one gather gives the contraction and the (diagonal) adjoint sources
      g.lam = lam_d_at(p, ws, L, l);
      g.wm = wm;
      g.FJ = FJ;
      g.src = src;
      MP3_HIP(timed(p, MP3_PASS_GATHER, st, [&] { return mp3::launch_gather_contract(p->prec, g, st); }), "gather");
      MP3_HIP(mp3::launch_reduce_partials(partials, gwg, nb2, zeta, l, p->lmax, wm * kFourPi, p->batch, st), "reduce");
      MP3_HIP(timed(p, MP3_PASS_SCATTER, st, [&] {
                return mp3::launch_scatter_source(p->prec, tcell, twt, toff, src, p->n, p->nbins, p->batch, F, st);
              }),
              "scatter (adjoint sources)");
      MP3_HIP(timed(p, MP3_PASS_Z_ADJOINT, st, [&] { return mp3::launch_fft_z(p->n, p->prec, +1, F, F, p->batch * p->nbins, p->tw, st); }),
              "adjoint z pass");
      MP3_HIP(timed(p, MP3_PASS_X, st, [&] { return mp3::launch_fft_x(p->n, p->prec, +1, F, p->batch * p->nbins, p->tw, p->tune[MP3_TUNE_FFT_X_PLAN], st); }),
              "adjoint x pass");
      mp3::FilterArgs a = filter_args(p, ws, L, F, G, item_index(l, m), 1, true);
      MP3_HIP(timed(p, MP3_PASS_ADJOINT, st, [&] { return mp3::launch_adjoint_y(p->n, p->prec, a, st); }), "adjoint window pass");
    }
  }
  // the value was summed over the rotated fields: back to the bins, then the volume means
  MP3_HIP(mp3::launch_rotate_zeta(zeta, reinterpret_cast<const double*>(at(ws, L.evec)), p->nbins, p->lmax, p->batch,
                                  st),
          "zeta out of the eigenbasis");
  for (int l = 0; l <= p->lmax; ++l)
    MP3_HIP(mp3::launch_fbar_subtract(p->prec, P, p->jtab, nq2, p->nbp, p->nbins, l, p->lmax, n3d * n3d, zeta, p->batch, st),
            "volume mean");
  MP3_HIP(mp3::launch_fbar_adjoint(p->prec, dzeta, p->jtab, p->nq2, p->nbp, p->nbins, p->lmax, at(ws, L.dhat), p->n,
                                   -1.0 / (kFourPi * n3d), reinterpret_cast<double*>(at(ws, L.hq)), G, p->batch,
                                   p->phi, p->acf, st),
          "volume-mean adjoint");
  MP3_HIP(timed(p, MP3_PASS_DFT, st, [&] { return mp3::launch_fft3d(p->n, p->prec, -1, false, G, G, p->batch, p->tw, st); }), "adjoint final FFT");
  MP3_HIP(mp3::launch_grad_combine(p->prec, direct, G, ddelta, n3 * p->batch, kFourPi / n3d, st), "combine");
  if (dw) {
    double* S = reinterpret_cast<double*>(at(ws, L.S));
    double* SF = reinterpret_cast<double*>(at(ws, L.SF));
    MP3_HIP(mp3::launch_fill_f64(S, p->batch, 0.0, st), "zero S");
    MP3_HIP(mp3::launch_fill_f64(SF, p->batch, 0.0, st), "zero SF");
    MP3_HIP(mp3::launch_dot_rho_g(p->prec, delta, ddelta, n3, S, p->batch, st), "dot");
    MP3_HIP(mp3::launch_gather_dw(p->prec, pos, off, p->batch, np_total, p->n, sc, ddelta, W, S, dw, p->btab, st), "gather dw");
    MP3_HIP(mp3::launch_weighted_sum(w, FJ, off, p->batch, np_max, SF, st), "sum w F_J");
    MP3_HIP(mp3::launch_primary_dw(p->prec, off, p->batch, np_total, FJ, W, SF, dw, st), "primary dw");
  }
  return MP3_OK;
}

// zeta != NULL: one sweep, the adjoint kernel also contracts the node values
// for zeta (float32 or float64 inputs, not the BF16-split option)
int backward_gamma(mp3_plan_t p, const void* delta, const double* dzeta, void* ddelta, const float* pos,
                   const float* w, const int64_t* np_off, void* dw, void* ws, size_t wsb, void* stream,
                   double* zeta = nullptr) {
  // tiles that do not hold every bin: the adjoint by bin chunks (and, for
  // zeta, the contraction by pairs of chunks)
  const bool chunked = gamma_stencil_adjoint(p) || mp3::gamma_adjoint_lds_need(p->prec, p->nbins) > kLdsLimit;
  long long np_total = 0, np_max = 0;
  if (dw) {
    if (int s = check_offsets(p, np_off, &np_total, &np_max)) return s;
    if (!pos) return fail(MP3_EINVAL, "pos is NULL while dw is requested");
  }
  const Layout L = layout(p, np_total);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n3 = (long long)p->n * p->n * p->n;
  if (int s = check_finite(p, ws, L.flag, st, delta, n3 * p->batch, p->prec)) return s;
  if (int s = forward_dft(p, delta, ws, L, st)) return s;
  if (int s = lam_all(p, dzeta, ws, L, st)) return s;
  int ps = MP3_OK;
  const void* prim = primary_field(p, delta, ws, L, st, &ps);
  if (ps) return ps;
  void* F = at(ws, L.fields);
  void* Fi = at(ws, L.fields_i);
  void* G = at(ws, L.G);
  void* direct = at(ws, L.direct);
  double* partials = zeta ? reinterpret_cast<double*>(at(ws, L.partials)) : nullptr;
  const int nb2 = p->nbins * p->nbins;
  if (zeta) MP3_HIP(mp3::launch_fill_f64(zeta, (long long)p->batch * (p->lmax + 1) * nb2, 0.0, st), "zero zeta");
  MP3_HIP(mp3::launch_fill(p->prec, G, 2 * n3 * p->batch, 0.0, st), "zero G");
  MP3_HIP(mp3::launch_fill(p->prec, direct, n3 * p->batch, 0.0, st), "zero direct");
  const long long tiles = (long long)(p->n / 4) * (p->n / 4) * (p->n / 4);
  long long gwg = (long long)contract_wgs(p);
  if (gwg < 1) gwg = 1;
  if (gwg > tiles) gwg = tiles;
  for (int l = 0; l <= p->lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      const double wm = m == 0 ? 1.0 : 2.0;
      if (int s = fields_xy(p, ws, L, F, item_index(l, m), 1, st)) return s;
      mp3::ZpassArgs z{};
      z.fields = F;
      z.tw = p->tw;
      z.nbins = p->nbins;
      z.nwg = L.nwg;
      z.ppw = L.ppw;
      z.batch = p->batch;
      MP3_HIP(timed(p, MP3_PASS_Z_STORE, st, [&] { return mp3::launch_zpass_store(p->n, p->prec, z, Fi, st); }), "z pass (store)");
      MP3_HIP(mp3::launch_fill(p->prec, F, 2 * n3 * p->batch * p->nbins, 0.0, st), "zero sources");
      if (chunked) {
        if (zeta)
          if (int s = gamma_contract_all(p, Fi, prim, partials, (int)gwg, zeta, l, wm * kFourPi / (double)n3, st))
            return s;
        void* U = at(ws, L.fields_u);
        MP3_HIP(mp3::launch_bin_mix(p->prec, Fi, lam_at(p, ws, L, l), U, n3, p->nbins, p->batch, st), "bin mix");
        const int cb = gamma_adjoint_chunk(p);
        for (int b0 = 0; b0 < p->nbins; b0 += cb) {
          const int nbc = std::min(cb, p->nbins - b0);
          MP3_HIP(timed(p, MP3_PASS_GAMMA, st, [&] {
                    if (gamma_stencil_adjoint(p))
                      return mp3::launch_stencil_adjoint(p->prec, Fi, U, prim, p->n, p->nbins, b0, nbc, p->sgam, wm,
                                                         (int)gwg, p->batch, F, direct, st);
                    return mp3::launch_gamma_adjoint_bins(p->prec, Fi, U, prim, p->n, p->nbins, b0, nbc, p->gm, p->gw,
                                                          wm, (int)gwg, p->batch, F, direct, st);
                  }),
                  "grid-Gamma adjoint (bin chunk)");
        }
      } else {
        MP3_HIP(timed(p, MP3_PASS_GAMMA, st, [&] {
                  return mp3::launch_gamma_adjoint(p->prec, Fi, prim, lam_at(p, ws, L, l), p->n, p->nbins, p->gm, p->gw, wm,
                                                   (int)gwg, p->batch, F, direct, partials, st);
                }),
                "grid-Gamma adjoint");
        if (zeta)
          MP3_HIP(mp3::launch_reduce_partials(partials, (int)gwg, nb2, zeta, l, p->lmax, wm * kFourPi / (double)n3,
                                              p->batch, st),
                  "reduce");
      }
      MP3_HIP(timed(p, MP3_PASS_Z_ADJOINT, st, [&] { return mp3::launch_fft_z(p->n, p->prec, +1, F, F, p->batch * p->nbins, p->tw, st); }),
              "adjoint z pass");
      MP3_HIP(timed(p, MP3_PASS_X, st, [&] { return mp3::launch_fft_x(p->n, p->prec, +1, F, p->batch * p->nbins, p->tw, p->tune[MP3_TUNE_FFT_X_PLAN], st); }),
              "adjoint x pass");
      mp3::FilterArgs a = filter_args(p, ws, L, F, G, item_index(l, m), 1);
      MP3_HIP(timed(p, MP3_PASS_ADJOINT, st, [&] { return mp3::launch_adjoint_y(p->n, p->prec, a, st); }), "adjoint window pass");
    }
  }
  MP3_HIP(timed(p, MP3_PASS_DFT, st, [&] { return mp3::launch_fft3d(p->n, p->prec, -1, false, G, G, p->batch, p->tw, st); }), "adjoint final FFT");
  if (int s = filter_direct(p, direct, ws, L, st)) return s;
  MP3_HIP(mp3::launch_grad_combine(p->prec, direct, G, ddelta, n3 * p->batch, kFourPi / (double)n3, st), "combine");
  if (dw) {
    if (int s = upload_offsets(p, np_off, ws, L, st)) return s;
    const long long* off = reinterpret_cast<const long long*>(at(ws, L.off));
    double* W = reinterpret_cast<double*>(at(ws, L.W));
    double* S = reinterpret_cast<double*>(at(ws, L.S));
    MP3_HIP(mp3::launch_fill_f64(W, p->batch, 0.0, st), "zero W");
    MP3_HIP(mp3::launch_fill_f64(S, p->batch, 0.0, st), "zero S");
    MP3_HIP(mp3::launch_weight_sum(w, off, p->batch, np_max, W, st), "weight sum");
    MP3_HIP(mp3::launch_dot_rho_g(p->prec, delta, ddelta, n3, S, p->batch, st), "dot");
    MP3_HIP(mp3::launch_gather_dw(p->prec, pos, off, p->batch, np_total, p->n, (double)p->n / p->box, ddelta, W, S, dw, p->btab, st),
            "gather dw");
  }
  return MP3_OK;
}

}  // namespace

int mp3_zeta_backward(mp3_plan_t p, const void* delta, const double* dzeta, void* ddelta, const float* pos,
                      const float* w, const int64_t* np_off, void* dw, void* ws, size_t wsb, void* stream) {
  if (int s = check_plan(p)) return s;
  if (!delta || !dzeta || !ddelta) return fail(MP3_EINVAL, "delta, dzeta and ddelta must not be NULL");
  if (p->summation == MP3_SUM_PARTICLE) return backward_particle(p, delta, dzeta, ddelta, pos, w, np_off, dw, ws, wsb, stream);
  if (p->summation == MP3_SUM_GRID_GAMMA) return backward_gamma(p, delta, dzeta, ddelta, pos, w, np_off, dw, ws, wsb, stream);
  long long np_total = 0, np_max = 0;
  if (dw) {
    if (int s = check_offsets(p, np_off, &np_total, &np_max)) return s;
    if (!pos) return fail(MP3_EINVAL, "pos is NULL while dw is requested");
  }
  const Layout L = layout(p, np_total);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n3 = (long long)p->n * p->n * p->n;
  if (int s = check_finite(p, ws, L.flag, st, delta, n3 * p->batch, p->prec)) return s;
  if (int s = forward_dft(p, delta, ws, L, st)) return s;
  if (int s = lam_eig_all(p, dzeta, ws, L, st)) return s;
  int ps = MP3_OK;
  const void* prim = primary_field(p, delta, ws, L, st, &ps);
  if (ps) return ps;
  void* F = at(ws, L.fields);
  void* G = at(ws, L.G);
  void* direct = at(ws, L.direct);
  MP3_HIP(mp3::launch_fill(p->prec, G, 2 * n3 * p->batch, 0.0, st), "zero G");
  MP3_HIP(mp3::launch_fill(p->prec, direct, n3 * p->batch, 0.0, st), "zero direct");
  const int nitems_all = (int)p->items.size();
  for (int item0 = 0; item0 < nitems_all; item0 += L.group) {
    const int ni = std::min(L.group, nitems_all - item0);
    if (int s = fields_xy(p, ws, L, F, item0, ni, st, true)) return s;
    mp3::ZpassArgs z = adjoint_zargs(p, ws, L, F, prim, dzeta, direct, item0, ni);
    MP3_HIP(timed(p, MP3_PASS_Z_ADJOINT, st, [&] { return mp3::launch_zpass_adjoint(p->n, p->prec, z, st); }), "z pass (adjoint)");
    MP3_HIP(timed(p, MP3_PASS_X, st, [&] { return mp3::launch_fft_x(p->n, p->prec, +1, F, ni * p->batch * p->nbins, p->tw, p->tune[MP3_TUNE_FFT_X_PLAN], st); }), "adjoint x pass");
    mp3::FilterArgs a = filter_args(p, ws, L, F, G, item0, ni, true);
    MP3_HIP(timed(p, MP3_PASS_ADJOINT, st, [&] { return mp3::launch_adjoint_y(p->n, p->prec, a, st); }), "adjoint window pass");
  }
  return nodal_gradient_tail(p, delta, ddelta, pos, w, np_off, dw, ws, L, np_total, np_max, st);
}

int mp3_zeta_value_and_grad(mp3_plan_t p, const void* delta, const double* dzeta, double* zeta, void* ddelta,
                            const float* pos, const float* w, const int64_t* np_off, void* dw, void* ws, size_t wsb,
                            void* stream) {
  if (int s = check_plan(p)) return s;
  if (!delta || !dzeta || !zeta || !ddelta) return fail(MP3_EINVAL, "delta, dzeta, zeta and ddelta must not be NULL");
  if (p->summation == MP3_SUM_PARTICLE)
    return value_and_grad_particle(p, delta, dzeta, zeta, ddelta, pos, w, np_off, dw, ws, wsb,
                                   static_cast<hipStream_t>(stream));
  if (p->summation == MP3_SUM_GRID_GAMMA && !p->split)
    return backward_gamma(p, delta, dzeta, ddelta, pos, w, np_off, dw, ws, wsb, stream, zeta);
  const int storage = p->prec;
  const bool one_sweep = p->summation == MP3_SUM_NODAL && !p->split && p->nbins <= 32 &&
                         mp3::zpass_fused_lds_need(p->n, storage, p->nbins) <= kLdsLimit;
  if (!one_sweep) {
    if (int s = mp3_zeta(p, delta, pos, w, np_off, zeta, ws, wsb, stream)) return s;
    return mp3_zeta_backward(p, delta, dzeta, ddelta, pos, w, np_off, dw, ws, wsb, stream);
  }
  long long np_total = 0, np_max = 0;
  if (dw) {
    if (int s = check_offsets(p, np_off, &np_total, &np_max)) return s;
    if (!pos) return fail(MP3_EINVAL, "pos is NULL while dw is requested");
  }
  const Layout L = layout(p, np_total);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n3 = (long long)p->n * p->n * p->n;
  const int nb2 = p->nbins * p->nbins;
  if (int s = check_finite(p, ws, L.flag, st, delta, n3 * p->batch, p->prec)) return s;
  if (int s = forward_dft(p, delta, ws, L, st)) return s;
  if (int s = lam_eig_all(p, dzeta, ws, L, st)) return s;
  int ps = MP3_OK;
  const void* prim = primary_field(p, delta, ws, L, st, &ps);
  if (ps) return ps;
  void* F = at(ws, L.fields);
  void* G = at(ws, L.G);
  void* direct = at(ws, L.direct);
  double* partials = reinterpret_cast<double*>(at(ws, L.partials));
  MP3_HIP(mp3::launch_fill_f64(zeta, (long long)p->batch * (p->lmax + 1) * nb2, 0.0, st), "zero zeta");
  MP3_HIP(mp3::launch_fill(p->prec, G, 2 * n3 * p->batch, 0.0, st), "zero G");
  MP3_HIP(mp3::launch_fill(p->prec, direct, n3 * p->batch, 0.0, st), "zero direct");
  const int nitems_all = (int)p->items.size();
  for (int item0 = 0; item0 < nitems_all; item0 += L.group) {
    const int ni = std::min(L.group, nitems_all - item0);
    if (int s = fields_xy(p, ws, L, F, item0, ni, st, true)) return s;
    mp3::ZpassArgs z = adjoint_zargs(p, ws, L, F, prim, dzeta, direct, item0, ni);
    z.partials = partials;
    z.waves = p->tune[MP3_TUNE_FUSED_WAVES];
    MP3_HIP(timed(p, MP3_PASS_Z_FUSED, st, [&] { return mp3::launch_zpass_fused(p->n, p->prec, z, st); }),
            "z pass (contraction and adjoint)");
    MP3_HIP(mp3::launch_reduce_items(partials, L.nwg, nb2, zeta, p->lmax, kFourPi / (double)n3, p->items_dev, item0, ni,
                                     p->batch, st),
            "reduce");
    MP3_HIP(timed(p, MP3_PASS_X, st, [&] { return mp3::launch_fft_x(p->n, p->prec, +1, F, ni * p->batch * p->nbins, p->tw, p->tune[MP3_TUNE_FFT_X_PLAN], st); }), "adjoint x pass");
    mp3::FilterArgs a = filter_args(p, ws, L, F, G, item0, ni, true);
    MP3_HIP(timed(p, MP3_PASS_ADJOINT, st, [&] { return mp3::launch_adjoint_y(p->n, p->prec, a, st); }), "adjoint window pass");
  }
  // the value was summed over the rotated fields: back to the bins
  MP3_HIP(mp3::launch_rotate_zeta(zeta, reinterpret_cast<const double*>(at(ws, L.evec)), p->nbins, p->lmax, p->batch,
                                  st),
          "zeta out of the eigenbasis");
  return nodal_gradient_tail(p, delta, ddelta, pos, w, np_off, dw, ws, L, np_total, np_max, st);
}

namespace {

// plain |dhat|^2 histogram of delta (forward transform included) into L.pplain
int power_plain(mp3_plan_t p, const void* delta, void* ws, const Layout& L, hipStream_t st) {
  if (int s = forward_dft(p, delta, ws, L, st)) return s;
  double* P = reinterpret_cast<double*>(at(ws, L.pplain));
  const int nq2 = mp3::nq2_count(p->n);
  MP3_HIP(mp3::launch_fill_f64(P, (long long)p->batch * nq2, 0.0, st), "zero histogram");
  MP3_HIP(mp3::launch_power_plain(p->prec, at(ws, L.dhat), p->n, nq2, P, p->batch, p->phi, st), "power histogram");
  return MP3_OK;
}

bool primary_smoothed(const mp3_plan_s* p) { return p->smoothing > 0.0 && p->summation != MP3_SUM_PARTICLE; }

}  // namespace

int mp3_xi(mp3_plan_t p, const void* delta, const double* radii, int32_t nr, double* xi, void* ws, size_t wsb,
           void* stream) {
  if (int s = check_plan(p)) return s;
  if (!delta || !radii || !xi) return fail(MP3_EINVAL, "delta, radii and xi must not be NULL");
  if (nr < 1 || nr > kMaxAux) return fail(MP3_EINVAL, "nr must be in [1, 4096]");
  for (int i = 0; i < nr; ++i) {
    if (!std::isfinite(radii[i])) return fail(MP3_ENONFINITE, "radii must be finite");
    if (radii[i] < 0.0) return fail(MP3_EINVAL, "radii must be >= 0");
  }
  const Layout L = layout(p);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n3 = (long long)p->n * p->n * p->n;
  if (int s = check_finite(p, ws, L.flag, st, delta, n3 * p->batch, p->prec)) return s;
  if (int s = power_plain(p, delta, ws, L, st)) return s;
  double* dr = reinterpret_cast<double*>(at(ws, L.aux));
  MP3_HIP(hipMemcpyAsync(dr, radii, (size_t)nr * sizeof(double), hipMemcpyHostToDevice, st), "copy radii");
  const double n6 = (double)n3 * (double)n3;
  MP3_HIP(mp3::launch_xi(reinterpret_cast<const double*>(at(ws, L.pplain)), mp3::nq2_count(p->n), 2.0 * M_PI / p->box,
                         p->smoothing, primary_smoothed(p), dr, nr, n6, xi, p->batch, st),
          "xi");
  return MP3_OK;
}

int mp3_xi_multipoles(mp3_plan_t p, const void* delta, const double* radii, int32_t nr, int32_t ell_max, double* xi,
                      void* ws, size_t wsb, void* stream) {
  if (int s = check_plan(p)) return s;
  if (!delta || !radii || !xi) return fail(MP3_EINVAL, "delta, radii and xi must not be NULL");
  if (nr < 1 || nr > kMaxAux) return fail(MP3_EINVAL, "nr must be in [1, 4096]");
  if (ell_max < 0 || ell_max > 16) return fail(MP3_EINVAL, "ell_max must be in [0, 16]");
  for (int i = 0; i < nr; ++i) {
    if (!std::isfinite(radii[i])) return fail(MP3_ENONFINITE, "radii must be finite");
    if (radii[i] < 0.0) return fail(MP3_EINVAL, "radii must be >= 0");
  }
  const Layout L = layout(p);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n3 = (long long)p->n * p->n * p->n;
  if (int s = check_finite(p, ws, L.flag, st, delta, n3 * p->batch, p->prec)) return s;
  if (int s = forward_dft(p, delta, ws, L, st)) return s;
  // the moments [batch][ell][nq2] fit in the (idle) field buffer: N^3 > 17 * 3 (N/2)^2 for N >= 16
  const int nq2 = mp3::nq2_count(p->n);
  double* H = reinterpret_cast<double*>(at(ws, L.fields));
  MP3_HIP(mp3::launch_fill_f64(H, (long long)p->batch * (ell_max + 1) * nq2, 0.0, st), "zero moments");
  MP3_HIP(mp3::launch_power_multipoles(p->prec, at(ws, L.dhat), p->n, nq2, ell_max, H, p->batch, p->phi, st),
          "power moments");
  double* dr = reinterpret_cast<double*>(at(ws, L.aux));
  MP3_HIP(hipMemcpyAsync(dr, radii, (size_t)nr * sizeof(double), hipMemcpyHostToDevice, st), "copy radii");
  const double n6 = (double)n3 * (double)n3;
  MP3_HIP(mp3::launch_xi_multipoles(H, nq2, ell_max, 2.0 * M_PI / p->box, p->smoothing, primary_smoothed(p), dr, nr, n6,
                                    xi, p->batch, st),
          "xi multipoles");
  return MP3_OK;
}

int mp3_reduced_3pcf(mp3_plan_t p, const void* delta, const double* zeta, int32_t lt, const double* mu, int32_t nth,
                     double* zeta_theta, double* q, void* ws, size_t wsb, void* stream) {
  if (int s = check_plan(p)) return s;
  if (!zeta || !mu || !zeta_theta) return fail(MP3_EINVAL, "zeta, mu and zeta_theta must not be NULL");
  if (q && !delta) return fail(MP3_EINVAL, "Q needs delta (for xi)");
  if (lt < 0 || lt > p->lmax) return fail(MP3_EINVAL, "need 0 <= lt <= lmax");
  if (nth < 1 || nth > kMaxAux) return fail(MP3_EINVAL, "nth must be in [1, 4096]");
  for (int i = 0; i < nth; ++i) {
    if (!std::isfinite(mu[i])) return fail(MP3_ENONFINITE, "mu must be finite");
    if (mu[i] < -1.0 || mu[i] > 1.0) return fail(MP3_EINVAL, "mu must lie in [-1, 1]");
  }
  const Layout L = layout(p);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n3 = (long long)p->n * p->n * p->n;
  double* dmu = reinterpret_cast<double*>(at(ws, L.aux));
  double* drb = dmu + kMaxAux;
  std::vector<double> rb(p->nbins);
  for (int b = 0; b < p->nbins; ++b) rb[b] = 0.5 * (p->edges[b] + p->edges[b + 1]);
  MP3_HIP(hipMemcpyAsync(dmu, mu, (size_t)nth * sizeof(double), hipMemcpyHostToDevice, st), "copy mu");
  MP3_HIP(hipMemcpyAsync(drb, rb.data(), (size_t)p->nbins * sizeof(double), hipMemcpyHostToDevice, st), "copy radii");
  const double n6 = (double)n3 * (double)n3;
  const int nq2 = mp3::nq2_count(p->n);
  const double kf = 2.0 * M_PI / p->box;
  const double* P = reinterpret_cast<const double*>(at(ws, L.pplain));
  double* xib = reinterpret_cast<double*>(at(ws, L.xib));
  if (q) {
    if (int s = check_finite(p, ws, L.flag, st, delta, n3 * p->batch, p->prec)) return s;
    if (int s = power_plain(p, delta, ws, L, st)) return s;
    MP3_HIP(mp3::launch_xi(P, nq2, kf, p->smoothing, primary_smoothed(p), drb, p->nbins, n6, xib, p->batch, st),
            "xi at the bins");
  }
  MP3_HIP(mp3::launch_reduced_3pcf(zeta, p->lmax, lt, p->nbins, dmu, nth, drb, xib, P, nq2, kf, p->smoothing,
                                   primary_smoothed(p), n6, zeta_theta, q, p->batch, st),
          "reduced 3PCF");
  return MP3_OK;
}

int mp3_ss_fields(mp3_plan_t p, const void* delta_d, const void* delta_r, void* f, void* r, void* stream) {
  if (int s = check_plan(p)) return s;
  if (!delta_d || !delta_r || !f || !r) return fail(MP3_EINVAL, "delta_d, delta_r, f and r must not be NULL");
  const long long n3 = (long long)p->n * p->n * p->n;
  MP3_HIP(mp3::launch_ss_fields(p->prec, delta_d, delta_r, f, r, n3 * p->batch, static_cast<hipStream_t>(stream)),
          "edge-corrected fields");
  return MP3_OK;
}

int mp3_ss_multipoles(mp3_plan_t p, const double* zeta_n, const double* zeta_r, int32_t lt, int32_t nquad,
                      double* zeta_ss, void* ws, size_t wsb, void* stream) {
  if (int s = check_plan(p)) return s;
  if (!zeta_n || !zeta_r || !zeta_ss) return fail(MP3_EINVAL, "zeta_n, zeta_r and zeta_ss must not be NULL");
  if (lt < 0 || lt > p->lmax) return fail(MP3_EINVAL, "need 0 <= lt <= lmax");
  if (nquad < 1 || nquad > kMaxAux) return fail(MP3_EINVAL, "nquad must be in [1, 4096]");
  const Layout L = layout(p);
  if (int s = check_ws(p, ws, wsb, L.total)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<double> xq, wq, both;
  mp3::gauss_legendre(nquad, xq, wq);
  both.insert(both.end(), xq.begin(), xq.end());
  both.insert(both.end(), wq.begin(), wq.end());
  double* dq = reinterpret_cast<double*>(at(ws, L.aux));
  MP3_HIP(hipMemcpyAsync(dq, both.data(), both.size() * sizeof(double), hipMemcpyHostToDevice, st), "copy nodes");
  MP3_HIP(mp3::launch_ss_multipoles(zeta_n, zeta_r, p->lmax, lt, p->nbins, dq, dq + nquad, nquad, zeta_ss, p->batch,
                                    st),
          "edge-corrected multipoles");
  return MP3_OK;
}

int mp3_sph_bessel(int32_t lmax, double x, double* out) {
  if (!out) return fail(MP3_EINVAL, "out is NULL");
  if (lmax < 0 || lmax > 64) return fail(MP3_EINVAL, "lmax must be in [0, 64]");
  if (!std::isfinite(x)) return fail(MP3_ENONFINITE, "x is not finite");
  if (x < 0.0) return fail(MP3_EINVAL, "x must be >= 0");
  mp3::sph_bessel_all(lmax, x, out);
  return MP3_OK;
}

int mp3_basis_tables(int32_t basis, int32_t n, double* table, size_t table_count, double* acf, double* phi_hat,
                     double* gamma) {
  if (basis != MP3_BASIS_BSPLINE3 && basis != MP3_BASIS_DAUBECHIES4) return fail(MP3_EINVAL, "unknown basis");
  if (phi_hat && !pow2_supported(n)) return fail(MP3_EUNSUPPORTED, "n must be one of 16, 32, 64, 128, 256, 512");
  if (basis == MP3_BASIS_BSPLINE3) {
    if (table) return fail(MP3_EINVAL, "the cubic B-spline has no tabulated values");
    if (gamma) {
      double g[7][7];
      mp3::b3_gamma(g);
      for (int s = 0; s < 7; ++s)
        for (int t = 0; t < 7; ++t) gamma[s * 7 + t] = g[s][t];
    }
    if (acf) {
      const double b7[4] = {2416.0 / 5040.0, 1191.0 / 5040.0, 120.0 / 5040.0, 1.0 / 5040.0};
      for (int s = 0; s < 4; ++s) acf[s] = b7[s];
    }
    if (phi_hat) {
      std::vector<double> ph;
      mp3::phi_hat_axis(n, ph);
      std::copy(ph.begin(), ph.end(), phi_hat);
    }
    return MP3_OK;
  }
  if (table && table_count != (size_t)mp3::kD4TableSize) return fail(MP3_EINVAL, "table_count must be 3073");
  if (table || acf) {
    std::vector<double> tab;
    mp3::d4_table(mp3::kD4Level, tab);
    if (table) std::copy(tab.begin(), tab.end(), table);
    if (acf) mp3::d4_autocorr(tab, mp3::kD4Level, acf);
  }
  if (phi_hat) {
    std::vector<double> ph;
    mp3::d4_phi_hat_axis(n, ph);
    std::copy(ph.begin(), ph.end(), phi_hat);
  }
  if (gamma) {
    double g[5][5];
    mp3::d4_gamma(g);
    for (int e = 0; e < 49; ++e) gamma[e] = 0.0;
    for (int s = 0; s < 5; ++s)
      for (int t = 0; t < 5; ++t) gamma[(s + 1) * 7 + t + 1] = g[s][t];
  }
  return MP3_OK;
}

int mp3_window_table(const mp3_plan_desc* d, double* out, size_t count) {
  if (!d || !out) return fail(MP3_EINVAL, "desc and out must not be NULL");
  if (int s = validate_desc(d)) return s;
  const size_t need = (size_t)(d->lmax + 1) * mp3::nq2_count(d->n) * d->nbins;
  if (count != need) return fail(MP3_EINVAL, "count must be (lmax+1) * nq2 * nbins = " + std::to_string(need));
  std::vector<double> edges(d->edges, d->edges + d->nbins + 1), jt;
  mp3::jbar_table(d->n, d->box, d->lmax, edges, jt, d->binning, d->smoothing);
  std::memcpy(out, jt.data(), need * sizeof(double));
  return MP3_OK;
}

}  // extern "C"
