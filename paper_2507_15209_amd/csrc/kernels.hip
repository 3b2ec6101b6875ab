// kernels.hip -- gfx950 kernels of the in-situ multipole 3PCF path.
//
// Data layout (per mock, per bin): complex fields of N^3 elements, index
// (ix * N + iy) * N + iz, batches of fields contiguous.  The inverse 3-D
// transform of each filtered field is done in three passes, one per axis:
//
//   pass y  (k_filter_y)   : k-space tile [qy column][16 or 8 contiguous qz] of
//                            dhat at fixed qx, read ONCE per (l, m); for every
//                            radial bin the window K_{lm,b} is applied and the
//                            y-transform done; writes field [qx][y][qz] per bin
//   pass x  (k_fft_strided): x-transform in place           -> [x][y][qz]
//   pass z  (k_zpass_*)    : per (x, y) pencil all bins are z-transformed into
//                            LDS and consumed there: nodal contraction
//                            (forward) or the adjoint source terms (backward)
//
// so a field element crosses HBM as: written by pass y, read+written by pass
// x, read by pass z (32 bytes per complex64 element in the forward).  The
// bin-looping kernels run along y, whose columns lie in one contiguous x-slab;
// the 512 KB-strided x axis is left to the one-field-per-tile plain pass.
#include "fft_core.hpp"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <type_traits>

namespace mp3 {

// contiguous complex values per strided-pass row: 128 bytes
template <typename T> constexpr int zc_of() { return 128 / (int)sizeof(c2<T>); }
// columns-tiles per workgroup so that small lengths still fill >= 256 threads
template <int N, typename T, int V = 0> constexpr int tiles_per_wg() {
  constexpr int t = Fft<N, V>::TPC * zc_of<T>();
  return t >= 256 ? 1 : 256 / t;
}

// LDS row stride (in complex elements) of a padded pencil: N plus one pad per
// 16 elements plus one, odd so that consecutive rows start in different banks
template <int N> constexpr int zrow() { return N + N / 16 + 1; }

// pencils per workgroup of the contiguous pass: fill 256 threads within 32 KB of LDS
template <int N, typename T> constexpr int contig_pencils() {
  constexpr int byt = zrow<N>() * (int)sizeof(c2<T>);
  constexpr int p = Fft<N>::TPC >= 256 ? 1 : 256 / Fft<N>::TPC;
  constexpr int cap = 32768 / byt;
  return p < cap ? p : (cap < 1 ? 1 : cap);
}

template <int N, typename T, int V = 0> constexpr int strided_threads() {
  return Fft<N, V>::TPC * zc_of<T>() * tiles_per_wg<N, T, V>();
}
// rows of the plain strided transforms (x pass, y and 3-D transforms): 256
// contiguous bytes, which HBM serves measurably faster than 128 in the
// in-place x pass, capped by N, 1024 threads and 64 KB of static LDS
template <int N, typename T, int V = 0> constexpr int zcx_of() {
  int z = 256 / (int)sizeof(c2<T>);
  if (z > N) z = N;
  while (z > 1 && (z * Fft<N, V>::TPC > 1024 || (long long)z * N * (long long)sizeof(c2<T>) > 65536)) z /= 2;
  return z;
}
template <int N, typename T, int V = 0> constexpr int tiles_x() {
  constexpr int t = Fft<N, V>::TPC * zcx_of<N, T, V>();
  return t >= 256 ? 1 : 256 / t;
}
template <int N, typename T, int V = 0> constexpr int strided_threads_x() {
  return Fft<N, V>::TPC * zcx_of<N, T, V>() * tiles_x<N, T, V>();
}
// plan variants by kernel (measured): radix 8 for the window passes and the
// nodal z pass; the adjoint z pass takes radix 16 in float32 and radix 8 in
// float64 (radix 16 spills there)
constexpr int VB = 1;
constexpr int VZN = 1;   // nodal z pass
template <typename T> constexpr int VZA = std::is_same<T, double>::value ? 1 : 0;   // adjoint z pass

__device__ __forceinline__ int sfreq(int i, int n) { return i < n / 2 ? i : i - n; }

// i^l conj(Y_lm(q_hat)) * scale for m >= 0, in float64.
// conj(Y_lm) = norm * Q_l^m(cos th) * (sin th e^{-i phi})^m with the reduced
// associated Legendre polynomial Q_l^m = P_l^m / (1 - x^2)^{m/2}
// (Condon-Shortley phase), which has no singularity at the poles.  At q = 0
// the direction is taken along +z (only m = 0 survives; the radial window
// then decides: jbar_{l>0}(0) = 0).
__device__ double2 ylm_conj_il(int qx, int qy, int qz, int l, int m, double norm, double scale, const YlmRec& yr) {
  const double q2 = (double)qx * qx + (double)qy * qy + (double)qz * qz;
  double x = 1.0, sre = 0.0, sim = 0.0;
  if (q2 > 0.0) {
    const double inv = 1.0 / sqrt(q2);
    x = qz * inv;
    sre = qx * inv;
    sim = -qy * inv;
  }
  const double pmm = yr.pmm;
  double q = pmm;
  if (l > m) {
    double p0 = pmm, p1 = x * (2.0 * m + 1.0) * pmm;
    for (int ll = m + 2; ll <= l; ++ll) {
      const double p2 = yr.c1[ll] * x * p1 - yr.c2[ll] * p0;
      p0 = p1;
      p1 = p2;
    }
    q = p1;
  }
  double cr = 1.0, ci = 0.0;
  for (int k = 0; k < m; ++k) {
    const double t = cr * sre - ci * sim;
    ci = cr * sim + ci * sre;
    cr = t;
  }
  const double a = norm * q * scale;
  double re = a * cr, im = a * ci;
  double2 r;
  switch (l & 3) {
    case 0: r.x = re; r.y = im; break;
    case 1: r.x = -im; r.y = re; break;
    case 2: r.x = -re; r.y = -im; break;
    default: r.x = im; r.y = -re; break;
  }
  return r;
}

// window factor at grid index (ix, iy, iz): i^l conj(Y) * scale with the
// Nyquist planes set to zero; also returns |q|^2 for the radial table
// phi != NULL: times the scaling function's power spectrum, a product of
// per-axis factors phi[ix] phi[iy] phi[iz] (Eq. SFC-3PCF-vertex)
template <typename T>
__device__ __forceinline__ c2<T> window_angular(int ix, int iy, int iz, int n, int l, int m, double norm,
                                                double scale, const YlmRec& yr, int& q2, const T* phi = nullptr) {
  const int qx = sfreq(ix, n), qy = sfreq(iy, n), qz = sfreq(iz, n);
  q2 = qx * qx + qy * qy + qz * qz;
  const int h = -n / 2;
  if (qx == h || qy == h || qz == h) return mk<T>((T)0, (T)0);
  double sc = scale;
  if (phi) sc *= (double)phi[ix] * (double)phi[iy] * (double)phi[iz];
  const double2 f = ylm_conj_il(qx, qy, qz, l, m, norm, sc, yr);
  return mk<T>((T)f.x, (T)f.y);
}

// streaming accesses: bulk data that is read or written once per pass goes
// through the caches with the non-temporal hint, so that the radial-window
// table (3.9 MB per l at 256^3, 20 bins) stays in L2
typedef double mp3_nt_d2 __attribute__((ext_vector_type(2)));
template <typename V> __device__ __forceinline__ void nt_store(V* p, V v) {
  if constexpr (sizeof(V) == 8) __builtin_nontemporal_store(__builtin_bit_cast(double, v), reinterpret_cast<double*>(p));
  else __builtin_nontemporal_store(__builtin_bit_cast(mp3_nt_d2, v), reinterpret_cast<mp3_nt_d2*>(p));
}
template <typename V> __device__ __forceinline__ V nt_load(const V* p) {
  if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const double*>(p)));
  else return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const mp3_nt_d2*>(p)));
}

// four consecutive radial-window values (the table's bin axis is padded to a
// multiple of four and 16-byte aligned per |q|^2 row)
template <typename T> __device__ __forceinline__ void load_quad(const T* p, T* o);
template <> __device__ __forceinline__ void load_quad<float>(const float* p, float* o) {
  const float4 q = *reinterpret_cast<const float4*>(p);
  o[0] = q.x; o[1] = q.y; o[2] = q.z; o[3] = q.w;
}
template <> __device__ __forceinline__ void load_quad<double>(const double* p, double* o) {
  const double2 a = reinterpret_cast<const double2*>(p)[0];
  const double2 b = reinterpret_cast<const double2*>(p)[1];
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

// copy the N twiddles to LDS (the multi-bin kernels reuse them for every bin)
template <int N, typename T>
__device__ __forceinline__ void stage_twiddles(const c2<T>* tw, c2<T>* tws) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) tws[i] = tw[i];
}

// ---------------------------------------------------------------------------
// fills and small reductions
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, long long count, T value) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    p[i] = value;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = warpSize / 2; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x % warpSize, wid = threadIdx.x / warpSize;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < (int)(blockDim.x + warpSize - 1) / warpSize; ++i) t += sh[i];
  }
  __syncthreads();
  return t;
}

// W[j] = sum of the weights of mock j (unit weights if w == nullptr)
// (times f[i] when f is given)
__global__ void k_weight_sum(const float* w, const double* f, const long long* off, int batch, double* W) {
  __shared__ double sh[32];
  const int j = blockIdx.y;
  const long long a = off[j], b = off[j + 1];
  double s = 0.0;
  for (long long i = a + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < b; i += (long long)gridDim.x * blockDim.x)
    s += (w ? (double)w[i] : 1.0) * (f ? f[i] : 1.0);
  s = block_sum(s, sh);
  if (threadIdx.x == 0 && s != 0.0) atomicAdd(&W[j], s);
}

// S[j] = sum_x (1 + delta_x) g_x for mock j
template <typename T>
__global__ void k_dot_rho_g(const T* delta, const T* g, long long n3, double* S) {
  __shared__ double sh[32];
  const int j = blockIdx.y;
  const T* d = delta + j * n3;
  const T* gg = g + j * n3;
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n3; i += (long long)gridDim.x * blockDim.x)
    s += (1.0 + (double)d[i]) * (double)gg[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) atomicAdd(&S[j], s);
}

// ---------------------------------------------------------------------------
// deposit: cubic B-spline, 4 taps per axis, periodic, float64 coordinates
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_mock(const long long* off, int batch, long long i) {
  int lo = 0, hi = batch;  // off[lo] <= i < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

struct Taps {
  int base[3];
  double wt[3][4];
  double f[3];     // fractional position in the cell
  bool ok;
};

// Daubechies-4: phi at x by linear interpolation of its values at the dyadic
// points i / 2^kD4Level of [0, 3] (tab), zero outside [0, 3)
__device__ __forceinline__ double d4_phi(const double* tab, double x) {
  if (!(x >= 0.0) || x >= 3.0) return 0.0;
  const double s = x * (double)(1 << kD4Level);
  const double fl = floor(s);
  const int i = (int)fl;
  const double fr = s - fl;
  return (1.0 - fr) * tab[i] + fr * tab[i + 1];
}

// Stencil of a particle: nodes base .. base + 3 per axis (base = floor(u) - 1)
// with the cubic B-spline weights B3(u - node), or with btab (Daubechies-4,
// node l carrying phi(u - l + 1)) the weights phi(f + 2 - a), the last zero.
__device__ __forceinline__ Taps make_taps(const float* p, int n, double sc, const double* btab) {
  Taps t;
  t.ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double u = (double)p[d] * sc;
    if (!(u == u) || fabs(u) > 1e15) { t.ok = false; u = 0.0; }
    u -= (double)n * floor(u / (double)n);          // periodic wrap into [0, n]
    double fl = floor(u);
    double f = u - fl;
    int ib = (int)fl;
    if (ib >= n) { ib -= n; }
    t.base[d] = ib - 1;
    t.f[d] = f;
    if (btab) {
#pragma unroll
      for (int a = 0; a < 4; ++a) t.wt[d][a] = d4_phi(btab, f + 2.0 - (double)a);
    } else {
      const double g = 1.0 - f;
      t.wt[d][0] = g * g * g / 6.0;
      t.wt[d][1] = (4.0 - 6.0 * f * f + 3.0 * f * f * f) / 6.0;
      t.wt[d][2] = (4.0 - 6.0 * g * g + 3.0 * g * g * g) / 6.0;
      t.wt[d][3] = f * f * f / 6.0;
    }
  }
  return t;
}

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T>
__global__ void k_normalise(T* eps, const double* W, long long n3) {
  const int j = blockIdx.y;
  const double f = (double)n3 / W[j];
  T* e = eps + j * n3;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n3; i += (long long)gridDim.x * blockDim.x)
    e[i] = (T)((double)e[i] * f - 1.0);
}

// dw_i = (N^3 / W) sum_taps B g - S / W
template <typename T>
__global__ void k_gather_dw(const float* pos, const long long* off, int batch, long long np_total, int n, double sc,
                            const T* g, const double* W, const double* S, T* dw, const double* btab) {
  const long long n3 = (long long)n * n * n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < np_total; i += (long long)gridDim.x * blockDim.x) {
    const int mock = find_mock(off, batch, i);
    Taps t = make_taps(pos + 3 * i, n, sc, btab);
    double acc = 0.0;
    if (t.ok) {
      const T* gg = g + mock * n3;
      for (int a = 0; a < 4; ++a) {
        const int ix = wrapi(t.base[0] + a, n);
        for (int b = 0; b < 4; ++b) {
          const int iy = wrapi(t.base[1] + b, n);
          const long long row = ((long long)ix * n + iy) * n;
          const double wab = t.wt[0][a] * t.wt[1][b];
          double s = 0.0;
          for (int c = 0; c < 4; ++c) s += t.wt[2][c] * (double)gg[row + wrapi(t.base[2] + c, n)];
          acc += wab * s;
        }
      }
    }
    const double Wj = W[mock];
    dw[i] = (T)((double)n3 / Wj * acc - S[mock] / Wj);
  }
}

// ---------------------------------------------------------------------------
// FFT along a strided axis (x: astride = N^2, outer = N; y: astride = N, outer = N^2);
// the twiddles are staged in LDS while the column loads are in flight
// ---------------------------------------------------------------------------
template <int N, typename T, int DIR, bool REAL_IN, int V = 0>
__global__ void __launch_bounds__((strided_threads_x<N, T, V>())) k_fft_strided(const void* in, c2<T>* out, long long fstride_in,
                                                       long long fstride_out, int astride, int outer, const c2<T>* tw) {
  using F = Fft<N, V>;
  constexpr int ZC = zcx_of<N, T, V>();
  constexpr int G = tiles_x<N, T, V>();
  constexpr int RMAX = F::RMAX;
  extern __shared__ __align__(16) char smem_x[];
  c2<T>* lds = reinterpret_cast<c2<T>*>(smem_x);
  c2<T>* tws = lds + G * N * ZC;
  const int tid = threadIdx.x;
  const int cc = tid % ZC;
  const int j = (tid / ZC) % F::TPC;
  const int g = tid / (ZC * F::TPC);
  const int tile = blockIdx.x * G + g;
  constexpr int chunks = N / ZC;
  const bool active = tile < N * chunks;
  const int o = active ? tile / chunks : 0;
  const int ch = active ? tile % chunks : 0;
  const long long base = (long long)o * outer + ch * ZC + cc;
  const long long f = blockIdx.y;
  c2<T> v[RMAX];
  if (active) {
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      const long long idx = f * fstride_in + base + (long long)F::in_index(j, r) * astride;
      if (REAL_IN) v[r] = mk<T>(static_cast<const T*>(in)[idx], (T)0);
      else v[r] = static_cast<const c2<T>*>(in)[idx];
    }
  }
  stage_twiddles<N, T>(tw, tws);
  __syncthreads();
  fft_column<N, DIR, T, false, V>(v, lds + g * N * ZC + cc, ZC, j, tws, active);
  if (active) {
#pragma unroll
    for (int e = 0; e < RMAX; ++e)
      out[f * fstride_out + base + (long long)F::out_index(j, e) * astride] = v[e];
  }
}

// FFT along the contiguous axis z, one pencil per TPC threads
template <int N, typename T, int DIR>
__global__ void __launch_bounds__((contig_pencils<N, T>() * Fft<N>::TPC)) k_fft_contig(const c2<T>* in, c2<T>* out, long long npencils, const c2<T>* tw) {
  using F = Fft<N>;
  constexpr int P = contig_pencils<N, T>();
  constexpr int RS = zrow<N>();
  constexpr int RMAX = F::RMAX;
  __shared__ c2<T> lds[P * RS];
  const int tid = threadIdx.x;
  const int j = tid % F::TPC;
  const int p = tid / F::TPC;
  const long long pen = (long long)blockIdx.x * P + p;
  const bool active = pen < npencils;
  c2<T> v[RMAX];
  if (active) {
#pragma unroll
    for (int r = 0; r < RMAX; ++r) v[r] = in[pen * N + F::in_index(j, r)];
  }
  fft_column<N, DIR, T, true, 0, 64 % Fft<N>::TPC == 0>(v, lds + p * RS, 1, j, tw, active);
  if (active) {
#pragma unroll
    for (int e = 0; e < RMAX; ++e) out[pen * N + F::out_index(j, e)] = v[e];
  }
}

// ---------------------------------------------------------------------------
// first pass of the forward: window K_{lm,b} on the k-space tile, all bins,
// transform along y
// ---------------------------------------------------------------------------
template <int N, typename T>
__global__ void __launch_bounds__((strided_threads<N, T, VB>())) k_filter_y(const c2<T>* dhat, c2<T>* fields,
                                                                         const T* jtab, int jmocks, int nq2, int nbins,
                                                                         int nbp, const ItemRec* items, int item0,
                                                                         int batch, double scale, const c2<T>* tw,
                                                                         const T* phi) {
  using F = Fft<N, VB>;
  constexpr int ZC = zc_of<T>();
  constexpr int G = tiles_per_wg<N, T, VB>();
  constexpr int RMAX = F::RMAX;
  constexpr long long N3 = (long long)N * N * N;
  __shared__ c2<T> lds[G * N * ZC];
  __shared__ c2<T> tws[N];
  const int tid = threadIdx.x;
  const int cc = tid % ZC;
  const int j = (tid / ZC) % F::TPC;
  const int g = tid / (ZC * F::TPC);
  const int tile = blockIdx.x * G + g;
  constexpr int chunks = N / ZC;
  const bool active = tile < N * chunks;
  const int qx = active ? tile / chunks : 0;
  const int qz = (active ? tile % chunks : 0) * ZC + cc;
  // grid.y runs over (item of the group, mock)
  const long long mock = blockIdx.y % batch;
  const int gi = blockIdx.y / batch;
  const ItemRec& it = items[item0 + gi];
  stage_twiddles<N, T>(tw, tws);
  __syncthreads();
  c2<T> v0[RMAX];
  int q2[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    const int qy = F::in_index(j, r);
    const c2<T> d = active ? nt_load(&dhat[mock * N3 + ((long long)qx * N + qy) * N + qz]) : mk<T>(0, 0);
    const c2<T> f = window_angular<T>(qx, qy, qz, N, it.l, it.m, it.norm, scale, it.yr, q2[r], phi);
    v0[r] = cmul<T>(d, f);
  }
  // radial window of this thread's elements, four bins per load, one quad
  // ahead (jmocks tables per l: one, or one per mock in the cotangent's eigenbasis)
  const T* jl = jtab + ((long long)it.l * jmocks + mock % jmocks) * nq2 * nbp;
  T jq[RMAX][4];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) load_quad<T>(jl + (long long)q2[r] * nbp, jq[r]);
  c2<T>* fbase = fields + ((long long)gi * batch + mock) * nbins * N3 + (long long)qx * N * N + qz;
  for (int bq = 0; bq < nbins; bq += 4) {
    T jn[RMAX][4];
    if (bq + 4 < nbins) {
#pragma unroll
      for (int r = 0; r < RMAX; ++r) load_quad<T>(jl + (long long)q2[r] * nbp + bq + 4, jn[r]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (bq + k < nbins) {
        c2<T> v[RMAX];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) v[r] = cscale<T>(v0[r], jq[r][k]);
        int jj = j;
        asm volatile("" : "+v"(jj));
        fft_column<N, +1, T, false, VB>(v, lds + g * N * ZC + cc, ZC, jj, tws, active);
        if (active) {
          c2<T>* out = fbase + (bq + k) * N3;
#pragma unroll
          for (int e = 0; e < RMAX; ++e) nt_store(&out[F::out_index(jj, e) * N], v[e]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) jq[r][k] = jn[r][k];
  }
}

// ---------------------------------------------------------------------------
// pass z of the forward: z-transform of every bin of a pencil into LDS, then
// the nodal contraction  P[b1,b2] += sum_z delta_z Re(a_b1 conj(a_b2))
// in 4x4 register blocks (float32 per pencil, float64 across pencils).
// ---------------------------------------------------------------------------
struct PairBlocks {
  int nblk, npb, zch;
  __device__ void init(int nbins, int nthreads) {
    nblk = (nbins + 3) / 4;
    npb = nblk * (nblk + 1) / 2;
    zch = nthreads / npb;
    if (zch < 1) zch = 1;
  }
  __device__ void block_of(int beta, int& b1, int& b2) const {
    int r = 0, rem = beta;
    while (rem >= nblk - r) { rem -= nblk - r; ++r; }
    b1 = r;
    b2 = r + rem;
  }
};

// Bins of a pencil are transformed in rounds of nbc = blockDim / TPC columns.
template <int N, int V>
__device__ __forceinline__ int pencil_rounds(int nbins) {
  const int nbc = blockDim.x / Fft<N, V>::TPC;
  return (nbins + nbc - 1) / nbc;
}

// Load round rr of a pencil: thread (bin b = rr * nbc + tid / TPC, j) loads its
// column's first-stage elements.
template <int N, typename T, int V>
__device__ __forceinline__ void load_pencil_round(const c2<T>* src, long long fstride, int nbins, int rr,
                                                  c2<T>* v) {
  using F = Fft<N, V>;
  const int nbc = blockDim.x / F::TPC;
  const int b = rr * nbc + threadIdx.x / F::TPC;
  const int j = threadIdx.x % F::TPC;
  if (b < nbins) {
#pragma unroll
    for (int r = 0; r < F::RMAX; ++r) v[r] = src[b * fstride + F::in_index(j, r)];
  }
}

// Rounds prefetched into registers ahead of use: one with radix-16 columns
// (16 values per thread), two with radix-8 columns.
template <int N, int V> constexpr int prefetch_rounds() { return Fft<N, V>::RMAX >= 16 ? 1 : 2; }

template <int N, typename T, int V>
__device__ __forceinline__ void prefetch_pencil(const c2<T>* src, long long fstride, int nbins,
                                                c2<T> (*vpre)[Fft<N, V>::RMAX]) {
  const int rounds = pencil_rounds<N, V>(nbins);
  load_pencil_round<N, T, V>(src, fstride, nbins, 0, vpre[0]);
  if constexpr (prefetch_rounds<N, V>() > 1) {
    if (rounds > 1) load_pencil_round<N, T, V>(src, fstride, nbins, 1, vpre[1]);
  }
}

// the z-pass workgroup has at least N threads (zpass_threads), so thread
// z = tid owns one value of a real pencil (DPRE = 1)
constexpr int DPRE = 1;
template <int N, typename T>
__device__ __forceinline__ void prefetch_delta(const T* src, T* d) {
#pragma unroll
  for (int k = 0; k < DPRE; ++k) {
    const int z = threadIdx.x + k * blockDim.x;
    d[k] = z < N ? src[z] : (T)0;
  }
}

// z-transform one round of bins of a pencil into LDS rows A[b] (padded).
template <int N, typename T, int V>
__device__ __forceinline__ void transform_round(int nbins, int rr, c2<T>* v, c2<T>* A, const c2<T>* tw) {
  using F = Fft<N, V>;
  constexpr int RS = zrow<N>();
  const int nbc = blockDim.x / F::TPC;
  int j = threadIdx.x % F::TPC;
  // keep per-thread LDS index arithmetic inside the pencil loop: hoisting it
  // out of the loop would pin dozens of registers for the whole kernel
  asm volatile("" : "+v"(j));
  const int b = rr * nbc + threadIdx.x / F::TPC;
  const bool active = b < nbins;
  fft_column<N, +1, T, true, V, 64 % Fft<N, V>::TPC == 0>(v, A + (active ? b : 0) * RS, 1, j, tw, active);
  if (active) {
#pragma unroll
    for (int e = 0; e < F::RMAX; ++e) A[b * RS + lds_pos<true>(F::out_index(j, e))] = v[e];
  }
}

// z-transform every bin of one pencil into LDS rows A[b]; rounds 0 and 1
// come from the prefetched registers.
template <int N, typename T, int V>
__device__ __forceinline__ void transform_pencil_bins(const c2<T>* src, long long fstride, int nbins, c2<T>* A,
                                                      const c2<T>* tw, c2<T> (*vpre)[Fft<N, V>::RMAX]) {
  constexpr int PR = prefetch_rounds<N, V>();
  const int rounds = pencil_rounds<N, V>(nbins);
  transform_round<N, T, V>(nbins, 0, vpre[0], A, tw);
  if constexpr (PR > 1) {
    if (rounds > 1) transform_round<N, T, V>(nbins, 1, vpre[1], A, tw);
  }
  for (int rr = PR; rr < rounds; ++rr) {
    c2<T> v[Fft<N, V>::RMAX];
    load_pencil_round<N, T, V>(src, fstride, nbins, rr, v);
    transform_round<N, T, V>(nbins, rr, v, A, tw);
  }
}

typedef float mp3_f4 __attribute__((ext_vector_type(4)));

// Nodal contraction on the matrix cores (float32, nbins <= 32): per pair of z,
// one v_mfma_f32_16x16x4f32 per upper-triangular 16x16 block of (b1, b2),
// k = (z, re/im):  A[b1][k] = delta_z c_k(a_b1(z)),  B[k][b2] = c_k(a_b2(z)).
// Lane l supplies A[l%16][l/16] and B[l/16][l%16]; D register i of lane l is
// C[4 (l/16) + i][l%16].
struct MfmaAcc {
  mp3_f4 c00, c01, c11;
};

__device__ __forceinline__ void mfma_contract_pencil(const float2* A, const float* dl, int nbins, int RS, int N,
                                                     MfmaAcc& acc) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int zz = kq >> 1, comp = kq & 1;
  const bool two = nbins > 16;
  const bool ok0 = col < nbins, ok1 = 16 + col < nbins;
  // lanes of bins beyond nbins read row 0 (finite values): they only feed
  // entries of P that the reduction drops, and the loads need no mask
  const float* r0 = reinterpret_cast<const float*>(A + (ok0 ? col : 0) * RS) + comp;
  const float* r1 = reinterpret_cast<const float*>(A + (ok1 ? 16 + col : 0) * RS) + comp;
  for (int zp = w; zp < N / 2; zp += nw) {
    const int z = 2 * zp + zz;
    const int off = 2 * lds_pos<true>(z);
    const float d = dl[z];
    const float v0 = r0[off];
    acc.c00 = __builtin_amdgcn_mfma_f32_16x16x4f32(d * v0, v0, acc.c00, 0, 0, 0);
    if (two) {
      const float v1 = r1[off];
      acc.c01 = __builtin_amdgcn_mfma_f32_16x16x4f32(d * v0, v1, acc.c01, 0, 0, 0);
      acc.c11 = __builtin_amdgcn_mfma_f32_16x16x4f32(d * v1, v1, acc.c11, 0, 0, 0);
    }
  }
}

// the same for z in [z0, z1) (even bounds), all by the calling wave
__device__ __forceinline__ void mfma_contract_pencil_range(const float2* A, const float* dl, int nbins, int RS, int z0,
                                                           int z1, MfmaAcc& acc) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  const int zz = kq >> 1, comp = kq & 1;
  const bool two = nbins > 16;
  const bool ok0 = col < nbins, ok1 = 16 + col < nbins;
  // lanes of bins beyond nbins read row 0 (finite values): they only feed
  // entries of P that the reduction drops, and the loads need no mask
  const float* r0 = reinterpret_cast<const float*>(A + (ok0 ? col : 0) * RS) + comp;
  const float* r1 = reinterpret_cast<const float*>(A + (ok1 ? 16 + col : 0) * RS) + comp;
#pragma unroll 8
  for (int zp = z0 / 2; zp < z1 / 2; ++zp) {
    const int z = 2 * zp + zz;
    const int off = 2 * lds_pos<true>(z);
    const float d = dl[z];
    const float v0 = r0[off];
    acc.c00 = __builtin_amdgcn_mfma_f32_16x16x4f32(d * v0, v0, acc.c00, 0, 0, 0);
    if (two) {
      const float v1 = r1[off];
      acc.c01 = __builtin_amdgcn_mfma_f32_16x16x4f32(d * v0, v1, acc.c01, 0, 0, 0);
      acc.c11 = __builtin_amdgcn_mfma_f32_16x16x4f32(d * v1, v1, acc.c11, 0, 0, 0);
    }
  }
}

// 17..20 bins: the 15 upper-triangle 4x4 blocks (g1 <= g2 of 5 bin groups)
// of P on v_mfma_f32_4x4x1f32, 16 independent 4x4 outer products per
// instruction, one instruction per k = (z, re/im): a third of the matrix-core
// cycles of three 16x16 blocks.  K must be even.  Lane l supplies A[4 g1 + l%4][k] of block
// beta = l/4 and B[k][4 g2 + l%4]; D register i of lane l is block l/4, row i,
// column l%4.  Block 15 is idle.
__device__ __forceinline__ void pair_group(int beta, int& g1, int& g2) {
  // beta = 0..14 over (g1, g2), 0 <= g1 <= g2 < 5, row-major
  int r = 0, rem = beta;
  while (rem >= 5 - r) { rem -= 5 - r; ++r; }
  g1 = r;
  g2 = r + rem;
}

__device__ __forceinline__ void mfma_contract_4x4(const float2* A, const float* dl, int nbins, int RS, int K,
                                                  MfmaAcc& acc) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int beta = lane >> 2, i = lane & 3;
  int g1 = 0, g2 = 0;
  if (beta < 15) pair_group(beta, g1, g2);
  const int ba = 4 * g1 + i, bb = 4 * g2 + i;
  const bool oka = beta < 15 && ba < nbins, okb = beta < 15 && bb < nbins;
  // lanes of block 15 and of bins beyond nbins read row 0 (finite values):
  // they only feed entries of P that the reduction drops, so no load is masked
  const float2* ra = A + (oka ? ba : 0) * RS;
  const float2* rb = A + (okb ? bb : 0) * RS;
  // three accumulators in rotation keep dependent matrix-core issues apart
  for (int z = 2 * w; z < K; z += 2 * nw) {
    const int zp0 = lds_pos<true>(z), zp1 = lds_pos<true>(z + 1);
    const float d0 = dl[z], d1 = dl[z + 1];
    const float2 u0 = ra[zp0], v0 = rb[zp0], u1 = ra[zp1], v1 = rb[zp1];
    acc.c00 = __builtin_amdgcn_mfma_f32_4x4x1f32(d0 * u0.x, v0.x, acc.c00, 0, 0, 0);
    acc.c01 = __builtin_amdgcn_mfma_f32_4x4x1f32(d0 * u0.y, v0.y, acc.c01, 0, 0, 0);
    acc.c11 = __builtin_amdgcn_mfma_f32_4x4x1f32(d1 * u1.x, v1.x, acc.c11, 0, 0, 0);
    acc.c00 = __builtin_amdgcn_mfma_f32_4x4x1f32(d1 * u1.y, v1.y, acc.c00, 0, 0, 0);
  }
}

// the same for z in [z0, z1) (even bounds), all by the calling wave
__device__ __forceinline__ void mfma_contract_4x4_range(const float2* A, const float* dl, int nbins, int RS, int z0,
                                                        int z1, MfmaAcc& acc) {
  const int lane = threadIdx.x & 63;
  const int beta = lane >> 2, i = lane & 3;
  int g1 = 0, g2 = 0;
  if (beta < 15) pair_group(beta, g1, g2);
  const int ba = 4 * g1 + i, bb = 4 * g2 + i;
  const bool oka = beta < 15 && ba < nbins, okb = beta < 15 && bb < nbins;
  // lanes of block 15 and of bins beyond nbins read row 0 (finite values):
  // they only feed entries of P that the reduction drops, so no load is masked
  const float2* ra = A + (oka ? ba : 0) * RS;
  const float2* rb = A + (okb ? bb : 0) * RS;
#pragma unroll 8
  for (int z = z0; z < z1; z += 2) {
    const int zp0 = lds_pos<true>(z), zp1 = lds_pos<true>(z + 1);
    const float d0 = dl[z], d1 = dl[z + 1];
    const float2 u0 = ra[zp0], v0 = rb[zp0], u1 = ra[zp1], v1 = rb[zp1];
    acc.c00 = __builtin_amdgcn_mfma_f32_4x4x1f32(d0 * u0.x, v0.x, acc.c00, 0, 0, 0);
    acc.c01 = __builtin_amdgcn_mfma_f32_4x4x1f32(d0 * u0.y, v0.y, acc.c01, 0, 0, 0);
    acc.c11 = __builtin_amdgcn_mfma_f32_4x4x1f32(d1 * u1.x, v1.x, acc.c11, 0, 0, 0);
    acc.c00 = __builtin_amdgcn_mfma_f32_4x4x1f32(d1 * u1.y, v1.y, acc.c00, 0, 0, 0);
  }
}

// BF16-split variant: every float operand x is carried as hi = bf16(x) and
// lo = bf16(x - hi) and each product as hi*hi + hi*lo + lo*hi on the bf16
// matrix cores (v_mfma_f32_16x16x16bf16_1k, k = 8 z values x (re, im) per
// instruction), accumulating in float32.  The dropped lo*lo term and the
// rounding of lo leave a relative error of about 2^-16 per product.
typedef short mp3_s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_float(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ void bf16_split4(const float* x, mp3_s4& hi, mp3_s4& lo) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned short h = bf16_rne(x[i]);
    hi[i] = (short)h;
    lo[i] = (short)bf16_rne(x[i] - bf16_to_float(h));
  }
}

__device__ __forceinline__ mp3_f4 mfma3(const mp3_s4& ah, const mp3_s4& al, const mp3_s4& bh, const mp3_s4& bl,
                                        mp3_f4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
  return c;
}

// K must be a multiple of 8.  Lane l supplies A[l%16][4 (l/16) + j] and
// B[4 (l/16) + j][l%16], j = 0..3: k = 2 (z - z0) + comp over z = z0 + 2 (l/16) + {0, 1}.
__device__ __forceinline__ void mfma_contract_bf16x3(const float2* A, const float* dl, int nbins, int RS, int K,
                                                     MfmaAcc& acc) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const bool two = nbins > 16;
  const bool ok0 = col < nbins, ok1 = 16 + col < nbins;
  const float2* r0 = A + col * RS;
  const float2* r1 = A + (16 + col) * RS;
  for (int zc = w; zc < K / 8; zc += nw) {
    const int z = 8 * zc + 2 * kq;
    const int p0 = lds_pos<true>(z), p1 = lds_pos<true>(z + 1);
    const float d0 = dl[z], d1 = dl[z + 1];
    float2 u0 = ok0 ? r0[p0] : make_float2(0.f, 0.f);
    float2 u1 = ok0 ? r0[p1] : make_float2(0.f, 0.f);
    float xa[4] = {d0 * u0.x, d0 * u0.y, d1 * u1.x, d1 * u1.y};
    float xb[4] = {u0.x, u0.y, u1.x, u1.y};
    mp3_s4 ah, al, bh, bl;
    bf16_split4(xa, ah, al);
    bf16_split4(xb, bh, bl);
    acc.c00 = mfma3(ah, al, bh, bl, acc.c00);
    if (two) {
      u0 = ok1 ? r1[p0] : make_float2(0.f, 0.f);
      u1 = ok1 ? r1[p1] : make_float2(0.f, 0.f);
      float ya[4] = {d0 * u0.x, d0 * u0.y, d1 * u1.x, d1 * u1.y};
      float yb[4] = {u0.x, u0.y, u1.x, u1.y};
      mp3_s4 ch, cl, dh, dlo;
      bf16_split4(ya, ch, cl);
      bf16_split4(yb, dh, dlo);
      acc.c01 = mfma3(ah, al, dh, dlo, acc.c01);
      acc.c11 = mfma3(ch, cl, dh, dlo, acc.c11);
    }
  }
}

// Per-workgroup accumulator of  P[b1,b2] = sum_k w_k Re(a_b1(k) conj(a_b2(k)))
// over LDS rows A[b * RS + lds_pos(k)], either on the matrix cores (MF) or in
// 4x4 register blocks on the vector ALUs.  Partial sums stay in the working
// precision over the workgroup's slices and are written as float64.
// QUAD: 4x4 blocks on the matrix cores (float32 inputs, 17..20 bins)
template <typename T, bool MF, bool SPLIT = false, bool QUAD = false>
struct Contractor {
  static __host__ __device__ bool quad(int) { return QUAD; }
  PairBlocks pb;
  int bb1 = 0, bb2 = 0, zc = 0;
  bool has_item = false;
  T acc[MF ? 1 : 16];
  MfmaAcc macc;

  __device__ void init(int nbins) {
    pb.init(nbins, blockDim.x);
    has_item = !MF && (int)threadIdx.x < pb.npb * pb.zch;
    if (has_item) {
      pb.block_of(threadIdx.x / pb.zch, bb1, bb2);
      zc = threadIdx.x % pb.zch;
    }
#pragma unroll
    for (int i = 0; i < (MF ? 1 : 16); ++i) acc[i] = (T)0;
    macc.c00 = mp3_f4{0.f, 0.f, 0.f, 0.f};
    macc.c01 = macc.c00;
    macc.c11 = macc.c00;
  }

  // K positions (even), weights w[k] in LDS
  __device__ void add(const c2<T>* A, const T* w, int nbins, int RS, int K) {
    if constexpr (MF && SPLIT) {
      mfma_contract_bf16x3(reinterpret_cast<const float2*>(A), reinterpret_cast<const float*>(w), nbins, RS, K, macc);
    } else if constexpr (MF && QUAD) {
      mfma_contract_4x4(reinterpret_cast<const float2*>(A), reinterpret_cast<const float*>(w), nbins, RS, K, macc);
    } else if constexpr (MF) {
      mfma_contract_pencil(reinterpret_cast<const float2*>(A), reinterpret_cast<const float*>(w), nbins, RS, K, macc);
    } else if (has_item) {
      const int b1o = 4 * bb1, b2o = 4 * bb2;
      for (int z = zc; z < K; z += pb.zch) {
        const T d = w[z];
        const int zp = lds_pos<true>(z);
        c2<T> x1[4], x2[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          x1[i] = (b1o + i < nbins) ? A[(b1o + i) * RS + zp] : mk<T>(0, 0);
          x2[i] = (b2o + i < nbins) ? A[(b2o + i) * RS + zp] : mk<T>(0, 0);
          x1[i] = cscale<T>(x1[i], d);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[i * 4 + k] += x1[i].x * x2[k].x + x1[i].y * x2[k].y;
      }
    }
  }

  // matrix-core forms only: z in [z0, z1) by the calling wave alone
  __device__ void add_range(const c2<T>* A, const T* w, int nbins, int RS, int z0, int z1) {
    static_assert(MF && !SPLIT, "range contraction: matrix-core float32 forms");
    if constexpr (QUAD)
      mfma_contract_4x4_range(reinterpret_cast<const float2*>(A), reinterpret_cast<const float*>(w), nbins, RS, z0, z1,
                              macc);
    else
      mfma_contract_pencil_range(reinterpret_cast<const float2*>(A), reinterpret_cast<const float*>(w), nbins, RS, z0,
                                 z1, macc);
  }

  // LDS bytes finish() needs as scratch
  static __host__ __device__ size_t scratch_bytes(int threads) {
    return MF ? (size_t)(threads / 64) * 3 * 256 * sizeof(double) : (size_t)threads * 16 * sizeof(double);
  }

  // workgroup reduction through LDS scratch red, symmetric partial to out[nbins^2]
  __device__ void finish(double* red, double* out, int nbins) {
    const int tid = threadIdx.x;
    if constexpr (MF && QUAD) {
      // red[w][beta][row][col] for the 15 (g1, g2) 4x4 blocks
      const int lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        red[(w * 16 + (lane >> 2)) * 16 + i * 4 + (lane & 3)] =
            (double)macc.c00[i] + (double)macc.c01[i] + (double)macc.c11[i];
      __syncthreads();
      for (int t = tid; t < 15 * 16; t += blockDim.x) {
        const int beta = t / 16, row = (t / 4) % 4, col = t % 4;
        double sacc = 0.0;
        for (int ww = 0; ww < nw; ++ww) sacc += red[(ww * 16 + beta) * 16 + row * 4 + col];
        int g1, g2;
        pair_group(beta, g1, g2);
        const int b1 = 4 * g1 + row, b2 = 4 * g2 + col;
        // diagonal blocks hold both orders of a pair: keep b1 <= b2 and mirror
        if (b1 < nbins && b2 < nbins && b1 <= b2) {
          out[b1 * nbins + b2] = sacc;
          out[b2 * nbins + b1] = sacc;
        }
      }
    } else if constexpr (MF) {
      // red[w][blk][row][col], blk 0 = (0,0), 1 = (0,1), 2 = (1,1)
      const int lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 4 * (lane >> 4) + i, col = lane & 15;
        red[((w * 3 + 0) * 16 + row) * 16 + col] = (double)macc.c00[i];
        red[((w * 3 + 1) * 16 + row) * 16 + col] = (double)macc.c01[i];
        red[((w * 3 + 2) * 16 + row) * 16 + col] = (double)macc.c11[i];
      }
      __syncthreads();
      for (int t = tid; t < 3 * 256; t += blockDim.x) {
        const int blk = t / 256, row = (t / 16) % 16, col = t % 16;
        double sacc = 0.0;
        for (int ww = 0; ww < nw; ++ww) sacc += red[((ww * 3 + blk) * 16 + row) * 16 + col];
        const int b1 = row + (blk == 2 ? 16 : 0), b2 = col + (blk >= 1 ? 16 : 0);
        if (b1 < nbins && b2 < nbins && b1 <= b2) {
          out[b1 * nbins + b2] = sacc;
          out[b2 * nbins + b1] = sacc;
        }
      }
    } else {
      if (has_item) {
#pragma unroll
        for (int i = 0; i < 16; ++i) red[tid * 16 + i] = (double)acc[i];
      }
      __syncthreads();
      for (int t = tid; t < pb.npb * 16; t += blockDim.x) {
        const int beta = t / 16, ik = t % 16;
        double sacc = 0.0;
        for (int c = 0; c < pb.zch; ++c) sacc += red[(beta * pb.zch + c) * 16 + ik];
        int c1, c2b;
        pb.block_of(beta, c1, c2b);
        const int b1 = 4 * c1 + ik / 4, b2 = 4 * c2b + ik % 4;
        // diagonal blocks hold both orders of a pair: keep b1 <= b2 and mirror,
        // so the partial is exactly symmetric
        if (b1 < nbins && b2 < nbins && b1 <= b2) {
          out[b1 * nbins + b2] = sacc;
          out[b2 * nbins + b1] = sacc;
        }
      }
    }
  }
};

template <int N, typename T, bool MF, bool SPLIT = false, bool QUAD = false>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(MF ? 4 : 1))) k_zpass_nodal(
    const c2<T>* fields, const T* delta, double* partials, int nbins, int ppw, const c2<T>* tw) {
  using F = Fft<N, VZN>;
  constexpr int RS = zrow<N>();
  constexpr long long N3 = (long long)N * N * N;
  extern __shared__ __align__(16) char smem[];
  c2<T>* A = reinterpret_cast<c2<T>*>(smem);
  c2<T>* tws = A + nbins * RS;
  T* dl = reinterpret_cast<T*>(tws + N);
  const int tid = threadIdx.x;
  const long long mock = blockIdx.y;
  stage_twiddles<N, T>(tw, tws);
  Contractor<T, MF, SPLIT, QUAD> ctr;
  ctr.init(nbins);
  const int p0 = blockIdx.x * ppw;
  const int p1 = min(p0 + ppw, N * N);
  const c2<T>* fmock = fields + mock * nbins * N3;
  c2<T> vpre[prefetch_rounds<N, VZN>()][F::RMAX];
  T dpre[DPRE];
  const T* dmock = delta + mock * N3;
  if (p0 < p1) {
    prefetch_pencil<N, T, VZN>(fmock + (long long)p0 * N, N3, nbins, vpre);
    prefetch_delta<N, T>(dmock + (long long)p0 * N, dpre);
  }
  for (int p = p0; p < p1; ++p) {
    // this pencil's data moves to vcur; the next pencil's loads are issued
    // before the transform so they stay in flight for the whole iteration
    c2<T> vcur[prefetch_rounds<N, VZN>()][F::RMAX];
#pragma unroll
    for (int q = 0; q < prefetch_rounds<N, VZN>(); ++q)
#pragma unroll
      for (int r = 0; r < F::RMAX; ++r) vcur[q][r] = vpre[q][r];
#pragma unroll
    for (int k = 0; k < DPRE; ++k) {
      const int z = tid + k * blockDim.x;
      if (z < N) dl[z] = dpre[k];
    }
    if (p + 1 < p1) {
      prefetch_pencil<N, T, VZN>(fmock + (long long)(p + 1) * N, N3, nbins, vpre);
      prefetch_delta<N, T>(dmock + (long long)(p + 1) * N, dpre);
    }
    __syncthreads();
    transform_pencil_bins<N, T, VZN>(fmock + (long long)p * N, N3, nbins, A, tws, vcur);
    __syncthreads();
    ctr.add(A, dl, nbins, RS, N);
    __syncthreads();
  }
  ctr.finish(reinterpret_cast<double*>(smem), partials + ((long long)mock * gridDim.x + blockIdx.x) * nbins * nbins,
             nbins);
}

// ---------------------------------------------------------------------------
// particle summation
// ---------------------------------------------------------------------------
// z pass that stores the fields bin-interleaved, out[mock][cell][b], so that a
// B-spline tap reads all bins of a node contiguously.  One launch handles bins
// b0 .. b0 + nbins - 1 of nbt (the pencil of those bins is held in LDS).
template <int N, typename T>
__global__ void __launch_bounds__(512) k_zpass_store(const c2<T>* fields, c2<T>* out, int nbins, int nbt, int b0,
                                                      int ppw, const c2<T>* tw) {
  using F = Fft<N, VZN>;
  constexpr int RS = zrow<N>();
  constexpr long long N3 = (long long)N * N * N;
  extern __shared__ __align__(16) char smem[];
  c2<T>* A = reinterpret_cast<c2<T>*>(smem);
  c2<T>* tws = A + nbins * RS;
  const long long mock = blockIdx.y;
  stage_twiddles<N, T>(tw, tws);
  const int p0 = blockIdx.x * ppw;
  const int p1 = min(p0 + ppw, N * N);
  const c2<T>* fmock = fields + (mock * nbt + b0) * N3;
  c2<T>* omock = out + mock * nbt * N3;
  c2<T> vpre[prefetch_rounds<N, VZN>()][F::RMAX];
  if (p0 < p1) prefetch_pencil<N, T, VZN>(fmock + (long long)p0 * N, N3, nbins, vpre);
  for (int p = p0; p < p1; ++p) {
    c2<T> vcur[prefetch_rounds<N, VZN>()][F::RMAX];
#pragma unroll
    for (int q = 0; q < prefetch_rounds<N, VZN>(); ++q)
#pragma unroll
      for (int r = 0; r < F::RMAX; ++r) vcur[q][r] = vpre[q][r];
    if (p + 1 < p1) prefetch_pencil<N, T, VZN>(fmock + (long long)(p + 1) * N, N3, nbins, vpre);
    __syncthreads();
    transform_pencil_bins<N, T, VZN>(fmock + (long long)p * N, N3, nbins, A, tws, vcur);
    __syncthreads();
    c2<T>* dst = omock + (long long)p * N * nbt + b0;
    for (int idx = threadIdx.x; idx < N * nbins; idx += blockDim.x) {
      const int z = idx / nbins, b = idx - z * nbins;
      dst[(long long)z * nbt + b] = A[b * RS + lds_pos<true>(z)];
    }
  }
}

// particles per (2^shift)^3-cell tile (sort key), tile id mock * NT + (tx * NTd + ty) * NTd + tz
__device__ __forceinline__ int tile_of(const float* p, int n, double sc, int ntd, int shift) {
  int t = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double u = (double)p[d] * sc;
    if (!(u == u) || fabs(u) > 1e15) u = 0.0;
    u -= (double)n * floor(u / (double)n);
    int c = (int)floor(u);
    if (c >= n) c -= n;
    if (c < 0) c = 0;
    t = t * ntd + (c >> shift);
  }
  return t;
}

__global__ void k_tile_count(const float* pos, const long long* off, int batch, long long np_total, int n, double sc,
                             int shift, int* counts) {
  const int ntd = n >> shift;
  const long long nt = (long long)ntd * ntd * ntd;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < np_total; i += (long long)gridDim.x * blockDim.x) {
    const int mock = find_mock(off, batch, i);
    atomicAdd(&counts[mock * nt + tile_of(pos + 3 * i, n, sc, ntd, shift)], 1);
  }
}

// exclusive scan of counts[0..m) into offs (and a copy into cursor), one block
__global__ void k_scan_counts(const int* counts, int* offs, int* cursor, long long m) {
  __shared__ long long part[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long seg = (m + nt - 1) / nt;
  const long long a = tid * seg, b = min(m, a + seg);
  long long s = 0;
  for (long long i = a; i < b; ++i) s += counts[i];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    long long run = 0;
    for (int t = 0; t < nt; ++t) {
      const long long v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  long long run = part[tid];
  for (long long i = a; i < b; ++i) {
    offs[i] = (int)run;
    cursor[i] = (int)run;
    run += counts[i];
  }
}

__global__ void k_tile_scatter(const float* pos, const long long* off, int batch, long long np_total, int n, double sc,
                               int shift, int* cursor, int* perm) {
  const int ntd = n >> shift;
  const long long nt = (long long)ntd * ntd * ntd;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < np_total; i += (long long)gridDim.x * blockDim.x) {
    const int mock = find_mock(off, batch, i);
    const int slot = atomicAdd(&cursor[mock * nt + tile_of(pos + 3 * i, n, sc, ntd, shift)], 1);
    perm[slot] = (int)i;
  }
}

// Per-particle stencil records in sorted order, computed once per call by
// make_taps: the cell (floor of x n / box per axis, packed 10 bits each; -1
// for a position that is not finite) and the 12 tap weights in the working
// precision.  The gathers and the scatter read these instead of re-deriving
// the stencil in float64 for every lane and (l, m).
__device__ __forceinline__ int pack_cell(const Taps& t) {
  return t.ok ? ((t.base[0] + 1) | ((t.base[1] + 1) << 10) | ((t.base[2] + 1) << 20)) : -1;
}

template <typename T>
__global__ void k_tap_records(const float* pos, const int* perm, long long np_total, int n, double sc, int* tcell,
                              T* twt, const double* btab) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < np_total; k += (long long)gridDim.x * blockDim.x) {
    const Taps t = make_taps(pos + 3 * (long long)perm[k], n, sc, btab);
    tcell[k] = pack_cell(t);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int a = 0; a < 4; ++a) twt[k * 12 + d * 4 + a] = (T)t.wt[d][a];
  }
}

// sum over the 64 taps of record k of w_tap * f[node][b] (bin-interleaved
// fields of one mock, nbins per node), separably: the four z taps of each
// (x, y) row with the z weights, the rows with the y weights, then x.  A row
// whose z taps do not wrap is read at one base address plus multiples of the
// node stride.
template <typename T>
__device__ __forceinline__ c2<T> gather_record(const c2<T>* fm, int cell, const T* wt, int n, int nbins, int b) {
  const int cx = cell & 1023, cy = (cell >> 10) & 1023, cz = cell >> 20;
  T w[8];                                               // y and z weights (x weights read per row)
#pragma unroll
  for (int e = 0; e < 8; ++e) w[e] = wt[4 + e];
  const long long rowy = (long long)n * nbins;          // elements per y step
  const long long rowx = (long long)n * rowy;           // elements per x step
  const bool zin = cz >= 1 && cz + 2 < n;
  long long oz[4];
#pragma unroll
  for (int az = 0; az < 4; ++az) oz[az] = (long long)(zin ? cz - 1 + az : wrapi(cz - 1 + az, n)) * nbins + b;
  c2<T> acc = mk<T>(0, 0);
  // all four x rows unrolled: the 64 loads of a record are in flight together
#pragma unroll
  for (int ax = 0; ax < 4; ++ax) {
    const c2<T>* px = fm + wrapi(cx - 1 + ax, n) * rowx;
    c2<T> sy = mk<T>(0, 0);
#pragma unroll
    for (int ay = 0; ay < 4; ++ay) {
      const c2<T>* py = px + wrapi(cy - 1 + ay, n) * rowy;
      c2<T> v[4];
      if (zin) {
        const c2<T>* q = py + oz[0];
#pragma unroll
        for (int az = 0; az < 4; ++az) v[az] = q[az * nbins];
      } else {
#pragma unroll
        for (int az = 0; az < 4; ++az) v[az] = py[oz[az]];
      }
      c2<T> sz = mk<T>(0, 0);
#pragma unroll
      for (int az = 0; az < 4; ++az) {
        sz.x += w[4 + az] * v[az].x;
        sz.y += w[4 + az] * v[az].y;
      }
      sy.x += w[ay] * sz.x;
      sy.y += w[ay] * sz.y;
    }
    const T wx = wt[ax];
    acc.x += wx * sy.x;
    acc.y += wx * sy.y;
  }
  return acc;
}

// particle slots of one contraction slice of the gather (LDS rows of nbins x slots)
constexpr int kGatherSlots = 256;

// Gather the B-spline interpolants of the (bin-interleaved) fields at the
// particles, one lane per (particle, bin), into LDS rows, then contract with
// the weights w_i / W.  Particles are visited in tile order (perm).
// SRC: the same gathered values also give the adjoint sources of
// k_gather_source (value and gradient in one sweep, fields in the eigenbasis
// of the cotangent, lam_d its eigenvalues): per lane v_b = d_b conj(atilde_b),
// src = N^3 (w_i / W) v_b, and wm sum_b d_b |atilde_b|^2 added to F_J(u_i),
// all at gather time.
template <typename T, bool MF, bool SPLIT = false, bool QUAD = false, bool SRC = false>
__global__ void __launch_bounds__(256) k_gather_contract(const c2<T>* fields, const int* tcell, const T* twt,
                                                          const float* w, const int* perm, const long long* off,
                                                          const double* W, int n, int nbins, double* partials,
                                                          const T* lam_d, T wm, double* FJ, c2<T>* src) {
  constexpr int K = kGatherSlots;                       // particle slots per contraction slice
  constexpr int RS = K + K / 16 + 1;
  extern __shared__ __align__(16) char smem[];
  c2<T>* A = reinterpret_cast<c2<T>*>(smem);
  T* wk = reinterpret_cast<T*>(A + nbins * RS);
  int* pk = reinterpret_cast<int*>(wk + K);             // SRC: particle of slot k (-1: none)
  T* lam = reinterpret_cast<T*>(pk + K);                // SRC: the eigenvalues d_b
  const long long mock = blockIdx.y;
  const long long n3 = (long long)n * n * n;
  const long long a0 = off[mock], a1 = off[mock + 1];
  const long long per = (a1 - a0 + gridDim.x - 1) / gridDim.x;
  const long long s0 = a0 + per * blockIdx.x, s1 = min(a1, s0 + per);
  const double invW = 1.0 / W[mock];
  // nbins lanes per particle, 64 / nbins particles per wave (the rest idle)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // slots per slice: a multiple of the particles per pass and of 8 (fewer
  // particles per wave where no multiple fits the slice)
  int ppw = 64 / nbins;
  if (ppw * nw > K) ppw = K / nw;
  int kcount = 0;
  for (;;) {
    const int pp = nw * ppw;
    kcount = pp * (K / pp);
    while (kcount > 0 && kcount % 8) kcount -= pp;
    if (kcount > 0 || ppw == 1) break;
    --ppw;
  }
  const int pw = lane / nbins, b = lane - pw * nbins;
  const bool lane_ok = pw < ppw;
  const int ppp = nw * ppw;                             // particles per pass
  const c2<T>* fm = fields + mock * n3 * nbins;
  const double fw = (double)n3 / W[mock];
  const T dl = (SRC && lane_ok) ? lam_d[mock * nbins + b] : (T)0;
  if constexpr (SRC) {
    for (int t = threadIdx.x; t < nbins; t += blockDim.x) lam[t] = lam_d[mock * nbins + t];
  }
  Contractor<T, MF, SPLIT, QUAD> ctr;
  ctr.init(nbins);
  for (long long c0 = s0; c0 < s1; c0 += kcount) {
    for (int k0 = 0; k0 < kcount; k0 += ppp) {
      const int k = k0 + wv * ppw + pw;
      const long long si = c0 + k;
      c2<T> acc = mk<T>(0, 0);
      T wgt = 0;
      int i = -1;
      if (lane_ok && si < s1) {
        i = perm[si];
        const int cell = tcell[si];
        if (cell >= 0) acc = gather_record<T>(fm, cell, twt + si * 12, n, nbins, b);
        const double wi = w ? (double)w[i] : 1.0;
        wgt = (T)(wi * invW);
        if constexpr (SRC) {
          const T e = dl * acc.x, f2 = dl * acc.y;
          const T f = (T)(fw * wi);
          src[si * nbins + b] = mk<T>(f * e, -(f * f2));
        }
      }
      if (lane_ok) {
        A[b * RS + lds_pos<true>(k)] = acc;
        if (b == 0) {
          wk[k] = wgt;
          if constexpr (SRC) pk[k] = i;
        }
      }
    }
    __syncthreads();
    ctr.add(A, wk, nbins, RS, kcount);
    if constexpr (SRC) {
      // the primary vertex's share: F_J(u_i) += wm sum_b d_b |atilde_b|^2, one thread per slot
      for (int k = threadIdx.x; k < kcount; k += blockDim.x) {
        const int ip = pk[k];
        if (ip >= 0) {
          const int kp = lds_pos<true>(k);
          T fj = 0;
          for (int bb = 0; bb < nbins; ++bb) {
            const c2<T> a = A[bb * RS + kp];
            fj += lam[bb] * (a.x * a.x + a.y * a.y);
          }
          FJ[ip] += (double)wm * (double)fj;
        }
      }
    }
    __syncthreads();
  }
  ctr.finish(reinterpret_cast<double*>(smem), partials + ((long long)mock * gridDim.x + blockIdx.x) * nbins * nbins,
             nbins);
}

// ---------------------------------------------------------------------------
// grid summation with connection coefficients
// ---------------------------------------------------------------------------
// sum_x delta_x sum_{s,t} Gamma(s,t) a(x+s) conj(b(x+t)) equals the integral of
// the three cubic B-spline interpolants, a degree-9 polynomial per axis on each
// cell, integrated exactly by 5-point Gauss-Legendre.  A workgroup takes a
// tile of 4^3 cells, holds the 7^3 coefficients it touches (all bins) in LDS
// and, per x node, interpolates along x, y (half of the y nodes at a time)
// and z into LDS rows A[b][node] with weights w_node delta_B(node), which the
// contraction consumes.  Interpolation weights M[s][t] = B3(xi_s + 1 - t) and
// node weights are set on the host.
struct GammaQuad {
  float m[5][4];     // B3 weight of tap t at node s (node xi_s in the unit cell)
  float wq[5];       // Gauss-Legendre weights on [0, 1]
  double md[5][4];
  double wqd[5];
};

template <typename T> __device__ __forceinline__ T gq_m(const GammaQuad& q, int s, int t);
template <> __device__ __forceinline__ float gq_m<float>(const GammaQuad& q, int s, int t) { return q.m[s][t]; }
template <> __device__ __forceinline__ double gq_m<double>(const GammaQuad& q, int s, int t) { return q.md[s][t]; }
template <typename T> __device__ __forceinline__ T gq_w(const GammaQuad& q, int s);
template <> __device__ __forceinline__ float gq_w<float>(const GammaQuad& q, int s) { return q.wq[s]; }
template <> __device__ __forceinline__ double gq_w<double>(const GammaQuad& q, int s) { return q.wqd[s]; }

constexpr int GT = 4;              // cells per tile edge
constexpr int GC = GT + 3;         // coefficients per tile edge
constexpr int GN = 5 * GT;         // quadrature nodes per tile edge
constexpr int GYH = GN / 2;        // y nodes per half
constexpr int GK = GYH * GN;       // nodes per contraction slice (200)
constexpr int GRS = GK + GK / 16 + 1;

template <typename T>
struct GammaLds {
  // byte offsets into dynamic LDS for nbins bins
  size_t C, D, P, Pd, Q, Qd, A, W, total;
  __host__ __device__ GammaLds(int nbins) {
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = (o + b + 15) & ~(size_t)15; return r; };
    C = take((size_t)GC * GC * GC * nbins * sizeof(c2<T>));
    D = take((size_t)GC * GC * GC * sizeof(T));
    P = take((size_t)GC * GC * nbins * sizeof(c2<T>));
    Pd = take((size_t)GC * GC * sizeof(T));
    Q = take((size_t)GYH * GC * nbins * sizeof(c2<T>));
    Qd = take((size_t)GYH * GC * sizeof(T));
    A = take((size_t)nbins * GRS * sizeof(c2<T>));
    W = take((size_t)GK * sizeof(T));
    total = o;
  }
};

// 1024 threads: the per-node phases are short, and one workgroup fills the
// CU's LDS, so the waves of that one workgroup are what hides LDS latency
// Bins: the workgroup contracts nbins local bins, local bin b < na being
// field bin a0 + b and the rest field bins c0 + (b - na) of the nbt stored
// bins (all of them with a0 = 0, na = nbins = nbt), so that plans with more
// bins than the tile's LDS holds take them in pairs of chunks.
template <typename T, bool MF, bool SPLIT = false, bool QUAD = false>
__global__ void __launch_bounds__(1024) k_gamma_contract(const c2<T>* fields, const T* delta, int n, int nbins,
                                                         GammaQuad gq, double* partials, int nbt, int a0, int na,
                                                         int c0) {
  extern __shared__ __align__(16) char smem[];
  const GammaLds<T> L(nbins);
  c2<T>* C = reinterpret_cast<c2<T>*>(smem + L.C);
  T* D = reinterpret_cast<T*>(smem + L.D);
  c2<T>* P = reinterpret_cast<c2<T>*>(smem + L.P);
  T* Pd = reinterpret_cast<T*>(smem + L.Pd);
  c2<T>* Q = reinterpret_cast<c2<T>*>(smem + L.Q);
  T* Qd = reinterpret_cast<T*>(smem + L.Qd);
  c2<T>* A = reinterpret_cast<c2<T>*>(smem + L.A);
  T* W = reinterpret_cast<T*>(smem + L.W);
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long mock = blockIdx.y;
  const long long n3 = (long long)n * n * n;
  const c2<T>* fm = fields + mock * n3 * nbt;
  const T* dm = delta + mock * n3;
  const int td = n / GT;
  const long long ntiles = (long long)td * td * td;
  Contractor<T, MF, SPLIT, QUAD> ctr;
  ctr.init(nbins);
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int tx = (int)(tile / ((long long)td * td)), ty = (int)((tile / td) % td), tz = (int)(tile % td);
    const int x0 = tx * GT - 1, y0 = ty * GT - 1, z0 = tz * GT - 1;     // first coefficient (periodic)
    __syncthreads();
    for (int e = tid; e < GC * GC * GC * nbins; e += nt) {
      const int b = e % nbins, c = e / nbins;
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      const long long cell = ((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n);
      C[e] = fm[cell * nbt + (b < na ? a0 + b : c0 + b - na)];
    }
    for (int c = tid; c < GC * GC * GC; c += nt) {
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      D[c] = dm[((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n)];
    }
    for (int xn = 0; xn < GN; ++xn) {
      const int cx = xn / 5, sx = xn % 5;
      __syncthreads();
      // x interpolation: P[j][k][b], Pd[j][k]
      for (int e = tid; e < GC * GC * nbins; e += nt) {
        const int b = e % nbins, jk = e / nbins;
        c2<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const c2<T> v = C[((cx + t) * GC * GC + jk) * nbins + b];
          const T m = gq_m<T>(gq, sx, t);
          acc.x += m * v.x;
          acc.y += m * v.y;
        }
        P[e] = acc;
      }
      for (int jk = tid; jk < GC * GC; jk += nt) {
        T acc = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc += gq_m<T>(gq, sx, t) * D[(cx + t) * GC * GC + jk];
        Pd[jk] = acc;
      }
      for (int half = 0; half < 2; ++half) {
        __syncthreads();
        // y interpolation for this half of the y nodes: Q[yh][k][b], Qd[yh][k]
        for (int e = tid; e < GYH * GC * nbins; e += nt) {
          const int b = e % nbins, yk = e / nbins;
          const int yh = yk / GC, k = yk % GC;
          const int yn = half * GYH + yh, cy = yn / 5, sy = yn % 5;
          c2<T> acc = mk<T>(0, 0);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const c2<T> v = P[((cy + t) * GC + k) * nbins + b];
            const T m = gq_m<T>(gq, sy, t);
            acc.x += m * v.x;
            acc.y += m * v.y;
          }
          Q[e] = acc;
        }
        for (int yk = tid; yk < GYH * GC; yk += nt) {
          const int yh = yk / GC, k = yk % GC;
          const int yn = half * GYH + yh, cy = yn / 5, sy = yn % 5;
          T acc = 0;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc += gq_m<T>(gq, sy, t) * Pd[(cy + t) * GC + k];
          Qd[yk] = acc;
        }
        __syncthreads();
        // z interpolation into the contraction rows; weights w_x w_y w_z delta_B
        for (int e = tid; e < GK * nbins; e += nt) {
          const int b = e % nbins, node = e / nbins;
          const int yh = node / GN, zn = node % GN, cz = zn / 5, sz = zn % 5;
          c2<T> acc = mk<T>(0, 0);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const c2<T> v = Q[(yh * GC + cz + t) * nbins + b];
            const T m = gq_m<T>(gq, sz, t);
            acc.x += m * v.x;
            acc.y += m * v.y;
          }
          A[b * GRS + lds_pos<true>(node)] = acc;
        }
        for (int node = tid; node < GK; node += nt) {
          const int yh = node / GN, zn = node % GN, cz = zn / 5, sz = zn % 5;
          const int sy = (half * GYH + yh) % 5;
          T acc = 0;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc += gq_m<T>(gq, sz, t) * Qd[yh * GC + cz + t];
          W[node] = acc * gq_w<T>(gq, sx) * gq_w<T>(gq, sy) * gq_w<T>(gq, sz);
        }
        __syncthreads();
        ctr.add(A, W, nbins, GRS, GK);
      }
    }
  }
  __syncthreads();
  ctr.finish(reinterpret_cast<double*>(smem), partials + ((long long)mock * gridDim.x + blockIdx.x) * nbins * nbins,
             nbins);
}

// sum_s A(s) e^{-i theta s} over the autocorrelation samples of the basis
__device__ __forceinline__ double acf_hat(const Acf& c, double th) {
  return c.a[0] + 2.0 * (c.a[1] * cos(th) + c.a[2] * cos(2.0 * th) + c.a[3] * cos(3.0 * th));
}

// P[mock][s] += |dhat(q)|^2 Ahat(q) over q with |q|^2 = s, Nyquist planes excluded,
// Ahat = prod_d acf_hat(theta_d) (for the cubic B-spline the samples are
// A(0..3) = (2416, 1191, 120, 1) / 5040).
// phi != NULL: each term also carries phi-hat(q)^2 (both secondary vertices
// of the volume mean carry the scaling function's power spectrum)
template <typename T>
__global__ void k_power_hist(const c2<T>* dhat, int n, int nq2, double* P, const T* phi, Acf acf) {
  const long long n3 = (long long)n * n * n;
  const int mock = blockIdx.y;
  const c2<T>* d = dhat + mock * n3;
  double* pm = P + (long long)mock * nq2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n3; i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i / ((long long)n * n)), iy = (int)((i / n) % n), iz = (int)(i % n);
    const int qx = sfreq(ix, n), qy = sfreq(iy, n), qz = sfreq(iz, n);
    const int h = -n / 2;
    if (qx == h || qy == h || qz == h) continue;
    const double tp = 2.0 * 3.14159265358979323846 / n;
    double b7 = 1.0;
    const int qs[3] = {qx, qy, qz};
#pragma unroll
    for (int a = 0; a < 3; ++a) b7 *= acf_hat(acf, tp * qs[a]);
    if (phi) {
      const double ph = (double)phi[ix] * (double)phi[iy] * (double)phi[iz];
      b7 *= ph * ph;
    }
    const c2<T> v = d[i];
    const double p2 = (double)v.x * v.x + (double)v.y * v.y;
    atomicAdd(&pm[qx * qx + qy * qy + qz * qz], p2 * b7);
  }
}

// zeta[mock][l][b1][b2] -= (2l+1)/N^6 sum_s P[s] jbar_{l,b1}(s) jbar_{l,b2}(s)
// (4 pi times the volume mean of F_l); one block per (b1 b2, mock)
template <typename T>
__global__ void k_fbar_subtract(const double* P, const T* jtab, int nq2, int nbp, int nbins, int l, int lmax,
                                double n6, double* zeta) {
  __shared__ double sh[32];
  const int e = blockIdx.x, mock = blockIdx.y;
  const int b1 = e / nbins, b2 = e % nbins;
  const double* pm = P + (long long)mock * nq2;
  const T* jl = jtab + (long long)l * nq2 * nbp;
  double s = 0.0;
  for (int q = threadIdx.x; q < nq2; q += blockDim.x) s += pm[q] * (double)jl[(long long)q * nbp + b1] * (double)jl[(long long)q * nbp + b2];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) zeta[((long long)mock * (lmax + 1) + l) * nbins * nbins + e] -= (2.0 * l + 1.0) / n6 * s;
}

// zeta[j][l][e] += scale * sum_w partials[j][w][e]; one block per (e, j),
// the partials of a group of items ([item][mock][wg][nb2]) into zeta at each item's l, times its m weight
__global__ void k_reduce_items(const double* partials, int nwg, int nb2, double* zeta, int lmax, double scale,
                               const ItemRec* items, int item0, int nitems, int batch) {
  // one block per (entry, mock) walks the group's items in order: items that
  // share an l add into the same entry, so no two blocks write one entry
  __shared__ double sh[32];
  const int e = blockIdx.x, j = blockIdx.y;
  for (int g = 0; g < nitems; ++g) {
    const ItemRec& it = items[item0 + g];
    const double* p = partials + ((long long)g * batch + j) * nwg * nb2 + e;
    double s = 0.0;
    for (int w = threadIdx.x; w < nwg; w += blockDim.x) s += p[(long long)w * nb2];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) zeta[((long long)j * (lmax + 1) + it.l) * nb2 + e] += scale * it.wm * s;
  }
}

// fixed summation order (deterministic)
__global__ void k_reduce_partials(const double* partials, int nwg, int nb2, double* zeta, int l, int lmax, double scale) {
  __shared__ double sh[32];
  const int e = blockIdx.x;
  const int j = blockIdx.y;
  const double* p = partials + (long long)j * nwg * nb2 + e;
  double s = 0.0;
  for (int w = threadIdx.x; w < nwg; w += blockDim.x) s += p[(long long)w * nb2];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) zeta[((long long)j * (lmax + 1) + l) * nb2 + e] += scale * s;
}

// ---------------------------------------------------------------------------
// backward pass z: recompute a_b on the pencil, then per z (one thread owns a
// z column, so no atomics and no read/write hazards)
//   u_b = sum_b' lam_s[b,b'] conj(a_b'),  direct += wm Re(sum_b a_b u_b),
//   c_b = delta u_b,
// and z-transform every c_b (the adjoint's first axis), written over the field.
// lam_s is read with wave-uniform indices (scalar loads).
// FUSED: the same sweep also contracts the pencil for zeta (the partials of
// k_zpass_nodal), so that value and gradient share one computation of the
// fields when dJ/dzeta is fixed before the forward (J linear in zeta).
// ---------------------------------------------------------------------------
template <int N, typename T, int MAXNB, bool FUSED = false, bool MF = false, bool QUAD = false>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(FUSED && MF ? 3 : 1)))
k_zpass_adjoint(c2<T>* fields, const T* delta, const T* __restrict__ lam_d, T* direct, int nbins, int ppw,
                const c2<T>* tw, double* partials, const ItemRec* items, int item0, int nitems, int batch, int nwg,
                int* counter) {
  using F = Fft<N, VZA<T>>;
  constexpr int RS = zrow<N>();
  constexpr int NBP = (MAXNB + 3) / 4 * 4;
  constexpr long long N3 = (long long)N * N * N;
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_unit;
  c2<T>* A = reinterpret_cast<c2<T>*>(smem);
  c2<T>* tws = A + nbins * RS;
  T* lam = reinterpret_cast<T*>(tws + N);             // [NBP] eigenvalues of the cotangent, zero padded
  T* dl = lam + NBP;                                  // FUSED: delta of the pencil
  const int tid = threadIdx.x;
  const int nbc = blockDim.x / F::TPC;
  const int nb2 = nbins * nbins;
  // several items of a group update the same direct term: atomically then
  const bool shared_direct = nitems > 1;
  // the next pencil's loads are issued at the top of each iteration, so they
  // stay in flight for the whole of it; the matrix-core one sweep instead
  // loads each pencil when it starts (no registers held across the
  // iteration: three workgroups per CU hide the latency instead)
  constexpr bool NO_PREFETCH = FUSED && MF;
  // persistent: work units (item of the group, mock, chunk of ppw pencils) from an atomic counter
  const int total = nitems * batch * nwg;
  for (;;) {
    __syncthreads();                          // the previous unit is done with the LDS
    if (tid == 0) s_unit = atomicAdd(counter, 1);
    __syncthreads();
    const int unit = s_unit;
    if (unit >= total) break;
    const int g = unit / (batch * nwg);
    const int mock = (unit / nwg) % batch;
    const int chunk = unit % nwg;
    const ItemRec& it = items[item0 + g];
    const T wm = (T)it.wm;
    stage_twiddles<N, T>(tw, tws);
    const T* ls = lam_d + ((long long)it.l * batch + mock) * nbins;
    for (int t = tid; t < NBP; t += blockDim.x) lam[t] = t < nbins ? ls[t] : (T)0;
    __syncthreads();
    Contractor<T, MF, false, QUAD> ctr;
    if constexpr (FUSED) ctr.init(nbins);
    const int p0 = chunk * ppw;
    const int p1 = min(p0 + ppw, N * N);
    c2<T>* fmock = fields + ((long long)g * batch + mock) * nbins * N3;
    const T* dmock = delta + (long long)mock * N3;
    T* rmock = direct + (long long)mock * N3;
    c2<T> vpre[prefetch_rounds<N, VZA<T>>()][F::RMAX];
    T dpre[DPRE], rpre[DPRE];
    if (!NO_PREFETCH && p0 < p1) {
      prefetch_pencil<N, T, VZA<T>>(fmock + (long long)p0 * N, N3, nbins, vpre);
      prefetch_delta<N, T>(dmock + (long long)p0 * N, dpre);
      prefetch_delta<N, T>(rmock + (long long)p0 * N, rpre);
    }
    for (int p = p0; p < p1; ++p) {
      c2<T>* fbase = fmock + (long long)p * N;
      c2<T> vcur[prefetch_rounds<N, VZA<T>>()][F::RMAX];
      T dcur[DPRE], rcur[DPRE];
      if constexpr (NO_PREFETCH) {
        prefetch_delta<N, T>(dmock + (long long)p * N, dcur);
        prefetch_delta<N, T>(rmock + (long long)p * N, rcur);
      } else {
#pragma unroll
        for (int q = 0; q < prefetch_rounds<N, VZA<T>>(); ++q)
#pragma unroll
          for (int r = 0; r < F::RMAX; ++r) vcur[q][r] = vpre[q][r];
#pragma unroll
        for (int k = 0; k < DPRE; ++k) {
          dcur[k] = dpre[k];
          rcur[k] = rpre[k];
        }
      }
      if (!NO_PREFETCH && p + 1 < p1) {
        prefetch_pencil<N, T, VZA<T>>(fbase + N, N3, nbins, vpre);
        prefetch_delta<N, T>(dmock + (long long)(p + 1) * N, dpre);
        prefetch_delta<N, T>(rmock + (long long)(p + 1) * N, rpre);
      }
      if constexpr (FUSED) {
#pragma unroll
        for (int k = 0; k < DPRE; ++k) {
          const int z = tid + k * blockDim.x;
          if (z < N) dl[z] = dcur[k];
        }
      }
      if constexpr (NO_PREFETCH) {
        const int rounds = pencil_rounds<N, VZA<T>>(nbins);
        for (int rr = 0; rr < rounds; ++rr) {
          c2<T> v[F::RMAX];
          load_pencil_round<N, T, VZA<T>>(fbase, N3, nbins, rr, v);
          transform_round<N, T, VZA<T>>(nbins, rr, v, A, tws);
        }
      } else {
        transform_pencil_bins<N, T, VZA<T>>(fbase, N3, nbins, A, tws, vcur);
      }
      __syncthreads();
      if constexpr (FUSED) {
        // contraction of the fields before the sources overwrite them.  On the
        // matrix cores each wave contracts the 64 z columns whose sources its
        // own threads form next, so no barrier separates the two steps.
        if constexpr (MF) {
          const int z0 = 64 * (tid >> 6);
          if (z0 < N) ctr.add_range(A, dl, nbins, RS, z0, z0 + 64 < N ? z0 + 64 : N);
        } else {
          ctr.add(A, dl, nbins, RS, N);
          __syncthreads();
        }
      }
#pragma unroll
      for (int k = 0; k < DPRE; ++k) {
        const int z = tid + k * blockDim.x;
        if (z >= N) continue;
        const int zp = lds_pos<true>(z);
        // in the eigenbasis of the cotangent the source of field k is
        // d_k conj(a_k) delta and the direct term sum_k d_k |a_k|^2
        const T d = dcur[k];
        T dir = 0;
#pragma unroll
        for (int bq = 0; bq < NBP; bq += 4) {
          T lq[4];
          load_quad<T>(lam + bq, lq);                // LDS broadcast
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int b = bq + i;
            if (b < nbins) {
              const c2<T> a = A[b * RS + zp];
              const T e = lq[i] * a.x, f = lq[i] * a.y;
              dir += e * a.x + f * a.y;
              A[b * RS + zp] = mk<T>(d * e, -(d * f));
            }
          }
        }
        if (shared_direct) atomicAdd(&rmock[(long long)p * N + z], wm * dir);
        else rmock[(long long)p * N + z] = rcur[k] + wm * dir;
      }
      __syncthreads();
      // adjoint z-transform of every c_b, read from LDS, written over the field
      const int rounds = (nbins + nbc - 1) / nbc;
      for (int rr = 0; rr < rounds; ++rr) {
        int j = tid % F::TPC;
        asm volatile("" : "+v"(j));
        const int b = rr * nbc + tid / F::TPC;
        const bool active = b < nbins;
        c2<T> v[F::RMAX];
        if (active) {
#pragma unroll
          for (int r = 0; r < F::RMAX; ++r) v[r] = A[b * RS + lds_pos<true>(F::in_index(j, r))];
        }
        __syncthreads();
        fft_column<N, +1, T, true, VZA<T>, 64 % F::TPC == 0>(v, A + (active ? b : 0) * RS, 1, j, tws, active);
        if (active) {
#pragma unroll
          for (int e = 0; e < F::RMAX; ++e) fbase[b * N3 + F::out_index(j, e)] = v[e];
        }
      }
      __syncthreads();
    }
    if constexpr (FUSED)
      ctr.finish(reinterpret_cast<double*>(smem), partials + (((long long)g * batch + mock) * nwg + chunk) * nb2,
                 nbins);
  }
}

// lam_s[l][j][b][b'] = (dzeta[j][l][b][b'] + dzeta[j][l][b'][b]) / 2 for every l (blockIdx.x = l)
template <typename T>
__global__ void k_lam_sym(const double* dzeta, T* lam_s, int nbins, int lmax, int batch) {
  const int j = blockIdx.y, l = blockIdx.x;
  const double* dz = dzeta + ((long long)j * (lmax + 1) + l) * nbins * nbins;
  for (int t = threadIdx.x; t < nbins * nbins; t += blockDim.x) {
    const int b = t / nbins, bp = t % nbins;
    lam_s[((long long)l * batch + j) * nbins * nbins + t] = (T)(0.5 * (dz[b * nbins + bp] + dz[bp * nbins + b]));
  }
}

// ---------------------------------------------------------------------------
// The nodal gradient in the eigenbasis of the cotangent.  The symmetrised
// cotangent of multipole l and mock j is real symmetric, lam_s = V diag(d) V^T
// with V orthogonal, so sum_{b,b'} lam_s[b][b'] a_b conj(a_b') equals
// sum_k d_k |abar_k|^2 for the rotated fields abar_k = sum_b V[b][k] a_b.  The
// window pass is linear in the radial table, so the rotated fields come from
// the rotated table jbar_{l,k} = sum_b V[b][k] jbar_{l,b}; the adjoint sources
// become diagonal, and the value in the rotated basis is turned back by
// zeta = V zetabar V^T.
// ---------------------------------------------------------------------------
constexpr int kEigMaxBins = 64;

// LDS bytes of k_lam_eig for nbins bins
inline size_t lam_eig_lds(int nbins) {
  const int half = (nbins + 1) / 2;
  return (size_t)2 * nbins * (nbins + 1) * sizeof(double) + (size_t)2 * half * sizeof(double) +
         (size_t)2 * 8 * sizeof(double) + (size_t)2 * half * sizeof(int);
}

// One workgroup per (l, mock): cyclic Jacobi in float64 with the round-robin
// pair order (each round rotates nbins / 2 disjoint index pairs at once, which
// commute), until the off-diagonal norm is below 1e-14 of the matrix norm or
// after kEigSweeps sweeps.  Writes the eigenvalues d [l][mock][nbins] at the
// plan precision and the eigenvectors V [l][mock][nbins][nbins] (columns) in
// float64.
constexpr int kEigSweeps = 40;

template <typename T>
__global__ void __launch_bounds__(256) k_lam_eig(const double* dzeta, T* lam_d, double* evec, int nbins, int lmax,
                                                 int batch) {
  extern __shared__ __align__(16) char smem[];
  const int l = blockIdx.x, j = blockIdx.y, nb = nbins, ld = nbins + 1;
  const int m = (nb + 1) & ~1, half = m / 2;   // an even index count: index nb is a dummy when nb is odd
  double* A = reinterpret_cast<double*>(smem);
  double* V = A + nb * ld;
  double* cs = V + nb * ld;
  double* sn = cs + half;
  double* red = sn + half;                      // [2][8]: per-wave partial norms
  int* pp = reinterpret_cast<int*>(red + 16);
  int* pq = pp + half;
  const int tid = threadIdx.x, nt = blockDim.x;
  const double* dz = dzeta + ((long long)j * (lmax + 1) + l) * nb * nb;
  for (int t = tid; t < nb * nb; t += nt) {
    const int b = t / nb, c = t % nb;
    A[b * ld + c] = 0.5 * (dz[b * nb + c] + dz[c * nb + b]);
    V[b * ld + c] = b == c ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < kEigSweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int t = tid; t < nb * nb; t += nt) {
      const int b = t / nb, c = t % nb;
      const double a2 = A[b * ld + c] * A[b * ld + c];
      tot += a2;
      if (b != c) off += a2;
    }
    for (int o = warpSize / 2; o > 0; o >>= 1) {
      off += __shfl_down(off, o);
      tot += __shfl_down(tot, o);
    }
    if (tid % warpSize == 0) {
      red[tid / warpSize] = off;
      red[8 + tid / warpSize] = tot;
    }
    __syncthreads();
    off = 0.0;
    tot = 0.0;
    for (int w = 0; w < (nt + warpSize - 1) / warpSize; ++w) {
      off += red[w];
      tot += red[8 + w];
    }
    __syncthreads();   // every thread has read red before it is written again
    if (!(off > 1e-28 * tot)) break;   // also ends on an all-zero matrix
    for (int r = 0; r + 1 < m; ++r) {
      // round r pairs index m - 1 with r and (r + k) with (r - k) modulo m - 1
      if (tid < half) {
        int p = tid == 0 ? r : (r + tid) % (m - 1);
        int q = tid == 0 ? m - 1 : (r - tid + (m - 1)) % (m - 1);
        if (p > q) {
          const int s = p;
          p = q;
          q = s;
        }
        double c = 1.0, s = 0.0;
        if (q < nb) {
          const double apq = A[p * ld + q];
          if (apq != 0.0) {
            // the rotation that zeroes the (p, q) entry, the smaller of the two angles
            const double tau = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
            const double at = fabs(tau);
            const double tt = at > 1e150 ? 0.5 / tau : (tau >= 0.0 ? 1.0 : -1.0) / (at + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        } else {
          q = -1;   // the dummy index: no rotation
        }
        pp[tid] = p;
        pq[tid] = q;
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // columns p, q of A and of V (A J, V J)
      for (int t = tid; t < nb * half; t += nt) {
        const int i = t / half, k = t % half;
        const int p = pp[k], q = pq[k];
        if (q < 0) continue;
        const double c = cs[k], s = sn[k];
        const double ap = A[i * ld + p], aq = A[i * ld + q];
        A[i * ld + p] = c * ap - s * aq;
        A[i * ld + q] = s * ap + c * aq;
        const double vp = V[i * ld + p], vq = V[i * ld + q];
        V[i * ld + p] = c * vp - s * vq;
        V[i * ld + q] = s * vp + c * vq;
      }
      __syncthreads();
      // rows p, q of A (J^T A J); the rotated pair's own entries are zero
      for (int t = tid; t < nb * half; t += nt) {
        const int k = t / nb, c2i = t % nb;
        const int p = pp[k], q = pq[k];
        if (q < 0) continue;
        const double c = cs[k], s = sn[k];
        const double ap = A[p * ld + c2i], aq = A[q * ld + c2i];
        A[p * ld + c2i] = (c2i == q) ? 0.0 : c * ap - s * aq;
        A[q * ld + c2i] = (c2i == p) ? 0.0 : s * ap + c * aq;
      }
      __syncthreads();
    }
  }
  const long long lj = (long long)l * batch + j;
  for (int b = tid; b < nb; b += nt) lam_d[lj * nb + b] = (T)A[b * ld + b];
  for (int t = tid; t < nb * nb; t += nt) evec[lj * nb * nb + t] = V[(t / nb) * ld + t % nb];
}

// jrot[l][mock][q2][k] = sum_b jtab[l][q2][b] V_{l,mock}[b][k], zero for k >= nbins
// (grid.y = (l, mock)); MB >= nbins bins held in registers
template <typename T, int MB>
__global__ void __launch_bounds__(256) k_rotate_jtab(const T* jtab, T* jrot, const double* evec, int nq2, int nbins,
                                                     int nbp, int batch) {
  __shared__ double v[MB * MB];
  const int lj = blockIdx.y, l = lj / batch;
  const double* V = evec + (long long)lj * nbins * nbins;
  for (int t = threadIdx.x; t < nbins * nbins; t += blockDim.x) v[(t / nbins) * MB + t % nbins] = V[t];
  __syncthreads();
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq2; q += gridDim.x * blockDim.x) {
    const T* src = jtab + ((long long)l * nq2 + q) * nbp;
    T* dst = jrot + ((long long)lj * nq2 + q) * nbp;
    double jb[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) jb[b] = b < nbins ? (double)src[b] : 0.0;
    for (int k = 0; k < nbp; ++k) {
      double acc = 0.0;
      if (k < nbins) {
#pragma unroll
        for (int b = 0; b < MB; ++b)
          if (b < nbins) acc += jb[b] * v[b * MB + k];
      }
      dst[k] = (T)acc;
    }
  }
}

// zeta[mock][l] = V zetabar V^T in place, written symmetric (one workgroup per (l, mock))
__global__ void __launch_bounds__(256) k_rotate_zeta(double* zeta, const double* evec, int nbins, int lmax, int batch) {
  extern __shared__ __align__(16) char smem[];
  const int l = blockIdx.x, j = blockIdx.y, nb = nbins, nb2 = nbins * nbins;
  double* zt = reinterpret_cast<double*>(smem);   // zetabar
  double* v = zt + nb2;
  double* w = v + nb2;                             // V zetabar
  double* z = zeta + ((long long)j * (lmax + 1) + l) * nb2;
  const double* V = evec + ((long long)l * batch + j) * nb2;
  for (int t = threadIdx.x; t < nb2; t += blockDim.x) {
    zt[t] = z[t];
    v[t] = V[t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb2; t += blockDim.x) {
    const int b = t / nb, kp = t % nb;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += v[b * nb + k] * zt[k * nb + kp];
    w[t] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb2; t += blockDim.x) {
    const int b = t / nb, bp = t % nb;
    if (b > bp) continue;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += w[b * nb + k] * v[bp * nb + k];
    z[b * nb + bp] = s;
    z[bp * nb + b] = s;
  }
}

// ---------------------------------------------------------------------------
// last adjoint pass: y-transform of every adjoint source c_b, summed over the
// bins with the radial window, times the angular factor (common to the bins),
// accumulated into G(q) (one read-modify-write per (l, m))
// ---------------------------------------------------------------------------
// float32: four waves per SIMD (128 registers; the angular factors wait in
// LDS, so the bin loop holds the bin sum, the column and the window values)
template <int N, typename T>
__global__ void __launch_bounds__((strided_threads<N, T, VB>())) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
k_adjoint_y(const c2<T>* fields, c2<T>* G,
                                                                          const T* jtab, int jmocks, int nq2, int nbins,
                                                                          int nbp, const ItemRec* items, int item0,
                                                                          int nitems, int batch, double scale,
                                                                          const c2<T>* tw, const T* phi) {
  using F = Fft<N, VB>;
  constexpr int ZC = zc_of<T>();
  constexpr int GT = tiles_per_wg<N, T, VB>();
  constexpr int RMAX = F::RMAX;
  constexpr long long N3 = (long long)N * N * N;
  __shared__ c2<T> lds[GT * N * ZC];
  __shared__ c2<T> tws[N];
  // each thread's angular factors, parked in LDS while the bins are summed
  // (registers hold the bin sum only): [RMAX][threads]
  extern __shared__ __align__(16) char dyn[];
  c2<T>* facs = reinterpret_cast<c2<T>*>(dyn);
  stage_twiddles<N, T>(tw, tws);
  __syncthreads();
  const int tid = threadIdx.x;
  const int cc = tid % ZC;
  const int j = (tid / ZC) % F::TPC;
  const int g = tid / (ZC * F::TPC);
  const int tile = blockIdx.x * GT + g;
  constexpr int chunks = N / ZC;
  const bool active = tile < N * chunks;
  const int qx = active ? tile / chunks : 0;
  const int qz = (active ? tile % chunks : 0) * ZC + cc;
  const long long mock = blockIdx.y;
  c2<T>* dst = G + mock * N3 + (long long)qx * N * N + qz;
  int q2[RMAX];
#pragma unroll
  for (int e = 0; e < RMAX; ++e) {
    const int qxs = sfreq(qx, N), qys = sfreq(F::out_index(j, e), N), qzs = sfreq(qz, N);
    q2[e] = qxs * qxs + qys * qys + qzs * qzs;
  }
  for (int gi = 0; gi < nitems; ++gi) {
    const ItemRec& it = items[item0 + gi];
    // one element at a time: the float64 recurrences of the elements do not
    // run side by side (registers)
#pragma unroll 1
    for (int e = 0; e < RMAX; ++e) {
      int q2e;
      facs[e * blockDim.x + tid] =
          window_angular<T>(qx, F::out_index(j, e), qz, N, it.l, it.m, it.norm, scale * it.wm, it.yr, q2e, phi);
    }
    c2<T> acc[RMAX];
#pragma unroll
    for (int e = 0; e < RMAX; ++e) acc[e] = mk<T>(0, 0);
    const T* jl = jtab + ((long long)it.l * jmocks + mock % jmocks) * nq2 * nbp;
    const c2<T>* src = fields + ((long long)gi * batch + mock) * nbins * N3 + (long long)qx * N * N + qz;
    // next bin's column, one bin ahead
    c2<T> vn[RMAX];
    if (active) {
#pragma unroll
      for (int r = 0; r < RMAX; ++r) vn[r] = nt_load(&src[F::in_index(j, r) * N]);
    }
    for (int bq = 0; bq < nbins; bq += 4) {
      T jq[RMAX][4];
#pragma unroll
      for (int e = 0; e < RMAX; ++e) load_quad<T>(jl + (long long)q2[e] * nbp + bq, jq[e]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int b = bq + k;
        if (b < nbins) {
          c2<T> v[RMAX];
#pragma unroll
          for (int r = 0; r < RMAX; ++r) v[r] = vn[r];
          if (b + 1 < nbins && active) {
#pragma unroll
            for (int r = 0; r < RMAX; ++r) vn[r] = nt_load(&src[(b + 1) * N3 + F::in_index(j, r) * N]);
          }
          int jj = j;
          asm volatile("" : "+v"(jj));
          fft_column<N, +1, T, false, VB>(v, lds + g * N * ZC + cc, ZC, jj, tws, active);
#pragma unroll
          for (int e = 0; e < RMAX; ++e) {
            acc[e].x += jq[e][k] * v[e].x;
            acc[e].y += jq[e][k] * v[e].y;
          }
        }
      }
    }
    // the window's angular factor is common to every bin: applied once, into G
    if (active) {
#pragma unroll
      for (int e = 0; e < RMAX; ++e) {
        c2<T>* p = dst + F::out_index(j, e) * N;
        nt_store(p, cadd<T>(nt_load(p), cmul<T>(acc[e], facs[e * blockDim.x + tid])));
      }
    }
  }
}

// ddelta = scale (direct + 2 Re Ghat)
template <typename T>
__global__ void k_grad_combine(const T* direct, const c2<T>* ghat, T* ddelta, long long count, double scale) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    ddelta[i] = (T)(scale * ((double)direct[i] + 2.0 * (double)ghat[i].x));
}

// ---------------------------------------------------------------------------
// adjoint of the particle summation
// ---------------------------------------------------------------------------
// Per particle (tile order), in the eigenbasis of the cotangent (the fields
// come from the rotated radial tables, lam_d holds the eigenvalues): gather
// atilde_b(u_i), form v_b = d_b conj(atilde_b), add wm sum_b d_b |atilde_b|^2
// to F_J(u_i) (the primary vertex's share of J) and store the adjoint source
// s_b(i) = N^3 (w_i / W) v_b at the particle's sorted slot.  One lane per
// (particle, bin), 32 or 64 lanes per particle.
template <typename T>
__global__ void __launch_bounds__(256) k_gather_source(const c2<T>* fields, const int* tcell, const T* twt,
                                                        const float* w, const int* perm, const long long* off,
                                                        const double* W, const T* lam_d, int n, int nbins, T wm,
                                                        double* FJ, c2<T>* src) {
  const int lpp = nbins <= 32 ? 32 : 64;
  const int ppp = blockDim.x / lpp;
  const long long mock = blockIdx.y;
  const long long n3 = (long long)n * n * n;
  const long long a0 = off[mock], a1 = off[mock + 1];
  const long long per = (a1 - a0 + gridDim.x - 1) / gridDim.x;
  const long long s0 = a0 + per * blockIdx.x, s1 = min(a1, s0 + per);
  const double fw = (double)n3 / W[mock];
  const int b = threadIdx.x % lpp, g = threadIdx.x / lpp;
  const T d = b < nbins ? lam_d[mock * nbins + b] : (T)0;
  const c2<T>* fm = fields + mock * n3 * nbins;
  for (long long c0 = s0; c0 < s1; c0 += ppp) {
    const long long si = c0 + g;
    const bool has = si < s1;
    const int i = has ? perm[si] : 0;
    T fj = 0;
    if (has && b < nbins) {
      c2<T> acc = mk<T>(0, 0);
      const int cell = tcell[si];
      if (cell >= 0) acc = gather_record<T>(fm, cell, twt + si * 12, n, nbins, b);
      const T e = d * acc.x, f2 = d * acc.y;
      fj = e * acc.x + f2 * acc.y;
      const T f = (T)(fw * (w ? (double)w[i] : 1.0));
      src[si * nbins + b] = mk<T>(f * e, -(f * f2));
    }
    for (int o = lpp / 2; o > 0; o >>= 1) fj += __shfl_xor(fj, o, lpp);
    if (has && b == 0) FJ[i] += (double)wm * (double)fj;
  }
}

// Adjoint source on the grid, c_b(x) = sum_i B3(u_i - x) s_b(i), by pulling:
// a workgroup owns an 8^3-node tile and BC bins, and every thread owns two of
// its nodes with BC complex accumulators in registers (no atomics on values).
// Candidates are the particles of the 4^3-cell sort tiles covering cells
// x0 - 4 .. x0 + 11 per axis, taken 256 at a time through a prefix sum over
// the 64 tiles' counts.  The ones whose stencil reaches the tile (first tap
// at local offset -3 .. 7 per axis) are staged in LDS with their tap weights
// and sources, bucketed by first-tap cell (11^3 buckets, counting sort), and
// each node then visits the 4^3 buckets that can reach it.  Batches of up to
// SCQ particles keep the LDS bounded in dense regions.  Every node has one
// owner: the tile is written once, empty tiles as zeros.
__device__ __forceinline__ int tap_offset(int base, int o, int n) {
  int r = (base - o) % n;
  return r < 0 ? r + n : r;
}

constexpr int SCT = 8;                    // owner tile side (nodes)
constexpr int SCB = (SCT + 3) * (SCT + 3) * (SCT + 3);   // first-tap buckets
// bins per owner workgroup: float32 8, or 10 where that saves a pass over the
// candidates (17..20 bins: two passes instead of three, 23 % faster at 512^3);
// float64 4 up to 8 bins, 10 beyond (scatter_bc_f64)
template <typename T> constexpr int scatter_bc() { return sizeof(T) == 4 ? 8 : 4; }
inline int scatter_bc_f32(int nbins) { return (nbins + 9) / 10 < (nbins + 7) / 8 ? 10 : 8; }
// float64 beyond 8 bins: 10 bins per workgroup (two workgroups per CU by LDS)
// instead of 4, so that 20 bins take two passes over the candidates, not five
inline int scatter_bc_f64(int nbins) { return nbins > 8 ? 10 : 4; }
template <typename T> constexpr int scatter_q() { return sizeof(T) == 4 ? 256 : 256; }

template <typename T, int BC>
struct ScatterLds {
  size_t key, wt, sv, cnt, ord, total;
  __host__ __device__ ScatterLds() {
    constexpr int Q = scatter_q<T>();
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = (o + b + 15) & ~(size_t)15; return r; };
    key = take((size_t)Q * sizeof(int));
    wt = take((size_t)Q * 12 * sizeof(T));
    sv = take((size_t)Q * BC * sizeof(c2<T>));
    cnt = take((size_t)(SCB + 1) * sizeof(int));
    ord = take((size_t)Q * sizeof(int));
    total = o;
  }
};

template <typename T, int BC>
__global__ void __launch_bounds__(256) k_scatter_source(const int* tcell, const T* twt, const int* toff,
                                                         const c2<T>* src, int n, int nbins, int nchunk, c2<T>* out) {
  constexpr int TO = SCT, TB = SCT + 3;
  constexpr int NODES = TO * TO * TO;
  constexpr int Q = scatter_q<T>();
  extern __shared__ __align__(16) char smem[];
  const ScatterLds<T, BC> L;
  int* qkey = reinterpret_cast<int*>(smem + L.key);          // bucket of each staged particle
  T* qwt = reinterpret_cast<T*>(smem + L.wt);                // [q][3][4] tap weights
  c2<T>* qsv = reinterpret_cast<c2<T>*>(smem + L.sv);        // [q][BC] sources
  int* cnt = reinterpret_cast<int*>(smem + L.cnt);           // bucket counts, then starts
  int* ord = reinterpret_cast<int*>(smem + L.ord);           // staged particles in bucket order
  __shared__ int pre[65];
  __shared__ int cbase[64];
  __shared__ int qn;
  __shared__ int wsum[4];
  const int tid = threadIdx.x;
  const int no = n / TO;
  const int ot = blockIdx.x;
  const int oxi = ot / (no * no), oyi = (ot / no) % no, ozi = ot % no;
  const int o0[3] = {oxi * TO, oyi * TO, ozi * TO};
  const int mock = blockIdx.y / nchunk, b0 = (blockIdx.y % nchunk) * BC;
  const int nbc = min(BC, nbins - b0);
  const int ntd = n / 4;
  const long long ns = (long long)ntd * ntd * ntd;
  if (tid < 64) {
    const int sx = wrapi(2 * oxi - 1 + tid / 16, ntd), sy = wrapi(2 * oyi - 1 + (tid / 4) % 4, ntd);
    const int sz = wrapi(2 * ozi - 1 + tid % 4, ntd);
    const long long tile = mock * ns + ((long long)sx * ntd + sy) * ntd + sz;
    const int a = toff[tile];
    cbase[tid] = a;
    pre[tid + 1] = toff[tile + 1] - a;
  }
  if (tid == 0) qn = 0;
  __syncthreads();
  if (tid == 0) {
    pre[0] = 0;
    for (int c = 1; c <= 64; ++c) pre[c] += pre[c - 1];
  }
  __syncthreads();
  const int total = pre[64];
  // owned nodes: tid and tid + 256
  c2<T> acc[2][BC];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) acc[h][bb] = mk<T>(0, 0);
  for (int t0 = 0; t0 <= total; t0 += blockDim.x) {
    // stage this pass's candidates that reach the tile
    const int t = t0 + tid;
    if (t < total) {
      int lo = 0, hi = 64;                      // pre[lo] <= t < pre[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= t) lo = mid; else hi = mid;
      }
      const int k = cbase[lo] + (t - pre[lo]);
      const int cell = tcell[k];
      const int cb[3] = {(cell & 1023) - 1, ((cell >> 10) & 1023) - 1, (cell >> 20) - 1};   // first tap per axis
      int rl[3];
      bool reach = cell >= 0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int r = tap_offset(cb[d], o0[d], n);
        rl[d] = r < TO ? r : r - n;             // -3 .. 7 when the stencil reaches the tile
        reach = reach && (r < TO || r >= n - 3);
      }
      if (reach) {
        const int q = atomicAdd(&qn, 1);
        qkey[q] = ((rl[0] + 3) * TB + (rl[1] + 3)) * TB + (rl[2] + 3);
        const T* wr = twt + (long long)k * 12;
#pragma unroll
        for (int e = 0; e < 12; ++e) qwt[q * 12 + e] = wr[e];
        const c2<T>* sp = src + (long long)k * nbins + b0;
#pragma unroll
        for (int bb = 0; bb < BC; ++bb) qsv[q * BC + bb] = bb < nbc ? sp[bb] : mk<T>(0, 0);
      }
    }
    __syncthreads();
    const int nq = qn;
    __syncthreads();                              // every thread has read qn before it changes
    // pull when the next pass might overflow the stage, and at the end
    if (nq > Q - (int)blockDim.x || t0 + (int)blockDim.x > total) {
      for (int c = tid; c <= SCB; c += blockDim.x) cnt[c] = 0;
      __syncthreads();
      for (int q = tid; q < nq; q += blockDim.x) atomicAdd(&cnt[qkey[q] + 1], 1);
      __syncthreads();
      // exclusive starts: cnt[c] = first slot of bucket c (c = 0 .. SCB)
      {
        constexpr int PER = (SCB + 1 + 255) / 256;
        int loc[PER];
        int run = 0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          const int c = tid * PER + e;
          loc[e] = c <= SCB ? cnt[c] : 0;
          run += loc[e];
        }
        // block-wide exclusive scan of the per-thread sums
        int incl = run;
        for (int o = 1; o < 64; o <<= 1) {
          const int v = __shfl_up(incl, o, 64);
          if ((tid & 63) >= o) incl += v;
        }
        if ((tid & 63) == 63) wsum[tid >> 6] = incl;
        __syncthreads();
        int woff = 0;
        for (int w = 0; w < (tid >> 6); ++w) woff += wsum[w];
        int ex = woff + incl - run;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
          const int c = tid * PER + e;
          ex += loc[e];
          if (c <= SCB) cnt[c] = ex;              // sum of the counts of buckets 0 .. c - 1
        }
      }
      __syncthreads();
      // cnt[c] is now the start of bucket c (counts were stored at c + 1)
      for (int q = tid; q < nq; q += blockDim.x) {
        const int slot = atomicAdd(&cnt[qkey[q]], 1);
        ord[slot] = q;
      }
      __syncthreads();
      // after the fill cnt[c] is the end of bucket c = start of bucket c + 1;
      // bucket c spans [c == 0 ? 0 : cnt[c - 1], cnt[c])
      // the 4 buckets (z taps c = 0..3) of one (a, b) row are consecutive keys,
      // so their particles form one contiguous range of ord
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int node = tid + h * 256;
        const int i = node / (TO * TO), j = (node / TO) % TO, kz = node % TO;
        for (int a = 0; a < 4; ++a) {
          for (int b = 0; b < 4; ++b) {
            const int rowc = ((i - a + 3) * TB + (j - b + 3)) * TB + 3 + kz;   // key of tap c = 0
            const int k0 = rowc - 3;
            const int e0 = k0 == 0 ? 0 : cnt[k0 - 1], e1 = cnt[rowc];
            for (int e = e0; e < e1; ++e) {
              const int q = ord[e];
              const int c = rowc - qkey[q];
              const T w = qwt[(q * 3 + 0) * 4 + a] * qwt[(q * 3 + 1) * 4 + b] * qwt[(q * 3 + 2) * 4 + c];
#pragma unroll
              for (int bb = 0; bb < BC; ++bb) {
                const c2<T> v = qsv[q * BC + bb];
                acc[h][bb].x += w * v.x;
                acc[h][bb].y += w * v.y;
              }
            }
          }
        }
      }
      __syncthreads();
      if (tid == 0) qn = 0;
      __syncthreads();
    }
  }
  const long long n3 = (long long)n * n * n;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int node = tid + h * 256;
    const int i = node / (TO * TO), j = (node / TO) % TO, k = node % TO;
    const long long cell = ((long long)(o0[0] + i) * n + o0[1] + j) * n + o0[2] + k;
#pragma unroll
    for (int bb = 0; bb < BC; ++bb)
      if (bb < nbc) out[((long long)mock * nbins + b0 + bb) * n3 + cell] = acc[h][bb];
  }
}

// ---------------------------------------------------------------------------
// adjoint of the grid summation with connection coefficients
// ---------------------------------------------------------------------------
// zeta is the exact 5-point Gauss-Legendre quadrature over every cell of
// delta_B(u) sum lam atilde_{b1}(u) conj(atilde_{b2}(u)), so for one (l, m)
//   c_b(x)    = sum_q B3(u_q - x) w_q delta_B(u_q) v_b(u_q),   v_b = sum_b' lam_s[b][b'] conj(atilde_b'),
//   direct(x) += wm sum_q B3(u_q - x) w_q F(u_q),               F = sum_b Re(atilde_b v_b):
// the transposes of the three interpolations of k_gamma_contract applied to
// the node sources.  A workgroup takes a 4^3-cell tile as the forward does,
// per x node and per y cell (5 y nodes x 20 z nodes) interpolates the fields
// to the nodes, forms v and F there, and folds the sources back through the
// transposed z, y and x interpolations into a 7^3-coefficient LDS accumulator,
// which it adds to c and direct with global atomics (neighbouring tiles
// overlap by three coefficients per axis).
constexpr int AGY = 5;                      // y nodes per adjoint slice (one y cell)
constexpr int AGK = AGY * GN;               // nodes per slice (100)
constexpr int AGRS = AGK + AGK / 16 + 1;
constexpr int AGH = 4;                      // bins per thread in the per-node step
constexpr int AGP = 5;                      // threads per node in that step (AGP * AGH >= bins)

template <typename T>
struct GammaAdjLds {
  size_t C, D, Ct, Dt, P, Pd, Pt, Pdt, Q, Qd, Qt, Qdt, A, W, Wq, Fh, lam, total;
  __host__ __device__ GammaAdjLds(int nbins) {
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = (o + b + 15) & ~(size_t)15; return r; };
    const size_t c = sizeof(c2<T>), r = sizeof(T);
    C = take((size_t)GC * GC * GC * nbins * c);
    D = take((size_t)GC * GC * GC * r);
    Ct = take((size_t)GC * GC * GC * nbins * c);
    Dt = take((size_t)GC * GC * GC * r);
    P = take((size_t)GC * GC * nbins * c);
    Pd = take((size_t)GC * GC * r);
    Pt = take((size_t)GC * GC * nbins * c);
    Pdt = take((size_t)GC * GC * r);
    Q = take((size_t)AGY * GC * nbins * c);
    Qd = take((size_t)AGY * GC * r);
    Qt = take((size_t)AGY * GC * nbins * c);
    Qdt = take((size_t)AGY * GC * r);
    A = take((size_t)nbins * AGRS * c);
    W = take((size_t)AGK * r);
    Wq = take((size_t)AGK * r);
    Fh = take((size_t)AGP * AGK * r);
    lam = take((size_t)nbins * nbins * r);
    total = o;
  }
};

// float: 1024 threads, for the same reason as k_gamma_contract; double needs
// more than the 128 registers a 1024-thread workgroup leaves each lane.
// FUSED: the node values and weights of each slice are also contracted for
// zeta (the partials of k_gamma_contract), so value and gradient share one
// interpolation of the fields.
template <typename T, bool FUSED = false, bool MF = false, bool QUAD = false>
__global__ void __launch_bounds__(sizeof(T) == 4 ? 1024 : 512) k_gamma_adjoint(const c2<T>* fields, const T* delta, const T* lam_s, int n,
                                                        int nbins, GammaQuad gq, T wm, c2<T>* cout, T* direct,
                                                        double* partials) {
  extern __shared__ __align__(16) char smem[];
  const GammaAdjLds<T> L(nbins);
  c2<T>* C = reinterpret_cast<c2<T>*>(smem + L.C);
  T* D = reinterpret_cast<T*>(smem + L.D);
  c2<T>* Ct = reinterpret_cast<c2<T>*>(smem + L.Ct);
  T* Dt = reinterpret_cast<T*>(smem + L.Dt);
  c2<T>* P = reinterpret_cast<c2<T>*>(smem + L.P);
  T* Pd = reinterpret_cast<T*>(smem + L.Pd);
  c2<T>* Pt = reinterpret_cast<c2<T>*>(smem + L.Pt);
  T* Pdt = reinterpret_cast<T*>(smem + L.Pdt);
  c2<T>* Q = reinterpret_cast<c2<T>*>(smem + L.Q);
  T* Qd = reinterpret_cast<T*>(smem + L.Qd);
  c2<T>* Qt = reinterpret_cast<c2<T>*>(smem + L.Qt);
  T* Qdt = reinterpret_cast<T*>(smem + L.Qdt);
  c2<T>* A = reinterpret_cast<c2<T>*>(smem + L.A);
  T* W = reinterpret_cast<T*>(smem + L.W);
  T* Wq = reinterpret_cast<T*>(smem + L.Wq);
  T* Fh = reinterpret_cast<T*>(smem + L.Fh);
  T* lam = reinterpret_cast<T*>(smem + L.lam);
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long mock = blockIdx.y;
  const long long n3 = (long long)n * n * n;
  const c2<T>* fm = fields + mock * n3 * nbins;
  const T* dm = delta + mock * n3;
  c2<T>* cm = cout + mock * nbins * n3;
  T* rm = direct + mock * n3;
  const int nb2 = nbins * nbins;
  for (int t = tid; t < nb2; t += nt) lam[t] = lam_s[mock * nb2 + t];
  Contractor<T, MF, false, QUAD> ctr;
  if constexpr (FUSED) ctr.init(nbins);
  const int td = n / GT;
  const long long ntiles = (long long)td * td * td;
  constexpr int NC = GC * GC * GC;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int tx = (int)(tile / ((long long)td * td)), ty = (int)((tile / td) % td), tz = (int)(tile % td);
    const int x0 = tx * GT - 1, y0 = ty * GT - 1, z0 = tz * GT - 1;     // first coefficient (periodic)
    __syncthreads();
    for (int e = tid; e < NC * nbins; e += nt) {
      const int b = e % nbins, c = e / nbins;
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      const long long cell = ((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n);
      C[e] = fm[cell * nbins + b];
      Ct[e] = mk<T>(0, 0);
    }
    for (int c = tid; c < NC; c += nt) {
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      D[c] = dm[((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n)];
      Dt[c] = (T)0;
    }
    for (int xn = 0; xn < GN; ++xn) {
      const int cx = xn / 5, sx = xn % 5;
      __syncthreads();
      // x interpolation: P[j][k][b], Pd[j][k]; clear the transposed accumulators
      for (int e = tid; e < GC * GC * nbins; e += nt) {
        const int b = e % nbins, jk = e / nbins;
        c2<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const c2<T> v = C[((cx + t) * GC * GC + jk) * nbins + b];
          const T m = gq_m<T>(gq, sx, t);
          acc.x += m * v.x;
          acc.y += m * v.y;
        }
        P[e] = acc;
        Pt[e] = mk<T>(0, 0);
      }
      for (int jk = tid; jk < GC * GC; jk += nt) {
        T acc = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc += gq_m<T>(gq, sx, t) * D[(cx + t) * GC * GC + jk];
        Pd[jk] = acc;
        Pdt[jk] = (T)0;
      }
      for (int cy = 0; cy < GT; ++cy) {
        __syncthreads();
        // y interpolation for the 5 y nodes of cell cy: Q[yh][k][b], Qd[yh][k]
        for (int e = tid; e < AGY * GC * nbins; e += nt) {
          const int b = e % nbins, yk = e / nbins;
          const int yh = yk / GC, k = yk % GC;
          c2<T> acc = mk<T>(0, 0);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const c2<T> v = P[((cy + t) * GC + k) * nbins + b];
            const T m = gq_m<T>(gq, yh, t);
            acc.x += m * v.x;
            acc.y += m * v.y;
          }
          Q[e] = acc;
        }
        for (int yk = tid; yk < AGY * GC; yk += nt) {
          const int yh = yk / GC, k = yk % GC;
          T acc = 0;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc += gq_m<T>(gq, yh, t) * Pd[(cy + t) * GC + k];
          Qd[yk] = acc;
        }
        __syncthreads();
        // z interpolation to the nodes: A[b][node], node = yh * GN + zn; weights
        for (int e = tid; e < AGK * nbins; e += nt) {
          const int b = e % nbins, node = e / nbins;
          const int yh = node / GN, zn = node % GN, cz = zn / 5, sz = zn % 5;
          c2<T> acc = mk<T>(0, 0);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const c2<T> v = Q[(yh * GC + cz + t) * nbins + b];
            const T m = gq_m<T>(gq, sz, t);
            acc.x += m * v.x;
            acc.y += m * v.y;
          }
          A[b * AGRS + lds_pos<true>(node)] = acc;
        }
        for (int node = tid; node < AGK; node += nt) {
          const int yh = node / GN, zn = node % GN, cz = zn / 5, sz = zn % 5;
          T acc = 0;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc += gq_m<T>(gq, sz, t) * Qd[yh * GC + cz + t];
          const T wq = gq_w<T>(gq, sx) * gq_w<T>(gq, yh) * gq_w<T>(gq, sz);
          W[node] = acc * wq;                  // w_q delta_B(u_q)
          Wq[node] = wq;
        }
        __syncthreads();
        // FUSED: contraction of the node values (read only in this phase)
        if constexpr (FUSED) ctr.add(A, W, nbins, AGRS, AGK);
        // per node and AGH bins: v_b = sum_b' lam_s[b][b'] conj(a_b'), F; the
        // node's field values are read from LDS once into registers
        c2<T> vh[AGH];
        const bool vthread = tid < AGP * AGK;
        const int vnode = tid / AGP, vh0 = (tid % AGP) * AGH;
        if (vthread) {
          const int zp = lds_pos<true>(vnode);
          c2<T> av[AGP * AGH];
#pragma unroll
          for (int bp = 0; bp < AGP * AGH; ++bp) av[bp] = bp < nbins ? A[bp * AGRS + zp] : mk<T>(0, 0);
          T f = 0;
#pragma unroll
          for (int i = 0; i < AGH; ++i) {
            const int b = vh0 + i;
            c2<T> v = mk<T>(0, 0);
            if (b < nbins) {
              const T* lrow = lam + b * nbins;
#pragma unroll
              for (int bp = 0; bp < AGP * AGH; ++bp) {
                if (bp < nbins) {
                  const T lv = lrow[bp];
                  v.x += lv * av[bp].x;
                  v.y -= lv * av[bp].y;
                }
              }
              const c2<T> a = A[b * AGRS + zp];
              f += a.x * v.x - a.y * v.y;
            }
            vh[i] = v;
          }
          Fh[tid] = f;
        }
        __syncthreads();
        // node sources: S_b = w_q delta_B v_b over A; direct source w_q F into Fh[AGP node]
        if (vthread) {
          const int zp = lds_pos<true>(vnode);
          const T wv = W[vnode];
#pragma unroll
          for (int i = 0; i < AGH; ++i) {
            const int b = vh0 + i;
            if (b < nbins) A[b * AGRS + zp] = mk<T>(wv * vh[i].x, wv * vh[i].y);
          }
        }
        __syncthreads();
        if (tid < AGK) {
          T f = 0;
#pragma unroll
          for (int q = 0; q < AGP; ++q) f += Fh[AGP * tid + q];
          Fh[AGP * tid] = Wq[tid] * f;
        }
        __syncthreads();
        // transposed z: Qt[yh][kz][b] = sum_{tz, sz} M[sz][tz] S_b(yh, 5 (kz - tz) + sz)
        for (int e = tid; e < AGY * GC * nbins; e += nt) {
          const int b = e % nbins, yk = e / nbins;
          const int yh = yk / GC, kz = yk % GC;
          c2<T> acc = mk<T>(0, 0);
#pragma unroll
          for (int tz = 0; tz < 4; ++tz) {
            const int cz = kz - tz;
            if (cz < 0 || cz >= GT) continue;
#pragma unroll
            for (int sz = 0; sz < 5; ++sz) {
              const c2<T> v = A[b * AGRS + lds_pos<true>(yh * GN + 5 * cz + sz)];
              const T m = gq_m<T>(gq, sz, tz);
              acc.x += m * v.x;
              acc.y += m * v.y;
            }
          }
          Qt[e] = acc;
        }
        for (int yk = tid; yk < AGY * GC; yk += nt) {
          const int yh = yk / GC, kz = yk % GC;
          T acc = 0;
#pragma unroll
          for (int tz = 0; tz < 4; ++tz) {
            const int cz = kz - tz;
            if (cz < 0 || cz >= GT) continue;
#pragma unroll
            for (int sz = 0; sz < 5; ++sz) acc += gq_m<T>(gq, sz, tz) * Fh[AGP * (yh * GN + 5 * cz + sz)];
          }
          Qdt[yk] = acc;
        }
        __syncthreads();
        // transposed y: Pt[cy + ty][kz][b] += sum_yh M[yh][ty] Qt[yh][kz][b]
        for (int e = tid; e < 4 * GC * nbins; e += nt) {
          const int b = e % nbins, tk = e / nbins;
          const int tyy = tk / GC, kz = tk % GC;
          c2<T> acc = mk<T>(0, 0);
#pragma unroll
          for (int yh = 0; yh < AGY; ++yh) {
            const c2<T> v = Qt[(yh * GC + kz) * nbins + b];
            const T m = gq_m<T>(gq, yh, tyy);
            acc.x += m * v.x;
            acc.y += m * v.y;
          }
          c2<T>& o = Pt[((cy + tyy) * GC + kz) * nbins + b];
          o.x += acc.x;
          o.y += acc.y;
        }
        for (int tk = tid; tk < 4 * GC; tk += nt) {
          const int tyy = tk / GC, kz = tk % GC;
          T acc = 0;
#pragma unroll
          for (int yh = 0; yh < AGY; ++yh) acc += gq_m<T>(gq, yh, tyy) * Qdt[yh * GC + kz];
          Pdt[(cy + tyy) * GC + kz] += acc;
        }
      }
      __syncthreads();
      // transposed x: Ct[cx + tx][j][k][b] += M[sx][tx] Pt[j][k][b]
      for (int e = tid; e < 4 * GC * GC * nbins; e += nt) {
        const int b = e % nbins, r = e / nbins;
        const int txx = r / (GC * GC), jk = r % (GC * GC);
        const c2<T> v = Pt[jk * nbins + b];
        const T m = gq_m<T>(gq, sx, txx);
        c2<T>& o = Ct[((cx + txx) * GC * GC + jk) * nbins + b];
        o.x += m * v.x;
        o.y += m * v.y;
      }
      for (int r = tid; r < 4 * GC * GC; r += nt) {
        const int txx = r / (GC * GC), jk = r % (GC * GC);
        Dt[(cx + txx) * GC * GC + jk] += gq_m<T>(gq, sx, txx) * Pdt[jk];
      }
    }
    __syncthreads();
    // fold the tile into the grid (neighbouring tiles share coefficients)
    for (int e = tid; e < NC * nbins; e += nt) {
      const int b = e % nbins, c = e / nbins;
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      const long long cell = ((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n);
      c2<T>* o = cm + (long long)b * n3 + cell;
      atomicAdd(&o->x, Ct[e].x);
      atomicAdd(&o->y, Ct[e].y);
    }
    for (int c = tid; c < NC; c += nt) {
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      atomicAdd(&rm[((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n)], wm * Dt[c]);
    }
  }
  if constexpr (FUSED) {
    __syncthreads();
    ctr.finish(reinterpret_cast<double*>(smem), partials + ((long long)mock * gridDim.x + blockIdx.x) * nbins * nbins,
               nbins);
  }
}

// ---------------------------------------------------------------------------
// grid-Gamma adjoint by bin chunks (plans whose tiles of every bin do not fit
// the LDS): v_b = sum_b' lam_s[b][b'] conj(atilde_b') is the conjugate of the
// interpolant of U_b = sum_b' lam_s[b][b'] a_b' (the interpolation is real
// and linear), so with U mixed on the grid first, each bin's sources
//   c_b(x) = sum_q B3(u_q - x) w_q delta_B(u_q) conj(U~_b(u_q))
// and each bin's share of the primary term
//   F = sum_b Re(atilde_b conj(U~_b))
// need only that bin's a and U: a tile takes the bins in chunks.
// ---------------------------------------------------------------------------
// U[mock][x][b] = sum_b' lam_s[mock][b][b'] F[mock][x][b'] (bin-interleaved)
template <typename T>
__global__ void k_bin_mix(const c2<T>* F, const T* lam_s, c2<T>* U, long long n3, int nbins) {
  extern __shared__ __align__(16) char smem_mix[];
  T* lam = reinterpret_cast<T*>(smem_mix);
  const long long mock = blockIdx.y;
  const int nb2 = nbins * nbins;
  for (int t = threadIdx.x; t < nb2; t += blockDim.x) lam[t] = lam_s[mock * nb2 + t];
  __syncthreads();
  const c2<T>* fm = F + mock * n3 * nbins;
  c2<T>* um = U + mock * n3 * nbins;
  const long long total = n3 * nbins;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long x = e / nbins;
    const int b = (int)(e - x * nbins);
    const c2<T>* row = fm + x * nbins;
    const T* lrow = lam + b * nbins;
    T re = 0, im = 0;
    for (int bp = 0; bp < nbins; ++bp) {
      const c2<T> a = row[bp];
      re += lrow[bp] * a.x;
      im += lrow[bp] * a.y;
    }
    um[e] = mk<T>(re, im);
  }
}

template <typename T>
struct GammaBinsLds {
  size_t C, Cu, Ct, D, Dt, P, Pu, Pt, Pd, Pdt, Q, Qu, Qt, Qd, Qdt, A, Au, W, Wq, Fn, total;
  __host__ __device__ GammaBinsLds(int nbc) {
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = (o + b + 15) & ~(size_t)15; return r; };
    const size_t c = sizeof(c2<T>), r = sizeof(T);
    const size_t nc = (size_t)GC * GC * GC;
    C = take(nc * nbc * c);
    Cu = take(nc * nbc * c);
    Ct = take(nc * nbc * c);
    D = take(nc * r);
    Dt = take(nc * r);
    P = take((size_t)GC * GC * nbc * c);
    Pu = take((size_t)GC * GC * nbc * c);
    Pt = take((size_t)GC * GC * nbc * c);
    Pd = take((size_t)GC * GC * r);
    Pdt = take((size_t)GC * GC * r);
    Q = take((size_t)AGY * GC * nbc * c);
    Qu = take((size_t)AGY * GC * nbc * c);
    Qt = take((size_t)AGY * GC * nbc * c);
    Qd = take((size_t)AGY * GC * r);
    Qdt = take((size_t)AGY * GC * r);
    A = take((size_t)nbc * AGRS * c);
    Au = take((size_t)nbc * AGRS * c);
    W = take((size_t)AGK * r);
    Wq = take((size_t)AGK * r);
    Fn = take((size_t)AGK * r);
    total = o;
  }
};

// bins b0 .. b0 + nbc - 1 of nbt; adds the sources into cout (zeroed by the
// caller) and wm times this chunk's share of the primary term into direct
template <typename T>
__global__ void __launch_bounds__(512) k_gamma_adjoint_bins(const c2<T>* fields, const c2<T>* U, const T* delta,
                                                            int n, int nbt, int b0, int nbc, GammaQuad gq, T wm,
                                                            c2<T>* cout, T* direct) {
  extern __shared__ __align__(16) char smem[];
  const GammaBinsLds<T> L(nbc);
  c2<T>* C = reinterpret_cast<c2<T>*>(smem + L.C);
  c2<T>* Cu = reinterpret_cast<c2<T>*>(smem + L.Cu);
  c2<T>* Ct = reinterpret_cast<c2<T>*>(smem + L.Ct);
  T* D = reinterpret_cast<T*>(smem + L.D);
  T* Dt = reinterpret_cast<T*>(smem + L.Dt);
  c2<T>* P = reinterpret_cast<c2<T>*>(smem + L.P);
  c2<T>* Pu = reinterpret_cast<c2<T>*>(smem + L.Pu);
  c2<T>* Pt = reinterpret_cast<c2<T>*>(smem + L.Pt);
  T* Pd = reinterpret_cast<T*>(smem + L.Pd);
  T* Pdt = reinterpret_cast<T*>(smem + L.Pdt);
  c2<T>* Q = reinterpret_cast<c2<T>*>(smem + L.Q);
  c2<T>* Qu = reinterpret_cast<c2<T>*>(smem + L.Qu);
  c2<T>* Qt = reinterpret_cast<c2<T>*>(smem + L.Qt);
  T* Qd = reinterpret_cast<T*>(smem + L.Qd);
  T* Qdt = reinterpret_cast<T*>(smem + L.Qdt);
  c2<T>* A = reinterpret_cast<c2<T>*>(smem + L.A);
  c2<T>* Au = reinterpret_cast<c2<T>*>(smem + L.Au);
  T* W = reinterpret_cast<T*>(smem + L.W);
  T* Wq = reinterpret_cast<T*>(smem + L.Wq);
  T* Fn = reinterpret_cast<T*>(smem + L.Fn);
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long mock = blockIdx.y;
  const long long n3 = (long long)n * n * n;
  const c2<T>* fm = fields + mock * n3 * nbt;
  const c2<T>* um = U + mock * n3 * nbt;
  const T* dm = delta + mock * n3;
  c2<T>* cm = cout + mock * nbt * n3;
  T* rm = direct + mock * n3;
  const int td = n / GT;
  const long long ntiles = (long long)td * td * td;
  constexpr int NC = GC * GC * GC;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int tx = (int)(tile / ((long long)td * td)), ty = (int)((tile / td) % td), tz = (int)(tile % td);
    const int x0 = tx * GT - 1, y0 = ty * GT - 1, z0 = tz * GT - 1;
    __syncthreads();
    for (int e = tid; e < NC * nbc; e += nt) {
      const int b = e % nbc, c = e / nbc;
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      const long long cell = ((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n);
      C[e] = fm[cell * nbt + b0 + b];
      Cu[e] = um[cell * nbt + b0 + b];
      Ct[e] = mk<T>(0, 0);
    }
    for (int c = tid; c < NC; c += nt) {
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      D[c] = dm[((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n)];
      Dt[c] = (T)0;
    }
    for (int xn = 0; xn < GN; ++xn) {
      const int cx = xn / 5, sx = xn % 5;
      __syncthreads();
      // x interpolation of a, U and delta; clear the transposed accumulators
      for (int e = tid; e < GC * GC * nbc; e += nt) {
        const int b = e % nbc, jk = e / nbc;
        c2<T> acc = mk<T>(0, 0), accu = mk<T>(0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int src = ((cx + t) * GC * GC + jk) * nbc + b;
          const T m = gq_m<T>(gq, sx, t);
          const c2<T> v = C[src], u = Cu[src];
          acc.x += m * v.x;
          acc.y += m * v.y;
          accu.x += m * u.x;
          accu.y += m * u.y;
        }
        P[e] = acc;
        Pu[e] = accu;
        Pt[e] = mk<T>(0, 0);
      }
      for (int jk = tid; jk < GC * GC; jk += nt) {
        T acc = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc += gq_m<T>(gq, sx, t) * D[(cx + t) * GC * GC + jk];
        Pd[jk] = acc;
        Pdt[jk] = (T)0;
      }
      for (int cy = 0; cy < GT; ++cy) {
        __syncthreads();
        // y interpolation for the 5 y nodes of cell cy
        for (int e = tid; e < AGY * GC * nbc; e += nt) {
          const int b = e % nbc, yk = e / nbc;
          const int yh = yk / GC, k = yk % GC;
          c2<T> acc = mk<T>(0, 0), accu = mk<T>(0, 0);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int src = ((cy + t) * GC + k) * nbc + b;
            const T m = gq_m<T>(gq, yh, t);
            const c2<T> v = P[src], u = Pu[src];
            acc.x += m * v.x;
            acc.y += m * v.y;
            accu.x += m * u.x;
            accu.y += m * u.y;
          }
          Q[e] = acc;
          Qu[e] = accu;
        }
        for (int yk = tid; yk < AGY * GC; yk += nt) {
          const int yh = yk / GC, k = yk % GC;
          T acc = 0;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc += gq_m<T>(gq, yh, t) * Pd[(cy + t) * GC + k];
          Qd[yk] = acc;
        }
        __syncthreads();
        // z interpolation to the 100 nodes of this (x node, y cell) slice
        for (int e = tid; e < AGK * nbc; e += nt) {
          const int b = e % nbc, node = e / nbc;
          const int yh = node / GN, zn = node % GN, cz = zn / 5, sz = zn % 5;
          c2<T> acc = mk<T>(0, 0), accu = mk<T>(0, 0);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int src = (yh * GC + cz + t) * nbc + b;
            const T m = gq_m<T>(gq, sz, t);
            const c2<T> v = Q[src], u = Qu[src];
            acc.x += m * v.x;
            acc.y += m * v.y;
            accu.x += m * u.x;
            accu.y += m * u.y;
          }
          A[b * AGRS + lds_pos<true>(node)] = acc;
          Au[b * AGRS + lds_pos<true>(node)] = accu;
        }
        for (int node = tid; node < AGK; node += nt) {
          const int yh = node / GN, zn = node % GN, cz = zn / 5, sz = zn % 5;
          T acc = 0;
#pragma unroll
          for (int t = 0; t < 4; ++t) acc += gq_m<T>(gq, sz, t) * Qd[yh * GC + cz + t];
          const T wq = gq_w<T>(gq, sx) * gq_w<T>(gq, yh) * gq_w<T>(gq, sz);
          W[node] = acc * wq;
          Wq[node] = wq;
        }
        __syncthreads();
        // per node: F (this chunk's bins) and the sources S_b = w delta_B conj(U~_b), over A
        for (int node = tid; node < AGK; node += nt) {
          const int zp = lds_pos<true>(node);
          const T wv = W[node];
          T f = 0;
          for (int b = 0; b < nbc; ++b) {
            const c2<T> a = A[b * AGRS + zp], u = Au[b * AGRS + zp];
            f += a.x * u.x + a.y * u.y;
            A[b * AGRS + zp] = mk<T>(wv * u.x, -wv * u.y);
          }
          Fn[node] = Wq[node] * f;
        }
        __syncthreads();
        // transposed z
        for (int e = tid; e < AGY * GC * nbc; e += nt) {
          const int b = e % nbc, yk = e / nbc;
          const int yh = yk / GC, kz = yk % GC;
          c2<T> acc = mk<T>(0, 0);
#pragma unroll
          for (int tz = 0; tz < 4; ++tz) {
            const int cz = kz - tz;
            if (cz < 0 || cz >= GT) continue;
#pragma unroll
            for (int sz = 0; sz < 5; ++sz) {
              const c2<T> v = A[b * AGRS + lds_pos<true>(yh * GN + 5 * cz + sz)];
              const T m = gq_m<T>(gq, sz, tz);
              acc.x += m * v.x;
              acc.y += m * v.y;
            }
          }
          Qt[e] = acc;
        }
        for (int yk = tid; yk < AGY * GC; yk += nt) {
          const int yh = yk / GC, kz = yk % GC;
          T acc = 0;
#pragma unroll
          for (int tz = 0; tz < 4; ++tz) {
            const int cz = kz - tz;
            if (cz < 0 || cz >= GT) continue;
#pragma unroll
            for (int sz = 0; sz < 5; ++sz) acc += gq_m<T>(gq, sz, tz) * Fn[yh * GN + 5 * cz + sz];
          }
          Qdt[yk] = acc;
        }
        __syncthreads();
        // transposed y
        for (int e = tid; e < 4 * GC * nbc; e += nt) {
          const int b = e % nbc, tk = e / nbc;
          const int tyy = tk / GC, kz = tk % GC;
          c2<T> acc = mk<T>(0, 0);
#pragma unroll
          for (int yh = 0; yh < AGY; ++yh) {
            const c2<T> v = Qt[(yh * GC + kz) * nbc + b];
            const T m = gq_m<T>(gq, yh, tyy);
            acc.x += m * v.x;
            acc.y += m * v.y;
          }
          c2<T>& o = Pt[((cy + tyy) * GC + kz) * nbc + b];
          o.x += acc.x;
          o.y += acc.y;
        }
        for (int tk = tid; tk < 4 * GC; tk += nt) {
          const int tyy = tk / GC, kz = tk % GC;
          T acc = 0;
#pragma unroll
          for (int yh = 0; yh < AGY; ++yh) acc += gq_m<T>(gq, yh, tyy) * Qdt[yh * GC + kz];
          Pdt[(cy + tyy) * GC + kz] += acc;
        }
      }
      __syncthreads();
      // transposed x
      for (int e = tid; e < 4 * GC * GC * nbc; e += nt) {
        const int b = e % nbc, r = e / nbc;
        const int txx = r / (GC * GC), jk = r % (GC * GC);
        const c2<T> v = Pt[jk * nbc + b];
        const T m = gq_m<T>(gq, sx, txx);
        c2<T>& o = Ct[((cx + txx) * GC * GC + jk) * nbc + b];
        o.x += m * v.x;
        o.y += m * v.y;
      }
      for (int r = tid; r < 4 * GC * GC; r += nt) {
        const int txx = r / (GC * GC), jk = r % (GC * GC);
        Dt[(cx + txx) * GC * GC + jk] += gq_m<T>(gq, sx, txx) * Pdt[jk];
      }
    }
    __syncthreads();
    // fold the tile into the grid (neighbouring tiles share coefficients)
    for (int e = tid; e < NC * nbc; e += nt) {
      const int b = e % nbc, c = e / nbc;
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      const long long cell = ((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n);
      c2<T>* o = cm + (long long)(b0 + b) * n3 + cell;
      atomicAdd(&o->x, Ct[e].x);
      atomicAdd(&o->y, Ct[e].y);
    }
    for (int c = tid; c < NC; c += nt) {
      const int i = c / (GC * GC), j = (c / GC) % GC, k = c % GC;
      atomicAdd(&rm[((long long)wrapi(x0 + i, n) * n + wrapi(y0 + j, n)) * n + wrapi(z0 + k, n)], wm * Dt[c]);
    }
  }
}

// zeta[mock][l][g(i)][g(j)] += scale sum_w partials[mock][w][i][j] for the local
// pairs (i, j) of a chunk-pair contraction that this pass owns: the cross
// block always, the diagonal block of the first chunk when own_a, of the
// second when own_c (local i < na is field bin a0 + i, else c0 + i - na)
__global__ void k_reduce_partials_map(const double* partials, int nwg, int nl, double* zeta, int l, int lmax,
                                      double scale, int nbt, int a0, int na, int c0, int own_a, int own_c) {
  __shared__ double sh[32];
  const int e = blockIdx.x, mock = blockIdx.y;
  const int i = e / nl, j = e % nl;
  const bool ia = i < na, ja = j < na;
  if (ia && ja && !own_a) return;
  if (!ia && !ja && !own_c) return;
  const int nl2 = nl * nl;
  const double* p = partials + (long long)mock * nwg * nl2 + e;
  double s = 0.0;
  for (int w = threadIdx.x; w < nwg; w += blockDim.x) s += p[(long long)w * nl2];
  s = block_sum(s, sh);
  const int gi = ia ? a0 + i : c0 + i - na, gj = ja ? a0 + j : c0 + j - na;
  if (threadIdx.x == 0) zeta[((long long)mock * (lmax + 1) + l) * nbt * nbt + (long long)gi * nbt + gj] += scale * s;
}

// h[mock][s] = sum_l (2l+1) sum_{b1,b2} dzeta[mock][l][b1][b2] jbar_{l,b1}(s) jbar_{l,b2}(s):
// the weight of |dhat(q)|^2 B7hat(q) in sum_l <dzeta_l, 4 pi Fbar_l>
template <typename T>
__global__ void k_fbar_weight(const double* dzeta, const T* jtab, int nq2, int nbp, int nbins, int lmax, double* h) {
  const int mock = blockIdx.y;
  const int nb2 = nbins * nbins;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nq2; s += gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int l = 0; l <= lmax; ++l) {
      const T* jl = jtab + ((long long)l * nq2 + s) * nbp;
      const double* dz = dzeta + ((long long)mock * (lmax + 1) + l) * nb2;
      double al = 0.0;
      for (int b1 = 0; b1 < nbins; ++b1) {
        double r = 0.0;
        for (int b2 = 0; b2 < nbins; ++b2) r += dz[b1 * nbins + b2] * (double)jl[b2];
        al += (double)jl[b1] * r;
      }
      acc += (2.0 * l + 1.0) * al;
    }
    h[(long long)mock * nq2 + s] = acc;
  }
}

// G(q) += scale B7hat(q) h(|q|^2) conj(dhat(q)), Nyquist planes excluded: the
// volume-mean term of the particle form's gradient, added in k-space before
// the final transform
template <typename T>
__global__ void k_fbar_adjoint(const c2<T>* dhat, const double* h, int n, int nq2, double scale, c2<T>* G,
                               const T* phi, Acf acf) {
  const long long n3 = (long long)n * n * n;
  const int mock = blockIdx.y;
  const c2<T>* d = dhat + mock * n3;
  c2<T>* gm = G + mock * n3;
  const double* hm = h + (long long)mock * nq2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n3; i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i / ((long long)n * n)), iy = (int)((i / n) % n), iz = (int)(i % n);
    const int qx = sfreq(ix, n), qy = sfreq(iy, n), qz = sfreq(iz, n);
    const int hh = -n / 2;
    if (qx == hh || qy == hh || qz == hh) continue;
    const double tp = 2.0 * 3.14159265358979323846 / n;
    double b7 = 1.0;
    const int qs[3] = {qx, qy, qz};
#pragma unroll
    for (int a = 0; a < 3; ++a) b7 *= acf_hat(acf, tp * qs[a]);
    if (phi) {
      const double ph = (double)phi[ix] * (double)phi[iy] * (double)phi[iz];
      b7 *= ph * ph;
    }
    const double f = scale * b7 * hm[qx * qx + qy * qy + qz * qz];
    const c2<T> v = d[i];
    c2<T> o = gm[i];
    o.x = (T)((double)o.x + f * (double)v.x);
    o.y = (T)((double)o.y - f * (double)v.y);
    gm[i] = o;
  }
}

// dw_i += 4 pi [ F_J(u_i) / W - sum_j w_j F_J(u_j) / W^2 ]: the primary vertex's weights
template <typename T>
__global__ void k_primary_dw(const long long* off, int batch, long long np_total, const double* FJ, const double* W,
                             const double* SF, T* dw) {
  const double fp = 12.566370614359172953850573533118011536788677597500;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < np_total; i += (long long)gridDim.x * blockDim.x) {
    const int mock = find_mock(off, batch, i);
    const double Wj = W[mock];
    dw[i] = (T)((double)dw[i] + fp * (FJ[i] / Wj - SF[mock] / (Wj * Wj)));
  }
}

}  // namespace mp3

// ===========================================================================
// host launchers
// ===========================================================================
namespace mp3 {

namespace {

inline unsigned grid_for(long long count, int threads, unsigned cap = 65535u * 4) {
  long long g = (count + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > (long long)cap) g = cap;
  return (unsigned)g;
}

template <typename T> using CT = c2<T>;

// dynamic LDS of the strided transform: the column tiles plus the twiddles
template <int N, typename T, int V> inline size_t xlds() {
  return ((size_t)tiles_x<N, T, V>() * N * zcx_of<N, T, V>() + N) * sizeof(CT<T>);
}
// above 64 KB the kernels must be allowed the larger dynamic LDS
template <int N, typename T, int V> inline hipError_t allow_x() {
  const size_t b = xlds<N, T, V>();
  if (b <= 65536) return hipSuccess;
  const void* ks[4] = {reinterpret_cast<const void*>(k_fft_strided<N, T, -1, false, V>),
                       reinterpret_cast<const void*>(k_fft_strided<N, T, +1, false, V>),
                       reinterpret_cast<const void*>(k_fft_strided<N, T, -1, true, V>),
                       reinterpret_cast<const void*>(k_fft_strided<N, T, +1, true, V>)};
  for (const void* k : ks) {
    const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int N, typename T>
hipError_t fft3d_t(int dir, bool real_in, const void* in, void* out, int nfields, const void* tw, hipStream_t st) {
  if (const hipError_t e = allow_x<N, T, 0>(); e != hipSuccess) return e;
  constexpr int ZC = zcx_of<N, T>();
  constexpr int G = tiles_x<N, T>();
  constexpr int threads = Fft<N>::TPC * ZC * G;
  constexpr long long N3 = (long long)N * N * N;
  const dim3 gs((N * (N / ZC) + G - 1) / G, nfields);
  CT<T>* o = static_cast<CT<T>*>(out);
  const CT<T>* t = static_cast<const CT<T>*>(tw);
  // x axis (stride N^2), tiles over (y, z-chunk)
  if (dir < 0) {
    if (real_in) k_fft_strided<N, T, -1, true><<<gs, threads, xlds<N, T, 0>(), st>>>(in, o, N3, N3, N * N, N, t);
    else k_fft_strided<N, T, -1, false><<<gs, threads, xlds<N, T, 0>(), st>>>(in, o, N3, N3, N * N, N, t);
    k_fft_strided<N, T, -1, false><<<gs, threads, xlds<N, T, 0>(), st>>>(o, o, N3, N3, N, N * N, t);
  } else {
    if (real_in) k_fft_strided<N, T, +1, true><<<gs, threads, xlds<N, T, 0>(), st>>>(in, o, N3, N3, N * N, N, t);
    else k_fft_strided<N, T, +1, false><<<gs, threads, xlds<N, T, 0>(), st>>>(in, o, N3, N3, N * N, N, t);
    k_fft_strided<N, T, +1, false><<<gs, threads, xlds<N, T, 0>(), st>>>(o, o, N3, N3, N, N * N, t);
  }
  constexpr int P = contig_pencils<N, T>();
  const long long npen = (long long)nfields * N * N;
  const unsigned gz = (unsigned)((npen + P - 1) / P);
  if (dir < 0) k_fft_contig<N, T, -1><<<gz, P * Fft<N>::TPC, 0, st>>>(o, o, npen, t);
  else k_fft_contig<N, T, +1><<<gz, P * Fft<N>::TPC, 0, st>>>(o, o, npen, t);
  return hipGetLastError();
}

template <int N, typename T, int V>
hipError_t fft_x_v(int dir, void* buf, int nfields, const void* tw, hipStream_t st) {
  if (const hipError_t e = allow_x<N, T, V>(); e != hipSuccess) return e;
  constexpr int ZC = zcx_of<N, T, V>();
  constexpr int G = tiles_x<N, T, V>();
  constexpr int threads = Fft<N, V>::TPC * ZC * G;
  constexpr long long N3 = (long long)N * N * N;
  const dim3 gs((N * (N / ZC) + G - 1) / G, nfields);
  CT<T>* o = static_cast<CT<T>*>(buf);
  const CT<T>* t = static_cast<const CT<T>*>(tw);
  if (dir < 0) k_fft_strided<N, T, -1, false, V><<<gs, threads, xlds<N, T, V>(), st>>>(o, o, N3, N3, N * N, N, t);
  else k_fft_strided<N, T, +1, false, V><<<gs, threads, xlds<N, T, V>(), st>>>(o, o, N3, N3, N * N, N, t);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t fft_x_t(int dir, void* buf, int nfields, const void* tw, int variant, hipStream_t st) {
  return variant ? fft_x_v<N, T, 1>(dir, buf, nfields, tw, st) : fft_x_v<N, T, 0>(dir, buf, nfields, tw, st);
}

template <int N, typename T>
hipError_t fft_y_t(int dir, void* buf, int nfields, const void* tw, hipStream_t st) {
  if (const hipError_t e = allow_x<N, T, 0>(); e != hipSuccess) return e;
  constexpr int ZC = zcx_of<N, T>();
  constexpr int G = tiles_x<N, T>();
  constexpr int threads = Fft<N>::TPC * ZC * G;
  constexpr long long N3 = (long long)N * N * N;
  const dim3 gs((N * (N / ZC) + G - 1) / G, nfields);
  CT<T>* o = static_cast<CT<T>*>(buf);
  const CT<T>* t = static_cast<const CT<T>*>(tw);
  if (dir < 0) k_fft_strided<N, T, -1, false><<<gs, threads, xlds<N, T, 0>(), st>>>(o, o, N3, N3, N, N * N, t);
  else k_fft_strided<N, T, +1, false><<<gs, threads, xlds<N, T, 0>(), st>>>(o, o, N3, N3, N, N * N, t);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t fft_z_t(int dir, const void* in, void* out, int nfields, const void* tw, hipStream_t st) {
  constexpr int P = contig_pencils<N, T>();
  const long long npen = (long long)nfields * N * N;
  const unsigned gz = (unsigned)((npen + P - 1) / P);
  const CT<T>* i = static_cast<const CT<T>*>(in);
  CT<T>* o = static_cast<CT<T>*>(out);
  const CT<T>* t = static_cast<const CT<T>*>(tw);
  if (dir < 0) k_fft_contig<N, T, -1><<<gz, P * Fft<N>::TPC, 0, st>>>(i, o, npen, t);
  else k_fft_contig<N, T, +1><<<gz, P * Fft<N>::TPC, 0, st>>>(i, o, npen, t);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t filter_y_t(const FilterArgs& a, hipStream_t st) {
  constexpr int ZC = zc_of<T>();
  constexpr int G = tiles_per_wg<N, T, VB>();
  constexpr int threads = Fft<N, VB>::TPC * ZC * G;
  const dim3 gs((N * (N / ZC) + G - 1) / G, a.batch * a.nitems);
  k_filter_y<N, T><<<gs, threads, 0, st>>>(static_cast<const CT<T>*>(a.src), static_cast<CT<T>*>(a.dst),
                                          static_cast<const T*>(a.jtab), a.jmocks, a.nq2, a.nbins, a.nbp, a.items,
                                          a.item0, a.batch, a.scale, static_cast<const CT<T>*>(a.tw),
                                          static_cast<const T*>(a.phi));
  return hipGetLastError();
}

template <int N, typename T>
hipError_t adjoint_y_t(const FilterArgs& a, hipStream_t st) {
  constexpr int ZC = zc_of<T>();
  constexpr int G = tiles_per_wg<N, T, VB>();
  constexpr int threads = Fft<N, VB>::TPC * ZC * G;
  const dim3 gs((N * (N / ZC) + G - 1) / G, a.batch);
  const size_t dyn = (size_t)threads * Fft<N, VB>::RMAX * sizeof(CT<T>);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_adjoint_y<N, T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
  if (e != hipSuccess) return e;
  k_adjoint_y<N, T><<<gs, threads, dyn, st>>>(static_cast<const CT<T>*>(a.src), static_cast<CT<T>*>(a.dst),
                                           static_cast<const T*>(a.jtab), a.jmocks, a.nq2, a.nbins, a.nbp, a.items,
                                           a.item0, a.nitems, a.batch, a.scale, static_cast<const CT<T>*>(a.tw),
                                           static_cast<const T*>(a.phi));
  return hipGetLastError();
}

// z-pass workgroup: nbc columns (bins) per round, rounds balanced, <= 512 threads
template <int N, int V> inline int zpass_threads(int nbins) {
  constexpr int TPC = Fft<N, V>::TPC;
  const int hi = 512 / TPC;
  const int rounds = (nbins + hi - 1) / hi;
  int nbc = (nbins + rounds - 1) / rounds;
  int lo = TPC >= 64 ? 1 : 64 / TPC;
  const int lo_delta = (N / DPRE + TPC - 1) / TPC;   // at least N / DPRE threads
  if (lo < lo_delta) lo = lo_delta;
  if (lo > hi) lo = hi;
  if (nbc < lo) nbc = lo;
  return nbc * TPC;
}

template <int N, typename T> inline size_t zpass_nodal_lds(int nbins, int threads) {
  constexpr int RS = zrow<N>();
  size_t a = (size_t)nbins * RS * sizeof(CT<T>) + (size_t)N * sizeof(CT<T>) + (size_t)N * sizeof(T);
  size_t r = (size_t)threads * 16 * sizeof(double);
  return a > r ? a : r;
}

template <int N, typename T> inline size_t zpass_adjoint_lds(int nbins) {
  constexpr int RS = zrow<N>();
  // the cotangent's eigenvalues, padded to the largest MAXNB that serves nbins
  const size_t maxnb = nbins <= 8 ? 8 : nbins <= 12 ? 12 : nbins <= 16 ? 16 : nbins <= 20 ? 20 : nbins <= 24 ? 24
                       : nbins <= 32 ? 32 : nbins <= 48 ? 48 : 64;
  return (size_t)nbins * RS * sizeof(CT<T>) + (size_t)N * sizeof(CT<T>) + maxnb * sizeof(T);
}

template <typename K> hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int N, typename T, bool MF, bool SPLIT = false, bool QUAD = false>
hipError_t zpass_nodal_mf(const ZpassArgs& a, hipStream_t st) {
  const int threads = zpass_threads<N, VZN>(a.nbins);
  size_t lds = zpass_nodal_lds<N, T>(a.nbins, threads);
  const size_t red = Contractor<T, MF, SPLIT, QUAD>::scratch_bytes(threads);
  if (lds < red) lds = red;
  hipError_t e = allow_lds(k_zpass_nodal<N, T, MF, SPLIT, QUAD>, lds);
  if (e != hipSuccess) return e;
  const dim3 gs(a.nwg, a.batch);
  k_zpass_nodal<N, T, MF, SPLIT, QUAD><<<gs, threads, lds, st>>>(static_cast<const CT<T>*>(a.fields),
                                                                static_cast<const T*>(a.delta), a.partials, a.nbins,
                                                                a.ppw, static_cast<const CT<T>*>(a.tw));
  return hipGetLastError();
}

// bins per launch of the store pass: as many as the LDS holds
template <int N, typename T> inline int zpass_store_bins(int nbins) {
  const size_t per = (size_t)zrow<N>() * sizeof(CT<T>);
  const size_t room = (size_t)160 * 1024 - (size_t)N * sizeof(CT<T>);
  const int cb = (int)(room / per);
  return nbins < cb ? nbins : cb;
}

template <int N, typename T>
hipError_t zpass_store_t(const ZpassArgs& a, void* out, hipStream_t st) {
  const int cb = zpass_store_bins<N, T>(a.nbins);
  for (int b0 = 0; b0 < a.nbins; b0 += cb) {
    const int nb = a.nbins - b0 < cb ? a.nbins - b0 : cb;
    const int threads = zpass_threads<N, VZN>(nb);
    const size_t lds = (size_t)nb * zrow<N>() * sizeof(CT<T>) + (size_t)N * sizeof(CT<T>);
    hipError_t e = allow_lds(k_zpass_store<N, T>, lds);
    if (e != hipSuccess) return e;
    const dim3 gs(a.nwg, a.batch);
    k_zpass_store<N, T><<<gs, threads, lds, st>>>(static_cast<const CT<T>*>(a.fields), static_cast<CT<T>*>(out), nb,
                                                 a.nbins, b0, a.ppw, static_cast<const CT<T>*>(a.tw));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// float32 with at most 32 bins contracts on the matrix cores (float32 or
// BF16-split inputs); otherwise on the vector ALUs
template <int N, typename T>
hipError_t zpass_nodal_t(const ZpassArgs& a, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (a.nbins <= 32 && zpass_threads<N, VZN>(a.nbins) % 64 == 0) {
      if (a.split) return zpass_nodal_mf<N, T, true, true>(a, st);
      if (a.nbins > 16 && a.nbins <= 20) return zpass_nodal_mf<N, T, true, false, true>(a, st);
      return zpass_nodal_mf<N, T, true>(a, st);
    }
  }
  return zpass_nodal_mf<N, T, false>(a, st);
}

// fused sweeps round the workgroup up to whole waves (the matrix-core
// contractions split the work by wave); the extra threads hold no column
template <int N, typename T> inline int zpass_fused_threads(int nbins, int waves = 0) {
  if (waves > 0) {
    // at least one thread per z point and one column; at most 8 waves (the launch bound)
    int need = N / DPRE > Fft<N, VZA<T>>::TPC ? N / DPRE : Fft<N, VZA<T>>::TPC;
    int t = 64 * waves;
    if (t < need) t = (need + 63) / 64 * 64;
    return t > 512 ? 512 : t;
  }
  return (zpass_threads<N, VZA<T>>(nbins) + 63) / 64 * 64;
}

template <int N, typename T> inline size_t zpass_fused_lds(int nbins, int threads, size_t scratch) {
  const size_t a = zpass_adjoint_lds<N, T>(nbins) + (size_t)N * sizeof(T);
  (void)threads;
  return a > scratch ? a : scratch;
}

// persistent launch over the group's (item, mock, chunk) units: at most
// kZpassResident workgroups take units from the counter (zeroed here first)
constexpr int kZpassResident = 2048;

template <int N, typename T, int MAXNB, bool FUSED = false, bool MF = false, bool QUAD = false>
hipError_t zpass_adjoint_nb(const ZpassArgs& a, hipStream_t st) {
  const int threads = FUSED ? zpass_fused_threads<N, T>(a.nbins, a.waves) : zpass_threads<N, VZA<T>>(a.nbins);
  const size_t lds = FUSED ? zpass_fused_lds<N, T>(a.nbins, threads,
                                                    Contractor<T, MF, false, QUAD>::scratch_bytes(threads))
                           : zpass_adjoint_lds<N, T>(a.nbins);
  hipError_t e = allow_lds(k_zpass_adjoint<N, T, MAXNB, FUSED, MF, QUAD>, lds);
  if (e != hipSuccess) return e;
  k_fill<int><<<1, 64, 0, st>>>(a.counter, 1, 0);
  const long long units = (long long)a.nitems * a.batch * a.nwg;
  const unsigned grid = (unsigned)(units < kZpassResident ? units : kZpassResident);
  k_zpass_adjoint<N, T, MAXNB, FUSED, MF, QUAD><<<grid, threads, lds, st>>>(
      static_cast<CT<T>*>(const_cast<void*>(a.fields)), static_cast<const T*>(a.delta), static_cast<const T*>(a.lam),
      static_cast<T*>(a.direct), a.nbins, a.ppw, static_cast<const CT<T>*>(a.tw), a.partials, a.items, a.item0,
      a.nitems, a.batch, a.nwg, a.counter);
  return hipGetLastError();
}

// value-and-gradient sweep, <= 32 bins: float32 contracts on the matrix cores
// (4x4 blocks at 17..20 bins), float64 on the vector ALUs
template <int N, typename T>
hipError_t zpass_fused_t(const ZpassArgs& a, hipStream_t st) {
  if (a.nbins > 32) return hipErrorInvalidValue;
  constexpr bool MF = std::is_same<T, float>::value;
  if (a.nbins <= 8) return zpass_adjoint_nb<N, T, 8, true, MF, false>(a, st);
  if (a.nbins <= 12) return zpass_adjoint_nb<N, T, 12, true, MF, false>(a, st);
  if (a.nbins <= 16) return zpass_adjoint_nb<N, T, 16, true, MF, false>(a, st);
  if (a.nbins <= 20) return zpass_adjoint_nb<N, T, 20, true, MF, MF>(a, st);
  if (a.nbins <= 24) return zpass_adjoint_nb<N, T, 24, true, MF, false>(a, st);
  return zpass_adjoint_nb<N, T, 32, true, MF, false>(a, st);
}

template <int N, typename T>
hipError_t zpass_adjoint_t(const ZpassArgs& a, hipStream_t st) {
  if (a.nbins <= 8) return zpass_adjoint_nb<N, T, 8>(a, st);
  if (a.nbins <= 12) return zpass_adjoint_nb<N, T, 12>(a, st);
  if (a.nbins <= 16) return zpass_adjoint_nb<N, T, 16>(a, st);
  if (a.nbins <= 20) return zpass_adjoint_nb<N, T, 20>(a, st);
  if (a.nbins <= 24) return zpass_adjoint_nb<N, T, 24>(a, st);
  if (a.nbins <= 32) return zpass_adjoint_nb<N, T, 32>(a, st);
  if (a.nbins <= 48) return zpass_adjoint_nb<N, T, 48>(a, st);
  return zpass_adjoint_nb<N, T, 64>(a, st);
}

template <int N, typename T> size_t zpass_lds_need_t(int nbins) {
  const size_t a = zpass_nodal_lds<N, T>(nbins, zpass_threads<N, VZN>(nbins));
  const size_t b = zpass_adjoint_lds<N, T>(nbins);
  return a > b ? a : b;
}

// dispatch over the grid length and the precision
#define MP3_DISPATCH(fn, n, prec, ...)                                                              \
  do {                                                                                              \
    switch (n) {                                                                                    \
      case 16: return prec ? fn<16, double>(__VA_ARGS__) : fn<16, float>(__VA_ARGS__);              \
      case 32: return prec ? fn<32, double>(__VA_ARGS__) : fn<32, float>(__VA_ARGS__);              \
      case 64: return prec ? fn<64, double>(__VA_ARGS__) : fn<64, float>(__VA_ARGS__);              \
      case 128: return prec ? fn<128, double>(__VA_ARGS__) : fn<128, float>(__VA_ARGS__);           \
      case 256: return prec ? fn<256, double>(__VA_ARGS__) : fn<256, float>(__VA_ARGS__);           \
      case 512: return prec ? fn<512, double>(__VA_ARGS__) : fn<512, float>(__VA_ARGS__);           \
      default: return hipErrorInvalidValue;                                                         \
    }                                                                                               \
  } while (0)

}  // namespace

hipError_t launch_fft3d(int n, int prec, int dir, bool real_in, const void* in, void* out, int nfields, const void* tw,
                        hipStream_t st) {
  MP3_DISPATCH(fft3d_t, n, prec, dir, real_in, in, out, nfields, tw, st);
}

hipError_t launch_fft_x(int n, int prec, int dir, void* buf, int nfields, const void* tw, int variant, hipStream_t st) {
  MP3_DISPATCH(fft_x_t, n, prec, dir, buf, nfields, tw, variant, st);
}

hipError_t launch_fft_y(int n, int prec, int dir, void* buf, int nfields, const void* tw, hipStream_t st) {
  MP3_DISPATCH(fft_y_t, n, prec, dir, buf, nfields, tw, st);
}

hipError_t launch_fft_z(int n, int prec, int dir, const void* in, void* out, int nfields, const void* tw, hipStream_t st) {
  MP3_DISPATCH(fft_z_t, n, prec, dir, in, out, nfields, tw, st);
}

hipError_t launch_filter_y(int n, int prec, const FilterArgs& a, hipStream_t st) { MP3_DISPATCH(filter_y_t, n, prec, a, st); }
hipError_t launch_adjoint_y(int n, int prec, const FilterArgs& a, hipStream_t st) { MP3_DISPATCH(adjoint_y_t, n, prec, a, st); }
hipError_t launch_zpass_nodal(int n, int prec, const ZpassArgs& a, hipStream_t st) { MP3_DISPATCH(zpass_nodal_t, n, prec, a, st); }
hipError_t launch_zpass_store(int n, int prec, const ZpassArgs& a, void* out, hipStream_t st) {
  MP3_DISPATCH(zpass_store_t, n, prec, a, out, st);
}
hipError_t launch_zpass_adjoint(int n, int prec, const ZpassArgs& a, hipStream_t st) { MP3_DISPATCH(zpass_adjoint_t, n, prec, a, st); }
hipError_t launch_zpass_fused(int n, int prec, const ZpassArgs& a, hipStream_t st) { MP3_DISPATCH(zpass_fused_t, n, prec, a, st); }

template <int N, typename T> size_t zpass_fused_lds_need_t(int nbins) {
  if (nbins > 32) return (size_t)1 << 40;
  const int threads = 512;   // the largest workgroup any waves setting gives
  constexpr bool MF = std::is_same<T, float>::value;
  const size_t red = nbins > 16 && nbins <= 20 ? Contractor<T, MF, false, MF>::scratch_bytes(threads)
                                                : Contractor<T, MF, false, false>::scratch_bytes(threads);
  return zpass_fused_lds<N, T>(nbins, threads, red);
}

size_t zpass_fused_lds_need(int n, int prec, int nbins) {
  switch (n) {
    case 16: return prec ? zpass_fused_lds_need_t<16, double>(nbins) : zpass_fused_lds_need_t<16, float>(nbins);
    case 32: return prec ? zpass_fused_lds_need_t<32, double>(nbins) : zpass_fused_lds_need_t<32, float>(nbins);
    case 64: return prec ? zpass_fused_lds_need_t<64, double>(nbins) : zpass_fused_lds_need_t<64, float>(nbins);
    case 128: return prec ? zpass_fused_lds_need_t<128, double>(nbins) : zpass_fused_lds_need_t<128, float>(nbins);
    case 256: return prec ? zpass_fused_lds_need_t<256, double>(nbins) : zpass_fused_lds_need_t<256, float>(nbins);
    case 512: return prec ? zpass_fused_lds_need_t<512, double>(nbins) : zpass_fused_lds_need_t<512, float>(nbins);
    default: return (size_t)-1;
  }
}

size_t zpass_lds_need(int n, int prec, int nbins) {
  switch (n) {
    case 16: return prec ? zpass_lds_need_t<16, double>(nbins) : zpass_lds_need_t<16, float>(nbins);
    case 32: return prec ? zpass_lds_need_t<32, double>(nbins) : zpass_lds_need_t<32, float>(nbins);
    case 64: return prec ? zpass_lds_need_t<64, double>(nbins) : zpass_lds_need_t<64, float>(nbins);
    case 128: return prec ? zpass_lds_need_t<128, double>(nbins) : zpass_lds_need_t<128, float>(nbins);
    case 256: return prec ? zpass_lds_need_t<256, double>(nbins) : zpass_lds_need_t<256, float>(nbins);
    case 512: return prec ? zpass_lds_need_t<512, double>(nbins) : zpass_lds_need_t<512, float>(nbins);
    default: return (size_t)-1;
  }
}

hipError_t launch_fill(int prec, void* p, long long count, double value, hipStream_t st) {
  const unsigned g = grid_for(count, 256, 8192);
  if (prec) k_fill<double><<<g, 256, 0, st>>>(static_cast<double*>(p), count, value);
  else k_fill<float><<<g, 256, 0, st>>>(static_cast<float*>(p), count, (float)value);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, long long count, int value, hipStream_t st) {
  const unsigned g = grid_for(count, 256, 8192);
  k_fill<int><<<g, 256, 0, st>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, long long count, double value, hipStream_t st) {
  const unsigned g = grid_for(count, 256, 8192);
  k_fill<double><<<g, 256, 0, st>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_lam_sym(int prec, const double* dzeta, void* lam_s, int nbins, int lmax, int batch, hipStream_t st) {
  const dim3 gs(lmax + 1, batch);
  if (prec) k_lam_sym<double><<<gs, 256, 0, st>>>(dzeta, static_cast<double*>(lam_s), nbins, lmax, batch);
  else k_lam_sym<float><<<gs, 256, 0, st>>>(dzeta, static_cast<float*>(lam_s), nbins, lmax, batch);
  return hipGetLastError();
}

hipError_t launch_lam_eig(int prec, const double* dzeta, void* lam_d, double* evec, int nbins, int lmax, int batch,
                          hipStream_t st) {
  if (nbins < 1 || nbins > kEigMaxBins) return hipErrorInvalidValue;
  const dim3 gs(lmax + 1, batch);
  const size_t lds = lam_eig_lds(nbins);
  if (prec) {
    hipError_t e = allow_lds(k_lam_eig<double>, lds);
    if (e != hipSuccess) return e;
    k_lam_eig<double><<<gs, 256, lds, st>>>(dzeta, static_cast<double*>(lam_d), evec, nbins, lmax, batch);
  } else {
    hipError_t e = allow_lds(k_lam_eig<float>, lds);
    if (e != hipSuccess) return e;
    k_lam_eig<float><<<gs, 256, lds, st>>>(dzeta, static_cast<float*>(lam_d), evec, nbins, lmax, batch);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t rotate_jtab_t(const void* jtab, void* jrot, const double* evec, int nq2, int nbins, int nbp, int lmax,
                         int batch, hipStream_t st) {
  const dim3 gs((unsigned)grid_for(nq2, 256, 64), (unsigned)((lmax + 1) * batch));
  const T* src = static_cast<const T*>(jtab);
  T* dst = static_cast<T*>(jrot);
  if (nbins <= 16) k_rotate_jtab<T, 16><<<gs, 256, 0, st>>>(src, dst, evec, nq2, nbins, nbp, batch);
  else if (nbins <= 32) k_rotate_jtab<T, 32><<<gs, 256, 0, st>>>(src, dst, evec, nq2, nbins, nbp, batch);
  else k_rotate_jtab<T, 64><<<gs, 256, 0, st>>>(src, dst, evec, nq2, nbins, nbp, batch);
  return hipGetLastError();
}

hipError_t launch_rotate_jtab(int prec, const void* jtab, void* jrot, const double* evec, int nq2, int nbins, int nbp,
                              int lmax, int batch, hipStream_t st) {
  if (nbins < 1 || nbins > kEigMaxBins || nbp < nbins) return hipErrorInvalidValue;
  return prec ? rotate_jtab_t<double>(jtab, jrot, evec, nq2, nbins, nbp, lmax, batch, st)
              : rotate_jtab_t<float>(jtab, jrot, evec, nq2, nbins, nbp, lmax, batch, st);
}

hipError_t launch_rotate_zeta(double* zeta, const double* evec, int nbins, int lmax, int batch, hipStream_t st) {
  if (nbins < 1 || nbins > kEigMaxBins) return hipErrorInvalidValue;
  const size_t lds = (size_t)3 * nbins * nbins * sizeof(double);
  hipError_t e = allow_lds(k_rotate_zeta, lds);
  if (e != hipSuccess) return e;
  k_rotate_zeta<<<dim3(lmax + 1, batch), 256, lds, st>>>(zeta, evec, nbins, lmax, batch);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partials, int nwg, int nb2, double* zeta, int l, int lmax, double scale,
                                  int batch, hipStream_t st) {
  const dim3 gs(nb2, batch);
  k_reduce_partials<<<gs, 256, 0, st>>>(partials, nwg, nb2, zeta, l, lmax, scale);
  return hipGetLastError();
}

hipError_t launch_reduce_items(const double* partials, int nwg, int nb2, double* zeta, int lmax, double scale,
                               const ItemRec* items, int item0, int nitems, int batch, hipStream_t st) {
  const dim3 gs(nb2, batch);
  k_reduce_items<<<gs, 256, 0, st>>>(partials, nwg, nb2, zeta, lmax, scale, items, item0, nitems, batch);
  return hipGetLastError();
}

hipError_t launch_weight_sum(const float* w, const long long* off, int batch, long long np_max, double* W, hipStream_t st) {
  const dim3 gs(grid_for(np_max, 256, 1024), batch);
  k_weight_sum<<<gs, 256, 0, st>>>(w, nullptr, off, batch, W);
  return hipGetLastError();
}

hipError_t launch_weighted_sum(const float* w, const double* f, const long long* off, int batch, long long np_max,
                               double* out, hipStream_t st) {
  const dim3 gs(grid_for(np_max, 256, 1024), batch);
  k_weight_sum<<<gs, 256, 0, st>>>(w, f, off, batch, out);
  return hipGetLastError();
}



hipError_t launch_normalise(int prec, void* eps, const double* W, long long n3, int batch, hipStream_t st) {
  const dim3 gs(grid_for(n3, 256, 4096), batch);
  if (prec) k_normalise<double><<<gs, 256, 0, st>>>(static_cast<double*>(eps), W, n3);
  else k_normalise<float><<<gs, 256, 0, st>>>(static_cast<float*>(eps), W, n3);
  return hipGetLastError();
}

hipError_t launch_grad_combine(int prec, const void* direct, const void* ghat, void* ddelta, long long count, double scale,
                               hipStream_t st) {
  const unsigned g = grid_for(count, 256, 16384);
  if (prec)
    k_grad_combine<double><<<g, 256, 0, st>>>(static_cast<const double*>(direct), static_cast<const double2*>(ghat),
                                              static_cast<double*>(ddelta), count, scale);
  else
    k_grad_combine<float><<<g, 256, 0, st>>>(static_cast<const float*>(direct), static_cast<const float2*>(ghat),
                                             static_cast<float*>(ddelta), count, scale);
  return hipGetLastError();
}

hipError_t launch_dot_rho_g(int prec, const void* delta, const void* g, long long n3, double* S, int batch, hipStream_t st) {
  const dim3 gs(grid_for(n3, 256, 1024), batch);
  if (prec) k_dot_rho_g<double><<<gs, 256, 0, st>>>(static_cast<const double*>(delta), static_cast<const double*>(g), n3, S);
  else k_dot_rho_g<float><<<gs, 256, 0, st>>>(static_cast<const float*>(delta), static_cast<const float*>(g), n3, S);
  return hipGetLastError();
}

hipError_t launch_gather_dw(int prec, const float* pos, const long long* off, int batch, long long np_total, int n,
                            double sc, const void* g, const double* W, const double* S, void* dw, const double* btab,
                            hipStream_t st) {
  const unsigned gr = grid_for(np_total, 256, 16384);
  if (prec)
    k_gather_dw<double><<<gr, 256, 0, st>>>(pos, off, batch, np_total, n, sc, static_cast<const double*>(g), W, S,
                                            static_cast<double*>(dw), btab);
  else
    k_gather_dw<float><<<gr, 256, 0, st>>>(pos, off, batch, np_total, n, sc, static_cast<const float*>(g), W, S,
                                           static_cast<float*>(dw), btab);
  return hipGetLastError();
}

hipError_t launch_tile_sort(const float* pos, const long long* off, int batch, long long np_total, int n, double sc,
                            int shift, int* counts, int* offs, int* cursor, int* perm, hipStream_t st) {
  const long long ntd = n >> shift;
  const long long nt = ntd * ntd * ntd * batch;
  k_fill<int><<<grid_for(nt + 1, 256, 8192), 256, 0, st>>>(counts, nt + 1, 0);
  const unsigned g = grid_for(np_total, 256, 16384);
  k_tile_count<<<g, 256, 0, st>>>(pos, off, batch, np_total, n, sc, shift, counts);
  k_scan_counts<<<1, 1024, 0, st>>>(counts, offs, cursor, nt + 1);
  k_tile_scatter<<<g, 256, 0, st>>>(pos, off, batch, np_total, n, sc, shift, cursor, perm);
  return hipGetLastError();
}

// Tiled deposit: a persistent grid takes TS^3-cell tiles (of every mock) from
// an atomic work counter, accumulates the tile's particles into an LDS block
// of (TS + 3)^3 nodes (the tile plus the B-spline halo) and flushes it with
// one global atomic per touched node.  Every workgroup leaves when the
// counter passes the number of tiles.  The particles of a tile were sorted
// there by the same cell arithmetic as make_taps, so their taps stay inside
// the block.
template <typename T, int TS>
__global__ void __launch_bounds__(256) k_deposit_tiled(const float* pos, const float* w, const int* perm,
                                                       const int* toff, int ntiles_total, int* counter, int n,
                                                       double sc, T* eps, const double* btab) {
  constexpr int TB = TS + 3;
  __shared__ T acc[TB * TB * TB];
  __shared__ int item_sh;
  const int ntd = n / TS;
  const int nt = ntd * ntd * ntd;
  const long long n3 = (long long)n * n * n;
  for (;;) {
    if (threadIdx.x == 0) item_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int item = item_sh;
    __syncthreads();                               // item_sh is rewritten by the next take
    if (item >= ntiles_total) break;
    const int a = toff[item], b = toff[item + 1];
    if (a == b) continue;                          // empty tile: nothing to add
    const int mock = item / nt, t = item % nt;
    const int tx = t / (ntd * ntd), ty = (t / ntd) % ntd, tz = t % ntd;
    const int ox = tx * TS - 1, oy = ty * TS - 1, oz = tz * TS - 1;   // node of local index 0
    for (int c = threadIdx.x; c < TB * TB * TB; c += blockDim.x) acc[c] = (T)0;
    __syncthreads();
    for (int k = a + threadIdx.x; k < b; k += blockDim.x) {
      const int i = perm[k];
      Taps tp = make_taps(pos + 3 * (long long)i, n, sc, btab);
      if (!tp.ok) continue;
      const double wi = w ? (double)w[i] : 1.0;
      const int lx = tp.base[0] - ox, ly = tp.base[1] - oy, lz = tp.base[2] - oz;   // in [0, TS)
#pragma unroll
      for (int ax = 0; ax < 4; ++ax) {
        const double wa = wi * tp.wt[0][ax];
#pragma unroll
        for (int ay = 0; ay < 4; ++ay) {
          const double wab = wa * tp.wt[1][ay];
          T* row = acc + ((lx + ax) * TB + (ly + ay)) * TB + lz;
#pragma unroll
          for (int az = 0; az < 4; ++az) atomicAdd(&row[az], (T)(wab * tp.wt[2][az]));
        }
      }
    }
    __syncthreads();
    T* em = eps + (long long)mock * n3;
    for (int c = threadIdx.x; c < TB * TB * TB; c += blockDim.x) {
      const T v = acc[c];
      if (v != (T)0) {
        const int i = c / (TB * TB), j = (c / TB) % TB, k = c % TB;
        atomicAdd(&em[((long long)wrapi(ox + i, n) * n + wrapi(oy + j, n)) * n + wrapi(oz + k, n)], v);
      }
    }
    __syncthreads();                               // acc is cleared by the next tile
  }
}

template <typename T>
hipError_t deposit_tiled_t(int tside, const float* pos, const float* w, const int* perm, const int* toff,
                           int ntiles_total, unsigned g, int* counter, int n, double sc, T* eps, const double* btab,
                           hipStream_t st) {
  switch (tside) {
    case 4: k_deposit_tiled<T, 4><<<g, 256, 0, st>>>(pos, w, perm, toff, ntiles_total, counter, n, sc, eps, btab); break;
    case 8: k_deposit_tiled<T, 8><<<g, 256, 0, st>>>(pos, w, perm, toff, ntiles_total, counter, n, sc, eps, btab); break;
    case 16: k_deposit_tiled<T, 16><<<g, 256, 0, st>>>(pos, w, perm, toff, ntiles_total, counter, n, sc, eps, btab); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_deposit_tiled(int prec, int tside, const float* pos, const float* w, const int* perm, const int* toff,
                                int ntiles_total, int wgs, int* counter, int n, double sc, void* eps, const double* btab,
                                hipStream_t st) {
  if (ntiles_total <= 0 || wgs <= 0 || tside <= 0 || n % tside != 0) return hipErrorInvalidValue;
  k_fill<int><<<1, 64, 0, st>>>(counter, 1, 0);
  const unsigned g = (unsigned)(ntiles_total < wgs ? ntiles_total : wgs);
  if (prec)
    return deposit_tiled_t<double>(tside, pos, w, perm, toff, ntiles_total, g, counter, n, sc,
                                   static_cast<double*>(eps), btab, st);
  return deposit_tiled_t<float>(tside, pos, w, perm, toff, ntiles_total, g, counter, n, sc, static_cast<float*>(eps),
                                btab, st);
}

template <typename T, bool MF, bool SPLIT, bool QUAD, bool SRC>
hipError_t gather_contract_v(const GatherArgs& a, hipStream_t st) {
  constexpr int K = kGatherSlots;
  const size_t rs = K + K / 16 + 1;
  size_t lds = (size_t)a.nbins * rs * sizeof(CT<T>) + K * sizeof(T);
  if (SRC) lds += K * sizeof(int) + (size_t)a.nbins * sizeof(T);
  const size_t red = Contractor<T, MF, SPLIT, QUAD>::scratch_bytes(256);
  if (lds < red) lds = red;
  hipError_t e = allow_lds(k_gather_contract<T, MF, SPLIT, QUAD, SRC>, lds);
  if (e != hipSuccess) return e;
  const dim3 gs(a.nwg, a.batch);
  k_gather_contract<T, MF, SPLIT, QUAD, SRC><<<gs, 256, lds, st>>>(
      static_cast<const CT<T>*>(a.fields), a.tcell, static_cast<const T*>(a.twt), a.w, a.perm, a.off, a.W, a.n, a.nbins,
      a.partials, static_cast<const T*>(a.lam), (T)a.wm, a.FJ, static_cast<CT<T>*>(a.src));
  return hipGetLastError();
}

template <typename T, bool MF, bool SPLIT = false, bool QUAD = false>
hipError_t gather_contract_t(const GatherArgs& a, hipStream_t st) {
  if (a.src) return gather_contract_v<T, MF, SPLIT, QUAD, true>(a, st);
  return gather_contract_v<T, MF, SPLIT, QUAD, false>(a, st);
}

hipError_t launch_gather_contract(int prec, const GatherArgs& a, hipStream_t st) {
  if (prec) return gather_contract_t<double, false>(a, st);
  if (a.nbins <= 32) {
    if (a.split) return gather_contract_t<float, true, true>(a, st);
    if (a.nbins > 16 && a.nbins <= 20) return gather_contract_t<float, true, false, true>(a, st);
    return gather_contract_t<float, true>(a, st);
  }
  return gather_contract_t<float, false>(a, st);
}

hipError_t launch_power_hist(int prec, const void* dhat, int n, int nq2, double* P, int batch, const void* phi,
                             const Acf& acf, hipStream_t st) {
  const long long n3 = (long long)n * n * n;
  const dim3 gs(grid_for(n3, 256, 8192), batch);
  if (prec) k_power_hist<double><<<gs, 256, 0, st>>>(static_cast<const double2*>(dhat), n, nq2, P,
                                                    static_cast<const double*>(phi), acf);
  else k_power_hist<float><<<gs, 256, 0, st>>>(static_cast<const float2*>(dhat), n, nq2, P,
                                                  static_cast<const float*>(phi), acf);
  return hipGetLastError();
}

hipError_t launch_fbar_subtract(int prec, const double* P, const void* jtab, int nq2, int nbp, int nbins, int l, int lmax,
                                double n6, double* zeta, int batch, hipStream_t st) {
  const dim3 gs(nbins * nbins, batch);
  if (prec)
    k_fbar_subtract<double><<<gs, 256, 0, st>>>(P, static_cast<const double*>(jtab), nq2, nbp, nbins, l, lmax, n6, zeta);
  else
    k_fbar_subtract<float><<<gs, 256, 0, st>>>(P, static_cast<const float*>(jtab), nq2, nbp, nbins, l, lmax, n6, zeta);
  return hipGetLastError();
}

template <typename T, bool MF, bool SPLIT = false, bool QUAD = false>
hipError_t gamma_contract_t(const void* fields, const void* delta, int n, const BinPair& bp, const GammaQuad& gq,
                            double* partials, int nwg, int batch, hipStream_t st) {
  const int threads = 1024;
  const int nbins = bp.na + bp.nc;
  size_t lds = GammaLds<T>(nbins).total;
  const size_t red = Contractor<T, MF, SPLIT, QUAD>::scratch_bytes(threads);
  if (lds < red) lds = red;
  hipError_t e = allow_lds(k_gamma_contract<T, MF, SPLIT, QUAD>, lds);
  if (e != hipSuccess) return e;
  const dim3 gs(nwg, batch);
  k_gamma_contract<T, MF, SPLIT, QUAD><<<gs, threads, lds, st>>>(static_cast<const CT<T>*>(fields),
                                                                static_cast<const T*>(delta), n, nbins, gq, partials,
                                                                bp.nbt, bp.a0, bp.na, bp.c0);
  return hipGetLastError();
}

GammaQuad make_gamma_quad(const double (*m)[4], const double* wq) {
  GammaQuad gq;
  for (int s = 0; s < 5; ++s) {
    for (int t = 0; t < 4; ++t) {
      gq.m[s][t] = (float)m[s][t];
      gq.md[s][t] = m[s][t];
    }
    gq.wq[s] = (float)wq[s];
    gq.wqd[s] = wq[s];
  }
  return gq;
}

hipError_t launch_gamma_contract(int prec, bool split, const void* fields, const void* delta, int n,
                                 const BinPair& bp, const double (*m)[4], const double* wq, double* partials, int nwg,
                                 int batch, hipStream_t st) {
  const GammaQuad gq = make_gamma_quad(m, wq);
  const int nbins = bp.na + bp.nc;
  if (prec) return gamma_contract_t<double, false>(fields, delta, n, bp, gq, partials, nwg, batch, st);
  if (nbins <= 32) {
    if (split) return gamma_contract_t<float, true, true>(fields, delta, n, bp, gq, partials, nwg, batch, st);
    if (nbins > 16 && nbins <= 20)
      return gamma_contract_t<float, true, false, true>(fields, delta, n, bp, gq, partials, nwg, batch, st);
    return gamma_contract_t<float, true>(fields, delta, n, bp, gq, partials, nwg, batch, st);
  }
  return gamma_contract_t<float, false>(fields, delta, n, bp, gq, partials, nwg, batch, st);
}

size_t gamma_lds_need(int prec, int nbins) {
  // the tile plus the contraction's reduction scratch (1024 threads)
  const size_t a = prec ? GammaLds<double>(nbins).total : GammaLds<float>(nbins).total;
  const size_t r = prec ? Contractor<double, false>::scratch_bytes(1024)
                        : (nbins <= 32 ? Contractor<float, true>::scratch_bytes(1024)
                                       : Contractor<float, false>::scratch_bytes(1024));
  return a > r ? a : r;
}

hipError_t launch_reduce_partials_map(const double* partials, int nwg, const BinPair& bp, double* zeta, int l,
                                      int lmax, double scale, bool own_a, bool own_c, int batch, hipStream_t st) {
  const int nl = bp.na + bp.nc;
  const dim3 gs(nl * nl, batch);
  k_reduce_partials_map<<<gs, 256, 0, st>>>(partials, nwg, nl, zeta, l, lmax, scale, bp.nbt, bp.a0, bp.na, bp.c0,
                                            own_a ? 1 : 0, own_c ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_bin_mix(int prec, const void* F, const void* lam_s, void* U, long long n3, int nbins, int batch,
                          hipStream_t st) {
  const size_t lds = (size_t)nbins * nbins * (prec ? 8 : 4);
  const dim3 gs(grid_for(n3 * nbins, 256, 16384), batch);
  if (prec)
    k_bin_mix<double><<<gs, 256, lds, st>>>(static_cast<const double2*>(F), static_cast<const double*>(lam_s),
                                            static_cast<double2*>(U), n3, nbins);
  else
    k_bin_mix<float><<<gs, 256, lds, st>>>(static_cast<const float2*>(F), static_cast<const float*>(lam_s),
                                           static_cast<float2*>(U), n3, nbins);
  return hipGetLastError();
}

template <typename T>
hipError_t gamma_adjoint_bins_t(const void* fields, const void* U, const void* delta, int n, int nbt, int b0, int nbc,
                                const GammaQuad& gq, double wm, int nwg, int batch, void* cout, void* direct,
                                hipStream_t st) {
  const size_t lds = GammaBinsLds<T>(nbc).total;
  hipError_t e = allow_lds(k_gamma_adjoint_bins<T>, lds);
  if (e != hipSuccess) return e;
  const dim3 gs(nwg, batch);
  k_gamma_adjoint_bins<T><<<gs, 512, lds, st>>>(static_cast<const CT<T>*>(fields), static_cast<const CT<T>*>(U),
                                                static_cast<const T*>(delta), n, nbt, b0, nbc, gq, (T)wm,
                                                static_cast<CT<T>*>(cout), static_cast<T*>(direct));
  return hipGetLastError();
}

hipError_t launch_gamma_adjoint_bins(int prec, const void* fields, const void* U, const void* delta, int n, int nbt,
                                     int b0, int nbc, const double (*m)[4], const double* wq, double wm, int nwg,
                                     int batch, void* cout, void* direct, hipStream_t st) {
  const GammaQuad gq = make_gamma_quad(m, wq);
  if (prec)
    return gamma_adjoint_bins_t<double>(fields, U, delta, n, nbt, b0, nbc, gq, wm, nwg, batch, cout, direct, st);
  return gamma_adjoint_bins_t<float>(fields, U, delta, n, nbt, b0, nbc, gq, wm, nwg, batch, cout, direct, st);
}

size_t gamma_adjoint_bins_lds_need(int prec, int nbc) {
  return prec ? GammaBinsLds<double>(nbc).total : GammaBinsLds<float>(nbc).total;
}

hipError_t launch_gather_source(int prec, const void* fields, const int* tcell, const void* twt, const float* w,
                                const int* perm, const long long* off, const double* W, const void* lam_d, int n,
                                int nbins, double wm, int nwg, int batch, double* FJ, void* src, hipStream_t st) {
  const dim3 gs(nwg, batch);
  if (prec)
    k_gather_source<double><<<gs, 256, 0, st>>>(static_cast<const double2*>(fields), tcell,
                                                static_cast<const double*>(twt), w, perm, off, W,
                                                static_cast<const double*>(lam_d), n, nbins, wm, FJ,
                                                static_cast<double2*>(src));
  else
    k_gather_source<float><<<gs, 256, 0, st>>>(static_cast<const float2*>(fields), tcell,
                                               static_cast<const float*>(twt), w, perm, off, W,
                                               static_cast<const float*>(lam_d), n, nbins, (float)wm, FJ,
                                               static_cast<float2*>(src));
  return hipGetLastError();
}

template <typename T, int BC>
hipError_t scatter_source_t(const int* tcell, const void* twt, const int* toff, const void* src, int n, int nbins,
                            int batch, void* out, hipStream_t st) {
  const int no = n / SCT;
  const int nchunk = (nbins + BC - 1) / BC;
  const size_t lds = ScatterLds<T, BC>().total;
  hipError_t e = allow_lds(k_scatter_source<T, BC>, lds);
  if (e != hipSuccess) return e;
  const dim3 gs(no * no * no, batch * nchunk);
  k_scatter_source<T, BC><<<gs, 256, lds, st>>>(tcell, static_cast<const T*>(twt), toff, static_cast<const CT<T>*>(src),
                                                n, nbins, nchunk, static_cast<CT<T>*>(out));
  return hipGetLastError();
}

hipError_t launch_scatter_source(int prec, const int* tcell, const void* twt, const int* toff, const void* src, int n,
                                 int nbins, int batch, void* out, hipStream_t st) {
  if (prec) {
    if (scatter_bc_f64(nbins) == 10) return scatter_source_t<double, 10>(tcell, twt, toff, src, n, nbins, batch, out, st);
    return scatter_source_t<double, scatter_bc<double>()>(tcell, twt, toff, src, n, nbins, batch, out, st);
  }
  if (scatter_bc_f32(nbins) == 10) return scatter_source_t<float, 10>(tcell, twt, toff, src, n, nbins, batch, out, st);
  return scatter_source_t<float, 8>(tcell, twt, toff, src, n, nbins, batch, out, st);
}

hipError_t launch_tap_records(int prec, const float* pos, const int* perm, long long np_total, int n, double sc,
                              int* tcell, void* twt, const double* btab, hipStream_t st) {
  const unsigned g = grid_for(np_total, 256, 16384);
  if (prec)
    k_tap_records<double><<<g, 256, 0, st>>>(pos, perm, np_total, n, sc, tcell, static_cast<double*>(twt), btab);
  else k_tap_records<float><<<g, 256, 0, st>>>(pos, perm, np_total, n, sc, tcell, static_cast<float*>(twt), btab);
  return hipGetLastError();
}

hipError_t launch_fbar_adjoint(int prec, const double* dzeta, const void* jtab, int nq2, int nbp, int nbins, int lmax,
                               const void* dhat, int n, double scale, double* h, void* G, int batch, const void* phi,
                               const Acf& acf, hipStream_t st) {
  const dim3 gh(grid_for(nq2, 256, 1024), batch);
  const long long n3 = (long long)n * n * n;
  const dim3 gs(grid_for(n3, 256, 8192), batch);
  if (prec) {
    k_fbar_weight<double><<<gh, 256, 0, st>>>(dzeta, static_cast<const double*>(jtab), nq2, nbp, nbins, lmax, h);
    k_fbar_adjoint<double><<<gs, 256, 0, st>>>(static_cast<const double2*>(dhat), h, n, nq2, scale,
                                               static_cast<double2*>(G), static_cast<const double*>(phi), acf);
  } else {
    k_fbar_weight<float><<<gh, 256, 0, st>>>(dzeta, static_cast<const float*>(jtab), nq2, nbp, nbins, lmax, h);
    k_fbar_adjoint<float><<<gs, 256, 0, st>>>(static_cast<const float2*>(dhat), h, n, nq2, scale,
                                              static_cast<float2*>(G), static_cast<const float*>(phi), acf);
  }
  return hipGetLastError();
}

hipError_t launch_primary_dw(int prec, const long long* off, int batch, long long np_total, const double* FJ,
                             const double* W, const double* SF, void* dw, hipStream_t st) {
  const unsigned gr = grid_for(np_total, 256, 16384);
  if (prec) k_primary_dw<double><<<gr, 256, 0, st>>>(off, batch, np_total, FJ, W, SF, static_cast<double*>(dw));
  else k_primary_dw<float><<<gr, 256, 0, st>>>(off, batch, np_total, FJ, W, SF, static_cast<float*>(dw));
  return hipGetLastError();
}

template <typename T, bool FUSED, bool MF, bool QUAD>
hipError_t gamma_adjoint_v(const void* fields, const void* delta, const void* lam_s, int n, int nbins,
                           const GammaQuad& gq, double wm, int nwg, int batch, void* cout, void* direct,
                           double* partials, hipStream_t st) {
  const int threads = sizeof(T) == 4 ? 1024 : 512;
  size_t lds = GammaAdjLds<T>(nbins).total;
  if (FUSED) {
    const size_t red = Contractor<T, MF, false, QUAD>::scratch_bytes(threads);
    if (lds < red) lds = red;
  }
  hipError_t e = allow_lds(k_gamma_adjoint<T, FUSED, MF, QUAD>, lds);
  if (e != hipSuccess) return e;
  const dim3 gs(nwg, batch);
  k_gamma_adjoint<T, FUSED, MF, QUAD><<<gs, threads, lds, st>>>(
      static_cast<const CT<T>*>(fields), static_cast<const T*>(delta), static_cast<const T*>(lam_s), n, nbins, gq, (T)wm,
      static_cast<CT<T>*>(cout), static_cast<T*>(direct), partials);
  return hipGetLastError();
}

hipError_t launch_gamma_adjoint(int prec, const void* fields, const void* delta, const void* lam_s, int n, int nbins,
                                const double (*m)[4], const double* wq, double wm, int nwg, int batch, void* cout,
                                void* direct, double* partials, hipStream_t st) {
  GammaQuad gq;
  for (int s = 0; s < 5; ++s) {
    for (int t = 0; t < 4; ++t) {
      gq.m[s][t] = (float)m[s][t];
      gq.md[s][t] = m[s][t];
    }
    gq.wq[s] = (float)wq[s];
    gq.wqd[s] = wq[s];
  }
  if (nbins > AGP * AGH) return hipErrorInvalidValue;
#define MP3_GAMMA_ADJ(T, F, M, Q) \
  gamma_adjoint_v<T, F, M, Q>(fields, delta, lam_s, n, nbins, gq, wm, nwg, batch, cout, direct, partials, st)
  // partials != NULL: also contract for zeta (float32 on the matrix cores)
  if (prec) return partials ? MP3_GAMMA_ADJ(double, true, false, false) : MP3_GAMMA_ADJ(double, false, false, false);
  if (!partials) return MP3_GAMMA_ADJ(float, false, false, false);
  return nbins > 16 ? MP3_GAMMA_ADJ(float, true, true, true) : MP3_GAMMA_ADJ(float, true, true, false);
#undef MP3_GAMMA_ADJ
}

size_t gamma_adjoint_lds_need(int prec, int nbins) {
  if (nbins > AGP * AGH) return (size_t)1 << 40;
  return prec ? GammaAdjLds<double>(nbins).total : GammaAdjLds<float>(nbins).total;
}

}  // namespace mp3
