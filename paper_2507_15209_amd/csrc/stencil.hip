// stencil.hip -- grid summation with connection coefficients (Sec. 2.2,
// Eqs. con-coeff and SFC-3PCF) for a scaling function of support 3 cells
// (Daubechies-4), evaluated as a stencil over the shifts Delta = t - s:
//
//   sum_x delta(x) sum_{s,t} Gamma(s, t) a_b(x + s) conj(a_b'(x + t))
//     = sum_y sum_Delta G_Delta(y) a_b(y) conj(a_b'(y + Delta)),
//   G_Delta(y) = sum_s delta(y - s) Gamma(s, s + Delta),
//
// with Gamma(s, t) = prod_d gamma(s_d, t_d) and gamma nonzero for
// |s|, |t|, |s - t| <= 2 (125 shifts).  Per tile of 4^3 cells a workgroup
// holds the primary and the fields on the 8^3 window (tile plus 2 cells of
// halo) in LDS, builds G_Delta on the tile separably (x, then y, then z, one
// x-shift slab of 25 shifts at a time) and contracts.  The adjoint reverses
// the same steps: sources c_b(y) = sum_Delta G_Delta(y) conj(U_b(y + Delta))
// with U_b = sum_b' lam_s[b][b'] a_b', and the primary's gradient, the
// transposed stencil of Q_Delta(y) = Re sum_b a_b(y) conj(U_b(y + Delta)),
// folded into the window and added atomically.
//
// (The cubic B-spline's grid summation uses the exact node quadrature of
// kernels.hip instead: it is a piecewise polynomial, the Daubechies-4
// function is not.)
#include "fft_core.hpp"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

namespace mp3 {

namespace {

constexpr int ST = 4;             // cells per tile edge
constexpr int ST3 = ST * ST * ST;
constexpr int kStencilThreads = 512;

// the geometry of halo H (shifts -H .. H per axis): window edge ST + 2H,
// NS = 2H + 1 shifts per axis, SLAB = NS^2 shifts per x-shift
#define STENCIL_GEOMETRY(H)                                                 \
  constexpr int SH = (H), SW = ST + 2 * (H), SW3 = SW * SW * SW;            \
  constexpr int NS = 2 * (H) + 1, SLAB = NS * NS;                           \
  (void)SW3;                                                                \
  (void)SLAB

__device__ __forceinline__ int wrap_s(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// gamma(s, t) for s, t in -H .. H at [(s + H) * (2H + 1) + t + H], held in
// LDS (indexed at run time)
template <typename T, int H>
struct StencilCoef {
  const T* g;
};

template <typename T, int H>
__device__ __forceinline__ StencilCoef<T, H> coef_of(const StencilGamma& sg, T* lds) {
  constexpr int NS = 2 * H + 1;
  for (int e = threadIdx.x; e < NS * NS; e += blockDim.x) lds[e] = (T)sg.g[e / NS - H + 3][e % NS - H + 3];
  __syncthreads();
  return StencilCoef<T, H>{lds};
}

// gamma(s, s + d) for s, d in -H .. H (zero when |s + d| > H)
template <typename T, int H>
__device__ __forceinline__ T gsd(const StencilCoef<T, H>& c, int s, int d) {
  const int t = s + d;
  return (t < -H || t > H) ? (T)0 : c.g[(s + H) * (2 * H + 1) + t + H];
}

template <typename T, int H>
struct StencilLds {
  size_t D, Gx, Gxy, Gs, R, C, total;
  // forward: R = rows on the tile, C = columns on the window, nl local bins;
  // adjoint: R = the chunk's fields on the tile, C = U on the window, plus the
  // Q slab and the transposed-stencil scratch
  __host__ __device__ StencilLds(int nl, bool adjoint) {
    STENCIL_GEOMETRY(H);
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = (o + b + 15) & ~(size_t)15; return r; };
    D = take(SW3 * sizeof(T));
    Gx = take((size_t)NS * ST * SW * SW * sizeof(T));
    Gxy = take((size_t)NS * ST * ST * SW * sizeof(T));
    Gs = take((size_t)SLAB * ST3 * sizeof(T));
    R = take((size_t)ST3 * nl * sizeof(c2<T>));
    C = take((size_t)SW3 * nl * sizeof(c2<T>));
    if (adjoint) {
      take((size_t)SLAB * ST3 * sizeof(T));              // Q slab
      take((size_t)NS * ST * ST * SW * sizeof(T));       // z-transposed
      take((size_t)ST * SW * SW * sizeof(T));            // y-transposed
      take((size_t)SW3 * sizeof(T));                     // direct-term window
    }
    total = o;
  }
};

// window index of window coordinates
template <int H>
__device__ __forceinline__ int widx(int i, int j, int k) {
  constexpr int SW = ST + 2 * H;
  return (i * SW + j) * SW + k;
}
// tile cell index of tile coordinates
__device__ __forceinline__ int tidx(int i, int j, int k) { return (i * ST + j) * ST + k; }

// primary on the window, and its x-convolutions for every x-shift:
// Gx[dx][xi][j][k] = sum_sx gamma(sx, sx + dx) delta(x0 + xi - sx, window j, k)
template <typename T, int H>
__device__ void stencil_prepare(const T* dm, int n, int x0, int y0, int z0, const StencilCoef<T, H>& c, T* D,
                                T* Gx) {
  STENCIL_GEOMETRY(H);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int w = tid; w < SW3; w += nt) {
    const int i = w / (SW * SW), j = (w / SW) % SW, k = w % SW;
    D[w] = dm[((long long)wrap_s(x0 - SH + i, n) * n + wrap_s(y0 - SH + j, n)) * n + wrap_s(z0 - SH + k, n)];
  }
  __syncthreads();
  for (int e = tid; e < NS * ST * SW * SW; e += nt) {
    const int dx = e / (ST * SW * SW) - SH, r = e % (ST * SW * SW);
    const int xi = r / (SW * SW), jk = r % (SW * SW);
    T acc = 0;
#pragma unroll
    for (int s = -SH; s <= SH; ++s) acc += gsd(c, s, dx) * D[(xi + SH - s) * SW * SW + jk];
    Gx[e] = acc;
  }
}

// G_Delta on the tile for the 25 shifts of x-shift dx: Gs[(dy+2)*5 + dz+2][cell]
template <typename T, int H>
__device__ void stencil_slab(int dx, const StencilCoef<T, H>& c, const T* Gx, T* Gxy, T* Gs) {
  STENCIL_GEOMETRY(H);
  const int tid = threadIdx.x, nt = blockDim.x;
  const T* gx = Gx + (dx + SH) * ST * SW * SW;
  for (int e = tid; e < NS * ST * ST * SW; e += nt) {
    const int dy = e / (ST * ST * SW) - SH, r = e % (ST * ST * SW);
    const int xi = r / (ST * SW), yi = (r / SW) % ST, k = r % SW;
    T acc = 0;
#pragma unroll
    for (int s = -SH; s <= SH; ++s) acc += gsd(c, s, dy) * gx[(xi * SW + yi + SH - s) * SW + k];
    Gxy[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < SLAB * ST3; e += nt) {
    const int sh = e / ST3, cell = e % ST3;
    const int dy = sh / NS - SH, dz = sh % NS - SH;
    const int xi = cell / (ST * ST), yi = (cell / ST) % ST, zi = cell % ST;
    const T* gxy = Gxy + (((dy + SH) * ST + xi) * ST + yi) * SW;
    T acc = 0;
#pragma unroll
    for (int s = -SH; s <= SH; ++s) acc += gsd(c, s, dz) * gxy[zi + SH - s];
    Gs[e] = acc;
  }
}

// Forward: partials [mock][wg][nl^2] of the symmetric local bin matrix
// (P + P^T) / 2, P[b][b'] = sum over the tiles' y and the 125 shifts of
// G_Delta(y) Re(a_b(y) conj(a_b'(y + Delta))).  Local bin b < na is stored bin
// a0 + b, the rest c0 + (b - na) (all bins: a0 = 0, na = nl = nbt).
// Threads own a 4x4 block of a pair (b-block i <= j) and a share of the
// (shift, cell) terms; both orders of the pair are accumulated so that the
// partial is symmetric exactly.
template <typename T, int H>
__global__ void __launch_bounds__(kStencilThreads) k_stencil_contract(const c2<T>* fields, const T* delta, int n,
                                                                     StencilGamma sg, double* partials, int nl,
                                                                     int nbt, int a0, int na, int c0) {
  STENCIL_GEOMETRY(H);
  extern __shared__ __align__(16) char smem[];
  const StencilLds<T, H> L(nl, false);
  T* D = reinterpret_cast<T*>(smem + L.D);
  T* Gx = reinterpret_cast<T*>(smem + L.Gx);
  T* Gxy = reinterpret_cast<T*>(smem + L.Gxy);
  T* Gs = reinterpret_cast<T*>(smem + L.Gs);
  c2<T>* Rw = reinterpret_cast<c2<T>*>(smem + L.R);
  c2<T>* Cw = reinterpret_cast<c2<T>*>(smem + L.C);
  __shared__ T gco[NS * NS];
  const StencilCoef<T, H> c = coef_of<T, H>(sg, gco);
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long mock = blockIdx.y;
  const long long n3 = (long long)n * n * n;
  const c2<T>* fm = fields + mock * n3 * nbt;
  const T* dm = delta + mock * n3;
  const int td = n / ST;
  const long long ntiles = (long long)td * td * td;
  // pair blocks of 4 bins
  const int nq = (nl + 3) / 4;
  const int npb = nq * (nq + 1) / 2;
  const int parts = nt / npb;
  const int pb = tid / parts, part = tid % parts;
  const bool active = pb < npb;
  int bi = 0, bj = 0;
  if (active) {                                   // pair block pb = (bi, bj), bi <= bj < nq
    int r = pb;
    while (r >= nq - bi) { r -= nq - bi; ++bi; }
    bj = bi + r;
  }
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[i][k] = 0;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int tx = (int)(tile / ((long long)td * td)), ty = (int)((tile / td) % td), tz = (int)(tile % td);
    const int x0 = tx * ST, y0 = ty * ST, z0 = tz * ST;
    __syncthreads();                              // the previous tile is done with the LDS
    for (int e = tid; e < SW3 * nl; e += nt) {
      const int b = e % nl, w = e / nl;
      const int i = w / (SW * SW), j = (w / SW) % SW, k = w % SW;
      const long long cell = ((long long)wrap_s(x0 - SH + i, n) * n + wrap_s(y0 - SH + j, n)) * n + wrap_s(z0 - SH + k, n);
      const c2<T> v = fm[cell * nbt + (b < na ? a0 + b : c0 + b - na)];
      Cw[e] = v;
      if (i >= SH && i < SH + ST && j >= SH && j < SH + ST && k >= SH && k < SH + ST)
        Rw[tidx(i - SH, j - SH, k - SH) * nl + b] = v;
    }
    stencil_prepare<T, H>(dm, n, x0, y0, z0, c, D, Gx);
    for (int dx = -SH; dx <= SH; ++dx) {
      __syncthreads();                            // Gx ready / the previous slab's Gs consumed
      stencil_slab<T, H>(dx, c, Gx, Gxy, Gs);
      __syncthreads();
      if (active) {
        for (int e = part; e < SLAB * ST3; e += parts) {
          const int sh = e / ST3, cell = e % ST3;
          const int dy = sh / NS - SH, dz = sh % NS - SH;
          const T g = Gs[e];
          const int xi = cell / (ST * ST), yi = (cell / ST) % ST, zi = cell % ST;
          const int ws = widx<H>(xi + SH + dx, yi + SH + dy, zi + SH + dz);
          c2<T> ri[4], rj[4], ci[4], cj[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int b1 = 4 * bi + q, b2 = 4 * bj + q;
            ri[q] = b1 < nl ? Rw[cell * nl + b1] : mk<T>(0, 0);
            rj[q] = b2 < nl ? Rw[cell * nl + b2] : mk<T>(0, 0);
            ci[q] = b1 < nl ? Cw[ws * nl + b1] : mk<T>(0, 0);
            cj[q] = b2 < nl ? Cw[ws * nl + b2] : mk<T>(0, 0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k)
              acc[i][k] += g * (ri[i].x * cj[k].x + ri[i].y * cj[k].y + rj[k].x * ci[i].x + rj[k].y * ci[i].y);
        }
      }
    }
  }
  // reduce the parts of every pair block; the scratch aliases the window
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);
  if (active) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) red[(pb * parts + part) * 16 + i * 4 + k] = (double)acc[i][k];
  }
  __syncthreads();
  double* out = partials + ((long long)mock * gridDim.x + blockIdx.x) * nl * nl;
  for (int t = tid; t < npb * 16; t += nt) {
    const int blk = t / 16, i = (t / 4) % 4, k = t % 4;
    double s = 0.0;
    for (int p = 0; p < parts; ++p) s += red[(blk * parts + p) * 16 + i * 4 + k];
    int qi = 0, r = blk;
    while (r >= nq - qi) { r -= nq - qi; ++qi; }
    const int qj = qi + r;
    const int b1 = 4 * qi + i, b2 = 4 * qj + k;
    // a diagonal block holds each unordered pair twice, (i, k) and (k, i),
    // both (P + P^T)[b1][b2]: the one with i <= k writes both mirror entries
    if (b1 < nl && b2 < nl && (qi != qj || i <= k)) {
      out[b1 * nl + b2] = 0.5 * s;
      out[b2 * nl + b1] = 0.5 * s;
    }
  }
}

// Adjoint for stored bins b0 .. b0 + nbc - 1: cout[b][y] = sum_Delta G_Delta(y)
// conj(U_b(y + Delta)) on the tile (written, every cell by its own tile), and
// wm times the transposed stencil of Q_Delta(y) = Re sum_b a_b(y)
// conj(U_b(y + Delta)) added atomically into direct over the window.
// Source items (cell, bin) per thread: at most kSrcItems.
constexpr int kSrcItems = 5;

template <typename T, int H>
__global__ void __launch_bounds__(kStencilThreads) k_stencil_adjoint(const c2<T>* fields, const c2<T>* U,
                                                                    const T* delta, int n, int nbt, int b0, int nbc,
                                                                    StencilGamma sg, double wm, c2<T>* cout,
                                                                    T* direct) {
  STENCIL_GEOMETRY(H);
  extern __shared__ __align__(16) char smem[];
  const StencilLds<T, H> L(nbc, true);
  T* D = reinterpret_cast<T*>(smem + L.D);
  T* Gx = reinterpret_cast<T*>(smem + L.Gx);
  T* Gxy = reinterpret_cast<T*>(smem + L.Gxy);
  T* Gs = reinterpret_cast<T*>(smem + L.Gs);
  c2<T>* Ar = reinterpret_cast<c2<T>*>(smem + L.R);
  c2<T>* Uw = reinterpret_cast<c2<T>*>(smem + L.C);
  T* Qs = reinterpret_cast<T*>(reinterpret_cast<char*>(Uw) + (((size_t)SW3 * nbc * sizeof(c2<T>) + 15) & ~(size_t)15));
  T* Tz = Qs + SLAB * ST3;
  T* Ty = Tz + NS * ST * ST * SW;
  T* Dw = Ty + ST * SW * SW;
  __shared__ T gco[NS * NS];
  const StencilCoef<T, H> c = coef_of<T, H>(sg, gco);
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long mock = blockIdx.y;
  const long long n3 = (long long)n * n * n;
  const c2<T>* fm = fields + mock * n3 * nbt;
  const c2<T>* um = U + mock * n3 * nbt;
  const T* dm = delta + mock * n3;
  T* rm = direct + mock * n3;
  const int td = n / ST;
  const long long ntiles = (long long)td * td * td;
  const int nsrc = ST3 * nbc;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int tx = (int)(tile / ((long long)td * td)), ty = (int)((tile / td) % td), tz = (int)(tile % td);
    const int x0 = tx * ST, y0 = ty * ST, z0 = tz * ST;
    __syncthreads();
    for (int e = tid; e < SW3 * nbc; e += nt) {
      const int b = e % nbc, w = e / nbc;
      const int i = w / (SW * SW), j = (w / SW) % SW, k = w % SW;
      const long long cell = ((long long)wrap_s(x0 - SH + i, n) * n + wrap_s(y0 - SH + j, n)) * n + wrap_s(z0 - SH + k, n);
      Uw[e] = um[cell * nbt + b0 + b];
      if (i >= SH && i < SH + ST && j >= SH && j < SH + ST && k >= SH && k < SH + ST)
        Ar[tidx(i - SH, j - SH, k - SH) * nbc + b] = fm[cell * nbt + b0 + b];
    }
    for (int w = tid; w < SW3; w += nt) Dw[w] = 0;
    stencil_prepare<T, H>(dm, n, x0, y0, z0, c, D, Gx);
    c2<T> src[kSrcItems];
#pragma unroll
    for (int q = 0; q < kSrcItems; ++q) src[q] = mk<T>(0, 0);
    for (int dx = -SH; dx <= SH; ++dx) {
      __syncthreads();
      stencil_slab<T, H>(dx, c, Gx, Gxy, Gs);
      __syncthreads();
      // sources: every (cell, bin) item of this thread, over the slab's shifts
#pragma unroll
      for (int q = 0; q < kSrcItems; ++q) {
        const int it = tid + q * nt;
        if (it < nsrc) {
          const int cell = it / nbc, b = it % nbc;
          const int xi = cell / (ST * ST), yi = (cell / ST) % ST, zi = cell % ST;
          c2<T> s = src[q];
          for (int sh = 0; sh < SLAB; ++sh) {
            const int dy = sh / NS - SH, dz = sh % NS - SH;
            const T g = Gs[sh * ST3 + cell];
            const c2<T> u = Uw[widx<H>(xi + SH + dx, yi + SH + dy, zi + SH + dz) * nbc + b];
            s.x += g * u.x;
            s.y -= g * u.y;
          }
          src[q] = s;
        }
      }
      // Q of the slab's shifts on the tile
      for (int e = tid; e < SLAB * ST3; e += nt) {
        const int sh = e / ST3, cell = e % ST3;
        const int dy = sh / NS - SH, dz = sh % NS - SH;
        const int xi = cell / (ST * ST), yi = (cell / ST) % ST, zi = cell % ST;
        const c2<T>* ua = Uw + widx<H>(xi + SH + dx, yi + SH + dy, zi + SH + dz) * nbc;
        const c2<T>* aa = Ar + cell * nbc;
        T qv = 0;
        for (int b = 0; b < nbc; ++b) qv += aa[b].x * ua[b].x + aa[b].y * ua[b].y;
        Qs[e] = qv;
      }
      __syncthreads();
      // transposed stencil, z: Tz[dy][xi][yi][wz] = sum_dz sum_sz gamma(sz, sz + dz) Q[dy, dz][xi, yi, zi],
      // zi = wz - 2 + sz on the tile
      for (int e = tid; e < NS * ST * ST * SW; e += nt) {
        const int dy = e / (ST * ST * SW), r = e % (ST * ST * SW);
        const int xi = r / (ST * SW), yi = (r / SW) % ST, wz = r % SW;
        T acc = 0;
        for (int dz = -SH; dz <= SH; ++dz) {
#pragma unroll
          for (int s = -SH; s <= SH; ++s) {
            const int zi = wz - SH + s;
            if (zi >= 0 && zi < ST) acc += gsd(c, s, dz) * Qs[(dy * NS + dz + SH) * ST3 + tidx(xi, yi, zi)];
          }
        }
        Tz[e] = acc;
      }
      __syncthreads();
      // y: Ty[xi][wy][wz] = sum_dy sum_sy gamma(sy, sy + dy) Tz[dy][xi][yi = wy - 2 + sy][wz]
      for (int e = tid; e < ST * SW * SW; e += nt) {
        const int xi = e / (SW * SW), wy = (e / SW) % SW, wz = e % SW;
        T acc = 0;
        for (int dy = -SH; dy <= SH; ++dy) {
#pragma unroll
          for (int s = -SH; s <= SH; ++s) {
            const int yi = wy - SH + s;
            if (yi >= 0 && yi < ST) acc += gsd(c, s, dy) * Tz[(((dy + SH) * ST + xi) * ST + yi) * SW + wz];
          }
        }
        Ty[e] = acc;
      }
      __syncthreads();
      // x: Dw[wx][wy][wz] += sum_sx gamma(sx, sx + dx) Ty[xi = wx - 2 + sx][wy][wz]
      for (int w = tid; w < SW3; w += nt) {
        const int wx = w / (SW * SW), r = w % (SW * SW);
        T acc = 0;
#pragma unroll
        for (int s = -SH; s <= SH; ++s) {
          const int xi = wx - SH + s;
          if (xi >= 0 && xi < ST) acc += gsd(c, s, dx) * Ty[xi * SW * SW + r];
        }
        Dw[w] += acc;
      }
    }
    // sources of the tile's cells (no other tile writes them)
#pragma unroll
    for (int q = 0; q < kSrcItems; ++q) {
      const int it = tid + q * nt;
      if (it < nsrc) {
        const int cell = it / nbc, b = it % nbc;
        const int xi = cell / (ST * ST), yi = (cell / ST) % ST, zi = cell % ST;
        const long long g = ((long long)(x0 + xi) * n + (y0 + yi)) * n + (z0 + zi);
        cout[(mock * nbt + b0 + b) * n3 + g] = src[q];
      }
    }
    __syncthreads();
    for (int w = tid; w < SW3; w += nt) {
      const int i = w / (SW * SW), j = (w / SW) % SW, k = w % SW;
      const long long g = ((long long)wrap_s(x0 - SH + i, n) * n + wrap_s(y0 - SH + j, n)) * n + wrap_s(z0 - SH + k, n);
      atomicAdd(&rm[g], (T)(wm * (double)Dw[w]));
    }
  }
}

template <typename T, int H>
size_t stencil_need(int nl, bool adjoint) {
  StencilLds<T, H> L(nl, adjoint);
  size_t need = L.total;
  if (!adjoint) {
    const int nq = (nl + 3) / 4, npb = nq * (nq + 1) / 2;
    const size_t red = (size_t)npb * (kStencilThreads / npb) * 16 * sizeof(double);
    if (red > need) need = red;
  }
  return need;
}

template <typename K>
hipError_t allow(K kern, size_t lds) {
  if (lds > 64 * 1024) return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return hipSuccess;
}

}  // namespace

// dynamic LDS plus the kernels' static coefficient table
constexpr size_t kStaticLds = 512;

size_t stencil_lds_need(int prec, int halo, int nl) {
  if (halo == 2) return kStaticLds + (prec ? stencil_need<double, 2>(nl, false) : stencil_need<float, 2>(nl, false));
  return kStaticLds + (prec ? stencil_need<double, 3>(nl, false) : stencil_need<float, 3>(nl, false));
}

size_t stencil_adjoint_lds_need(int prec, int halo, int nbc) {
  if ((ST3 * nbc + kStencilThreads - 1) / kStencilThreads > kSrcItems) return (size_t)1 << 40;
  if (halo == 2) return kStaticLds + (prec ? stencil_need<double, 2>(nbc, true) : stencil_need<float, 2>(nbc, true));
  return kStaticLds + (prec ? stencil_need<double, 3>(nbc, true) : stencil_need<float, 3>(nbc, true));
}

namespace {

template <typename T, int H>
hipError_t stencil_contract_t(const void* fields, const void* delta, int n, const BinPair& bp, const StencilGamma& sg,
                              double* partials, int nl, dim3 gs, hipStream_t st) {
  const size_t lds = stencil_need<T, H>(nl, false);
  if (hipError_t e = allow(k_stencil_contract<T, H>, lds)) return e;
  k_stencil_contract<T, H><<<gs, kStencilThreads, lds, st>>>(static_cast<const c2<T>*>(fields),
                                                             static_cast<const T*>(delta), n, sg, partials, nl, bp.nbt,
                                                             bp.a0, bp.na, bp.c0);
  return hipGetLastError();
}

template <typename T, int H>
hipError_t stencil_adjoint_t(const void* fields, const void* U, const void* delta, int n, int nbt, int b0, int nbc,
                             const StencilGamma& sg, double wm, dim3 gs, void* cout, void* direct, hipStream_t st) {
  const size_t lds = stencil_need<T, H>(nbc, true);
  if (hipError_t e = allow(k_stencil_adjoint<T, H>, lds)) return e;
  k_stencil_adjoint<T, H><<<gs, kStencilThreads, lds, st>>>(
      static_cast<const c2<T>*>(fields), static_cast<const c2<T>*>(U), static_cast<const T*>(delta), n, nbt, b0, nbc,
      sg, wm, static_cast<c2<T>*>(cout), static_cast<T*>(direct));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stencil_contract(int prec, const void* fields, const void* delta, int n, const BinPair& bp,
                                   const StencilGamma& sg, double* partials, int nwg, int batch, hipStream_t st) {
  const int nl = (bp.a0 == 0 && bp.na == bp.nbt) ? bp.nbt : bp.na + bp.nc;
  if (n % ST != 0 || nwg < 1 || nl < 1 || (sg.halo != 2 && sg.halo != 3)) return hipErrorInvalidValue;
  const dim3 gs((unsigned)nwg, (unsigned)batch);
  if (sg.halo == 2)
    return prec ? stencil_contract_t<double, 2>(fields, delta, n, bp, sg, partials, nl, gs, st)
                : stencil_contract_t<float, 2>(fields, delta, n, bp, sg, partials, nl, gs, st);
  return prec ? stencil_contract_t<double, 3>(fields, delta, n, bp, sg, partials, nl, gs, st)
              : stencil_contract_t<float, 3>(fields, delta, n, bp, sg, partials, nl, gs, st);
}

hipError_t launch_stencil_adjoint(int prec, const void* fields, const void* U, const void* delta, int n, int nbt,
                                  int b0, int nbc, const StencilGamma& sg, double wm, int nwg, int batch, void* cout,
                                  void* direct, hipStream_t st) {
  if (n % ST != 0 || nwg < 1 || nbc < 1 || (ST3 * nbc + kStencilThreads - 1) / kStencilThreads > kSrcItems ||
      (sg.halo != 2 && sg.halo != 3))
    return hipErrorInvalidValue;
  const dim3 gs((unsigned)nwg, (unsigned)batch);
  if (sg.halo == 2)
    return prec ? stencil_adjoint_t<double, 2>(fields, U, delta, n, nbt, b0, nbc, sg, wm, gs, cout, direct, st)
                : stencil_adjoint_t<float, 2>(fields, U, delta, n, nbt, b0, nbc, sg, wm, gs, cout, direct, st);
  return prec ? stencil_adjoint_t<double, 3>(fields, U, delta, n, nbt, b0, nbc, sg, wm, gs, cout, direct, st)
              : stencil_adjoint_t<float, 3>(fields, U, delta, n, nbt, b0, nbc, sg, wm, gs, cout, direct, st);
}

}  // namespace mp3
