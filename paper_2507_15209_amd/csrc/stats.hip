// stats.hip -- gfx950 kernels around the multipole path: input validation,
// the spherical top-hat filter of the primary vertex (Sec. 3, the
// triple-sphere binning), the two-point function xi(r) from the power
// spectrum (Sec. 2.1, Eqs. pair-counting and window-sphshell), its
// line-of-sight multipoles (Sec. 2.1, Eqs. DD-multipole and
// DD-windowfunction) and the
// reconstruction of zeta(r1, r2, theta) and of the reduced 3PCF Q from the
// multipoles (Sec. 2.2, Eq. triplet-counting; Sec. 3, Eq. Q-factor), and the
// edge-corrected (D - R)^3 / R^3 estimator with a random catalogue (Sec. 3,
// Eq. SSestimator).
//
// All are O(N^3) or smaller per call (the per-(l, m) work of the estimator
// is in kernels.hip).
#include "fft_core.hpp"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

namespace mp3 {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

__device__ __forceinline__ int sfreq_s(int i, int n) { return i < n / 2 ? i : i - n; }

__device__ __forceinline__ bool finite_d(double v) { return v == v && fabs(v) <= 1.7976931348623157e308; }

// flag[0] += 1 if any of the count values is NaN or infinite
template <typename T>
__global__ void k_count_nonfinite(const T* p, long long count, int* flag) {
  bool bad = false;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    bad = bad || !finite_d((double)p[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicAdd(flag, 1);
}

// 3 j_1(x) / x, the transform of the unit-volume sphere of radius R at x = k R
__device__ __forceinline__ double tophat_d(double x) {
  if (x < 1e-2) {
    const double x2 = x * x;
    return 1.0 - x2 / 10.0 + x2 * x2 / 280.0 - x2 * x2 * x2 / 15120.0;
  }
  return 3.0 * (sin(x) - x * cos(x)) / (x * x * x);
}

__device__ __forceinline__ double j0_d(double x) { return x < 1e-6 ? 1.0 - x * x / 6.0 : sin(x) / x; }

// X[q] *= scale * W_TH(|k| R) for every mock (k = 2 pi q / box), in place:
// the spherical top-hat filter in k-space (real, even: its own transpose)
template <typename T>
__global__ void k_tophat_filter(c2<T>* X, int n, double kf, double R, double scale) {
  const long long n3 = (long long)n * n * n;
  c2<T>* xm = X + blockIdx.y * n3;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n3; i += (long long)gridDim.x * blockDim.x) {
    const int qx = sfreq_s((int)(i / ((long long)n * n)), n), qy = sfreq_s((int)((i / n) % n), n);
    const int qz = sfreq_s((int)(i % n), n);
    const double k = kf * sqrt((double)(qx * qx + qy * qy + qz * qz));
    const double f = scale * tophat_d(k * R);
    const c2<T> v = xm[i];
    xm[i] = mk<T>((T)(f * (double)v.x), (T)(f * (double)v.y));
  }
}

template <typename T>
__global__ void k_real_part(const c2<T>* in, T* out, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    out[i] = in[i].x;
}

// P[mock][|q|^2] += |dhat(q)|^2 (times phi-hat(q) when phi != NULL), Nyquist
// planes excluded (the secondary vertex's window vanishes there)
template <typename T>
__global__ void k_power_plain(const c2<T>* dhat, int n, int nq2, double* P, const T* phi) {
  const long long n3 = (long long)n * n * n;
  const int mock = blockIdx.y;
  const c2<T>* d = dhat + mock * n3;
  double* pm = P + (long long)mock * nq2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n3; i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i / ((long long)n * n)), iy = (int)((i / n) % n), iz = (int)(i % n);
    const int qx = sfreq_s(ix, n), qy = sfreq_s(iy, n), qz = sfreq_s(iz, n);
    const int h = -n / 2;
    if (qx == h || qy == h || qz == h) continue;
    double f = 1.0;
    if (phi) f = (double)phi[ix] * (double)phi[iy] * (double)phi[iz];
    const c2<T> v = d[i];
    atomicAdd(&pm[qx * qx + qy * qy + qz * qz], f * ((double)v.x * v.x + (double)v.y * v.y));
  }
}

__device__ __forceinline__ double block_sum_d(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

// xi(r) = N^-6 sum_s P[s] Wp(k_s) Ws(k_s) j_0(k_s r): the primary's window Wp
// (top-hat when prim_smooth) and the secondary's top-hat Ws, k_s = kf sqrt(s)
__device__ double xi_at(const double* pm, int nq2, double kf, double R, bool prim_smooth, double r, double n6,
                        double* sh) {
  double s = 0.0;
  for (int q = threadIdx.x; q < nq2; q += blockDim.x) {
    const double p = pm[q];
    if (p == 0.0) continue;
    const double k = kf * sqrt((double)q);
    double w = R > 0.0 ? tophat_d(k * R) : 1.0;
    if (prim_smooth) w *= w;
    s += p * w * j0_d(k * r);
  }
  return block_sum_d(s, sh) / n6;
}

// xi[mock][i] at radii[i]; one block per (radius, mock)
__global__ void k_xi(const double* P, int nq2, double kf, double R, int prim_smooth, const double* radii, int nr,
                     double n6, double* xi) {
  __shared__ double sh[16];
  const int i = blockIdx.x, mock = blockIdx.y;
  const double v = xi_at(P + (long long)mock * nq2, nq2, kf, R, prim_smooth != 0, radii[i], n6, sh);
  if (threadIdx.x == 0) xi[(long long)mock * nr + i] = v;
}

// zeta(r_b1, r_b2, theta_t) = sum_{l <= lt} zeta_l[b1][b2] P_l(mu_t) and, when
// q != NULL, Q = zeta / (xi(r1) xi(r2) + xi(r2) xi(r3) + xi(r3) xi(r1)) with
// r3^2 = r1^2 + r2^2 - 2 r1 r2 mu_t.  One block per ((b1, b2, t), mock).
__global__ void k_reduced_3pcf(const double* zeta, int lmax, int lt, int nbins, const double* mu, int nth,
                               const double* rb, const double* xib, const double* P, int nq2, double kf, double R,
                               int prim_smooth, double n6, double* zt, double* q) {
  __shared__ double sh[16];
  const int e = blockIdx.x, mock = blockIdx.y;
  const int t = e % nth, b2 = (e / nth) % nbins, b1 = e / (nth * nbins);
  const double m = mu[t];
  const double* zm = zeta + (long long)mock * (lmax + 1) * nbins * nbins;
  double acc = 0.0, p0 = 1.0, p1 = m;
  for (int l = 0; l <= lt; ++l) {
    const double pl = l == 0 ? 1.0 : (l == 1 ? m : ((2.0 * l - 1.0) * m * p1 - (l - 1.0) * p0) / l);
    if (l >= 2) {
      p0 = p1;
      p1 = pl;
    }
    acc += zm[((long long)l * nbins + b1) * nbins + b2] * pl;
  }
  const long long o = (((long long)mock * nbins + b1) * nbins + b2) * nth + t;
  if (q) {
    const double r1 = rb[b1], r2 = rb[b2];
    double r3s = r1 * r1 + r2 * r2 - 2.0 * r1 * r2 * m;
    const double r3 = r3s > 0.0 ? sqrt(r3s) : 0.0;
    const double x3 = xi_at(P + (long long)mock * nq2, nq2, kf, R, prim_smooth != 0, r3, n6, sh);
    const double x1 = xib[(long long)mock * nbins + b1], x2 = xib[(long long)mock * nbins + b2];
    if (threadIdx.x == 0) q[o] = acc / (x1 * x2 + x2 * x3 + x3 * x1);
  }
  if (threadIdx.x == 0) zt[o] = acc;
}

// H[mock][ell][|q|^2] += |dhat(q)|^2 P_ell(q_z / |q|) (times phi-hat when phi != NULL), ell = 0..lmx,
// Nyquist planes excluded: the per-shell Legendre moments of the power along the line of sight z
template <typename T>
__global__ void k_power_multipoles(const c2<T>* dhat, int n, int nq2, int lmx, double* H, const T* phi) {
  const long long n3 = (long long)n * n * n;
  const int mock = blockIdx.y;
  const c2<T>* d = dhat + mock * n3;
  double* hm = H + (long long)mock * (lmx + 1) * nq2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n3; i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i / ((long long)n * n)), iy = (int)((i / n) % n), iz = (int)(i % n);
    const int qx = sfreq_s(ix, n), qy = sfreq_s(iy, n), qz = sfreq_s(iz, n);
    const int h = -n / 2;
    if (qx == h || qy == h || qz == h) continue;
    double f = 1.0;
    if (phi) f = (double)phi[ix] * (double)phi[iy] * (double)phi[iz];
    const c2<T> v = d[i];
    const double p = f * ((double)v.x * v.x + (double)v.y * v.y);
    const int q2 = qx * qx + qy * qy + qz * qz;
    const double mu = q2 > 0 ? (double)qz / sqrt((double)q2) : 1.0;
    double p0 = 1.0, p1 = mu;
    for (int l = 0; l <= lmx; ++l) {
      double pl;
      if (l == 0) pl = 1.0;
      else if (l == 1) pl = mu;
      else {
        pl = ((2.0 * l - 1.0) * mu * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = pl;
      }
      atomicAdd(&hm[(long long)l * nq2 + q2], p * pl);
    }
  }
}

// j_0(x) .. j_L(x), L < 17: upward recurrence for x > L, Miller's downward
// recurrence (normalised by the larger of the closed forms j_0, j_1) below
__device__ void sph_bessel_d(int L, double x, double* out) {
  if (x < 1e-8) {
    out[0] = 1.0;
    for (int l = 1; l <= L; ++l) out[l] = 0.0;
    return;
  }
  const double s = sin(x), c = cos(x);
  const double j0 = s / x, j1 = s / (x * x) - c / x;
  out[0] = j0;
  if (L == 0) return;
  if (x > (double)L) {
    out[1] = j1;
    for (int l = 1; l < L; ++l) out[l + 1] = (2.0 * l + 1.0) / x * out[l] - out[l - 1];
    return;
  }
  const int lstart = L + 30 + (int)x;
  double jp1 = 0.0, jl = 1e-200;
  for (int l = lstart; l >= 1; --l) {
    const double jm1 = (2.0 * l + 1.0) / x * jl - jp1;
    jp1 = jl;
    jl = jm1;
    if (l - 1 <= L) out[l - 1] = jl;
    if (fabs(jl) > 1e200) {
      jl *= 1e-200;
      jp1 *= 1e-200;
      for (int k = l - 1; k <= L; ++k) out[k] *= 1e-200;
    }
  }
  const double norm = fabs(j0) >= fabs(j1) ? j0 / out[0] : j1 / out[1];
  for (int l = 0; l <= L; ++l) out[l] *= norm;
}

constexpr int kMaxEll = 16;

// xi_ell(r) = (2 ell + 1) Re(i^ell) N^-6 sum_s H_ell[s] Wp Ws j_ell(k_s r); one block per (radius, mock)
__global__ void k_xi_multipoles(const double* H, int nq2, int lmx, double kf, double R, int prim_smooth,
                                const double* radii, int nr, double n6, double* out) {
  __shared__ double sh[16];
  const int i = blockIdx.x, mock = blockIdx.y;
  const double r = radii[i];
  const double* hm = H + (long long)mock * (lmx + 1) * nq2;
  double acc[kMaxEll + 1];
  double jl[kMaxEll + 1];
  for (int l = 0; l <= lmx; ++l) acc[l] = 0.0;
  for (int q = threadIdx.x; q < nq2; q += blockDim.x) {
    const double k = kf * sqrt((double)q);
    double w = R > 0.0 ? tophat_d(k * R) : 1.0;
    if (prim_smooth) w *= w;
    sph_bessel_d(lmx, k * r, jl);
    for (int l = 0; l <= lmx; ++l) acc[l] += hm[(long long)l * nq2 + q] * w * jl[l];
  }
  for (int l = 0; l <= lmx; ++l) {
    const double v = block_sum_d(acc[l], sh);
    const double ph = (l & 1) ? 0.0 : ((l & 2) ? -1.0 : 1.0);   // Re(i^l)
    if (threadIdx.x == 0) out[((long long)mock * (lmx + 1) + l) * nr + i] = (2.0 * l + 1.0) * ph * v / n6;
  }
}

// f = delta_D - delta_R (the field of D - R), r = 1 + delta_R (the field of R), for every mock
template <typename T>
__global__ void k_ss_fields(const T* dd, const T* dr, T* f, T* r, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x) {
    const T a = dd[i], b = dr[i];
    f[i] = a - b;
    r[i] = (T)1 + b;
  }
}

// zeta_SS_l[b1][b2] = (2l+1)/2 sum_k wq_k N(mu_k) / R(mu_k) P_l(mu_k), N and R summed over l <= lt;
// one thread per (b1, b2, mock) entry
__global__ void k_ss_multipoles(const double* zn, const double* zr, int lmax, int lt, int nbins, const double* xq,
                                const double* wq, int nq, double* out, int batch) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int nb2 = nbins * nbins;
  if (e >= nb2 * batch) return;
  const int mock = e / nb2, bb = e % nb2;
  const double* a = zn + (long long)mock * (lmax + 1) * nb2 + bb;
  const double* b = zr + (long long)mock * (lmax + 1) * nb2 + bb;
  double acc[21];
  for (int l = 0; l <= lt; ++l) acc[l] = 0.0;
  for (int k = 0; k < nq; ++k) {
    const double m = xq[k];
    double num = 0.0, den = 0.0, p0 = 1.0, p1 = m;
    for (int l = 0; l <= lt; ++l) {
      double pl;
      if (l == 0) pl = 1.0;
      else if (l == 1) pl = m;
      else {
        pl = ((2.0 * l - 1.0) * m * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = pl;
      }
      num += a[(long long)l * nb2] * pl;
      den += b[(long long)l * nb2] * pl;
    }
    const double ratio = wq[k] * num / den;
    p0 = 1.0;
    p1 = m;
    for (int l = 0; l <= lt; ++l) {
      double pl;
      if (l == 0) pl = 1.0;
      else if (l == 1) pl = m;
      else {
        pl = ((2.0 * l - 1.0) * m * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = pl;
      }
      acc[l] += ratio * pl;
    }
  }
  for (int l = 0; l <= lt; ++l) out[((long long)mock * (lt + 1) + l) * nb2 + bb] = 0.5 * (2.0 * l + 1.0) * acc[l];
}

unsigned grid_of(long long count, int block, unsigned cap) {
  long long g = (count + block - 1) / block;
  if (g < 1) g = 1;
  return (unsigned)(g < (long long)cap ? g : cap);
}

}  // namespace

hipError_t launch_count_nonfinite(int prec, const void* p, long long count, int* flag, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const unsigned g = grid_of(count, 256, 4096);
  if (prec) k_count_nonfinite<double><<<g, 256, 0, st>>>(static_cast<const double*>(p), count, flag);
  else k_count_nonfinite<float><<<g, 256, 0, st>>>(static_cast<const float*>(p), count, flag);
  return hipGetLastError();
}

hipError_t launch_tophat_filter(int prec, void* X, int n, double kf, double R, double scale, int batch, hipStream_t st) {
  const long long n3 = (long long)n * n * n;
  const dim3 gs(grid_of(n3, 256, 8192), batch);
  if (prec) k_tophat_filter<double><<<gs, 256, 0, st>>>(static_cast<double2*>(X), n, kf, R, scale);
  else k_tophat_filter<float><<<gs, 256, 0, st>>>(static_cast<float2*>(X), n, kf, R, scale);
  return hipGetLastError();
}

hipError_t launch_real_part(int prec, const void* in, void* out, long long count, hipStream_t st) {
  const unsigned g = grid_of(count, 256, 16384);
  if (prec) k_real_part<double><<<g, 256, 0, st>>>(static_cast<const double2*>(in), static_cast<double*>(out), count);
  else k_real_part<float><<<g, 256, 0, st>>>(static_cast<const float2*>(in), static_cast<float*>(out), count);
  return hipGetLastError();
}

hipError_t launch_power_plain(int prec, const void* dhat, int n, int nq2, double* P, int batch, const void* phi,
                              hipStream_t st) {
  const long long n3 = (long long)n * n * n;
  const dim3 gs(grid_of(n3, 256, 8192), batch);
  if (prec)
    k_power_plain<double><<<gs, 256, 0, st>>>(static_cast<const double2*>(dhat), n, nq2, P,
                                              static_cast<const double*>(phi));
  else
    k_power_plain<float><<<gs, 256, 0, st>>>(static_cast<const float2*>(dhat), n, nq2, P,
                                             static_cast<const float*>(phi));
  return hipGetLastError();
}

hipError_t launch_xi(const double* P, int nq2, double kf, double R, bool prim_smooth, const double* radii, int nr,
                     double n6, double* xi, int batch, hipStream_t st) {
  const dim3 gs(nr, batch);
  k_xi<<<gs, 256, 0, st>>>(P, nq2, kf, R, prim_smooth ? 1 : 0, radii, nr, n6, xi);
  return hipGetLastError();
}

hipError_t launch_power_multipoles(int prec, const void* dhat, int n, int nq2, int lmx, double* H, int batch,
                                  const void* phi, hipStream_t st) {
  if (lmx < 0 || lmx > kMaxEll) return hipErrorInvalidValue;
  const long long n3 = (long long)n * n * n;
  const dim3 gs(grid_of(n3, 256, 8192), batch);
  if (prec)
    k_power_multipoles<double><<<gs, 256, 0, st>>>(static_cast<const double2*>(dhat), n, nq2, lmx, H,
                                                   static_cast<const double*>(phi));
  else
    k_power_multipoles<float><<<gs, 256, 0, st>>>(static_cast<const float2*>(dhat), n, nq2, lmx, H,
                                                  static_cast<const float*>(phi));
  return hipGetLastError();
}

hipError_t launch_xi_multipoles(const double* H, int nq2, int lmx, double kf, double R, bool prim_smooth,
                                const double* radii, int nr, double n6, double* out, int batch, hipStream_t st) {
  if (lmx < 0 || lmx > kMaxEll) return hipErrorInvalidValue;
  const dim3 gs(nr, batch);
  k_xi_multipoles<<<gs, 256, 0, st>>>(H, nq2, lmx, kf, R, prim_smooth ? 1 : 0, radii, nr, n6, out);
  return hipGetLastError();
}

hipError_t launch_ss_fields(int prec, const void* dd, const void* dr, void* f, void* r, long long count,
                            hipStream_t st) {
  const unsigned g = grid_of(count, 256, 16384);
  if (prec)
    k_ss_fields<double><<<g, 256, 0, st>>>(static_cast<const double*>(dd), static_cast<const double*>(dr),
                                           static_cast<double*>(f), static_cast<double*>(r), count);
  else
    k_ss_fields<float><<<g, 256, 0, st>>>(static_cast<const float*>(dd), static_cast<const float*>(dr),
                                          static_cast<float*>(f), static_cast<float*>(r), count);
  return hipGetLastError();
}

hipError_t launch_ss_multipoles(const double* zn, const double* zr, int lmax, int lt, int nbins, const double* xq,
                                const double* wq, int nq, double* out, int batch, hipStream_t st) {
  if (lt < 0 || lt > 20) return hipErrorInvalidValue;
  const long long cnt = (long long)nbins * nbins * batch;
  k_ss_multipoles<<<grid_of(cnt, 64, 65535), 64, 0, st>>>(zn, zr, lmax, lt, nbins, xq, wq, nq, out, batch);
  return hipGetLastError();
}

hipError_t launch_reduced_3pcf(const double* zeta, int lmax, int lt, int nbins, const double* mu, int nth,
                               const double* rb, const double* xib, const double* P, int nq2, double kf, double R,
                               bool prim_smooth, double n6, double* zt, double* q, int batch, hipStream_t st) {
  const dim3 gs(nbins * nbins * nth, batch);
  k_reduced_3pcf<<<gs, 256, 0, st>>>(zeta, lmax, lt, nbins, mu, nth, rb, xib, P, nq2, kf, R, prim_smooth ? 1 : 0, n6,
                                     zt, q);
  return hipGetLastError();
}

}  // namespace mp3
