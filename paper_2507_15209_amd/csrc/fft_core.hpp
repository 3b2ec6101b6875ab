// fft_core.hpp -- workgroup-level Stockham FFT building blocks for gfx950.
//
// One column of N complex values is transformed by TPC = N / RMAX threads;
// each thread keeps RMAX values in registers and exchanges them through LDS
// between radix stages (one LDS round trip per stage boundary).  Radix
// sequences per length:
//     16: {16}   32: {8,4}   64: {8,8}   128: {16,8}   256: {16,16}   512: {8,8,8}
// and a low-register variant with radix <= 8 (see FftPlan).
// The first stage always has radix RMAX, so a thread's first-stage inputs are
// the strided elements j + r * (N / RMAX), r < RMAX, which is also the
// coalesced order for global loads.  After the last stage, register e of
// thread j holds output index out_index(j, e); consecutive j give consecutive
// indices for every e, so global stores coalesce too.
//
// Sign convention: DIR = -1 computes sum_n x_n exp(-2 pi i n k / N) (forward),
// DIR = +1 the same with +i (inverse, unnormalised).  Twiddles come from a
// table tw[i] = exp(-2 pi i i / N), generated in float64 on the host.
#pragma once
#include <hip/hip_runtime.h>

namespace mp3 {

template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename T> using c2 = typename cplx<T>::type;

template <typename T> __device__ __forceinline__ c2<T> mk(T re, T im) { c2<T> r; r.x = re; r.y = im; return r; }
template <typename T> __device__ __forceinline__ c2<T> cadd(c2<T> a, c2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ c2<T> csub(c2<T> a, c2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ c2<T> cscale(c2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// multiply by DIR * i
template <int DIR, typename T> __device__ __forceinline__ c2<T> mul_i(c2<T> a) {
  return DIR > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}
// twiddle from the forward table, conjugated for the inverse direction
template <int DIR, typename T> __device__ __forceinline__ c2<T> twid(const c2<T>* tw, int idx) {
  c2<T> w = tw[idx];
  if (DIR > 0) w.y = -w.y;
  return w;
}

// ---------------------------------------------------------------------------
// small DFTs in registers, natural order in and out
// ---------------------------------------------------------------------------
template <int DIR, typename T> __device__ __forceinline__ void dft2(c2<T>* v) {
  c2<T> a = v[0], b = v[1];
  v[0] = cadd<T>(a, b);
  v[1] = csub<T>(a, b);
}

template <int DIR, typename T> __device__ __forceinline__ void dft4(c2<T>& x0, c2<T>& x1, c2<T>& x2, c2<T>& x3) {
  c2<T> a = cadd<T>(x0, x2), b = csub<T>(x0, x2);
  c2<T> c = cadd<T>(x1, x3), d = mul_i<DIR, T>(csub<T>(x1, x3));
  x0 = cadd<T>(a, c);
  x2 = csub<T>(a, c);
  x1 = cadd<T>(b, d);
  x3 = csub<T>(b, d);
}

template <int DIR, typename T> __device__ __forceinline__ void dft4(c2<T>* v) { dft4<DIR, T>(v[0], v[1], v[2], v[3]); }

template <int DIR, typename T> __device__ __forceinline__ void dft8(c2<T>* v) {
  const T h = (T)0.70710678118654752440084436210484903928;
  c2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  c2<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR, T>(e0, e1, e2, e3);
  dft4<DIR, T>(o0, o1, o2, o3);
  // w8^1 = h (1 + DIR i), w8^2 = DIR i, w8^3 = h (-1 + DIR i)
  c2<T> t1 = cscale<T>(cadd<T>(o1, mul_i<DIR, T>(o1)), h);
  c2<T> t2 = mul_i<DIR, T>(o2);
  c2<T> t3 = cscale<T>(csub<T>(mul_i<DIR, T>(o3), o3), h);
  v[0] = cadd<T>(e0, o0); v[4] = csub<T>(e0, o0);
  v[1] = cadd<T>(e1, t1); v[5] = csub<T>(e1, t1);
  v[2] = cadd<T>(e2, t2); v[6] = csub<T>(e2, t2);
  v[3] = cadd<T>(e3, t3); v[7] = csub<T>(e3, t3);
}

template <int DIR, typename T> __device__ __forceinline__ void dft16(c2<T>* v) {
  // n = n2 + 4 n1, k = k1 + 4 k2: inner 4-point DFTs over n1, twiddle w16^(n2 k1),
  // outer 4-point DFTs over n2.
  const T c1 = (T)0.92387953251128675612818318939678828682;  // cos(pi/8)
  const T s1 = (T)0.38268343236508977172845998403039886676;  // sin(pi/8)
  const T h = (T)0.70710678118654752440084436210484903928;
  c2<T> y[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    c2<T> a0 = v[n2], a1 = v[n2 + 4], a2 = v[n2 + 8], a3 = v[n2 + 12];
    dft4<DIR, T>(a0, a1, a2, a3);
    y[n2 * 4 + 0] = a0; y[n2 * 4 + 1] = a1; y[n2 * 4 + 2] = a2; y[n2 * 4 + 3] = a3;
  }
  // twiddles w16^p, p = n2 * k1 in {0..9}; w16^p = cos(2 pi p/16) + DIR i sin(2 pi p/16)
  const T cs[10] = {(T)1, c1, h, s1, (T)0, -s1, -h, -c1, (T)-1, -c1};
  const T sn[10] = {(T)0, s1, h, c1, (T)1, c1, h, s1, (T)0, -s1};
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2) {
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) {
      const int p = n2 * k1;
      c2<T> w = mk<T>(cs[p], DIR > 0 ? sn[p] : -sn[p]);
      y[n2 * 4 + k1] = cmul<T>(y[n2 * 4 + k1], w);
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    c2<T> a0 = y[k1], a1 = y[4 + k1], a2 = y[8 + k1], a3 = y[12 + k1];
    dft4<DIR, T>(a0, a1, a2, a3);
    v[k1] = a0; v[k1 + 4] = a1; v[k1 + 8] = a2; v[k1 + 12] = a3;
  }
}

template <int R, int DIR, typename T> __device__ __forceinline__ void dft(c2<T>* v) {
  if constexpr (R == 2) dft2<DIR, T>(v);
  else if constexpr (R == 4) dft4<DIR, T>(v);
  else if constexpr (R == 8) dft8<DIR, T>(v);
  else if constexpr (R == 16) dft16<DIR, T>(v);
}

// ---------------------------------------------------------------------------
// per-length radix plans
// ---------------------------------------------------------------------------
// Radix plans.  Variant V = 0 favours few stages (radix 16), V = 1 keeps at
// most 8 values per thread (fewer registers, one more LDS exchange).
template <int N, int V> struct FftPlan;
template <> struct FftPlan<16, 0>  { static constexpr int RMAX = 16, S = 1; static constexpr int R[3] = {16, 1, 1}; };
template <> struct FftPlan<32, 0>  { static constexpr int RMAX = 8,  S = 2; static constexpr int R[3] = {8, 4, 1}; };
template <> struct FftPlan<64, 0>  { static constexpr int RMAX = 8,  S = 2; static constexpr int R[3] = {8, 8, 1}; };
template <> struct FftPlan<128, 0> { static constexpr int RMAX = 16, S = 2; static constexpr int R[3] = {16, 8, 1}; };
template <> struct FftPlan<256, 0> { static constexpr int RMAX = 16, S = 2; static constexpr int R[3] = {16, 16, 1}; };
template <> struct FftPlan<512, 0> { static constexpr int RMAX = 8,  S = 3; static constexpr int R[3] = {8, 8, 8}; };
template <> struct FftPlan<16, 1>  { static constexpr int RMAX = 4,  S = 2; static constexpr int R[3] = {4, 4, 1}; };
template <> struct FftPlan<32, 1>  { static constexpr int RMAX = 8,  S = 2; static constexpr int R[3] = {8, 4, 1}; };
template <> struct FftPlan<64, 1>  { static constexpr int RMAX = 8,  S = 2; static constexpr int R[3] = {8, 8, 1}; };
template <> struct FftPlan<128, 1> { static constexpr int RMAX = 8,  S = 3; static constexpr int R[3] = {8, 4, 4}; };
template <> struct FftPlan<256, 1> { static constexpr int RMAX = 8,  S = 3; static constexpr int R[3] = {8, 8, 4}; };
template <> struct FftPlan<512, 1> { static constexpr int RMAX = 8,  S = 3; static constexpr int R[3] = {8, 8, 8}; };

template <int N, int V = 0> struct Fft {
  static constexpr int RMAX = FftPlan<N, V>::RMAX;
  static constexpr int S = FftPlan<N, V>::S;
  static constexpr int TPC = N / RMAX;                 // threads per column
  static constexpr int RLAST = FftPlan<N, V>::R[S - 1];
  static constexpr int NSLAST = N / RLAST;
  // output index held in register e of thread j after the last stage
  __device__ __forceinline__ static int out_index(int j, int e) {
    const int t = e / RLAST, r = e % RLAST;
    return j + t * TPC + r * NSLAST;
  }
  // first-stage input index loaded into register r of thread j
  __device__ __forceinline__ static int in_index(int j, int r) { return j + r * TPC; }
};

// LDS addressing of a column: element i at base[(i + pad(i)) * ld]
template <bool PAD> __device__ __forceinline__ int lds_pos(int i) { return PAD ? i + (i >> 4) : i; }

// Synchronisation of a column's exchange: the workgroup, or, when all
// threads of the column are lanes of one wave (WAVE), that wave alone:
// workgroup-scope fences order the LDS accesses and the wave barrier keeps
// the compiler from moving them across.
template <bool WAVE> __device__ __forceinline__ void col_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __syncthreads();
  }
}

// One radix stage (compile-time stage index S_IDX, Ns = product of earlier
// radices): twiddle, butterflies, and -- unless it is the last stage -- the
// LDS exchange that gathers the next stage's inputs.
template <int N, int S_IDX, int DIR, typename T, bool PAD, int V, bool WAVE = false>
__device__ __forceinline__ void fft_stage(c2<T>* v, c2<T>* col, int ld, int j, const c2<T>* tw, bool active, int Ns) {
  using F = Fft<N, V>;
  constexpr int RMAX = F::RMAX;
  constexpr int TPC = F::TPC;
  constexpr int R = FftPlan<N, V>::R[S_IDX];
  constexpr int BPT = RMAX / R;
  if constexpr (S_IDX > 0) {
    if (active) {
      const int step = N / (Ns * R);
#pragma unroll
      for (int t = 0; t < BPT; ++t) {
        const int k = (j + t * TPC) % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) v[t * R + r] = cmul<T>(v[t * R + r], twid<DIR, T>(tw, k * r * step));
      }
    }
  }
#pragma unroll
  for (int t = 0; t < BPT; ++t) dft<R, DIR, T>(v + t * R);
  if constexpr (S_IDX + 1 < F::S) {
    if (active) {
#pragma unroll
      for (int t = 0; t < BPT; ++t) {
        const int jj = j + t * TPC;
        const int base = (jj / Ns) * Ns * R + (jj % Ns);
#pragma unroll
        for (int r = 0; r < R; ++r) col[lds_pos<PAD>(base + r * Ns) * ld] = v[t * R + r];
      }
    }
    col_sync<WAVE>();
    constexpr int Rn = FftPlan<N, V>::R[S_IDX + 1];
    constexpr int BPTn = RMAX / Rn;
    if (active) {
#pragma unroll
      for (int t = 0; t < BPTn; ++t) {
        const int jj = j + t * TPC;
#pragma unroll
        for (int r = 0; r < Rn; ++r) v[t * Rn + r] = col[lds_pos<PAD>(jj + r * (N / Rn)) * ld];
      }
    }
    col_sync<WAVE>();
    fft_stage<N, S_IDX + 1, DIR, T, PAD, V, WAVE>(v, col, ld, j, tw, active, Ns * R);
  }
}

// Transform one column.  v holds the first-stage inputs on entry and the
// outputs (see Fft<N>::out_index) on exit.  col is the column's LDS storage
// (element i at col[lds_pos<PAD>(i) * ld]); it is used as exchange space.
// Every thread of the workgroup must call this the same number of times
// (it contains __syncthreads when N has more than one stage); threads without
// a column pass active = false.  WAVE: the caller guarantees that the TPC
// threads of every column are lanes of one wave (consecutive thread indices,
// TPC dividing 64); the exchanges then synchronise that wave only.
template <int N, int DIR, typename T, bool PAD, int V = 0, bool WAVE = false>
__device__ __forceinline__ void fft_column(c2<T>* v, c2<T>* col, int ld, int j, const c2<T>* tw, bool active) {
  fft_stage<N, 0, DIR, T, PAD, V, WAVE>(v, col, ld, j, tw, active, 1);
}

}  // namespace mp3
