// Device-side FFT building blocks for gfx950: complex arithmetic, small DFT
// codelets, per-length radix plans and the per-thread Stockham stage driver.
//
// The prior operator S_L^-1 of the lognormal prior (section 2.3) is a
// convolution on the periodic grid, applied as forward FFT -> pointwise
// multiply -> inverse FFT (section 3: the expensive operations reduce to
// FFTs).  A length-N transform is split into radix stages R_0 R_1 ... with
// the self-sorting (Stockham) ordering: stage s, span Ns = R_0 ... R_{s-1},
// butterfly j reads x[j + r N/R], multiplies by w^{r (j mod Ns)} with
// w = exp(-+2 pi i / (Ns R)), does a radix-R DFT and writes
// y[(j - j mod Ns) R + j mod Ns + m Ns].  P threads cooperate on one
// transform; thread t owns butterflies j = t + P q.  Stages exchange data
// through LDS (or registers when P == 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pl {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }

// multiply by -i (forward) or +i (inverse)
template <bool INV, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> a) {
  if constexpr (INV) return {-a.y, a.x};
  else return {a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Small DFT codelets (in place on v[0..R-1], stride ST between entries)
// ---------------------------------------------------------------------------

template <bool INV, typename T>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a - b;
  a = a + b;
  b = t;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft3(cx<T>& a0, cx<T>& a1, cx<T>& a2) {
  const T h = T(0.86602540378443864676);  // sqrt(3)/2
  cx<T> s = a1 + a2;
  cx<T> t = {a0.x - T(0.5) * s.x, a0.y - T(0.5) * s.y};
  cx<T> u = scale(a1 - a2, h);
  a0 = a0 + s;
  cx<T> ru = rot<INV>(u);  // -+ i u
  a1 = t + ru;
  a2 = t - ru;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> s02 = a0 + a2, d02 = a0 - a2;
  cx<T> s13 = a1 + a3, d13 = rot<INV>(a1 - a3);
  a0 = s02 + s13;
  a2 = s02 - s13;
  a1 = d02 + d13;
  a3 = d02 - d13;
}

// 6 = 2 x 3: DFT3 of the even and of the odd inputs, then one radix-2 step
// with the twiddles w6^k (w6 = exp(-+ 2 pi i / 6)):
//   X[k] = E[k] + w6^k O[k],  X[k + 3] = E[k] - w6^k O[k],  k = 0, 1, 2
template <bool INV, typename T>
__device__ __forceinline__ void dft6(cx<T>* v) {
  const T h = T(0.86602540378443864676);  // sqrt(3)/2
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5];
  dft3<INV>(e0, e1, e2);
  dft3<INV>(o0, o1, o2);
  // w6 = 1/2 -+ i sqrt(3)/2, w6^2 = -1/2 -+ i sqrt(3)/2 (forward: minus)
  cx<T> t1, t2;
  if constexpr (INV) {
    t1 = {T(0.5) * o1.x - h * o1.y, T(0.5) * o1.y + h * o1.x};
    t2 = {-T(0.5) * o2.x - h * o2.y, -T(0.5) * o2.y + h * o2.x};
  } else {
    t1 = {T(0.5) * o1.x + h * o1.y, T(0.5) * o1.y - h * o1.x};
    t2 = {-T(0.5) * o2.x + h * o2.y, -T(0.5) * o2.y - h * o2.x};
  }
  v[0] = e0 + o0;
  v[3] = e0 - o0;
  v[1] = e1 + t1;
  v[4] = e1 - t1;
  v[2] = e2 + t2;
  v[5] = e2 - t2;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  const T r2 = T(0.70710678118654752440);
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  // twiddles w8^k, k = 0..3, w8 = exp(-+ 2 pi i / 8)
  cx<T> t1, t3;
  if constexpr (INV) {
    t1 = {r2 * (o1.x - o1.y), r2 * (o1.x + o1.y)};     // (1 + i)/sqrt2
    t3 = {-r2 * (o3.x + o3.y), r2 * (o3.x - o3.y)};    // (-1 + i)/sqrt2
  } else {
    t1 = {r2 * (o1.x + o1.y), r2 * (o1.y - o1.x)};     // (1 - i)/sqrt2
    t3 = {r2 * (o3.y - o3.x), -r2 * (o3.x + o3.y)};    // (-1 - i)/sqrt2
  }
  cx<T> t2 = rot<INV>(o2);
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = e1 + t1;
  v[5] = e1 - t1;
  v[2] = e2 + t2;
  v[6] = e2 - t2;
  v[3] = e3 + t3;
  v[7] = e3 - t3;
}

// w16^e for e = 0..9 (forward sign), as (cos, -sin) pairs; inverse conjugates
template <bool INV, typename T>
__device__ __forceinline__ cx<T> w16(int e) {
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
  const T r2 = T(0.70710678118654752440);
  cx<T> w;
  switch (e) {
    case 0: w = {T(1), T(0)}; break;
    case 1: w = {c1, -s1}; break;
    case 2: w = {r2, -r2}; break;
    case 3: w = {s1, -c1}; break;
    case 4: w = {T(0), T(-1)}; break;
    case 6: w = {-r2, -r2}; break;
    case 9: w = {-c1, s1}; break;
    default: w = {T(1), T(0)}; break;
  }
  if constexpr (INV) w.y = -w.y;
  return w;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft16(cx<T>* v) {
  // n = n1 + 4 n2, k = k2 + 4 k1
  cx<T> f[16];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    cx<T> a0 = v[n1], a1 = v[n1 + 4], a2 = v[n1 + 8], a3 = v[n1 + 12];
    dft4<INV>(a0, a1, a2, a3);
    f[n1 * 4 + 0] = a0;
    f[n1 * 4 + 1] = a1;
    f[n1 * 4 + 2] = a2;
    f[n1 * 4 + 3] = a3;
  }
#pragma unroll
  for (int n1 = 1; n1 < 4; ++n1)
#pragma unroll
    for (int k2 = 1; k2 < 4; ++k2) f[n1 * 4 + k2] = cmul(f[n1 * 4 + k2], w16<INV, T>(n1 * k2));
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    cx<T> a0 = f[0 * 4 + k2], a1 = f[1 * 4 + k2], a2 = f[2 * 4 + k2], a3 = f[3 * 4 + k2];
    dft4<INV>(a0, a1, a2, a3);
    v[k2 + 0] = a0;
    v[k2 + 4] = a1;
    v[k2 + 8] = a2;
    v[k2 + 12] = a3;
  }
}

template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_r(cx<T>* v) {
  if constexpr (R == 2) dft2<INV>(v[0], v[1]);
  else if constexpr (R == 3) dft3<INV>(v[0], v[1], v[2]);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 6) dft6<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 16) dft16<INV>(v);
  else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Radix plans per transform length: radices R_0..R_{S-1} and threads P per
// transform (each thread holds W = N/P values; every radix divides W).
// ---------------------------------------------------------------------------

template <int N>
struct Plan;
#define PL_PLAN(NN, PP, S, A, B, C)                         \
  template <>                                               \
  struct Plan<NN> {                                         \
    static constexpr int N = NN, P = PP, W = NN / PP, NS = S; \
    static constexpr int R0 = A, R1 = B, R2 = C;            \
  };
PL_PLAN(8, 1, 1, 8, 1, 1)
PL_PLAN(12, 1, 2, 4, 3, 1)
PL_PLAN(16, 1, 1, 16, 1, 1)
PL_PLAN(24, 1, 2, 8, 3, 1)
PL_PLAN(32, 4, 2, 8, 4, 1)
PL_PLAN(48, 4, 3, 4, 4, 3)
PL_PLAN(64, 8, 2, 8, 8, 1)
PL_PLAN(96, 8, 3, 4, 4, 6)
PL_PLAN(128, 8, 2, 16, 8, 1)
PL_PLAN(192, 8, 3, 8, 8, 3)
PL_PLAN(256, 16, 2, 16, 16, 1)
PL_PLAN(512, 32, 3, 8, 8, 8)
#undef PL_PLAN

template <class PL, int S>
struct StageInfo {
  static constexpr int R = S == 0 ? PL::R0 : (S == 1 ? PL::R1 : PL::R2);
  static constexpr int NS = S == 0 ? 1 : (S == 1 ? PL::R0 : PL::R0 * PL::R1);
};

template <class PL>
struct LastStage {
  static constexpr int R = StageInfo<PL, PL::NS - 1>::R;
};

// Position of the element a thread holds in slot (q, r) at the input of
// stage S and at its output.
template <class PL, int S>
__device__ __forceinline__ int in_pos(int t, int q, int r) {
  constexpr int R = StageInfo<PL, S>::R;
  return t + PL::P * q + r * (PL::N / R);
}
template <class PL, int S>
__device__ __forceinline__ int out_pos(int t, int q, int m) {
  constexpr int R = StageInfo<PL, S>::R;
  constexpr int Ns = StageInfo<PL, S>::NS;
  int j = t + PL::P * q;
  int k = j % Ns;
  return (j - k) * R + k + m * Ns;
}

// Twiddle tables: tw[e] = exp(-2 pi i e / N), e in [0, N).
template <class PL, int S, bool INV, typename T>
__device__ __forceinline__ void stage_compute(cx<T>* v, int t, const cx<T>* __restrict__ tw) {
  constexpr int R = StageInfo<PL, S>::R;
  constexpr int Ns = StageInfo<PL, S>::NS;
  constexpr int Q = PL::W / R;
  constexpr int STEP = PL::N / (Ns * R);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    cx<T>* b = v + q * R;
    if constexpr (Ns > 1) {
      int k = (t + PL::P * q) % Ns;
      // powers w^r, r = 1..R-1, of w = exp(-2 pi i k / (Ns R)): w^1, w^2,
      // w^4, w^8 from the table, the rest as products of at most three of
      // them (a few ulp, instead of one table load per power)
      cx<T> w[R];
      w[1] = tw[k * STEP];
      if constexpr (R > 2) w[2] = tw[2 * k * STEP];
      if constexpr (R == 3) {
      } else {
        if constexpr (R > 3) w[3] = cmul(w[1], w[2]);
        if constexpr (R > 4) {
          w[4] = tw[4 * k * STEP];
          w[5] = cmul(w[4], w[1]);
        }
        if constexpr (R > 6) {
          w[6] = cmul(w[4], w[2]);
          w[7] = cmul(w[4], w[3]);
        }
        if constexpr (R > 8) {
          w[8] = tw[8 * k * STEP];
#pragma unroll
          for (int r = 9; r < R; ++r) w[r] = cmul(w[8], w[r - 8]);
        }
      }
#pragma unroll
      for (int r = 1; r < R; ++r) b[r] = INV ? cmulc(b[r], w[r]) : cmul(b[r], w[r]);
    }
    dft_r<R, INV>(b);
  }
}

// LDS accessor: element e of the transform lives at base[e * STRIDE + pad],
// with one padding slot every 2^PL_ROW_PAD_SHIFT elements when PAD is set.
#ifndef PL_ROW_PAD_SHIFT
#define PL_ROW_PAD_SHIFT 4
#endif
template <int STRIDE, bool PAD>
struct LdsMap {
  __device__ __forceinline__ static int off(int e) {
    if constexpr (PAD && PL_ROW_PAD_SHIFT < 16) return (e + (e >> PL_ROW_PAD_SHIFT)) * STRIDE;
    else return e * STRIDE;
  }
};

template <int N, bool PAD>
struct PaddedLen {
  static constexpr int value = (PAD && PL_ROW_PAD_SHIFT < 16) ? (N + (N >> PL_ROW_PAD_SHIFT) + 1) : N + 1;
};

// Permute the block's data through LDS: slot (q, m) of every thread (QA
// groups of RA) goes to element POS_A(t, q, m), then slot (q, r) (QB groups
// of RB) is read back from element POS_B(t, q, r).
// SPLIT: the real parts go through LDS first, then the imaginary parts, so
// the exchange needs half the LDS (lds then points at real-valued slots,
// lds[MAP::off(e)] of a T array) at twice the barriers; every real part is
// in LDS before any is overwritten in registers.
template <int RA, int QA, int RB, int QB, class MAP, bool SPLIT = false, typename T, typename PA, typename PB>
__device__ __forceinline__ void lds_permute(cx<T>* v, cx<T>* lds, bool active, PA pos_a, PB pos_b) {
  if constexpr (SPLIT) {
    T* lt = reinterpret_cast<T*>(lds);
    __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < QA; ++q)
#pragma unroll
        for (int m = 0; m < RA; ++m) lt[MAP::off(pos_a(q, m))] = v[q * RA + m].x;
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < QB; ++q)
#pragma unroll
        for (int r = 0; r < RB; ++r) v[q * RB + r].x = lt[MAP::off(pos_b(q, r))];
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < QA; ++q)
#pragma unroll
        for (int m = 0; m < RA; ++m) lt[MAP::off(pos_a(q, m))] = v[q * RA + m].y;
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < QB; ++q)
#pragma unroll
        for (int r = 0; r < RB; ++r) v[q * RB + r].y = lt[MAP::off(pos_b(q, r))];
    }
  } else {
    __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < QA; ++q)
#pragma unroll
        for (int m = 0; m < RA; ++m) lds[MAP::off(pos_a(q, m))] = v[q * RA + m];
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < QB; ++q)
#pragma unroll
        for (int r = 0; r < RB; ++r) v[q * RB + r] = lds[MAP::off(pos_b(q, r))];
    }
  }
}

// Exchange between stage S-1 (outputs) and stage S (inputs).  Threads with
// active == false take part in the barriers only.
template <class PL, int S, class MAP, bool SPLIT = false, typename T>
__device__ __forceinline__ void stage_exchange(cx<T>* v, int t, cx<T>* lds, bool active) {
  constexpr int RP = StageInfo<PL, S - 1>::R;
  constexpr int R = StageInfo<PL, S>::R;
  if constexpr (PL::P == 1) {
    cx<T> tmp[PL::N];
#pragma unroll
    for (int q = 0; q < PL::W / RP; ++q)
#pragma unroll
      for (int m = 0; m < RP; ++m) tmp[out_pos<PL, S - 1>(0, q, m)] = v[q * RP + m];
#pragma unroll
    for (int q = 0; q < PL::W / R; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) v[q * R + r] = tmp[in_pos<PL, S>(0, q, r)];
  } else {
    lds_permute<RP, PL::W / RP, R, PL::W / R, MAP, SPLIT>(
        v, lds, active, [t](int q, int m) { return out_pos<PL, S - 1>(t, q, m); },
        [t](int q, int r) { return in_pos<PL, S>(t, q, r); });
  }
}

// Whole transform: v holds stage-0 inputs (slot (q,r) <-> in_pos<0>) and
// returns last-stage outputs (slot (q,m) <-> out_pos<NS-1>).  All threads of
// the block must call this together when P > 1 (it contains barriers).
template <class PL, bool INV, class MAP, bool SPLIT = false, typename T>
__device__ __forceinline__ void fft_thread(cx<T>* v, int t, cx<T>* lds, const cx<T>* __restrict__ tw,
                                           bool active = true) {
  if (active) stage_compute<PL, 0, INV>(v, t, tw);
  if constexpr (PL::NS > 1) {
    stage_exchange<PL, 1, MAP, SPLIT>(v, t, lds, active);
    if (active) stage_compute<PL, 1, INV>(v, t, tw);
  }
  if constexpr (PL::NS > 2) {
    stage_exchange<PL, 2, MAP, SPLIT>(v, t, lds, active);
    if (active) stage_compute<PL, 2, INV>(v, t, tw);
  }
}

// Move data held in last-stage output slots into stage-0 input slots (used
// between an inverse and a forward transform of the same data).
template <class PL, class MAP, bool SPLIT = false, typename T>
__device__ __forceinline__ void last_to_first(cx<T>* v, int t, cx<T>* lds, bool active = true) {
  constexpr int RL = LastStage<PL>::R;
  constexpr int R0 = PL::R0;
  if constexpr (RL == R0) {
    // out_pos<last>(t,q,m) = t + P q + m N/RL = in_pos<0>(t,q,m): same slots
    (void)v; (void)t; (void)lds;
  } else if constexpr (PL::P == 1) {
    cx<T> tmp[PL::N];
#pragma unroll
    for (int q = 0; q < PL::W / RL; ++q)
#pragma unroll
      for (int m = 0; m < RL; ++m) tmp[out_pos<PL, PL::NS - 1>(0, q, m)] = v[q * RL + m];
#pragma unroll
    for (int q = 0; q < PL::W / R0; ++q)
#pragma unroll
      for (int r = 0; r < R0; ++r) v[q * R0 + r] = tmp[in_pos<PL, 0>(0, q, r)];
  } else {
    lds_permute<RL, PL::W / RL, R0, PL::W / R0, MAP, SPLIT>(
        v, lds, active, [t](int q, int m) { return out_pos<PL, PL::NS - 1>(t, q, m); },
        [t](int q, int r) { return in_pos<PL, 0>(t, q, r); });
  }
}

}  // namespace pl
