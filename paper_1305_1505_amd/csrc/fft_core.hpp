// Device FFT engine for gfx950: mixed-radix (8/4/3/2) Stockham transforms of a tile of pencils
// staged in LDS.
//
// A workgroup transforms Q*P pencils of length N at once.  Two LDS layouts:
//   interleaved (IL = true):  element n of pencil p of transform q at (q*N + n)*P + p -- the
//       pencil index runs fastest, matching a strided global tile whose P pencils are P
//       consecutive (contiguous) z positions;
//   contiguous  (IL = false): at (q*P + p)*NPAD + n + n/16 -- the element index runs fastest,
//       matching a global tile of P contiguous lines; one pad element per 16 spreads the
//       stride-R accesses of the Stockham writes over the LDS banks.
// The first stage reads its inputs from registers (loaded from HBM by the caller, with any
// spectral multiplier already applied) and the last stage leaves its outputs in registers, in
// the same per-thread layout: thread t owns butterflies b = t + k*T (k < K0) of the first
// stage's radix R0, i.e. the elements n = j + s*N/R0 (s < R0) of pencil (q, p).  The radix
// order puts equal radices first and last so that this holds; otherwise the result is gathered
// back through LDS.  Middle stages run in place in LDS with a barrier between read and write.
//
// Stockham stage (radix R, Ns = product of the radices before it), for butterfly j < N/R:
//   inputs  x[j + s*N/R] * w^(s * (j mod Ns) * N/(Ns R)),  w = exp(DIR * 2 pi i / N),
//   radix-R DFT with root exp(DIR * 2 pi i / R),
//   outputs to (j / Ns) * Ns * R + (j mod Ns) + s*Ns.
// Twiddles come from a table of exp(2 pi i m/N), m < N, computed in float64 on the host and
// rounded once to the transform precision (conjugated for DIR = -1), staged in LDS per stage
// (load_stage_twiddles).
#pragma once

#include <hip/hip_runtime.h>

namespace pin {

template <typename R> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V, typename R> __device__ __forceinline__ V cscale(V a, R s) { return V{a.x * s, a.y * s}; }
template <typename V> __device__ __forceinline__ V conj(V a) { return V{a.x, -a.y}; }
// DIR * i * a
template <int DIR, typename V> __device__ __forceinline__ V mul_i(V a) {
  return DIR > 0 ? V{-a.y, a.x} : V{a.y, -a.x};
}

// ---------------------------------------------------------------------------------------------
// Radix factorisation: N = 2^e 3^t with radices 8, 4, 2, 3; equal radices at both ends.
struct Factor {
  int n;
  int r[16];
};

constexpr Factor factorize(int N) {
  Factor f{0, {}};
  int e = 0, t = 0, m = N;
  while (m > 1 && m % 2 == 0) { m /= 2; ++e; }
  while (m > 1 && m % 3 == 0) { m /= 3; ++t; }
  int n8 = e / 3, n4 = 0, n2 = 0;
  const int rem = e % 3;
  if (rem == 1) {
    if (n8 > 0) { --n8; n4 = 2; } else { n2 = 1; }
  } else if (rem == 2) {
    n4 = 1;
  }
  int list[16] = {};
  int c = 0;
  for (int i = 0; i < n8; ++i) list[c++] = 8;
  for (int i = 0; i < n4; ++i) list[c++] = 4;
  for (int i = 0; i < n2; ++i) list[c++] = 2;
  for (int i = 0; i < t; ++i) list[c++] = 3;
  // move one copy of a repeated radix to the end so that first == last
  int rep = 0;
  if (n8 >= 2) rep = 8; else if (n4 >= 2) rep = 4; else if (t >= 2) rep = 3;
  if (rep != 0) {
    int first = -1;
    for (int i = 0; i < c; ++i) if (list[i] == rep) { first = i; break; }
    // list[first] stays; take the last occurrence and move it to the end, put `rep` first
    int lastpos = -1;
    for (int i = c - 1; i >= 0; --i) if (list[i] == rep) { lastpos = i; break; }
    int tmp[16] = {};
    int k = 0;
    tmp[k++] = rep;
    for (int i = 0; i < c; ++i) if (i != first && i != lastpos) tmp[k++] = list[i];
    tmp[k++] = rep;
    for (int i = 0; i < c; ++i) list[i] = tmp[i];
  }
  f.n = c;
  for (int i = 0; i < c; ++i) f.r[i] = list[i];
  return f;
}

constexpr int radix_prefix(const Factor& f, int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= f.r[i];
  return p;
}

// Twiddles of the middle and last stages, laid out per stage in LDS as
//   [off(s) + (x - 1) * Ns + kk] = w^(x * kk * N/(Ns R)),   x in [1, R), kk in [0, Ns)
// for stage s >= 1 (radix R, Ns = product of the earlier radices): the lanes of a butterfly row
// read consecutive entries, free of the bank conflicts of strided reads into an N-entry table.
constexpr int tw_stage_offset(const Factor& f, int s) {
  int off = 0;
  for (int i = 1; i < s; ++i) off += (f.r[i] - 1) * radix_prefix(f, i);
  return off;
}
constexpr int tw_elems(int N) {
  const Factor f = factorize(N);
  const int e = tw_stage_offset(f, f.n);
  return e > 0 ? e : 1;
}

// Source index in the N-entry table of per-stage entry i (stage found by compile-time recursion,
// so that no stage parameter is indexed at run time).
template <int N, int S_> __device__ __forceinline__ int tw_source(int i) {
  constexpr Factor f = factorize(N);
  if constexpr (S_ >= f.n) {
    return 0;
  } else {
    constexpr int ns = radix_prefix(f, S_), R = f.r[S_], off = tw_stage_offset(f, S_);
    if (i < off + (R - 1) * ns) {
      const int l = i - off;
      return (l / ns + 1) * (l % ns) * (N / (ns * R));
    }
    return tw_source<N, S_ + 1>(i);
  }
}

// All of a thread's table entries are loaded before any is stored, so that a workgroup waits for
// one round trip to memory instead of one per stage.
template <int N, int T, typename V>
__device__ __forceinline__ void load_stage_twiddles(V* __restrict__ s_tw, const V* __restrict__ tw, int t) {
  constexpr int E = tw_elems(N);
  constexpr int K = (E + T - 1) / T;
  V v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t + k * T;
    v[k] = tw[i < E ? tw_source<N, 1>(i) : 0];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = t + k * T;
    if (i < E) s_tw[i] = v[k];
  }
  __syncthreads();
}

constexpr bool size_ok(int n) {
  if (n < 2) return false;
  int m = n;
  while (m % 2 == 0) m /= 2;
  while (m % 3 == 0) m /= 3;
  return m == 1;
}

// ---------------------------------------------------------------------------------------------
// Small DFTs with root exp(DIR 2 pi i / R), in place.
template <typename V, int DIR> __device__ __forceinline__ void dft2(V& a0, V& a1) {
  V t = a0;
  a0 = cadd(t, a1);
  a1 = csub(t, a1);
}

template <typename V, int DIR> __device__ __forceinline__ void dft4(V& a0, V& a1, V& a2, V& a3) {
  V t0 = cadd(a0, a2), t1 = csub(a0, a2);
  V t2 = cadd(a1, a3), t3 = mul_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <typename V, int DIR> __device__ __forceinline__ void dft3(V& a0, V& a1, V& a2) {
  using R = decltype(a0.x);
  const R h = R(0.5);
  const R s3 = R(0.86602540378443864676372317075294);  // sqrt(3)/2
  V s = cadd(a1, a2), d = csub(a1, a2);
  V m = V{a0.x - h * s.x, a0.y - h * s.y};
  V r = mul_i<DIR>(cscale(d, s3));
  a0 = cadd(a0, s);
  a1 = cadd(m, r);
  a2 = csub(m, r);
}

template <typename V, int DIR> __device__ __forceinline__ void dft8(V (&a)[8]) {
  using R = decltype(a[0].x);
  const R c = R(0.70710678118654752440084436210485);  // 1/sqrt(2)
  dft4<V, DIR>(a[0], a[2], a[4], a[6]);
  dft4<V, DIR>(a[1], a[3], a[5], a[7]);
  // odd half times exp(DIR 2 pi i k/8), k = 1, 2, 3 (a[3] holds k=1, a[5] k=2, a[7] k=3)
  V o1 = a[3], o2 = a[5], o3 = a[7];
  o1 = DIR > 0 ? V{c * (o1.x - o1.y), c * (o1.y + o1.x)} : V{c * (o1.x + o1.y), c * (o1.y - o1.x)};
  o2 = mul_i<DIR>(o2);
  o3 = DIR > 0 ? V{-c * (o3.x + o3.y), c * (o3.x - o3.y)} : V{c * (o3.y - o3.x), -c * (o3.y + o3.x)};
  V e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], q0 = a[1];
  a[0] = cadd(e0, q0);
  a[4] = csub(e0, q0);
  a[1] = cadd(e1, o1);
  a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2);
  a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3);
  a[7] = csub(e3, o3);
}

template <int R, int DIR, typename V> __device__ __forceinline__ void dft(V (&a)[R]) {
  if constexpr (R == 2) {
    dft2<V, DIR>(a[0], a[1]);
  } else if constexpr (R == 3) {
    dft3<V, DIR>(a[0], a[1], a[2]);
  } else if constexpr (R == 4) {
    dft4<V, DIR>(a[0], a[1], a[2], a[3]);
  } else {
    static_assert(R == 8, "radix");
    dft8<V, DIR>(a);
  }
}

// ---------------------------------------------------------------------------------------------
// Engine: Q*P pencils of length N, T threads, direction DIR (+1 inverse, -1 forward).
template <typename V, int N, int P, int Q, bool IL, int T, int DIR>
struct Engine {
  static constexpr Factor FAC = factorize(N);
  static constexpr int S = FAC.n;
  static constexpr int R0 = FAC.r[0];
  static constexpr int RL = FAC.r[S - 1];
  static constexpr bool SAME = (R0 == RL);
  static constexpr int nb(int R) { return Q * P * (N / R); }
  static constexpr int kcount(int R) { return (nb(R) + T - 1) / T; }
  static constexpr int K0 = kcount(R0);
  // most elements a thread holds in any stage
  static constexpr int max_held() {
    int m = 0;
    for (int i = 0; i < FAC.n; ++i) m = kcount(FAC.r[i]) * FAC.r[i] > m ? kcount(FAC.r[i]) * FAC.r[i] : m;
    return m;
  }
  static constexpr int NPAD = IL ? N : N + N / 16 + 1;
  static constexpr int LDS_ELEMS = Q * P * NPAD;

  __device__ static __forceinline__ int lds_index(int q, int p, int n) {
    return IL ? (q * N + n) * P + p : (q * P + p) * NPAD + n + (n >> 4);
  }

  // butterfly b of a radix-R stage -> (q, p, j)
  template <int R> __device__ static __forceinline__ void decomp(int b, int& q, int& p, int& j) {
    constexpr int M = N / R;
    if constexpr (IL) {
      p = b % P;
      j = (b / P) % M;
      q = b / (P * M);
    } else {
      j = b % M;
      p = (b / M) % P;
      q = b / (M * P);
    }
  }

  // element n of the first-stage layout for butterfly slot k, element s of thread t
  __device__ static __forceinline__ void first_layout(int t, int k, int& q, int& p, int& j, bool& ok) {
    const int b = t + k * T;
    ok = b < nb(R0);
    decomp<R0>(ok ? b : 0, q, p, j);
  }

  __device__ static __forceinline__ V twiddle(const V* __restrict__ tw, int m) {
    V w = tw[m];
    return DIR > 0 ? w : conj(w);
  }

  template <int s> __device__ static __forceinline__ void stage(V (&v)[K0][R0], V* lds, const V* __restrict__ tw, int t) {
    constexpr int R = FAC.r[s];
    constexpr int Ns = radix_prefix(FAC, s);
    constexpr int KS = kcount(R);
    constexpr int M = N / R;
    constexpr int TWO = tw_stage_offset(FAC, s);   // this stage's block of the twiddle table
    constexpr bool FIRST = (s == 0);
    constexpr bool LAST = (s == S - 1);
    V a[KS][R];
    int qq[KS], pp[KS], jj[KS];
    bool ok[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int b = t + k * T;
      ok[k] = b < nb(R);
      decomp<R>(ok[k] ? b : 0, qq[k], pp[k], jj[k]);
    }
    if constexpr (FIRST) {
      static_assert(KS == K0 && R == R0, "first stage layout");
#pragma unroll
      for (int k = 0; k < KS; ++k)
#pragma unroll
        for (int x = 0; x < R; ++x) a[k][x] = v[k][x];
    } else {
#pragma unroll
      for (int k = 0; k < KS; ++k)
        if (ok[k]) {
#pragma unroll
          for (int x = 0; x < R; ++x) a[k][x] = lds[lds_index(qq[k], pp[k], jj[k] + x * M)];
        }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      if constexpr (!FIRST) {
        int kk = jj[k] % Ns;
        // Strided (interleaved) tiles: the caller runs several transforms in a loop with one
        // transform's data live; an opaque index keeps the compiler from hoisting every stage's
        // twiddle addresses out of that loop, which would hold ~14 more VGPRs across it.
        if constexpr (IL) asm volatile("" : "+v"(kk));
#pragma unroll
        for (int x = 1; x < R; ++x) a[k][x] = cmul(a[k][x], twiddle(tw, TWO + (x - 1) * Ns + kk));
      }
      dft<R, DIR>(a[k]);
    }
    if constexpr (LAST && SAME) {
#pragma unroll
      for (int k = 0; k < KS; ++k)
#pragma unroll
        for (int x = 0; x < R; ++x) v[k][x] = a[k][x];
    } else {
#pragma unroll
      for (int k = 0; k < KS; ++k)
        if (ok[k]) {
          const int kk = jj[k] % Ns;
          const int idxd = (jj[k] / Ns) * Ns * R + kk;
#pragma unroll
          for (int x = 0; x < R; ++x) lds[lds_index(qq[k], pp[k], idxd + x * Ns)] = a[k][x];
        }
      __syncthreads();
      if constexpr (LAST) {
        // gather the result back into the first-stage layout
#pragma unroll
        for (int k = 0; k < K0; ++k) {
          int q, p, j;
          bool okk;
          first_layout(t, k, q, p, j, okk);
          if (okk) {
#pragma unroll
            for (int x = 0; x < R0; ++x) v[k][x] = lds[lds_index(q, p, j + x * (N / R0))];
          }
        }
        __syncthreads();
      }
    }
  }

  template <int s> __device__ static __forceinline__ void stages(V (&v)[K0][R0], V* lds, const V* __restrict__ tw, int t) {
    stage<s>(v, lds, tw, t);
    if constexpr (s + 1 < S) stages<s + 1>(v, lds, tw, t);
  }

  // In: v in the first-stage layout.  Out: the transform, same layout.  LDS is free on return.
  __device__ static __forceinline__ void run(V (&v)[K0][R0], V* lds, const V* __restrict__ tw, int t) {
    stages<0>(v, lds, tw, t);
  }
};

}  // namespace pin
