// HIP kernels of the collapse-time path for one grid size N and one precision.
//
// Layouts (C order, z fastest):
//   user half spectrum dk   [N][N][N/2+1] complex
//   half slot               [N][N][N/2]   complex -- the kz = N/2 (Nyquist) plane is zero by
//                                                    construction and is not stored
//   packed z slot           [N][N][N]     complex -- for one pair of real outputs (A, B), the
//       full-length z spectrum C = A + iB of each (x, y) line, stored as
//         P[k]       = C[k]       k in [0, N/2)
//         P[N/2 + k] = C[N - k]   k in [1, N/2)     (= conj(A[k]) + i conj(B[k]))
//       (P[N/2], the Nyquist term, is zero and is neither written nor read), so that both halves
//       are written as aligned runs by the y pass and the z pass loads each element once.
//   real field              [N][N][N]
//
// Inverse 3D transform of the six Hessian components with shared prefixes.  With
// g = M W dk / f^2 (M zeroes Nyquist modes, W the Gaussian window, f the integer wavevector),
// component (a, b, c) with a + b + c = 2 is the inverse transform of fx^a fy^b fz^c g, and the
// factors fx^a, fy^b, fz^c commute with the other axes' transforms:
//   x pass:  X_a = IFFT_x[fx^a g]                      a = 0, 1, 2         (1 -> 3 half slots)
//   y pass:  S_abc = IFFT_y[fy^b X_a] fz^c, written in pairs of components (3 -> 3 packed slots)
//   z pass:  IFFT_z of each packed pair gives two real components per complex transform; the six
//            real values of a point stay in registers for the per-point epilogue (collapse,
//            store, or the 2LPT source).
// Gradients (displacements) use the same passes with a + b + c = 1 and g = i c M dk / f^2.
// Every kernel first stages the twiddles it needs in LDS, laid out per FFT stage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "collapse_dev.hpp"
#include "fft_core.hpp"

namespace pin {

// ---------------------------------------------------------------------------------------------
// Tile shapes
// Tuning constants (measured at 512^3 on MI355X): 128-byte z rows for the strided passes; the z
// pass keeps one transform of 4 lines in LDS at a time (its three transforms run in turn), which
// keeps its LDS below 25 KB so that VGPRs, not LDS, bound its occupancy.
constexpr int kRowBytes = 128;
constexpr bool kZSequential = true;
constexpr int kZWaves = 4;
template <typename R> struct Tile {
  using V = typename Cplx<R>::type;
  static constexpr int PS = kRowBytes / (int)sizeof(V);   // strided passes: rows of z
};

// Blocks are dealt round-robin to the 8 XCDs (block b runs on XCD b mod 8).  The strided passes
// give XCD k the contiguous tile range [k G/8, (k+1) G/8): the tiles in flight on one XCD then
// cover whole rows of the same slabs, which spreads them over the L2 and lets the per-transform
// re-reads of an input tile (x and y passes) hit there.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  if (nblocks % 8 != 0) return b;
  return (b & 7) * (nblocks >> 3) + (b >> 3);
}

constexpr int round_up64(int x) { return (x + 63) / 64 * 64; }
constexpr int strided_threads(int nb0) { return round_up64(nb0 < 1024 ? nb0 : 1024); }
constexpr int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// Strided passes (x, y): a workgroup owns PS consecutive z (one 128-byte row) of one pencil set
// and all N elements along the transform axis.
template <typename R, int N, int DIR>
struct Strided {
  using V = typename Cplx<R>::type;
  static constexpr int PS = Tile<R>::PS;
  static constexpr int HZ = N / 2;
  static constexpr int NZT = (HZ + PS - 1) / PS;
  using E0 = Engine<V, N, PS, 1, true, 64, DIR>;
  static constexpr int T = strided_threads(E0::nb(E0::R0));
  using E = Engine<V, N, PS, 1, true, T, DIR>;
  // occupancy target (waves per SIMD): two 1024-thread workgroups per CU for float32 tiles where
  // each thread owns one butterfly and the transform ends in registers (the x and y passes keep
  // one transform's data live, within 64 VGPRs); otherwise 4 (float64 tiles are LDS-bound there)
  static constexpr int WPE = (sizeof(V) == 8 && E::K0 == 1 && E::SAME && E::max_held() <= E::R0) ? 8 : 4;
  // the float64 x pass keeps three outputs' multipliers and a transform live: at 4 waves per SIMD
  // it spills; 2 waves (1.37 -> 1.21 ms at 512^3).  The float32 Hessian x pass of workgroups
  // under 1024 threads (64^3, 256^3: 64 bytes a lane at 64 VGPRs, which made the 256^3 pass
  // fetch 5.6x its input) gets 6 waves per SIMD (80 VGPRs; three 512-thread workgroups a CU).
  static constexpr int XWPE = sizeof(V) == 16 ? 2 : (WPE == 8 && T < 1024 ? 6 : WPE);
  static constexpr int GRID = N * NZT;
  static constexpr size_t HSLOT = (size_t)N * N * HZ;
};

// z pass: P lines per workgroup so that T = P * N/R0 threads (<= 64 kZWaves) and the LDS tile
// stays within 96 KB.
template <typename R, int N, int Q> struct ZTile {
  using V = typename Cplx<R>::type;
  static constexpr int R0 = factorize(N).r[0];
  static constexpr int M0 = N / R0;
  static constexpr int NPAD = N + N / 16 + 1;
  static constexpr int QL = kZSequential ? 1 : Q;   // transforms resident in LDS at once
  static constexpr int P_by_threads = pow2_floor((kZWaves * 64) / M0 > 0 ? (kZWaves * 64) / M0 : 1);
  static constexpr int P_by_lds = pow2_floor((96 * 1024) / (QL * NPAD * (int)sizeof(V)) > 0
                                                 ? (96 * 1024) / (QL * NPAD * (int)sizeof(V)) : 1);
  static constexpr int P0 = P_by_threads < P_by_lds ? P_by_threads : P_by_lds;
  static constexpr int P = P0 < 2 ? 2 : P0;   // even: the 2LPT epilogue pairs lines
  static constexpr int T = P * M0;
};

// The prepared half slot g0 (k_prep's output, read only by the Hessian x pass): tiled where W
// divides N/2, so that an x-pass workgroup (one y, W consecutive z, all x) reads one contiguous
// block of N W elements instead of W elements every 1 MB at 512^3 (x pass 0.494 -> 0.463 ms);
// rows (x, y, z) otherwise.
template <typename R, int N> struct PrepLayout {
  static constexpr int W = Tile<R>::PS;
  static constexpr int HZ = N / 2;
  static constexpr bool TILED = HZ % W == 0;
  __device__ static __forceinline__ size_t index(int x, int y, int z) {
    if constexpr (TILED) {
      return (((size_t)y * (HZ / W) + z / W) * N + x) * W + z % W;
    } else {
      return ((size_t)x * N + y) * HZ + z;
    }
  }
};

// Packed z lines, the y pass's output and the z pass's input: N lines of N complex per x-plane,
// element n of line (x, y) at `index(x, y, n)`.  Tiled where the widths allow: positions in
// groups of W (one y-pass tile row, 128 bytes), and for each x and group the N lines' W elements
// one after another.  A y-pass workgroup then writes whole contiguous blocks (N W elements per
// group) instead of W elements every line (y pass 1.02 -> 0.96 ms at 512^3), and a z-pass wave
// still reads W consecutive elements per group.  The z pass steps through its elements
// M0 = N/R0 positions apart, which must stay in the same column of a group.
template <typename R, int N> struct PackedLayout {
  static constexpr int W = Tile<R>::PS;
  static constexpr int M0 = N / factorize(N).r[0];
  static constexpr bool TILED = (N / 2) % W == 0 && M0 % W == 0;
  // elements between positions n and n + M0 of a line
  static constexpr size_t STEP = TILED ? (size_t)(M0 / W) * N * W : (size_t)M0;
  // affine in n (also for n outside [0, N), so that offsets can be formed from a base)
  __device__ static __forceinline__ long long index(int x, int y, int n) {
    if constexpr (TILED) {
      const int g = n >= 0 ? n / W : -((W - 1 - n) / W);
      return (((long long)x * (N / W) + g) * N + y) * W + (n - g * W);
    } else {
      return ((long long)x * N + y) * N + n;
    }
  }
};

__device__ __forceinline__ int ifreq(int i, int n) { return i < (n >> 1) ? i : i - n; }

template <typename R> __device__ __forceinline__ R powf_int(R f, int e) {
  return e == 0 ? R(1) : (e == 1 ? f : f * f);
}

// Streaming store: the line is not retained in the caches.  Used for every output that the next
// pass reads only after much other traffic: plain stores would leave dirty lines that evict the
// tiles a pass re-reads, or that the next pass has to write back while it runs.
template <typename V> __device__ __forceinline__ void st_stream(V* p, V v) {
  using R = decltype(v.x);
  typedef R R2 __attribute__((ext_vector_type(2)));
  R2 w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<R2*>(p));
}

// Streaming load, for the last read of a tile (its lines need not stay in L2).
template <typename V> __device__ __forceinline__ V ld_stream(const V* p) {
  using R = decltype(p->x);
  typedef R R2 __attribute__((ext_vector_type(2)));
  const R2 w = __builtin_nontemporal_load(reinterpret_cast<const R2*>(p));
  return V{w.x, w.y};
}

template <int N, int T, typename V>
__device__ __forceinline__ void load_twiddles(V* __restrict__ s_tw, const V* __restrict__ tw, int t) {
  load_stage_twiddles<N, T>(s_tw, tw, t);
}

// ---------------------------------------------------------------------------------------------
// Radius-independent part of the Hessian multiplier, once per call: g0 = M dk scale / f^2 into
// a half slot in the x pass's tile order (PrepLayout; the user spectrum's rows of N/2+1 complex
// are neither aligned nor in that order), so the per-radius x pass reads contiguous blocks.
template <typename R, int N>
__global__ void k_prep(const typename Cplx<R>::type* __restrict__ dk, typename Cplx<R>::type* __restrict__ g0,
                       R scale) {
  using V = typename Cplx<R>::type;
  constexpr int HZ = N / 2, NH = N / 2 + 1;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)N * N * HZ) return;
  const int z = (int)(i % HZ);
  const int y = (int)((i / HZ) % N);
  const int x = (int)(i / ((size_t)HZ * N));
  V out = V{R(0), R(0)};
  if (x != N / 2 && y != N / 2) {
    const int fx = ifreq(x, N), fy = ifreq(y, N);
    const R f2 = R(fx * fx + fy * fy + z * z);
    if (f2 > R(0)) {
      const V d = dk[((size_t)x * N + y) * NH + z];
      const R m = scale / f2;
      out = V{d.x * m, d.y * m};
    }
  }
  st_stream(&g0[PrepLayout<R, N>::index(x, y, z)], out);
}

// ---------------------------------------------------------------------------------------------
// x pass.  MODE 0 (Hessian): input g0 (k_prep's tiled half slot), 3 outputs, multiplier
// W(x)W(y)W(z) from the window row wtab (never null; a row of ones for no smoothing).  MODE 1
// (gradient): input the user half spectrum, 2 outputs, multiplier i * scale / f^2 (wtab
// unused).  Outputs: half slots.  Loads are unconditional (lanes without an element read an
// in-bounds address and discard it): a load under a per-lane branch would make the compiler
// wait for each one before issuing the next.
template <typename R, int N, int MODE>
__global__ void __launch_bounds__((Strided<R, N, +1>::T))
__attribute__((amdgpu_waves_per_eu(Strided<R, N, +1>::XWPE, Strided<R, N, +1>::XWPE)))
k_xpass(const typename Cplx<R>::type* __restrict__ in, typename Cplx<R>::type* __restrict__ out,
        const R* __restrict__ wtab, const typename Cplx<R>::type* __restrict__ tw, R scale) {
  using S = Strided<R, N, +1>;
  using V = typename S::V;
  using E = typename S::E;
  constexpr int PS = S::PS, HZ = S::HZ, NH = N / 2 + 1, NA = MODE == 0 ? 3 : 2, M = N / E::R0;
  __shared__ V lds[E::LDS_ELEMS];
  __shared__ V s_tw[tw_elems(N)];
  const int t = threadIdx.x;
  load_twiddles<N, S::T>(s_tw, tw, t);
  const int bt = xcd_tile(blockIdx.x, S::GRID);
  const int zt = bt % S::NZT;
  const int y = bt / S::NZT;
  const int fy = ifreq(y, N);
  if constexpr (MODE == 0 && E::K0 == 1) {
    // Hessian, one butterfly per thread: same values as the general form below, in a form whose
    // schedule (data loads batched, the window loads kept out of that batch) measured 13% faster
    // at 512^3.  wtab is never null here; the test only shapes that schedule.
    int q, p, j;
    bool ok;
    E::first_layout(t, 0, q, p, j, ok);
    const int z = zt * PS + p;
    ok = ok && z < HZ;
    const R wyz = ok ? wtab[y] * wtab[z] : R(1);
#pragma unroll 1
    for (int a = 0; a < NA; ++a) {
      V u[1][E::R0];
#pragma unroll
      for (int s = 0; s < E::R0; ++s) {
        const int n = j + s * M;
        V val = V{R(0), R(0)};
        if (ok) {
          val = in[PrepLayout<R, N>::index(n, y, z)];
          if (wtab != nullptr) val = cscale(val, wtab[n] * wyz);
        }
        u[0][s] = cscale(val, powf_int(R(ifreq(n, N)), a));
      }
      E::run(u, lds, s_tw, t);
      // outputs streamed past the caches: left there, their dirty lines would be written back
      // while the y pass runs (y pass 1.04 -> 1.01 ms at 512^3)
      if (ok) {
#pragma unroll
        for (int s = 0; s < E::R0; ++s) st_stream(out + a * S::HSLOT + ((size_t)(j + s * M) * N + y) * HZ + z, u[0][s]);
      }
    }
    return;
  }
  int zz[E::K0], jj[E::K0];
  bool ok[E::K0];
  R wyz[E::K0];
#pragma unroll
  for (int k = 0; k < E::K0; ++k) {
    int q, p, j;
    E::first_layout(t, k, q, p, j, ok[k]);
    const int z = zt * PS + p;
    ok[k] = ok[k] && z < HZ;
    zz[k] = ok[k] ? z : 0;   // lanes without an element read (and never write) z = 0
    jj[k] = j;
    if constexpr (MODE == 0) wyz[k] = wtab[y] * wtab[zz[k]];
  }
  // One output at a time: the input tile is read again for each output (an L2 hit after the
  // first), so that only one transform's data is live and two workgroups fit on a CU.
#pragma unroll 1
  for (int a = 0; a < NA; ++a) {
    V u[E::K0][E::R0];
#pragma unroll
    for (int k = 0; k < E::K0; ++k) {
      // opaque copies: addresses and multipliers are computed per output, not hoisted
      int jv = jj[k], z = zz[k];
      asm volatile("" : "+v"(jv), "+v"(z));
#pragma unroll
      for (int s = 0; s < E::R0; ++s) {
        const int n = jv + s * M;
        const R fa = powf_int(R(ifreq(n, N)), a);
        V val;
        if constexpr (MODE == 0) {
          // no mask: a lane without an element never writes its values (to LDS or out)
          val = cscale(in[PrepLayout<R, N>::index(n, y, z)], wtab[n] * wyz[k] * fa);
        } else {
          const V d = in[((size_t)n * N + y) * NH + z];
          const int fx = ifreq(n, N);
          const int f2 = fx * fx + fy * fy + z * z;
          const bool keep = ok[k] && n != N / 2 && y != N / 2 && f2 > 0;
          const R m = keep ? scale / R(f2) * fa : R(0);
          val = V{-d.y * m, d.x * m};
        }
        u[k][s] = val;
      }
    }
    E::run(u, lds, s_tw, t);
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
      if (ok[k]) {
#pragma unroll
        for (int s = 0; s < E::R0; ++s)
          st_stream(out + a * S::HSLOT + ((size_t)(jj[k] + s * M) * N + y) * HZ + zz[k], u[k][s]);
      }
  }
}

// ---------------------------------------------------------------------------------------------
// Fused forward-x / inverse-x pass of a second-order source: reads the (z-forward, y-forward)
// transformed source from a half slot and completes the forward transform along x.  Gradient
// form (HESS false, the 2LPT displacement): multiplies by i * scale * M / f^2 and runs the two
// inverse x transforms of fx^a (a = 0, 1).  Hessian form (HESS true, the second-order tensor of
// the third-order displacement): multiplies by scale * M / f^2 and runs the three inverse x
// transforms of fx^a (a = 0, 1, 2), the outputs of the Hessian x pass.  Outputs: half slots.
template <typename R, int N, bool HESS>
__global__ void __launch_bounds__((Strided<R, N, +1>::T))
k_xpass_fwdinv(const typename Cplx<R>::type* __restrict__ in, typename Cplx<R>::type* __restrict__ out,
               const typename Cplx<R>::type* __restrict__ tw, R scale) {
  using S = Strided<R, N, +1>;
  using V = typename S::V;
  using E = typename S::E;
  using EF = Engine<V, N, S::PS, 1, true, S::T, -1>;
  constexpr int PS = S::PS, HZ = S::HZ, M = N / E::R0;
  __shared__ V lds[E::LDS_ELEMS];
  __shared__ V s_tw[tw_elems(N)];
  const int t = threadIdx.x;
  load_twiddles<N, S::T>(s_tw, tw, t);
  const int bt = xcd_tile(blockIdx.x, S::GRID);
  const int zt = bt % S::NZT;
  const int y = bt / S::NZT;
  const int fy = ifreq(y, N);
  V v[E::K0][E::R0];
  int zz[E::K0], jj[E::K0];
  bool ok[E::K0];
#pragma unroll
  for (int k = 0; k < E::K0; ++k) {
    int q, p, j;
    E::first_layout(t, k, q, p, j, ok[k]);
    const int z = zt * PS + p;
    ok[k] = ok[k] && z < HZ;
    zz[k] = z;
    jj[k] = j;
#pragma unroll
    for (int s = 0; s < E::R0; ++s)
      v[k][s] = ok[k] ? in[((size_t)(j + s * M) * N + y) * HZ + z] : V{R(0), R(0)};
  }
  EF::run(v, lds, s_tw, t);
#pragma unroll
  for (int k = 0; k < E::K0; ++k)
#pragma unroll
    for (int s = 0; s < E::R0; ++s) {
      const int n = jj[k] + s * M;
      const int fx = ifreq(n, N);
      const R f2 = R(fx * fx + fy * fy + zz[k] * zz[k]);
      const bool keep = ok[k] && n != N / 2 && y != N / 2 && f2 > R(0);
      const R m = keep ? scale / f2 : R(0);
      const V d = v[k][s];
      v[k][s] = HESS ? V{d.x * m, d.y * m} : V{-d.y * m, d.x * m};
    }
#pragma unroll 1
  for (int a = 0; a < (HESS ? 3 : 2); ++a) {
    V u[E::K0][E::R0];
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
#pragma unroll
      for (int s = 0; s < E::R0; ++s) u[k][s] = cscale(v[k][s], powf_int(R(ifreq(jj[k] + s * M, N)), a));
    E::run(u, lds, s_tw, t);
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
      if (ok[k]) {
#pragma unroll
        for (int s = 0; s < E::R0; ++s)
          st_stream(out + a * S::HSLOT + ((size_t)(jj[k] + s * M) * N + y) * HZ + zz[k], u[k][s]);
      }
  }
}

// ---------------------------------------------------------------------------------------------
// Fused forward-x / inverse-x pass of the third-order displacement: four half slots in, the
// (z-forward, y-forward) transforms of the divergence source s and of the transverse source
// c = (cx, cy, cz); forward transforms along x; per mode
//     psi_a = i scale M / f^2 (-f_a S + f_b C_d - f_d C_b),   (a, b, d) cyclic,
// and the three inverse x transforms of psi_a into half slots (the y and z passes finish them).
template <typename R, int N>
__global__ void __launch_bounds__((Strided<R, N, +1>::T))
k_xpass_lpt3(const typename Cplx<R>::type* __restrict__ in, typename Cplx<R>::type* __restrict__ out,
             const typename Cplx<R>::type* __restrict__ tw, R scale) {
  using S = Strided<R, N, +1>;
  using V = typename S::V;
  using E = typename S::E;
  using EF = Engine<V, N, S::PS, 1, true, S::T, -1>;
  constexpr int PS = S::PS, HZ = S::HZ, M = N / E::R0;
  __shared__ V lds[E::LDS_ELEMS];
  __shared__ V s_tw[tw_elems(N)];
  const int t = threadIdx.x;
  load_twiddles<N, S::T>(s_tw, tw, t);
  const int bt = xcd_tile(blockIdx.x, S::GRID);
  const int zt = bt % S::NZT;
  const int y = bt / S::NZT;
  const R fy = R(ifreq(y, N));
  V v[4][E::K0][E::R0];
  int zz[E::K0], jj[E::K0];
  bool ok[E::K0];
#pragma unroll
  for (int k = 0; k < E::K0; ++k) {
    int q, p, j;
    E::first_layout(t, k, q, p, j, ok[k]);
    const int z = zt * PS + p;
    ok[k] = ok[k] && z < HZ;
    zz[k] = z;
    jj[k] = j;
  }
  // each source is loaded just before its forward transform (all four in flight at once would
  // exceed the register budget of a 1024-thread workgroup)
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
#pragma unroll
      for (int s = 0; s < E::R0; ++s)
        v[c][k][s] = ok[k] ? in[c * S::HSLOT + ((size_t)(jj[k] + s * M) * N + y) * HZ + zz[k]] : V{R(0), R(0)};
    EF::run(v[c], lds, s_tw, t);
  }
  // psi3 components in place of (S, cx, cy), element by element
#pragma unroll
  for (int k = 0; k < E::K0; ++k)
#pragma unroll
    for (int s = 0; s < E::R0; ++s) {
      const int n = jj[k] + s * M;
      const R fx = R(ifreq(n, N)), fz = R(zz[k]);
      const R f2 = fx * fx + fy * fy + fz * fz;
      const bool keep = ok[k] && n != N / 2 && y != N / 2 && f2 > R(0);
      const R m = keep ? scale / f2 : R(0);
      const V sk = v[0][k][s], cx = v[1][k][s], cy = v[2][k][s], cz = v[3][k][s];
      // i m (-f_a S + f_b c_d - f_d c_b): w = the bracket, then times i m
      const V wx = V{fy * cz.x - fz * cy.x - fx * sk.x, fy * cz.y - fz * cy.y - fx * sk.y};
      const V wy = V{fz * cx.x - fx * cz.x - fy * sk.x, fz * cx.y - fx * cz.y - fy * sk.y};
      const V wz = V{fx * cy.x - fy * cx.x - fz * sk.x, fx * cy.y - fy * cx.y - fz * sk.y};
      v[0][k][s] = V{-wx.y * m, wx.x * m};
      v[1][k][s] = V{-wy.y * m, wy.x * m};
      v[2][k][s] = V{-wz.y * m, wz.x * m};
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    E::run(v[a], lds, s_tw, t);
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
      if (ok[k]) {
#pragma unroll
        for (int s = 0; s < E::R0; ++s)
          st_stream(out + a * S::HSLOT + ((size_t)(jj[k] + s * M) * N + y) * HZ + zz[k], v[a][k][s]);
      }
  }
}

// ---------------------------------------------------------------------------------------------
// y pass, packed output.  Packed component c of the recipe is (a, b, cz): input half slot a,
// fy^b before the transform, fz^cz after it; components (2q, 2q+1) go to packed slot q as
// C = A + iB.  The Hessian pairs are ordered so that each pair reads as few inputs as possible
// (pair 0 reads X_1 only, pair 1 X_0 only), which lets X_2 be fetched while pair 1 runs:
//   Hessian (RECIPE 0), packed order xy xz | yy yz | xx zz:
//       (1,1,0) (1,0,1) | (0,2,0) (0,1,1) | (2,0,0) (0,0,2)
//   gradient (RECIPE 1), packed order x y | z:  (1,0,0) (0,1,0) | (0,0,1)
//   gradient of the Hessian's x-pass outputs (RECIPE 3, v_max): RECIPE 1's components times i,
//       which the gradient x pass applies itself but the Hessian x pass does not (TI)
//   three finished components (RECIPE 4, the third-order displacement), packed order x y | z:
//       (0,0,0) (1,0,0) | (2,0,0)
//   Hessian and v_max gradient in one pass (RECIPE 5): RECIPE 0's pairs, then RECIPE 3's into a
//       second output (pairs from SPLIT on), so the Hessian x-pass outputs are read once
// The z pass maps the packed order back to (xx, xy, xz, yy, yz, zz) and (x, y, z).
// STREAM: the last transform that reads an input tile streams it (its lines need not stay in L2).
template <int RECIPE> struct YRecipe;
template <> struct YRecipe<0> {
  static constexpr bool STREAM = true;
  static constexpr int NIN = 3, NC = 6, Q = 3, SPLIT = 0;
  static constexpr int A[6] = {1, 1, 0, 0, 2, 0}, B[6] = {1, 0, 2, 1, 0, 0}, C[6] = {0, 1, 0, 1, 0, 2};
  static constexpr bool ti(int) { return false; }
};
template <> struct YRecipe<1> {
  static constexpr bool STREAM = false;
  static constexpr int NIN = 2, NC = 3, Q = 2, SPLIT = 0;
  static constexpr int A[3] = {1, 0, 0}, B[3] = {0, 1, 0}, C[3] = {0, 0, 1};
  static constexpr bool ti(int) { return false; }
};
template <> struct YRecipe<3> : YRecipe<1> {
  static constexpr bool ti(int) { return true; }
};
template <> struct YRecipe<4> {
  static constexpr bool STREAM = true;
  static constexpr int NIN = 3, NC = 3, Q = 2, SPLIT = 0;
  static constexpr int A[3] = {0, 1, 2}, B[3] = {0, 0, 0}, C[3] = {0, 0, 0};
  static constexpr bool ti(int) { return false; }
};
template <> struct YRecipe<5> {
  static constexpr bool STREAM = true;
  static constexpr int NIN = 3, NC = 9, Q = 5, SPLIT = 3;
  static constexpr int A[9] = {1, 1, 0, 0, 2, 0, 1, 0, 0}, B[9] = {1, 0, 2, 1, 0, 0, 0, 1, 0},
                       C[9] = {0, 1, 0, 1, 0, 2, 0, 0, 1};
  static constexpr bool ti(int c) { return c >= 6; }
};

// Pair of the last transform that reads input slot `a` under recipe RC.
template <class RC> constexpr int last_pair(int a) {
  int q = -1;
  for (int c = 0; c < RC::NC; ++c)
    if (RC::A[c] == a) q = c / 2;
  return q;
}

template <typename R, int N, int RECIPE>
__global__ void __launch_bounds__((Strided<R, N, +1>::T))
__attribute__((amdgpu_waves_per_eu(Strided<R, N, +1>::WPE, Strided<R, N, +1>::WPE)))
k_ypass_packed(const typename Cplx<R>::type* __restrict__ in, typename Cplx<R>::type* __restrict__ out,
               const typename Cplx<R>::type* __restrict__ tw, typename Cplx<R>::type* __restrict__ out2) {
  using S = Strided<R, N, +1>;
  using RC = YRecipe<RECIPE>;
  using V = typename S::V;
  using E = typename S::E;
  constexpr int PS = S::PS, HZ = S::HZ, M = N / E::R0;
  constexpr size_t PSLOT = (size_t)N * N * N;
  __shared__ V lds[E::LDS_ELEMS];
  __shared__ V s_tw[tw_elems(N)];
  const int t = threadIdx.x;
  load_twiddles<N, S::T>(s_tw, tw, t);
  const int bt = xcd_tile(blockIdx.x, S::GRID);
  const int zt = bt % S::NZT;
  const int x = bt / S::NZT;
  int zz[E::K0], jj[E::K0];
  bool ok[E::K0];
#pragma unroll
  for (int k = 0; k < E::K0; ++k) {
    int q, p, j;
    E::first_layout(t, k, q, p, j, ok[k]);
    const int z = zt * PS + p;
    ok[k] = ok[k] && z < HZ;
    zz[k] = z;
    jj[k] = j;
  }
  // One transform per (pair, sign): u = fy^bA fz^cA X_aA + sgn i fy^bB fz^cB X_aB.  By
  // linearity sgn = +1 gives C[kz] = A + iB and sgn = -1 gives conj(C[N - kz]) = A - iB.  Each
  // transform reads its inputs itself (L2 hits after the first read of a tile) so that only one
  // transform's data is live and two workgroups fit on a CU; the outputs are streamed past L2.
#pragma unroll
  for (int q = 0; q < RC::Q; ++q) {
    const int ca = 2 * q, cb = 2 * q + 1;
    const bool has_b = cb < RC::NC;
    const int aa = RC::A[ca];
    const int ab = RC::A[has_b ? cb : ca];
    V* dst = (RC::SPLIT > 0 && q >= RC::SPLIT) ? out2 + (size_t)(q - RC::SPLIT) * PSLOT : out + (size_t)q * PSLOT;
#pragma unroll
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      if (!has_b && sgn < 0) break;   // B = 0: C[N - kz] = conj(C[kz]), written below
      // opaque copies of the indices: the compiler would otherwise compute every transform's
      // multipliers and addresses up front and keep them live across all of them
      int jv[E::K0], zv[E::K0];
#pragma unroll
      for (int k = 0; k < E::K0; ++k) {
        jv[k] = jj[k];
        zv[k] = zz[k];
        asm volatile("" : "+v"(jv[k]), "+v"(zv[k])::"memory");
      }
      V u[E::K0][E::R0];
#pragma unroll
      for (int k = 0; k < E::K0; ++k) {
        const R fz = R(zv[k]);
#pragma unroll
        for (int s = 0; s < E::R0; ++s) {
          const R fy = R(ifreq(jv[k] + s * M, N));
          const size_t ubase = ((size_t)x * N + s * M) * HZ;   // uniform part of the address
          const unsigned off = (unsigned)(jv[k] * HZ + zv[k]);
          // the last transform that reads a tile streams it (Hessian: X_1 after pair 0, X_0 and
          // X_2 after pair 2)
          const bool final_sgn = sgn < 0 || !has_b;
          const bool last_a = RC::STREAM && final_sgn && q == last_pair<RC>(aa);
          const bool last_b = RC::STREAM && final_sgn && q == last_pair<RC>(ab);
          const V* pa = in + aa * S::HSLOT + ubase + off;
          const V xa = ok[k] ? (last_a ? ld_stream(pa) : *pa) : V{R(0), R(0)};
          V ta = cscale(xa, powf_int(fy, RC::B[ca]) * powf_int(fz, RC::C[ca]));
          if (RC::ti(ca)) ta = V{-ta.y, ta.x};
          if (has_b) {
            const V* pb = in + ab * S::HSLOT + ubase + off;
            const V xb = ab == aa ? xa : (ok[k] ? (last_b ? ld_stream(pb) : *pb) : V{R(0), R(0)});
            V tb = cscale(xb, powf_int(fy, RC::B[has_b ? cb : ca]) * powf_int(fz, RC::C[has_b ? cb : ca]));
            if (RC::ti(cb)) tb = V{-tb.y, tb.x};
            u[k][s] = sgn > 0 ? V{ta.x - tb.y, ta.y + tb.x} : V{ta.x + tb.y, ta.y - tb.x};
          } else {
            u[k][s] = ta;
          }
        }
      }
      E::run(u, lds, s_tw, t);
#pragma unroll
      for (int k = 0; k < E::K0; ++k)
        if (ok[k]) {
#pragma unroll
          for (int s = 0; s < E::R0; ++s) {
            // x-plane base (uniform) + 32-bit byte offsets within the plane
            using L = PackedLayout<R, N>;
            char* plane = reinterpret_cast<char*>(dst + (size_t)x * N * N);
            V* first = reinterpret_cast<V*>(plane + (unsigned)L::index(0, jv[k] + s * M, zv[k]) * (unsigned)sizeof(V));
            V* second =
                reinterpret_cast<V*>(plane + (unsigned)L::index(0, jv[k] + s * M, zv[k] + HZ) * (unsigned)sizeof(V));
            if (sgn > 0) {
              st_stream(first, u[k][s]);
              if (!has_b && zv[k] > 0) st_stream(second, conj(u[k][s]));
            } else if (zv[k] > 0) {
              st_stream(second, conj(u[k][s]));
            }
          }
        }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Forward y pass of the 2LPT source: half slot -> half slot, no multiplier.
template <typename R, int N>
__global__ void __launch_bounds__((Strided<R, N, -1>::T))
k_ypass_fwd(const typename Cplx<R>::type* __restrict__ in, typename Cplx<R>::type* __restrict__ out,
            const typename Cplx<R>::type* __restrict__ tw) {
  using S = Strided<R, N, -1>;
  using V = typename S::V;
  using E = typename S::E;
  constexpr int PS = S::PS, HZ = S::HZ, M = N / E::R0;
  __shared__ V lds[E::LDS_ELEMS];
  __shared__ V s_tw[tw_elems(N)];
  const int t = threadIdx.x;
  load_twiddles<N, S::T>(s_tw, tw, t);
  const int bt = xcd_tile(blockIdx.x, S::GRID);
  const int zt = bt % S::NZT;
  const int x = bt / S::NZT;
  V v[E::K0][E::R0];
  int zz[E::K0], jj[E::K0];
  bool ok[E::K0];
#pragma unroll
  for (int k = 0; k < E::K0; ++k) {
    int q, p, j;
    E::first_layout(t, k, q, p, j, ok[k]);
    const int z = zt * PS + p;
    ok[k] = ok[k] && z < HZ;
    zz[k] = z;
    jj[k] = j;
#pragma unroll
    for (int s = 0; s < E::R0; ++s)
      v[k][s] = ok[k] ? in[((size_t)x * N + j + s * M) * HZ + z] : V{R(0), R(0)};
  }
  E::run(v, lds, s_tw, t);
#pragma unroll
  for (int k = 0; k < E::K0; ++k)
    if (ok[k]) {
#pragma unroll
      for (int s = 0; s < E::R0; ++s) st_stream(out + ((size_t)x * N + jj[k] + s * M) * HZ + zz[k], v[k][s]);
    }
}

// ---------------------------------------------------------------------------------------------
// z pass: inverse transform along z of Q packed slots (two real components each) and the
// per-point epilogue.
enum ZEpi { EPI_COLLAPSE = 0, EPI_STORE = 1, EPI_MU2 = 2, EPI_COLLAPSE_V = 3, EPI_LPT3 = 4 };

template <typename R, int N, int Q, int EPI>
struct ZPass {
  using V = typename Cplx<R>::type;
  using ZT = ZTile<R, N, Q>;
  static constexpr int P = ZT::P;
  static constexpr int T = ZT::T;
  static constexpr int HZ = N / 2;
  using E = Engine<V, N, P, ZT::QL, false, T, +1>;
  static constexpr int LINES = N * N;
  static constexpr int GRID = (LINES + P - 1) / P;
  static_assert(E::K0 == ZT::QL, "z pass: one butterfly per transform per thread");
};

struct ZArgs {
  void* F;          // EPI_COLLAPSE: running F_max (R)
  uint8_t* ridx;    // EPI_COLLAPSE: running radius index
  int r;            // EPI_COLLAPSE: radius index of this launch
  int nc;           // EPI_STORE: number of real components to store (<= 2Q)
  void* out;        // EPI_STORE: [nc][N^3] real; EPI_MU2: one half slot (complex)
  CollapseConst cc;
  const void* gin;  // EPI_COLLAPSE_V: the two packed gradient slots (y-pass recipe 3)
  void* vout;       // EPI_COLLAPSE_V: v_max [3][N^3] (R)
  double vscale;    // EPI_COLLAPSE_V: L / 2 pi
  void* t6;         // EPI_MU2: when not null, the six components are stored to t6[6][N^3] (R);
                    // EPI_LPT3: the first-order tensor T1 [6][N^3] read at each point
};

// Sources of the third-order displacement at one point from the first-order tensor a and the
// second-order tensor b (xx, xy, xz, yy, yz, zz): the divergence
//     sl = det(a) / 3 - (10/21) ((tr a)(tr b) - tr(a b)) / 2
// and the curl c_i = eps_ijk (a b)_jk / 7.
template <typename R>
__device__ __forceinline__ void lpt3_sources(const R (&a)[6], const R (&b)[6], R& sl, R& cx, R& cy, R& cz) {
  const R axx = a[0], axy = a[1], axz = a[2], ayy = a[3], ayz = a[4], azz = a[5];
  const R bxx = b[0], bxy = b[1], bxz = b[2], byy = b[3], byz = b[4], bzz = b[5];
  const R det = axx * (ayy * azz - ayz * ayz) - axy * (axy * azz - ayz * axz) + axz * (axy * ayz - ayy * axz);
  const R trab = axx * bxx + ayy * byy + azz * bzz + R(2) * (axy * bxy + axz * bxz + ayz * byz);
  const R mixed = R(0.5) * ((axx + ayy + azz) * (bxx + byy + bzz) - trab);
  sl = det * R(1.0 / 3.0) - mixed * R(10.0 / 21.0);
  cx = (axy * bxz + ayy * byz + ayz * bzz - axz * bxy - ayz * byy - azz * byz) * R(1.0 / 7.0);
  cy = (axz * bxx + ayz * bxy + azz * bxz - axx * bxz - axy * byz - axz * bzz) * R(1.0 / 7.0);
  cz = (axx * bxy + axy * byy + axz * byz - axy * bxx - ayy * bxy - ayz * bxz) * R(1.0 / 7.0);
}

template <typename R, int N, int Q, int EPI>
__global__ void __launch_bounds__((ZPass<R, N, Q, EPI>::T))
k_zpass(const typename Cplx<R>::type* __restrict__ in, const typename Cplx<R>::type* __restrict__ tw, ZArgs args) {
  using Z = ZPass<R, N, Q, EPI>;
  using V = typename Z::V;
  using E = typename Z::E;
  constexpr int P = Z::P, HZ = Z::HZ, R0 = E::R0, M0 = N / R0;
  constexpr size_t PSLOT = (size_t)N * N * N;
  __shared__ V lds[E::LDS_ELEMS];
  __shared__ V s_tw[tw_elems(N)];
  const int t = threadIdx.x;
  load_twiddles<N, Z::T>(s_tw, tw, t);
  // thread t owns pencil position (p, j) of every transform q
  const int j = t % M0;
  const int p = t / M0;
  const int line = blockIdx.x * P + p;
  const bool line_ok = line < Z::LINES;
  V v[Q][R0];
  // collapse epilogue: the running maximum of this thread's points, fetched with the inputs so
  // that its latency hides behind the transforms
  R fold[R0];
  if constexpr (EPI == EPI_COLLAPSE || EPI == EPI_COLLAPSE_V) {
    const R* F = static_cast<const R*>(args.F);
#pragma unroll
    for (int s = 0; s < R0; ++s) fold[s] = F[(size_t)(line_ok ? line : Z::LINES - 1) * N + j + s * M0];
  }
  // Packed storage of C[n]: P[n] for n < N/2, P[3N/2 - n] for n > N/2; R0 is even, so elements
  // s < R0/2 are the first kind and s >= R0/2 the second.  Loads are unconditional (a wave past
  // the last line reads the last line and stores nothing); the Nyquist element n = N/2 (lane
  // j = 0, s = R0/2) reads P[N/2], which is never written, and is replaced by zero.
  static_assert(R0 % 2 == 0 && M0 * (R0 / 2) == HZ, "z pass: the first half of the elements is n < N/2");
  const int lineL = line_ok ? line : Z::LINES - 1;
  using L = PackedLayout<R, N>;
  static_assert(L::M0 == M0, "z pass: the packed layout's element stride");
  // Offsets of element j + s M0, of the Nyquist slot and of element 3N/2 - j - s M0 =
  // (3N/2 - j) - s M0, the same for every slot.  The workgroup's lines share one x-plane when P
  // divides N: the plane's base is then uniform and the offsets within it (bytes) fit 32 bits,
  // so each load adds one 32-bit offset to a scalar base.
  const int ly = lineL % N;
  constexpr bool PLANE = N % P == 0;
  const int lx = PLANE ? (int)(blockIdx.x * P / N) : lineL / N;
  const size_t plane = (size_t)lx * N * N;
  const unsigned o_lo = (unsigned)L::index(0, ly, j) * (unsigned)sizeof(V);
  const unsigned o_ny = (unsigned)L::index(0, ly, j == 0 ? HZ : N - j) * (unsigned)sizeof(V);
  const unsigned o_hi = (unsigned)L::index(0, ly, 3 * HZ - j) * (unsigned)sizeof(V);
  constexpr unsigned STEPB = (unsigned)(L::STEP * sizeof(V));
  static_assert((size_t)3 * N * N * sizeof(V) < ((size_t)1 << 32), "z pass: plane offsets must fit 32 bits");
  auto load_line = [&](const V* slot, V(&dst)[R0]) {
    const char* base = reinterpret_cast<const char*>(slot + plane);
#pragma unroll
    for (int s = 0; s < R0 / 2; ++s) dst[s] = *reinterpret_cast<const V*>(base + (o_lo + s * STEPB));
    {
      const V x = *reinterpret_cast<const V*>(base + o_ny);
      dst[R0 / 2] = j == 0 ? V{R(0), R(0)} : x;
    }
#pragma unroll
    for (int s = R0 / 2 + 1; s < R0; ++s) dst[s] = *reinterpret_cast<const V*>(base + (o_hi - s * STEPB));
  };
#pragma unroll
  for (int q = 0; q < Q; ++q) load_line(in + (size_t)q * PSLOT, v[q]);
  if constexpr (Z::ZT::QL == Q) {
    E::run(v, lds, s_tw, t);
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q) E::run(*reinterpret_cast<V(*)[1][R0]>(&v[q]), lds, s_tw, t);
  }
  // v[q][s] = (packed component 2q) + i (packed component 2q+1) at n = j + s*M0 of line `line`;
  // comp(c, s) is the canonical component c (Hessian xx xy xz yy yz zz; gradient x y z).
  auto comp = [&](int c, int s) -> R {
    if constexpr (Q == 3) {
      return c == 0 ? v[2][s].x : c == 1 ? v[0][s].x : c == 2 ? v[0][s].y : c == 3 ? v[1][s].x
                                                                 : c == 4 ? v[1][s].y : v[2][s].y;
    } else {
      return c == 0 ? v[0][s].x : c == 1 ? v[0][s].y : v[1][s].x;
    }
  };
  if constexpr (EPI == EPI_COLLAPSE || EPI == EPI_COLLAPSE_V) {
    static_assert(Q == 3, "collapse needs the six components");
    R* F = static_cast<R*>(args.F);
    bool upd[R0];
#pragma unroll
    for (int s = 0; s < R0; ++s) {
      const size_t idx = (size_t)line * N + j + s * M0;
      R fr;
      if constexpr (sizeof(R) == 4) {
        fr = collapse_point_mixed(comp(0, s), comp(1, s), comp(2, s), comp(3, s), comp(4, s), comp(5, s),
                                  (float)args.cc.sphere_gain);
      } else {
        fr = (R)collapse_point(comp(0, s), comp(1, s), comp(2, s), comp(3, s), comp(4, s), comp(5, s), args.cc);
      }
      upd[s] = line_ok && fr > fold[s];
      if (upd[s]) {
        // streamed: read again only at the next radius, after the x and y passes
        __builtin_nontemporal_store(fr, &F[idx]);
        __builtin_nontemporal_store((uint8_t)args.r, &args.ridx[idx]);
      }
    }
    if constexpr (EPI == EPI_COLLAPSE_V) {
      // v_max: the smoothed gradient at this radius, transformed only now (the Hessian data is
      // dead) and stored where F_max grew
      const V* gin = static_cast<const V*>(args.gin);
      V g[2][R0];
      load_line(gin, g[0]);
      load_line(gin + PSLOT, g[1]);
#pragma unroll
      for (int q = 0; q < 2; ++q) E::run(*reinterpret_cast<V(*)[1][R0]>(&g[q]), lds, s_tw, t);
      R* vout = static_cast<R*>(args.vout);
      constexpr size_t VOL = (size_t)N * N * N;
      const R vs = (R)args.vscale;
#pragma unroll
      for (int s = 0; s < R0; ++s) {
        if (upd[s]) {
          const size_t idx = (size_t)line * N + j + s * M0;
          __builtin_nontemporal_store(g[0][s].x * vs, &vout[idx]);
          __builtin_nontemporal_store(g[0][s].y * vs, &vout[VOL + idx]);
          __builtin_nontemporal_store(g[1][s].x * vs, &vout[2 * VOL + idx]);
        }
      }
    }
  } else if constexpr (EPI == EPI_STORE) {
    R* out = static_cast<R*>(args.out);
    constexpr size_t VOL = (size_t)N * N * N;
    if (line_ok) {
#pragma unroll
      for (int s = 0; s < R0; ++s) {
        const size_t idx = (size_t)line * N + j + s * M0;
#pragma unroll
        for (int c = 0; c < 2 * Q; ++c)
          if (c < args.nc) __builtin_nontemporal_store(comp(c, s), &out[(size_t)c * VOL + idx]);
      }
    }
  } else if constexpr (EPI == EPI_LPT3) {
    static_assert(Q == 3, "third-order sources need the six components of T2");
    // sources of the third-order displacement at each point from T2 (this pass) and T1 (read),
    // packed (sl + i cx), (cy + i cz) and transformed forward along z; the two real spectra of
    // each packed line are separated and written to four half slots (sl, cx, cy, cz)
    using EF = Engine<V, N, P, 1, false, Z::T, -1>;
    static_assert(EF::K0 == 1 && EF::LDS_ELEMS <= E::LDS_ELEMS, "forward z tile: the inverse one's layout");
    const R* t1 = static_cast<const R*>(args.t6);
    constexpr size_t VOL = (size_t)N * N * N;
    V w[2][R0];
#pragma unroll
    for (int s = 0; s < R0; ++s) {
      const size_t idx = (size_t)lineL * N + j + s * M0;
      R a6[6], b6[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        a6[c] = t1[c * VOL + idx];
        b6[c] = comp(c, s);
      }
      R sl, cx, cy, cz;
      lpt3_sources(a6, b6, sl, cx, cy, cz);
      w[0][s] = V{sl, cx};
      w[1][s] = V{cy, cz};
    }
    V* out = static_cast<V*>(args.out);
    constexpr size_t HSLOT = (size_t)N * N * HZ;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      EF::run(*reinterpret_cast<V(*)[1][R0]>(&w[q]), lds, s_tw, t);
#pragma unroll
      for (int s = 0; s < R0; ++s) lds[EF::lds_index(0, p, j + s * M0)] = w[q][s];
      __syncthreads();
#pragma unroll
      for (int s = 0; s < R0 / 2; ++s) {
        const int k = j + s * M0;
        const V zk = lds[EF::lds_index(0, p, k)];
        const V zn = lds[EF::lds_index(0, p, (N - k) % N)];
        const V A = V{R(0.5) * (zk.x + zn.x), R(0.5) * (zk.y - zn.y)};   // (Z_k + conj Z_{N-k})/2
        const V B = V{R(0.5) * (zk.y + zn.y), R(0.5) * (zn.x - zk.x)};   // (Z_k - conj Z_{N-k})/(2i)
        if (line_ok) {
          out[(size_t)(2 * q) * HSLOT + (size_t)line * HZ + k] = A;
          out[(size_t)(2 * q + 1) * HSLOT + (size_t)line * HZ + k] = B;
        }
      }
      __syncthreads();
    }
  } else {
    static_assert(EPI == EPI_MU2 && Q == 3, "2LPT source needs the six components");
    // mu2 at each point, then a forward real-to-complex transform along z of line pairs
    // (2u, 2u+1) packed as one complex line, written to a half slot.
    using EF = Engine<V, N, P / 2, 1, false, Z::T, -1>;
    static_assert(EF::LDS_ELEMS <= E::LDS_ELEMS, "forward z tile fits the LDS of the inverse one");
#pragma unroll
    for (int s = 0; s < R0; ++s) {
      const int n = j + s * M0;
      const R xx = comp(0, s), xy = comp(1, s), xz = comp(2, s), yy = comp(3, s), yz = comp(4, s), zz = comp(5, s);
      const R mu2 = line_ok ? (xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz) : R(0);
      if (args.t6 != nullptr && line_ok) {
        R* t6 = static_cast<R*>(args.t6);
        constexpr size_t VOL = (size_t)N * N * N;
        const size_t idx = (size_t)line * N + n;
        t6[idx] = xx;
        t6[VOL + idx] = xy;
        t6[2 * VOL + idx] = xz;
        t6[3 * VOL + idx] = yy;
        t6[4 * VOL + idx] = yz;
        t6[5 * VOL + idx] = zz;
      }
      reinterpret_cast<R*>(&lds[EF::lds_index(0, p >> 1, n)])[p & 1] = mu2;
    }
    __syncthreads();
    static_assert(EF::K0 == 1, "forward z: one butterfly per thread");
    V w[1][R0];
    {
      int q2, p2, j2;
      bool ok2;
      EF::first_layout(t, 0, q2, p2, j2, ok2);
#pragma unroll
      for (int s = 0; s < R0; ++s) w[0][s] = ok2 ? lds[EF::lds_index(0, p2, j2 + s * M0)] : V{R(0), R(0)};
      __syncthreads();
      EF::run(w, lds, s_tw, t);
      if (ok2) {
#pragma unroll
        for (int s = 0; s < R0; ++s) lds[EF::lds_index(0, p2, j2 + s * M0)] = w[0][s];
      }
    }
    __syncthreads();
    V* out = static_cast<V*>(args.out);
    constexpr int NOUT = (P / 2) * HZ;
    for (int o = t; o < NOUT; o += Z::T) {
      const int u = o / HZ, k = o % HZ;
      const V zk = lds[EF::lds_index(0, u, k)];
      const V zn = lds[EF::lds_index(0, u, (N - k) % N)];
      const V a = V{R(0.5) * (zk.x + zn.x), R(0.5) * (zk.y - zn.y)};   // (Z_k + conj Z_{N-k})/2
      const V b = V{R(0.5) * (zk.y + zn.y), R(0.5) * (zn.x - zk.x)};   // (Z_k - conj Z_{N-k})/(2i)
      const int l0 = blockIdx.x * P + 2 * u;
      if (l0 < Z::LINES) st_stream(out + (size_t)l0 * HZ + k, a);
      if (l0 + 1 < Z::LINES) st_stream(out + (size_t)(l0 + 1) * HZ + k, b);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Per-point collapse model on caller-given tensors T6 [6][count] (xx, xy, xz, yy, yz, zz): the
// same device functions as the z pass epilogue.
template <typename R>
__global__ void k_collapse_points(const R* __restrict__ t6, size_t count, R* __restrict__ F, CollapseConst cc) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const R xx = t6[i], xy = t6[count + i], xz = t6[2 * count + i];
  const R yy = t6[3 * count + i], yz = t6[4 * count + i], zz = t6[5 * count + i];
  if constexpr (sizeof(R) == 4) {
    F[i] = collapse_point_mixed(xx, xy, xz, yy, yz, zz, (float)cc.sphere_gain);
  } else {
    F[i] = collapse_point(xx, xy, xz, yy, yz, zz, cc);
  }
}

// ---------------------------------------------------------------------------------------------
// Running-maximum reset: F = 0, ridx = 255.
template <typename R>
__global__ void k_reset(R* __restrict__ F, uint8_t* __restrict__ ridx, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    F[i] = R(0);
    ridx[i] = 255;
  }
}

// ---------------------------------------------------------------------------------------------
// Collapse redshift: z_c with D(z_c) = 1/F, D the growing mode normalised to 1 at z = 0,
// tabulated (float64) on y = ln a at m nodes y0 + i h with D and dD/dy.  The interval holding
// 1/F is found by bisection on the monotone D, then y by Newton steps on the cubic Hermite
// interpolant of D(y) there.  Below the first node D = a (1 - (2/11)(Lambda/Om) a^3 + ...) / a_per_D
// is inverted directly; F <= 0, or 1/F beyond the last node (a > 1e6), gives z_c = -1.
struct GrowthArgs {
  const double* d;
  const double* dd;
  int m;
  double y0, h, a_per_D, lambda_over_m;
  const int32_t* guide;   // last node with d <= 2^(l0 + b / inv), per bucket b < k
  int k;
  float l0, inv;
};

template <typename R>
__global__ void k_redshift(const R* __restrict__ F, size_t count, GrowthArgs g, R* __restrict__ z) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double f = (double)F[i];
  double out = -1.0;
  if (f > 0.0) {
    const double t = 1.0 / f;
    if (t < g.d[0]) {
      const double a0 = t * g.a_per_D;
      const double a = a0 * (1.0 + (2.0 / 11.0) * g.lambda_over_m * a0 * a0 * a0);
      out = 1.0 / a - 1.0;
    } else if (t < g.d[g.m - 1]) {
      // the bucket of t in log2 narrows the node search to a few steps; the bounds are checked
      // against t so that a bucket taken one off by rounding only widens the search
      int b = (int)((__log2f((float)t) - g.l0) * g.inv);
      b = min(max(b, 0), g.k - 2);
      int lo = g.guide[b], hi = min(g.guide[b + 1] + 1, g.m - 1);   // d[lo] <= t < d[hi]
      if (!(g.d[lo] <= t)) lo = 0;
      if (!(t < g.d[hi])) hi = g.m - 1;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (g.d[mid] <= t) lo = mid; else hi = mid;
      }
      const double d0 = g.d[lo], d1 = g.d[hi], m0 = g.dd[lo] * g.h, m1 = g.dd[hi] * g.h;
      // Newton on the cubic Hermite segment from the chord: the chord is within h/4 of the root
      // in s, and each step squares the error times about h, so three steps reach rounding
      double s = (t - d0) / (d1 - d0);
#pragma unroll
      for (int it = 0; it < 3; ++it) {
        const double s2 = s * s, s3 = s2 * s;
        const double hv = (2 * s3 - 3 * s2 + 1) * d0 + (s3 - 2 * s2 + s) * m0 + (-2 * s3 + 3 * s2) * d1 + (s3 - s2) * m1;
        const double hp = (6 * s2 - 6 * s) * d0 + (3 * s2 - 4 * s + 1) * m0 + (-6 * s2 + 6 * s) * d1 + (3 * s2 - 2 * s) * m1;
        s = fmin(1.0, fmax(0.0, s - (hv - t) / hp));
      }
      out = exp(-(g.y0 + (lo + s) * g.h)) - 1.0;
    }
  }
  z[i] = (R)out;
}

template <typename R>
__global__ void k_zero(R* __restrict__ p, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = R(0);
}

}  // namespace pin
