// HIP kernels of the collapse-time path for one grid size N and one precision.
//
// Layouts (C order, z fastest):
//   user half spectrum dk      [N][N][N/2+1]   complex
//   workspace slot             [N][N][N/2]     complex -- the kz = N/2 (Nyquist) plane is zero
//                                                         by construction and is not stored
//   real field                 [N][N][N]
//
// Inverse 3D transform of the six Hessian components with shared prefixes.  With
// g = M W dk / f^2 (M zeroes Nyquist modes, W the Gaussian window, f the integer wavevector),
// component (a, b, c) with a + b + c = 2 is the inverse transform of fx^a fy^b fz^c g, and the
// factors fx^a, fy^b commute with the later axes' transforms:
//   x pass:  X_a  = IFFT_x[fx^a g]                    a = 0, 1, 2       (1 -> 3 arrays)
//   y pass:  Y_ab = IFFT_y[fy^b X_a]                  (a, b) with a + b <= 2 (3 -> 6 arrays)
//   z pass:  T_abc = C2R_z[fz^c Y_ab]                 6 real values per point, in registers,
//            consumed by the per-point epilogue (collapse, store, or the 2LPT source).
// Gradients (displacements) use the same passes with a + b + c = 1 and g = i c M dk / f^2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "collapse_dev.hpp"
#include "fft_core.hpp"

namespace pin {

// ---------------------------------------------------------------------------------------------
// Tile shapes
template <typename R> struct Tile {
  using V = typename Cplx<R>::type;
  static constexpr int PS = 128 / (int)sizeof(V);   // strided passes: 128-byte rows of z
};

constexpr int round_up64(int x) { return (x + 63) / 64 * 64; }
constexpr int strided_threads(int nb0) { return round_up64(nb0 < 512 ? nb0 : 512); }
constexpr int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}
// z pass: P lines per workgroup so that T = P * N/R0 threads (<= 256) and Q*P*N*sizeof(V) of LDS
// stays within 96 KB.
template <typename R, int N, int Q> struct ZTile {
  using V = typename Cplx<R>::type;
  static constexpr int R0 = factorize(N).r[0];
  static constexpr int M0 = N / R0;
  static constexpr int P_by_threads = pow2_floor(256 / M0 > 0 ? 256 / M0 : 1);
  static constexpr int P_by_lds = pow2_floor((96 * 1024) / (Q * N * (int)sizeof(V)) > 0
                                                 ? (96 * 1024) / (Q * N * (int)sizeof(V)) : 1);
  static constexpr int P0 = P_by_threads < P_by_lds ? P_by_threads : P_by_lds;
  static constexpr int P = P0 < 2 ? 2 : P0;   // even: the 2LPT epilogue pairs lines
  static constexpr int T = P * M0;
};

__device__ __forceinline__ int ifreq(int i, int n) { return i < (n >> 1) ? i : i - n; }

template <typename R> __device__ __forceinline__ R powf_int(R f, int e) {
  return e == 0 ? R(1) : (e == 1 ? f : f * f);
}

// ---------------------------------------------------------------------------------------------
// x pass from the user half spectrum.  MODE 0 (Hessian): NA = 3 outputs, multiplier
// W(x)W(y)W(z) scale / f^2 (wtab may be null: no smoothing).  MODE 1 (gradient): NA = 2,
// multiplier i * scale / f^2.
template <typename R, int N, int MODE>
struct XPass {
  using V = typename Cplx<R>::type;
  static constexpr int PS = Tile<R>::PS;
  static constexpr int HZ = N / 2;
  static constexpr int NZT = (HZ + PS - 1) / PS;
  static constexpr int NA = MODE == 0 ? 3 : 2;
  using E0 = Engine<V, N, PS, 1, true, 64, +1>;
  static constexpr int T = strided_threads(E0::nb(E0::R0));
  using E = Engine<V, N, PS, 1, true, T, +1>;
  static constexpr int GRID = N * NZT;
};

template <typename R, int N, int MODE>
__global__ void __launch_bounds__((XPass<R, N, MODE>::T))
k_xpass(const typename Cplx<R>::type* __restrict__ in, typename Cplx<R>::type* __restrict__ out,
        const R* __restrict__ wtab, const typename Cplx<R>::type* __restrict__ tw, R scale) {
  using X = XPass<R, N, MODE>;
  using V = typename X::V;
  using E = typename X::E;
  constexpr int PS = X::PS, HZ = X::HZ, NH = N / 2 + 1;
  constexpr size_t SLOT = (size_t)N * N * HZ;
  __shared__ V lds[E::LDS_ELEMS];
  const int zt = blockIdx.x % X::NZT;
  const int y = blockIdx.x / X::NZT;
  const int t = threadIdx.x;
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
    for (int s = 0; s < E::R0; ++s) {
      const int n = j + s * (N / E::R0);
      V val = V{R(0), R(0)};
      if (ok[k] && n != N / 2 && y != N / 2) {
        const int fx = ifreq(n, N);
        const R f2 = R(fx * fx + fy * fy + z * z);
        if (f2 > R(0)) {
          R m = scale / f2;
          if (MODE == 0 && wtab != nullptr) m *= wtab[n] * wtab[y] * wtab[z];
          const V d = in[((size_t)n * N + y) * NH + z];
          val = MODE == 0 ? V{d.x * m, d.y * m} : V{-d.y * m, d.x * m};
        }
      }
      v[k][s] = val;
    }
  }
#pragma unroll 1
  for (int a = 0; a < X::NA; ++a) {
    V u[E::K0][E::R0];
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
#pragma unroll
      for (int s = 0; s < E::R0; ++s) {
        const int n = jj[k] + s * (N / E::R0);
        const R fx = R(ifreq(n, N));
        u[k][s] = cscale(v[k][s], powf_int(fx, a));
      }
    E::run(u, lds, tw, t);
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
      if (ok[k]) {
#pragma unroll
        for (int s = 0; s < E::R0; ++s) {
          const int n = jj[k] + s * (N / E::R0);
          out[a * SLOT + ((size_t)n * N + y) * HZ + zz[k]] = u[k][s];
        }
      }
  }
}

// ---------------------------------------------------------------------------------------------
// Fused forward-x / inverse-x pass of the 2LPT displacement: reads the (z-forward, y-forward)
// transformed source, completes the forward transform along x, multiplies by
// i * scale * M / f^2 and runs the two inverse x transforms of fx^a (a = 0, 1).
template <typename R, int N>
__global__ void __launch_bounds__((XPass<R, N, 1>::T))
k_xpass_fwdinv(const typename Cplx<R>::type* __restrict__ in, typename Cplx<R>::type* __restrict__ out,
               const typename Cplx<R>::type* __restrict__ tw, R scale) {
  using X = XPass<R, N, 1>;
  using V = typename X::V;
  using E = typename X::E;
  using EF = Engine<V, N, X::PS, 1, true, X::T, -1>;
  constexpr int PS = X::PS, HZ = X::HZ;
  constexpr size_t SLOT = (size_t)N * N * HZ;
  __shared__ V lds[E::LDS_ELEMS];
  const int zt = blockIdx.x % X::NZT;
  const int y = blockIdx.x / X::NZT;
  const int t = threadIdx.x;
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
    for (int s = 0; s < E::R0; ++s) {
      const int n = j + s * (N / E::R0);
      v[k][s] = ok[k] ? in[((size_t)n * N + y) * HZ + z] : V{R(0), R(0)};
    }
  }
  EF::run(v, lds, tw, t);
#pragma unroll
  for (int k = 0; k < E::K0; ++k)
#pragma unroll
    for (int s = 0; s < E::R0; ++s) {
      const int n = jj[k] + s * (N / E::R0);
      const int fx = ifreq(n, N);
      const R f2 = R(fx * fx + fy * fy + zz[k] * zz[k]);
      const bool keep = ok[k] && n != N / 2 && y != N / 2 && f2 > R(0);
      const R m = keep ? scale / f2 : R(0);
      const V d = v[k][s];
      v[k][s] = V{-d.y * m, d.x * m};
    }
#pragma unroll 1
  for (int a = 0; a < 2; ++a) {
    V u[E::K0][E::R0];
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
#pragma unroll
      for (int s = 0; s < E::R0; ++s) {
        const int n = jj[k] + s * (N / E::R0);
        u[k][s] = cscale(v[k][s], powf_int(R(ifreq(n, N)), a));
      }
    E::run(u, lds, tw, t);
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
      if (ok[k]) {
#pragma unroll
        for (int s = 0; s < E::R0; ++s) {
          const int n = jj[k] + s * (N / E::R0);
          out[a * SLOT + ((size_t)n * N + y) * HZ + zz[k]] = u[k][s];
        }
      }
  }
}

// ---------------------------------------------------------------------------------------------
// y pass.  RECIPE 0 (Hessian): inputs a = 0, 1, 2 -> outputs b < 3 - a, slot base(a) = 0, 3, 5.
// RECIPE 1 (gradient): inputs a = 0, 1 -> b < 2 - a, base 0, 2.  RECIPE 2 (forward, 2LPT):
// one input, one output, DIR = -1, no multiplier.
template <int RECIPE> struct YRecipe;
template <> struct YRecipe<0> {
  static constexpr int NIN = 3, DIR = +1;
  __device__ static int nout(int a) { return 3 - a; }
  __device__ static int base(int a) { return a == 0 ? 0 : (a == 1 ? 3 : 5); }
};
template <> struct YRecipe<1> {
  static constexpr int NIN = 2, DIR = +1;
  __device__ static int nout(int a) { return 2 - a; }
  __device__ static int base(int a) { return a == 0 ? 0 : 2; }
};
template <> struct YRecipe<2> {
  static constexpr int NIN = 1, DIR = -1;
  __device__ static int nout(int) { return 1; }
  __device__ static int base(int) { return 0; }
};

template <typename R, int N, int RECIPE>
struct YPass {
  using V = typename Cplx<R>::type;
  static constexpr int PS = Tile<R>::PS;
  static constexpr int HZ = N / 2;
  static constexpr int NZT = (HZ + PS - 1) / PS;
  using E0 = Engine<V, N, PS, 1, true, 64, YRecipe<RECIPE>::DIR>;
  static constexpr int T = strided_threads(E0::nb(E0::R0));
  using E = Engine<V, N, PS, 1, true, T, YRecipe<RECIPE>::DIR>;
  static constexpr int GRID = N * NZT * YRecipe<RECIPE>::NIN;
};

template <typename R, int N, int RECIPE>
__global__ void __launch_bounds__((YPass<R, N, RECIPE>::T))
k_ypass(const typename Cplx<R>::type* __restrict__ in, typename Cplx<R>::type* __restrict__ out,
        const typename Cplx<R>::type* __restrict__ tw) {
  using Y = YPass<R, N, RECIPE>;
  using RC = YRecipe<RECIPE>;
  using V = typename Y::V;
  using E = typename Y::E;
  constexpr int PS = Y::PS, HZ = Y::HZ;
  constexpr size_t SLOT = (size_t)N * N * HZ;
  __shared__ V lds[E::LDS_ELEMS];
  const int zt = blockIdx.x % Y::NZT;
  const int x = (blockIdx.x / Y::NZT) % N;
  const int a = blockIdx.x / (Y::NZT * N);
  const int t = threadIdx.x;
  V v[E::K0][E::R0];
  int zz[E::K0], jj[E::K0];
  bool ok[E::K0];
  const V* src = in + a * SLOT;
#pragma unroll
  for (int k = 0; k < E::K0; ++k) {
    int q, p, j;
    E::first_layout(t, k, q, p, j, ok[k]);
    const int z = zt * PS + p;
    ok[k] = ok[k] && z < HZ;
    zz[k] = z;
    jj[k] = j;
#pragma unroll
    for (int s = 0; s < E::R0; ++s) {
      const int n = j + s * (N / E::R0);
      v[k][s] = ok[k] ? src[((size_t)x * N + n) * HZ + z] : V{R(0), R(0)};
    }
  }
  const int nout = RC::nout(a);
  const int base = RC::base(a);
#pragma unroll 1
  for (int b = 0; b < nout; ++b) {
    V u[E::K0][E::R0];
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
#pragma unroll
      for (int s = 0; s < E::R0; ++s) {
        const int n = jj[k] + s * (N / E::R0);
        u[k][s] = cscale(v[k][s], powf_int(R(ifreq(n, N)), b));
      }
    E::run(u, lds, tw, t);
    V* dst = out + (size_t)(base + b) * SLOT;
#pragma unroll
    for (int k = 0; k < E::K0; ++k)
      if (ok[k]) {
#pragma unroll
        for (int s = 0; s < E::R0; ++s) {
          const int n = jj[k] + s * (N / E::R0);
          dst[((size_t)x * N + n) * HZ + zz[k]] = u[k][s];
        }
      }
  }
}

// ---------------------------------------------------------------------------------------------
// z pass: complex-to-real along z of NC components, packed two per complex transform
// (c = A + iB over the full length-N spectrum, A(N-m) = conj A(m)).  Component recipes give
// (slot, kz power): Hessian (xx, xy, xz, yy, yz, zz) = (5,0) (4,0) (3,1) (2,0) (1,1) (0,2);
// gradient (x, y, z) = (2,0) (1,0) (0,1).
template <int NC> struct ZRecipe;
template <> struct ZRecipe<6> {
  static constexpr int Q = 3;
  __device__ static int slot(int c) { return c == 0 ? 5 : c == 1 ? 4 : c == 2 ? 3 : c == 3 ? 2 : c == 4 ? 1 : 0; }
  __device__ static int kpow(int c) { return c == 2 || c == 4 ? 1 : (c == 5 ? 2 : 0); }
};
template <> struct ZRecipe<3> {
  static constexpr int Q = 2;
  __device__ static int slot(int c) { return c == 0 ? 2 : (c == 1 ? 1 : 0); }
  __device__ static int kpow(int c) { return c == 2 ? 1 : 0; }
};

enum ZEpi { EPI_COLLAPSE = 0, EPI_STORE = 1, EPI_MU2 = 2 };

template <typename R, int N, int NC, int EPI>
struct ZPass {
  using V = typename Cplx<R>::type;
  static constexpr int Q = ZRecipe<NC>::Q;
  using ZT = ZTile<R, N, Q>;
  static constexpr int P = ZT::P;
  static constexpr int T = ZT::T;
  static constexpr int HZ = N / 2;
  using E = Engine<V, N, P, Q, false, T, +1>;
  static constexpr int LINES = N * N;
  static constexpr int GRID = (LINES + P - 1) / P;
  static_assert(E::K0 == Q, "z pass: one butterfly per transform per thread");
};

struct ZArgs {
  void* F;          // EPI_COLLAPSE: running F_max (R)
  uint8_t* ridx;    // EPI_COLLAPSE: running radius index
  int r;            // EPI_COLLAPSE: radius index of this launch
  void* out;        // EPI_STORE: [NC][N^3] real; EPI_MU2: one workspace slot (complex)
  CollapseConst cc;
};

template <typename R, int N, int NC, int EPI>
__global__ void __launch_bounds__((ZPass<R, N, NC, EPI>::T))
k_zpass(const typename Cplx<R>::type* __restrict__ in, const typename Cplx<R>::type* __restrict__ tw, ZArgs args) {
  using Z = ZPass<R, N, NC, EPI>;
  using RC = ZRecipe<NC>;
  using V = typename Z::V;
  using E = typename Z::E;
  constexpr int P = Z::P, HZ = Z::HZ, Q = Z::Q, R0 = E::R0, M0 = N / R0;
  constexpr size_t SLOT = (size_t)N * N * HZ;
  __shared__ V lds[E::LDS_ELEMS];
  const int t = threadIdx.x;
  // thread t owns pencil position (p, j) of every transform q
  const int j = t % M0;
  const int p = t / M0;
  const int line = blockIdx.x * P + p;
  const bool line_ok = line < Z::LINES;
  V v[Q][R0];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int ca = 2 * q, cb = 2 * q + 1;
    const bool has_b = cb < NC;
    const V* pa = in + (size_t)RC::slot(ca) * SLOT + (size_t)line * HZ;
    const V* pb = in + (size_t)RC::slot(has_b ? cb : ca) * SLOT + (size_t)line * HZ;
    const int ea = RC::kpow(ca), eb = RC::kpow(has_b ? cb : ca);
#pragma unroll
    for (int s = 0; s < R0; ++s) {
      const int n = j + s * M0;
      V c = V{R(0), R(0)};
      if (line_ok && n != N / 2) {
        const int m = n < N / 2 ? n : N - n;
        V A = pa[m];
        A = cscale(A, powf_int(R(m), ea));
        V B = has_b ? cscale(pb[m], powf_int(R(m), eb)) : V{R(0), R(0)};
        if (n > N / 2) {
          A = conj(A);
          B = conj(B);
        }
        c = V{A.x - B.y, A.y + B.x};
      }
      v[q][s] = c;
    }
  }
  E::run(v, lds, tw, t);
  // v[q][s] = T_{2q}(n) + i T_{2q+1}(n) at n = j + s*M0 of line `line`
  if constexpr (EPI == EPI_COLLAPSE) {
    R* F = static_cast<R*>(args.F);
    if (line_ok) {
#pragma unroll
      for (int s = 0; s < R0; ++s) {
        const int n = j + s * M0;
        const size_t idx = (size_t)line * N + n;
        const double f = collapse_point((double)v[0][s].x, (double)v[0][s].y, (double)v[1][s].x,
                                        (double)v[1][s].y, (double)v[2][s].x, (double)v[2][s].y, args.cc);
        const R fr = (R)f;
        if (fr > F[idx]) {
          F[idx] = fr;
          args.ridx[idx] = (uint8_t)args.r;
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
        for (int q = 0; q < Q; ++q) {
          out[(size_t)(2 * q) * VOL + idx] = v[q][s].x;
          if (2 * q + 1 < NC) out[(size_t)(2 * q + 1) * VOL + idx] = v[q][s].y;
        }
      }
    }
  } else {
    static_assert(EPI == EPI_MU2 && NC == 6, "2LPT source needs the six components");
    // mu2 at each point, then a forward real-to-complex transform along z of line pairs
    // (2u, 2u+1) packed as one complex line.
    R* ldsr = reinterpret_cast<R*>(lds);
#pragma unroll
    for (int s = 0; s < R0; ++s) {
      const int n = j + s * M0;
      const R xx = v[0][s].x, xy = v[0][s].y, xz = v[1][s].x, yy = v[1][s].y, yz = v[2][s].x, zz = v[2][s].y;
      const R mu2 = line_ok ? (xx * yy + xx * zz + yy * zz - xy * xy - xz * xz - yz * yz) : R(0);
      ldsr[2 * ((p >> 1) * N + n) + (p & 1)] = mu2;
    }
    __syncthreads();
    using EF = Engine<V, N, P / 2, 1, false, Z::T, -1>;
    static_assert(EF::K0 == 1, "forward z: one butterfly per thread");
    V w[1][R0];
    {
      int q2, p2, j2;
      bool ok2;
      EF::first_layout(t, 0, q2, p2, j2, ok2);
#pragma unroll
      for (int s = 0; s < R0; ++s) w[0][s] = ok2 ? lds[EF::lds_index(0, p2, j2 + s * M0)] : V{R(0), R(0)};
      __syncthreads();
      EF::run(w, lds, tw, t);
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
      const V zk = lds[u * N + k];
      const V zn = lds[u * N + ((N - k) % N)];
      const V a = V{R(0.5) * (zk.x + zn.x), R(0.5) * (zk.y - zn.y)};   // (Z_k + conj Z_{N-k})/2
      const V b = V{R(0.5) * (zk.y + zn.y), R(0.5) * (zn.x - zk.x)};   // (Z_k - conj Z_{N-k})/(2i)
      const int l0 = blockIdx.x * P + 2 * u;
      if (l0 < Z::LINES) out[(size_t)l0 * HZ + k] = a;
      if (l0 + 1 < Z::LINES) out[(size_t)(l0 + 1) * HZ + k] = b;
    }
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

}  // namespace pin
