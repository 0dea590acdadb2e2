// Fragmentation of the collapsed medium into halos (section "Fragmentation"), on the GPU.
//
// The method takes the particles (grid points) one at a time in decreasing F_max; each decision
// depends on the halos built by the particles before it.  The kernels reproduce that sequential
// result exactly with deterministic reservations: each round, every pending particle in a window
// of the order reserves the objects its step reads or writes -- its own cell, its six neighbour
// cells and the halos those neighbours belong to -- with an atomic minimum of its order
// position; a particle whose reservations all hold commits its step.  The earliest pending
// particle always commits, and a particle commits only when no earlier pending particle shares
// an object with it, so every step sees the same state as in the sequential order.  Keys carry
// the round in their high word (newer rounds smaller), so reservations never need clearing.
//
// Every floating-point decision is taken in float64 with the operations in the order the method
// states them (this file is compiled without contraction into fused multiply-adds); halo radii
// come from a host table computed with the C library's pow.
//
// Readings (the paper leaves these open or garbled): particles with F_max >= f_min take part,
// ties in F_max in increasing linear index; the event time is D = 1/F_max of the particle being
// processed; x = q + D u with u = v_max in grid units, periodic minimum image; a halo keeps N_h,
// the sum of its members' offsets from its founder and the sum of their u, and sits at
// q_founder + offsets/N_h + D u_sum/N_h; R = (3 N_h / 4 pi)^(1/3); sigma(R) is the top-hat rms of
// the linear field at R L/N Mpc/h times D, from 64 nodes per octave, linear in ln R; the merging
// constant is Table 1's f_rm; several touched halos are taken in increasing id, pairs (a < b) in
// that order with the halos as merged so far, the larger keeping its id (the smaller id on equal
// sizes); the smallest d/R takes the first halo in id order on equal values; a halo's id is the
// linear index of its founder.
#include "fragment.hpp"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "host_math.hpp"
#include "plan.hpp"

namespace pin {
namespace {

constexpr int kNotCollapsed = -2;
constexpr int kFilament = -1;
// Order positions considered per round: at 512^3 (z = 0) 2^16, 2^17, 2^18, 2^19 and 2^20 took
// 191, 150, 134, 137 and 148 ms, with identical labels for every size (each figure then included
// ~37 ms of host quadrature for the sigma nodes, now computed once per plan).
constexpr int kWindow = 1 << 18;
constexpr int kRoundsPerCheck = 32;    // rounds queued between host checks of progress
constexpr int kRadiusTable = 1 << 20;  // halo radii tabulated for N_h up to this
constexpr int kNodesPerOctave = 64;
constexpr int kFindLimit = 64;         // union by size keeps trees below 32 levels
constexpr double kPi = 3.141592653589793;

struct Dev {
  int n;
  size_t vol;
  int m;                                // participating particles
  int window;                           // order positions considered per round
  const int32_t* order;
  int32_t* label;
  int32_t* parent;
  int32_t* hn;
  double* hs;
  unsigned long long* res_cell;
  unsigned long long* res_halo;
  int32_t* items;
  int32_t* ctl;
  const double* rtab;
  const double* stab;
  int stab_n;
  double s_r0, s_step;
  double uscale;
  FragParams prm;
  unsigned long long* ev_key;
  double* ev_f;
  int32_t* ev_ids;
};

__device__ __forceinline__ void neighbours(int i, int n, int (&nb)[6]) {
  const int x = i / (n * n), y = (i / n) % n, z = i % n;
  nb[0] = ((x + 1) % n) * n * n + y * n + z;
  nb[1] = ((x - 1 + n) % n) * n * n + y * n + z;
  nb[2] = x * n * n + ((y + 1) % n) * n + z;
  nb[3] = x * n * n + ((y - 1 + n) % n) * n + z;
  nb[4] = x * n * n + y * n + (z + 1) % n;
  nb[5] = x * n * n + y * n + (z - 1 + n) % n;
}

__device__ __forceinline__ int find_root(const Dev& d, int h) {
  for (int it = 0; it < kFindLimit; ++it) {
    const int p = d.parent[h];
    if (p == h) return h;
    h = p;
  }
  d.ctl[2] = 1;   // not reachable with union by size; reported as an error by the host
  return h;
}

__device__ __forceinline__ void reserve(unsigned long long* slot, unsigned long long key) {
  if (__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > key) atomicMin(slot, key);
}

// sorted insert without duplicates into a list of at most 6
__device__ __forceinline__ void insert_sorted(int (&l)[6], int& c, int h) {
  int pos = 0;
  while (pos < c && l[pos] < h) ++pos;
  if (pos < c && l[pos] == h) return;
  for (int j = c; j > pos; --j) l[j] = l[j - 1];
  l[pos] = h;
  ++c;
}

// Sort keys: ascending key = descending F for the participants; every other point gets the
// largest key (`none`), so the participants come first.
template <typename R>
__global__ void k_keys(const R* __restrict__ F, size_t vol, double f_min, uint64_t* __restrict__ keys,
                       int32_t* __restrict__ vals) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vol) return;
  const R f = F[i];
  const bool in = (double)f >= f_min;
  uint64_t k;
  if constexpr (sizeof(R) == 4) {
    k = in ? 0xFFFFFFFFull - (uint64_t)__float_as_uint(f) : 0xFFFFFFFFull;
  } else {
    k = in ? ~(uint64_t)__double_as_longlong(f) : ~0ull;
  }
  keys[i] = k;
  vals[i] = (int32_t)i;
}

// Number of participants: the first sorted position holding `none` (binary search, one thread).
__global__ void k_count(const uint64_t* __restrict__ keys, size_t vol, uint64_t none, int32_t* __restrict__ m) {
  size_t lo = 0, hi = vol;
  while (lo < hi) {
    const size_t mid = lo + (hi - lo) / 2;
    if (keys[mid] < none) lo = mid + 1; else hi = mid;
  }
  *m = (int32_t)lo;
}

__global__ void k_state_init(size_t vol, int32_t* label, int32_t* parent, int32_t* hn,
                             unsigned long long* res_cell, unsigned long long* res_halo) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vol) return;
  label[i] = kNotCollapsed;
  parent[i] = (int32_t)i;
  hn[i] = 0;
  res_cell[i] = ~0ull;
  res_halo[i] = ~0ull;
}

__global__ void k_reserve(Dev d, unsigned long long hi) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = d.ctl[0] + k;
  if (k >= d.window || p >= d.m) return;
  const int i = d.order[p];
  if (d.label[i] != kNotCollapsed) return;   // committed in an earlier round
  const unsigned long long key = hi | (unsigned)p;
  int nb[6];
  neighbours(i, d.n, nb);
  reserve(&d.res_cell[i], key);
  int hl[6];
  int hc = 0;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    reserve(&d.res_cell[nb[c]], key);
    const int l = d.label[nb[c]];
    if (l >= 0) insert_sorted(hl, hc, find_root(d, l));
  }
  int32_t* it = d.items + (size_t)k * 7;
  it[0] = hc;
  for (int j = 0; j < hc; ++j) {
    reserve(&d.res_halo[hl[j]], key);
    it[1 + j] = hl[j];
  }
}

// ---- the sequential step of one particle (float64, operations in the method's order) --------

struct Step {
  const Dev& d;
  double D;

  __device__ double radius(int nh) const {
    return nh <= kRadiusTable ? d.rtab[nh - 1] : pow(3.0 * nh / (4.0 * kPi), 1.0 / 3.0);
  }
  __device__ double sigma(double r) const {
    const double t = log(r / d.s_r0) / d.s_step;
    int k = (int)floor(t);
    if (k > d.stab_n - 2) k = d.stab_n - 2;
    if (k < 0) k = 0;   // R >= R(1) always; keeps the index in the table
    const double w = t - k;
    return d.stab[k] + w * (d.stab[k + 1] - d.stab[k]);
  }
  __device__ double wrap(double x) const {
    const double n = (double)d.n;
    return x - n * floor(x / n + 0.5);
  }
  __device__ void coords(int i, double (&q)[3]) const {
    q[0] = (double)(i / (d.n * d.n));
    q[1] = (double)((i / d.n) % d.n);
    q[2] = (double)(i % d.n);
  }
  __device__ void position(int h, double (&x)[3]) const {
    double q[3];
    coords(h, q);
    const double nh = (double)d.hn[h];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double c = q[a] + d.hs[(size_t)a * d.vol + h] / nh;
      x[a] = c + D * (d.hs[(size_t)(3 + a) * d.vol + h] / nh);
    }
  }
  __device__ double dist(const double (&a)[3], const double (&b)[3]) const {
    const double x = wrap(a[0] - b[0]), y = wrap(a[1] - b[1]), z = wrap(a[2] - b[2]);
    return sqrt(x * x + y * y + z * z);
  }
  __device__ bool accretion_ok(double dd, int h) const {
    const double r = radius(d.hn[h]);
    return dd < d.prm.fa * r + d.prm.fra + d.prm.fs * pow(r * sigma(r) * D, 1.7);
  }
  __device__ void add(int h, int j, const double (&u)[3]) const {
    d.hn[h] += 1;
    double qj[3], qh[3];
    coords(j, qj);
    coords(h, qh);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d.hs[(size_t)a * d.vol + h] = d.hs[(size_t)a * d.vol + h] + wrap(qj[a] - qh[a]);
      d.hs[(size_t)(3 + a) * d.vol + h] = d.hs[(size_t)(3 + a) * d.vol + h] + u[a];
    }
    d.label[j] = h;
  }
};

template <typename R>
__device__ __forceinline__ void load_u(const R* v, size_t vol, int j, double uscale, double (&u)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = (double)v[(size_t)a * vol + j] * uscale;
}

template <typename R>
__device__ void execute(const Dev& d, const R* F, const R* v, int p, int i, const int (&nb)[6], const int (&halos)[6],
                        int hc) {
  const Step st{d, 1.0 / (double)F[i]};
  double q[3], ui[3], xi[3];
  st.coords(i, q);
  load_u(v, d.vol, i, d.uscale, ui);
#pragma unroll
  for (int a = 0; a < 3; ++a) xi[a] = q[a] + st.D * ui[a];
  bool has_fil = false;
#pragma unroll
  for (int c = 0; c < 6; ++c) has_fil = has_fil || d.label[nb[c]] == kFilament;

  auto accrete = [&](int h) {
    st.add(h, i, ui);
    for (int c = 0; c < 6; ++c) {
      if (d.label[nb[c]] == kFilament) {
        double uj[3];
        load_u(v, d.vol, nb[c], d.uscale, uj);
        st.add(h, nb[c], uj);
      }
    }
  };
  auto best_halo = [&](const int* list, int cnt, double& best_d) {
    int best = -1;
    double best_v = 0.0;
    for (int j = 0; j < cnt; ++j) {
      double xh[3];
      st.position(list[j], xh);
      const double dd = st.dist(xi, xh);
      const double val = dd / st.radius(d.hn[list[j]]);
      if (best < 0 || val < best_v) {
        best = list[j];
        best_v = val;
        best_d = dd;
      }
    }
    return best;
  };

  if (hc == 0 && !has_fil) {                       // (i) a peak: a new halo
    d.parent[i] = i;
    d.hn[i] = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d.hs[(size_t)a * d.vol + i] = 0.0;
      d.hs[(size_t)(3 + a) * d.vol + i] = ui[a];
    }
    d.label[i] = i;
  } else if (hc == 0) {                            // (iv) filaments only
    d.label[i] = kFilament;
  } else if (hc == 1) {                            // (ii) one halo
    double xh[3];
    st.position(halos[0], xh);
    if (st.accretion_ok(st.dist(xi, xh), halos[0])) {
      accrete(halos[0]);
    } else {
      d.label[i] = kFilament;
    }
  } else {                                         // (iii) several halos
    double dd = 0.0;
    const int h = best_halo(halos, hc, dd);
    const bool accreted = st.accretion_ok(dd, h);
    if (accreted) accrete(h);
    for (int a = 0; a < hc; ++a) {
      for (int b = a + 1; b < hc; ++b) {
        const int ha = find_root(d, halos[a]), hb = find_root(d, halos[b]);
        if (ha == hb) continue;
        double xa[3], xb[3];
        st.position(ha, xa);
        st.position(hb, xb);
        const double dab = st.dist(xa, xb);
        const double ra = st.radius(d.hn[ha]), rb = st.radius(d.hn[hb]);
        if (dab < d.prm.fm * (ra > rb ? ra : rb) + d.prm.frm) {
          const bool keep_a = d.hn[ha] > d.hn[hb] || (d.hn[ha] == d.hn[hb] && ha <= hb);
          const int keep = keep_a ? ha : hb, gone = keep_a ? hb : ha;
          // merger event, tagged with its place in the sequential order (particle, pair)
          const int e = atomicAdd(&d.ctl[6], 1);
          if (e < (int)d.vol) {
            d.ev_key[e] = ((unsigned long long)p << 8) | (unsigned)(a * 8 + b);
            d.ev_f[e] = (double)F[i];
            d.ev_ids[4 * (size_t)e + 0] = keep;
            d.ev_ids[4 * (size_t)e + 1] = gone;
            d.ev_ids[4 * (size_t)e + 2] = d.hn[keep];
            d.ev_ids[4 * (size_t)e + 3] = d.hn[gone];
          } else {
            d.ctl[7] = 1;
          }
          double qk[3], qg[3];
          st.coords(keep, qk);
          st.coords(gone, qg);
          const double ng = (double)d.hn[gone];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double off = st.wrap(qg[c] - qk[c]);
            d.hs[(size_t)c * d.vol + keep] = d.hs[(size_t)c * d.vol + keep] + d.hs[(size_t)c * d.vol + gone] + ng * off;
            d.hs[(size_t)(3 + c) * d.vol + keep] =
                d.hs[(size_t)(3 + c) * d.vol + keep] + d.hs[(size_t)(3 + c) * d.vol + gone];
          }
          d.hn[keep] += d.hn[gone];
          d.parent[gone] = keep;
        }
      }
    }
    if (!accreted) {
      int roots[6];
      int rc = 0;
      for (int j = 0; j < hc; ++j) insert_sorted(roots, rc, find_root(d, halos[j]));
      double d2 = 0.0;
      const int h2 = best_halo(roots, rc, d2);
      if (st.accretion_ok(d2, h2)) {
        accrete(h2);
      } else {
        d.label[i] = kFilament;
      }
    }
  }
}

template <typename R>
__global__ void k_commit(Dev d, unsigned long long hi, const R* __restrict__ F, const R* __restrict__ v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = d.ctl[0] + k;
  if (k >= d.window || p >= d.m) return;
  const int i = d.order[p];
  if (d.label[i] != kNotCollapsed) return;
  const unsigned long long key = hi | (unsigned)p;
  int nb[6];
  neighbours(i, d.n, nb);
  const int32_t* it = d.items + (size_t)k * 7;
  const int hc = it[0];
  int halos[6];
  bool own = d.res_cell[i] == key;
#pragma unroll
  for (int c = 0; c < 6; ++c) own = own && d.res_cell[nb[c]] == key;
  for (int j = 0; j < hc; ++j) {
    halos[j] = it[1 + j];
    own = own && d.res_halo[halos[j]] == key;
  }
  if (!own) {
    atomicMin(&d.ctl[1], p);
    return;
  }
  execute<R>(d, F, v, p, i, nb, halos, hc);
}

__global__ void k_advance(int32_t* ctl, int m, int window) {
  const int head = ctl[1];
  ctl[0] = head;
  ctl[1] = head + window < m ? head + window : m;
}

// Final labels (the root of each member's halo), halo sizes at the roots, and the number of roots
// per block of 256 points into block_count.
__global__ void __launch_bounds__(256) k_finish(Dev d, int32_t* __restrict__ halo_size, int32_t* __restrict__ block_count) {
  __shared__ int32_t wave_roots[4];
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool root = false;
  if (i < d.vol) {
    const int l = d.label[i];
    if (l >= 0) d.label[i] = find_root(d, l);
    root = l >= 0 && d.parent[i] == (int)i && d.hn[i] > 0;
    if (halo_size) halo_size[i] = root ? d.hn[i] : 0;
  }
  const unsigned long long ballot = __ballot(root);
  if ((threadIdx.x & 63) == 0) wave_roots[threadIdx.x >> 6] = (int32_t)__popcll(ballot);
  __syncthreads();
  if (threadIdx.x == 0) block_count[blockIdx.x] = wave_roots[0] + wave_roots[1] + wave_roots[2] + wave_roots[3];
}

// Sum of `count` ints into *out (one workgroup of 1024 threads).
__global__ void __launch_bounds__(1024) k_sum(const int32_t* __restrict__ in, int count, int32_t* __restrict__ out) {
  __shared__ long long part[1024];
  long long acc = 0;
  for (int i = threadIdx.x; i < count; i += 1024) acc += in[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (int32_t)part[0];
}

// Catalogue: flags of the halo roots, then one entry per selected id.
__global__ void k_root_flags(const int32_t* __restrict__ parent, const int32_t* __restrict__ hn, size_t vol,
                             uint8_t* __restrict__ flags) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vol) return;
  flags[i] = parent[i] == (int32_t)i && hn[i] > 0;
}

__global__ void k_catalog(const int32_t* __restrict__ id, const int32_t* __restrict__ count, int n, size_t vol,
                          const int32_t* __restrict__ hn, const double* __restrict__ hs, double cell, int capacity,
                          int32_t* __restrict__ nh_out, double* __restrict__ centre, double* __restrict__ disp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= *count || k >= capacity) return;
  const int h = id[k];
  const double nd = (double)n;
  const double nh = (double)hn[h];
  const double q[3] = {(double)(h / (n * n)), (double)((h / n) % n), (double)(h % n)};
  nh_out[k] = hn[h];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double c = q[a] + hs[(size_t)a * vol + h] / nh;
    centre[(size_t)a * capacity + k] = (c - nd * floor(c / nd)) * cell;
    disp[(size_t)a * capacity + k] = hs[(size_t)(3 + a) * vol + h] / nh * cell;
  }
}

__global__ void k_iota(int32_t* __restrict__ x, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) x[i] = i;
}

__global__ void k_gather_mergers(const int32_t* __restrict__ idx, int count, const double* __restrict__ ev_f,
                                 const int32_t* __restrict__ ev_ids, double* __restrict__ f, int32_t* __restrict__ keep,
                                 int32_t* __restrict__ gone, int32_t* __restrict__ n_keep, int32_t* __restrict__ n_gone) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int e = idx[k];
  f[k] = ev_f[e];
  keep[k] = ev_ids[4 * (size_t)e + 0];
  gone[k] = ev_ids[4 * (size_t)e + 1];
  n_keep[k] = ev_ids[4 * (size_t)e + 2];
  n_gone[k] = ev_ids[4 * (size_t)e + 3];
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Temporary storage of the radix sort and of the catalogue's selection (one buffer for both).
size_t sort_tmp_bytes(size_t vol) {
  size_t tmp = 0, sel = 0;
  hipcub::DoubleBuffer<uint64_t> kb(nullptr, nullptr);
  hipcub::DoubleBuffer<int32_t> vb(nullptr, nullptr);
  hip_check(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kb, vb, (int)vol, 0, 64), "radix sort size");
  hip_check(hipcub::DeviceSelect::Flagged(nullptr, sel, hipcub::CountingInputIterator<int32_t>(0),
                                          static_cast<const uint8_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                          static_cast<int32_t*>(nullptr), (int)vol),
            "select size");
  return tmp > sel ? tmp : sel;
}

}  // namespace

size_t fragment_workspace_bytes(int n) {
  const size_t vol = (size_t)n * n * n;
  size_t b = 0;
  b += 2 * align256(vol * 8) + 2 * align256(vol * 4);   // keys, values
  b += align256(sort_tmp_bytes(vol));
  b += 2 * align256(vol * 4) + align256(vol * 6 * 8);   // parent, hn, hs
  b += 2 * align256(vol * 8);                           // reservations
  b += align256((size_t)kWindow * 7 * 4) + 256;      // items, ctl
  b += 2 * align256(vol * 8) + align256(vol * 16);      // merger events
  b += align256((size_t)kRadiusTable * 8);
  b += align256(64 * 40 * 8);                           // sigma nodes (<= 40 octaves)
  return b;
}

void fragment_free(FragWorkspace& w) {
  if (w.block) (void)hipFree(w.block);
  if (w.host_ctl) (void)hipHostFree(w.host_ctl);
  w = FragWorkspace{};
}

void fragment_prepare(FragWorkspace& w, int n, double box, double amplitude, double gamma, double ns,
                      hipStream_t s) {
  const size_t vol = (size_t)n * n * n;
  if (w.block == nullptr || w.vol != vol) {
    fragment_free(w);
    w.vol = vol;
    w.bytes = fragment_workspace_bytes(n);
    w.sort_tmp_bytes = sort_tmp_bytes(vol);
    w.block = device_alloc(w.bytes, "fragmentation workspace");
    char* p = static_cast<char*>(w.block);
    auto take = [&](size_t bytes) {
      char* q = p;
      p += align256(bytes);
      return q;
    };
    w.keys[0] = reinterpret_cast<uint64_t*>(take(vol * 8));
    w.keys[1] = reinterpret_cast<uint64_t*>(take(vol * 8));
    w.vals[0] = reinterpret_cast<int32_t*>(take(vol * 4));
    w.vals[1] = reinterpret_cast<int32_t*>(take(vol * 4));
    w.sort_tmp = take(w.sort_tmp_bytes);
    w.parent = reinterpret_cast<int32_t*>(take(vol * 4));
    w.hn = reinterpret_cast<int32_t*>(take(vol * 4));
    w.hs = reinterpret_cast<double*>(take(vol * 6 * 8));
    w.res_cell = reinterpret_cast<unsigned long long*>(take(vol * 8));
    w.res_halo = reinterpret_cast<unsigned long long*>(take(vol * 8));
    w.items = reinterpret_cast<int32_t*>(take((size_t)kWindow * 7 * 4));
    w.ctl = reinterpret_cast<int32_t*>(take(256));
    w.ev_key = reinterpret_cast<unsigned long long*>(take(vol * 8));
    w.ev_f = reinterpret_cast<double*>(take(vol * 8));
    w.ev_ids = reinterpret_cast<int32_t*>(take(vol * 16));
    w.rtab = reinterpret_cast<double*>(take((size_t)kRadiusTable * 8));
    w.stab = reinterpret_cast<double*>(take(64 * 40 * 8));
    void* hc = nullptr;
    hip_check(hipHostMalloc(&hc, 64, hipHostMallocDefault), "hipHostMalloc");
    w.host_ctl = static_cast<int32_t*>(hc);
    // halo radii by N_h, with the C library's pow
    std::vector<double> rt(kRadiusTable);
    for (int nh = 1; nh <= kRadiusTable; ++nh) rt[nh - 1] = std::pow(3.0 * nh / (4.0 * kPi), 1.0 / 3.0);
    hip_check(hipMemcpyAsync(w.rtab, rt.data(), rt.size() * 8, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  }
  // sigma nodes: R_k = R(1) 2^(k/64) cells up to the radius of the whole grid (a host quadrature
  // per node, tens of milliseconds at 512^3: kept while the box and the spectrum stay the same)
  const double key[4] = {box, amplitude, gamma, ns};
  if (w.stab_n > 0 && std::equal(key, key + 4, w.s_for)) return;
  w.s_r0 = std::pow(3.0 * 1 / (4.0 * kPi), 1.0 / 3.0);
  w.s_step = std::log(2.0) / kNodesPerOctave;
  const double rmax = std::pow(3.0 * (double)vol / (4.0 * kPi), 1.0 / 3.0);
  w.stab_n = (int)std::ceil(std::log(rmax / w.s_r0) / w.s_step) + 2;
  if (w.stab_n > 64 * 40) fail(PIN_ERR_INVALID_ARG, "grid too large for the sigma table");
  const std::vector<double> st = tophat_sigma_nodes(w.s_r0 * box / n, w.s_step, w.stab_n, amplitude, gamma, ns);
  hip_check(hipMemcpyAsync(w.stab, st.data(), st.size() * 8, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  std::copy(key, key + 4, w.s_for);
}

int fragment_run(FragWorkspace& w, bool fp64, int n, const void* F, const void* v, double uscale, double f_min,
                 const FragParams& prm, int32_t* label, int32_t* halo_size, hipStream_t s) {
  const size_t vol = (size_t)n * n * n;
  const int block = 256;
  const int grid = (int)((vol + block - 1) / block);
  w.n_halos = -1;   // no catalogue until this run completes
  hip_check(hipMemsetAsync(w.ctl, 0, 64, s), "hipMemsetAsync");
  if (fp64) {
    hipLaunchKernelGGL(k_keys<double>, dim3(grid), dim3(block), 0, s, static_cast<const double*>(F), vol, f_min,
                       w.keys[0], w.vals[0]);
  } else {
    hipLaunchKernelGGL(k_keys<float>, dim3(grid), dim3(block), 0, s, static_cast<const float*>(F), vol, f_min,
                       w.keys[0], w.vals[0]);
  }
  hip_check(hipGetLastError(), "fragmentation keys");
  hipcub::DoubleBuffer<uint64_t> kb(w.keys[0], w.keys[1]);
  hipcub::DoubleBuffer<int32_t> vb(w.vals[0], w.vals[1]);
  size_t tmp = w.sort_tmp_bytes;
  hip_check(hipcub::DeviceRadixSort::SortPairs(w.sort_tmp, tmp, kb, vb, (int)vol, 0, fp64 ? 64 : 32, s),
            "radix sort");
  hipLaunchKernelGGL(k_count, dim3(1), dim3(1), 0, s, kb.Current(), vol, fp64 ? ~0ull : 0xFFFFFFFFull, w.ctl + 3);
  hipLaunchKernelGGL(k_state_init, dim3(grid), dim3(block), 0, s, vol, label, w.parent, w.hn, w.res_cell,
                     w.res_halo);
  hip_check(hipGetLastError(), "fragmentation init");
  hip_check(hipMemcpyAsync(w.host_ctl, w.ctl, 16, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  const int m = w.host_ctl[3];

  Dev d{};
  d.n = n;
  d.vol = vol;
  d.m = m;
  d.order = vb.Current();
  d.label = label;
  d.parent = w.parent;
  d.hn = w.hn;
  d.hs = w.hs;
  d.res_cell = w.res_cell;
  d.res_halo = w.res_halo;
  d.items = w.items;
  d.ctl = w.ctl;
  d.rtab = w.rtab;
  d.stab = w.stab;
  d.stab_n = w.stab_n;
  d.s_r0 = w.s_r0;
  d.s_step = w.s_step;
  d.uscale = uscale;
  d.prm = prm;
  d.ev_key = w.ev_key;
  d.ev_f = w.ev_f;
  d.ev_ids = w.ev_ids;
  const int window = kWindow;
  d.window = window;
  // head = 0, next head = end of the first window
  const int32_t init[2] = {0, m < window ? m : window};
  hip_check(hipMemcpyAsync(w.ctl, init, sizeof(init), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");

  const int wgrid = window / block;
  unsigned long long round = 0;
  // every round commits at least the earliest pending particle
  const unsigned long long max_rounds = (unsigned long long)m + 2 * kRoundsPerCheck;
  while (m > 0) {
    for (int r = 0; r < kRoundsPerCheck; ++r, ++round) {
      const unsigned long long hi = (0xFFFFFFFFull - round) << 32;
      hipLaunchKernelGGL(k_reserve, dim3(wgrid), dim3(block), 0, s, d, hi);
      if (fp64) {
        hipLaunchKernelGGL(k_commit<double>, dim3(wgrid), dim3(block), 0, s, d, hi, static_cast<const double*>(F),
                           static_cast<const double*>(v));
      } else {
        hipLaunchKernelGGL(k_commit<float>, dim3(wgrid), dim3(block), 0, s, d, hi, static_cast<const float*>(F),
                           static_cast<const float*>(v));
      }
      hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, w.ctl, m, window);
    }
    hip_check(hipGetLastError(), "fragmentation rounds");
    hip_check(hipMemcpyAsync(w.host_ctl, w.ctl, 16, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (w.host_ctl[2] != 0) fail(PIN_ERR_DEVICE, "fragmentation: halo tree deeper than expected");
    if (w.host_ctl[0] >= m) break;
    if (round > max_rounds) fail(PIN_ERR_DEVICE, "fragmentation made no progress");
  }
  // per-block root counts into the (now free) key buffer, then their sum
  int32_t* block_count = reinterpret_cast<int32_t*>(w.keys[0]);
  hipLaunchKernelGGL(k_finish, dim3(grid), dim3(block), 0, s, d, halo_size, block_count);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, s, block_count, grid, w.ctl + 4);
  hip_check(hipGetLastError(), "fragmentation finish");
  hip_check(hipMemcpyAsync(w.host_ctl, w.ctl, 32, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (w.host_ctl[7] != 0) fail(PIN_ERR_DEVICE, "fragmentation: merger events exceed the grid size");
  w.n_halos = w.host_ctl[4];
  w.n_mergers = w.host_ctl[6];
  w.n = n;
  return w.n_halos;
}

int fragment_mergers(FragWorkspace& w, double* f, int32_t* keep, int32_t* gone, int32_t* n_keep, int32_t* n_gone,
                     int capacity, hipStream_t s) {
  const int count = w.n_mergers;
  if (count == 0) return 0;
  const int block = 256;
  const int grid = (count + block - 1) / block;
  // sort copies of the keys (the events stay as recorded, so the call can be repeated)
  hip_check(hipMemcpyAsync(w.keys[0], w.ev_key, (size_t)count * 8, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
  hipLaunchKernelGGL(k_iota, dim3(grid), dim3(block), 0, s, w.vals[0], count);
  hipcub::DoubleBuffer<uint64_t> kb(w.keys[0], w.keys[1]);
  hipcub::DoubleBuffer<int32_t> vb(w.vals[0], w.vals[1]);
  size_t tmp = w.sort_tmp_bytes;
  hip_check(hipcub::DeviceRadixSort::SortPairs(w.sort_tmp, tmp, kb, vb, count, 0, 40, s), "merger sort");
  hipLaunchKernelGGL(k_gather_mergers, dim3(grid), dim3(block), 0, s, vb.Current(), count < capacity ? count : capacity,
                     w.ev_f, w.ev_ids, f, keep, gone, n_keep, n_gone);
  hip_check(hipGetLastError(), "merger gather");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  return count;
}

int fragment_catalog(FragWorkspace& w, double cell, int32_t* id, int32_t* nh, double* centre, double* disp,
                     int capacity, hipStream_t s) {
  const size_t vol = w.vol;
  const int block = 256;
  const int grid = (int)((vol + block - 1) / block);
  uint8_t* flags = reinterpret_cast<uint8_t*>(w.keys[1]);
  hipLaunchKernelGGL(k_root_flags, dim3(grid), dim3(block), 0, s, w.parent, w.hn, vol, flags);
  hip_check(hipGetLastError(), "catalogue flags");
  size_t tmp = w.sort_tmp_bytes;
  hip_check(hipcub::DeviceSelect::Flagged(w.sort_tmp, tmp, hipcub::CountingInputIterator<int32_t>(0), flags, id,
                                          w.ctl + 5, (int)vol, s),
            "catalogue select");
  const int cgrid = (w.n_halos + block - 1) / block;
  if (cgrid > 0) {
    hipLaunchKernelGGL(k_catalog, dim3(cgrid), dim3(block), 0, s, id, w.ctl + 5, w.n, vol, w.hn, w.hs, cell, capacity,
                       nh, centre, disp);
    hip_check(hipGetLastError(), "catalogue");
  }
  hip_check(hipMemcpyAsync(w.host_ctl, w.ctl, 32, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (w.host_ctl[5] != w.n_halos) fail(PIN_ERR_DEVICE, "catalogue: halo count differs from the fragmentation's");
  return w.n_halos;
}

}  // namespace pin
