// Scene build on the device: unit face normals, vertex normals (paper Eq. 13),
// and a linear BVH over the triangles (Morton order, binary radix tree,
// bottom-up box fit).  Everything here is deterministic: integer atomics
// only count, FP32 sums run in a fixed order.
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include "dt_internal.h"

namespace {

constexpr int SCAN_NB = 256;  // blocks (= partial sums) of the chunked device scan
constexpr int TREELET_PASSES = 4;  // treelet restructuring passes after the box fit
constexpr int SCAN_T = 256;

// ------------------------------------------------------------------ block scans
template <class T>
__device__ T block_incl_scan(T v, T* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    T x = t >= off ? sh[t - off] : T(0);
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  return sh[t];
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_scan_reduce(const int32_t* in, int32_t n, int32_t chunk, int32_t* part) {
  __shared__ int32_t sh[SCAN_T];
  int64_t lo = (int64_t)blockIdx.x * chunk;
  int64_t hi = lo + chunk < n ? lo + chunk : n;
  int32_t s = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += in[i];
  int32_t tot = block_incl_scan(s, sh);
  if (threadIdx.x == blockDim.x - 1) part[blockIdx.x] = tot;
}

// exclusive scan of part[0..nb) in place; part[nb] = total
__global__ void k_scan_partials(int32_t* part, int nb) {
  __shared__ int32_t sh[SCAN_NB];
  int t = threadIdx.x;
  int32_t v = t < nb ? part[t] : 0;
  int32_t inc = block_incl_scan(v, sh);
  __syncthreads();
  if (t < nb) part[t] = inc - v;
  if (t == (int)blockDim.x - 1) part[nb] = inc;
}

__global__ void k_scan_apply(const int32_t* in, int32_t* out, int32_t n, int32_t chunk,
                             const int32_t* part) {
  __shared__ int32_t sh[SCAN_T];
  int64_t lo = (int64_t)blockIdx.x * chunk;
  int64_t hi = lo + chunk < n ? lo + chunk : n;
  int32_t carry = part[blockIdx.x];
  for (int64_t base = lo; base < hi; base += blockDim.x) {
    int64_t i = base + threadIdx.x;
    int32_t v = i < hi ? in[i] : 0;
    int32_t inc = block_incl_scan(v, sh);
    int32_t tot = sh[blockDim.x - 1];
    if (i < hi) out[i] = carry + inc - v;
    carry += tot;
    __syncthreads();
  }
}

__global__ void k_copy_total(const int32_t* part, int nb, int32_t* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = part[nb];
}

// ------------------------------------------------------------------ normals
__device__ __forceinline__ bool face_ok(const int32_t* F, int f, int32_t nv) {
  int a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
  return a >= 0 && a < nv && b >= 0 && b < nv && c >= 0 && c < nv;
}

__global__ void k_face_normals(const float* V, const int32_t* F, int32_t nf, int32_t nv, float4* fn) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  if (!face_ok(F, f, nv)) {
    fn[f] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  v3 a = load3(V + 3 * F[3 * f]), b = load3(V + 3 * F[3 * f + 1]), c = load3(V + 3 * F[3 * f + 2]);
  v3 n = cross(b - a, c - a);
  float l2 = dot(n, n);
  if (l2 > 0.0f) {
    v3 u = n * (1.0f / sqrtf(l2));
    fn[f] = make_float4(u.x, u.y, u.z, 1.0f);
  } else {
    fn[f] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

__global__ void k_vcount(const int32_t* F, int32_t nf, int32_t nv, int32_t* cnt) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf || !face_ok(F, f, nv)) return;
  for (int k = 0; k < 3; ++k) atomicAdd(&cnt[F[3 * f + k]], 1);
}

__global__ void k_vfill(const int32_t* F, int32_t nf, int32_t nv, const int32_t* off,
                        int32_t* cursor, int32_t* idx) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf || !face_ok(F, f, nv)) return;
  for (int k = 0; k < 3; ++k) {
    int v = F[3 * f + k];
    int p = atomicAdd(&cursor[v], 1);
    idx[off[v] + p] = f;
  }
}

// each vertex's face list in ascending face order (fixed summation order)
__global__ void k_vsort(const int32_t* off, int32_t nv, int32_t* idx) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  int lo = off[v], hi = off[v + 1];
  for (int i = lo + 1; i < hi; ++i) {
    int x = idx[i];
    int j = i - 1;
    while (j >= lo && idx[j] > x) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = x;
  }
}

// Eq. 13: one third of the sum of the unit normals of the incident faces, in
// ascending face order (not renormalised: the shading normal normalises the
// barycentric blend of Eq. 12 instead)
__global__ void k_vnormals(const int32_t* off, const int32_t* idx, const float4* fn, int32_t nv,
                           float4* vn) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  v3 s = mk3(0.f, 0.f, 0.f);
  for (int i = off[v]; i < off[v + 1]; ++i) s += xyz(fn[idx[i]]);
  v3 n = s * (1.0f / 3.0f);
  vn[v] = make_float4(n.x, n.y, n.z, 0.0f);
}

// ------------------------------------------------------------------ Morton codes
constexpr int NBB = 256;  // blocks of the bounds reduction

__device__ __forceinline__ int vclamp(int i, int nv) { return i < 0 ? 0 : (i >= nv ? nv - 1 : i); }

__device__ __forceinline__ v3 centroid(const float* V, const int32_t* F, int f, int nv) {
  v3 a = load3(V + 3 * vclamp(F[3 * f], nv)), b = load3(V + 3 * vclamp(F[3 * f + 1], nv));
  v3 c = load3(V + 3 * vclamp(F[3 * f + 2], nv));
  return (a + b + c) * (1.0f / 3.0f);
}

__global__ void k_bounds(const float* V, const int32_t* F, int32_t nf, int32_t nv, float* part) {
  __shared__ float sh[6][256];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += gridDim.x * blockDim.x) {
    v3 c = centroid(V, F, f, nv);
    lo[0] = fminf(lo[0], c.x);
    lo[1] = fminf(lo[1], c.y);
    lo[2] = fminf(lo[2], c.z);
    hi[0] = fmaxf(hi[0], c.x);
    hi[1] = fmaxf(hi[1], c.y);
    hi[2] = fmaxf(hi[2], c.z);
  }
  int t = threadIdx.x;
  for (int k = 0; k < 3; ++k) {
    sh[k][t] = lo[k];
    sh[3 + k][t] = hi[k];
  }
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s)
      for (int k = 0; k < 3; ++k) {
        sh[k][t] = fminf(sh[k][t], sh[k][t + s]);
        sh[3 + k][t] = fmaxf(sh[3 + k][t], sh[3 + k][t + s]);
      }
    __syncthreads();
  }
  if (t < 6) part[blockIdx.x * 6 + t] = sh[t][0];
}

__device__ __forceinline__ uint64_t spread21(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t quant21(float c, float lo, float ext) {
  if (!(ext > 0.0f)) return 0u;
  float q = (c - lo) / ext * 2097152.0f;
  q = fminf(fmaxf(q, 0.0f), 2097151.0f);
  return (uint32_t)q;
}

// keys: 63-bit Morton codes of the centroids (21 bits per axis) shifted right
// by `drop` bits (31 keeps the top 32, about 11 bits per axis)
// the scene bounds of the centroids from the per-block partials (one block of
// NBB threads), into the header
__global__ void __launch_bounds__(NBB) k_bounds_final(const float* part, BvhHeader* hdr) {
  __shared__ float sh[6][NBB];
  const int t = threadIdx.x;
  for (int k = 0; k < 6; ++k) sh[k][t] = part[t * 6 + k];
  __syncthreads();
  for (int st = NBB / 2; st > 0; st >>= 1) {
    if (t < st)
      for (int k = 0; k < 3; ++k) {
        sh[k][t] = fminf(sh[k][t], sh[k][t + st]);
        sh[3 + k][t] = fmaxf(sh[3 + k][t], sh[3 + k][t + st]);
      }
    __syncthreads();
  }
  if (t < 3) hdr->lo[t] = sh[t][0];
  if (t >= 3 && t < 6) hdr->hi[t - 3] = sh[t][0];
}

__global__ void k_morton(const float* V, const int32_t* F, int32_t nf, int32_t nv, int drop,
                         const BvhHeader* hdr, uint64_t* keys, int32_t* vals) {
  const float bb[6] = {hdr->lo[0], hdr->lo[1], hdr->lo[2], hdr->hi[0], hdr->hi[1], hdr->hi[2]};
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  v3 c = centroid(V, F, f, nv);
  uint32_t qx = quant21(c.x, bb[0], bb[3] - bb[0]);
  uint32_t qy = quant21(c.y, bb[1], bb[4] - bb[1]);
  uint32_t qz = quant21(c.z, bb[2], bb[5] - bb[2]);
  keys[f] = ((spread21(qx) << 2) | (spread21(qy) << 1) | spread21(qz)) >> drop;
  vals[f] = f;
}

// ------------------------------------------------------------------ stable LSD radix sort
constexpr int RS_T = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_T * RS_ITEMS;
constexpr int RS_WAVES = RS_T / 64;

__global__ void k_rs_hist(const uint64_t* keys, int32_t n, int shift, int32_t* hist, int ntiles) {
  __shared__ uint32_t h[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int j = 0; j < RS_ITEMS; ++j) {
    int64_t i = base + (int64_t)j * RS_T + threadIdx.x;
    if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int dg = threadIdx.x; dg < 256; dg += blockDim.x)
    hist[(size_t)dg * ntiles + blockIdx.x] = (int32_t)h[dg];
}

// lanes of the wave holding the same 8-bit digit (restricted to valid lanes)
__device__ __forceinline__ uint64_t digit_peers(uint32_t dg, bool valid) {
  uint64_t m = __ballot(valid);
  for (int b = 0; b < 8; ++b) {
    bool bit = (dg >> b) & 1u;
    uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// Each wave owns RS_ITEMS*64 consecutive keys of the tile; ranks are stable.
__global__ void k_rs_scatter(const uint64_t* kin, const int32_t* vin, uint64_t* kout,
                             int32_t* vout, int32_t n, int shift, const int32_t* offs, int ntiles) {
  __shared__ uint32_t cnt[RS_WAVES][256];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < RS_WAVES * 256; i += blockDim.x) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const int64_t wbase = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * (RS_ITEMS * 64);
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int s = 0; s < RS_ITEMS; ++s) {
    int64_t i = wbase + s * 64 + lane;
    bool valid = i < n;
    uint32_t dg = valid ? ((uint32_t)(kin[i] >> shift) & 255u) : 0u;
    uint64_t peers = digit_peers(dg, valid);
    if (valid && (peers & lt) == 0) cnt[w][dg] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  for (int dg = threadIdx.x; dg < 256; dg += blockDim.x) {
    uint32_t run = (uint32_t)offs[(size_t)dg * ntiles + blockIdx.x];
    for (int ww = 0; ww < RS_WAVES; ++ww) {
      uint32_t c = cnt[ww][dg];
      cnt[ww][dg] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int s = 0; s < RS_ITEMS; ++s) {
    int64_t i = wbase + s * 64 + lane;
    bool valid = i < n;
    uint64_t k = valid ? kin[i] : 0ull;
    int32_t val = valid ? vin[i] : 0;
    uint32_t dg = (uint32_t)(k >> shift) & 255u;
    uint64_t peers = digit_peers(dg, valid);
    uint32_t pos = cnt[w][dg] + (uint32_t)__popcll(peers & lt);
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      kout[pos] = k;
      vout[pos] = val;
      if ((peers & lt) == 0) cnt[w][dg] += (uint32_t)__popcll(peers);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------------ binary radix tree
__device__ __forceinline__ int kdelta(const uint64_t* k, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  uint64_t a = k[i], b = k[j];
  if (a == b) return 64 + __clz((uint32_t)(i ^ j));
  return __clzll(a ^ b);
}

__global__ void k_karras(const uint64_t* keys, int n, BvhNode* nodes, int32_t* leaf_parent) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  int dl = kdelta(keys, n, i, i - 1), dr = kdelta(keys, n, i, i + 1);
  int d = dr > dl ? 1 : -1;
  int dmin = d > 0 ? dl : dr;
  int lmax = 2;
  while (kdelta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int l = 0;
  for (int t = lmax >> 1; t >= 1; t >>= 1)
    if (kdelta(keys, n, i, i + (l + t) * d) > dmin) l += t;
  int j = i + l * d;
  int dnode = kdelta(keys, n, i, j);
  int s = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (kdelta(keys, n, i, i + (s + t) * d) > dnode) s += t;
  } while (t > 1);
  int gamma = i + s * d + (d < 0 ? -1 : 0);
  int lo = i < j ? i : j, hi = i < j ? j : i;
  int* nd = (int*)&nodes[i].d;
  if (lo == gamma) {
    nd[0] = (int)((uint32_t)gamma | DT_LEAF_BIT);
    leaf_parent[gamma] = i;
  } else {
    nd[0] = gamma;
    ((int*)&nodes[gamma].d)[2] = i;
  }
  if (hi == gamma + 1) {
    nd[1] = (int)((uint32_t)(gamma + 1) | DT_LEAF_BIT);
    leaf_parent[gamma + 1] = i;
  } else {
    nd[1] = gamma + 1;
    ((int*)&nodes[gamma + 1].d)[2] = i;
  }
  nd[3] = 0;
  if (i == 0) nd[2] = -1;
}

__device__ __forceinline__ void put_box(BvhNode* P, int slot, v3 lo, v3 hi) {
  float* fp = (float*)P + slot * 6;
  fp[0] = lo.x;
  fp[1] = lo.y;
  fp[2] = lo.z;
  fp[3] = hi.x;
  fp[4] = hi.y;
  fp[5] = hi.z;
}

__device__ __forceinline__ v3 vmin(v3 a, v3 b) { return {fminf(a.x, b.x), fminf(a.y, b.y), fminf(a.z, b.z)}; }
__device__ __forceinline__ v3 vmax(v3 a, v3 b) { return {fmaxf(a.x, b.x), fmaxf(a.y, b.y), fmaxf(a.z, b.z)}; }

// Order-preserving map of floats to ints (for integer atomic min / max).
__device__ __forceinline__ int fenc(float f) {
  int i = __float_as_int(f);
  return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ __forceinline__ float fdec(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

__global__ void k_fit_init(int* acc, int n_nodes) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 6 * n_nodes; i += gridDim.x * blockDim.x)
    acc[i] = (i % 6) < 3 ? fenc(INFINITY) : fenc(-INFINITY);
}

// Leaves in Morton order get their triangle; boxes are fitted bottom-up.
// Each child writes its box into its slot of the parent node (read only by
// later kernels) and merges it into the parent's union accumulator with
// device-scope atomic min / max.  The second child to arrive (arrival
// counter) reads the finished union back with device-scope atomic loads and
// carries on upward.  No memory fence is needed: the accumulator is only
// touched by atomics, which are coherent across the chip, and a wait for
// their completion orders them before the arrival increment.
__global__ void k_fit(const float* V, const int32_t* F, int32_t nv, const int32_t* sorted, int n,
                      BvhNode* nodes, const int32_t* leaf_parent, int32_t* arrive, int* acc,
                      float4* leaves) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int f = sorted[j];
  v3 a = load3(V + 3 * vclamp(F[3 * f], nv)), b = load3(V + 3 * vclamp(F[3 * f + 1], nv));
  v3 c = load3(V + 3 * vclamp(F[3 * f + 2], nv));
  leaves[3 * j + 0] = make_float4(a.x, a.y, a.z, __int_as_float(f));
  leaves[3 * j + 1] = make_float4(b.x, b.y, b.z, 0.f);
  leaves[3 * j + 2] = make_float4(c.x, c.y, c.z, 0.f);
  if (n == 1) return;
  v3 lo = vmin(vmin(a, b), c), hi = vmax(vmax(a, b), c);
  int ref = (int)((uint32_t)j | DT_LEAF_BIT);
  int p = leaf_parent[j];
  // a binary radix tree over 63-bit keys + 31-bit indices is at most 95 deep
  for (int guard = 0; guard < 256 && p >= 0 && p < n - 1; ++guard) {
    BvhNode* P = &nodes[p];
    const int* pd = (const int*)&P->d;
    int slot = pd[0] == ref ? 0 : 1;
    put_box(P, slot, lo, hi);
    int* ac = acc + 6 * p;
    __hip_atomic_fetch_min(ac + 0, fenc(lo.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_min(ac + 1, fenc(lo.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_min(ac + 2, fenc(lo.z), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_max(ac + 3, fenc(hi.x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_max(ac + 4, fenc(hi.y), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_max(ac + 5, fenc(hi.z), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);  // the merges above are performed before the arrival below
    int old = __hip_atomic_fetch_add(&arrive[p], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == 0) return;
    lo = mk3(fdec(__hip_atomic_load(ac + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)),
             fdec(__hip_atomic_load(ac + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)),
             fdec(__hip_atomic_load(ac + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
    hi = mk3(fdec(__hip_atomic_load(ac + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)),
             fdec(__hip_atomic_load(ac + 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)),
             fdec(__hip_atomic_load(ac + 5, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
    if (p == 0) return;
    ref = p;
    p = pd[2];
  }
}

// 1 for an internal node at even depth (root = 0), else 0: walk to the root.
// With hdr, also the tree height (root = 1): the deepest internal node has a
// leaf child one level below it.
__global__ void k_even(int32_t n_int, const BvhNode* nodes, int32_t* flag, BvhHeader* hdr) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_int) return;
  int dep = 0, p = i;
  while (p > 0 && p < n_int && dep < 4096) {
    p = nodes[p].d.z;
    ++dep;
  }
  flag[i] = (dep & 1) == 0;
  if (hdr) atomicMax(&hdr->depth, dep + 2);
}

// ------------------------------------------------------------------ treelet restructuring
// The Morton-order tree groups triangles by space-filling-curve position, not
// by how much box surface the grouping costs, and the excess sits in the lower
// levels.  Each pass takes the nodes X at one depth parity as roots of
// disjoint two-level treelets: X, its internal children, and as treelet leaves
// the grandchildren (or a child that is itself a triangle), 3 or 4 of them.
// Among all binary trees over those leaves it keeps the one whose inner nodes
// have the least total surface area (the root's box, and every box below the
// treelet leaves, are unchanged), reusing X and its internal children as the
// inner nodes.  Treelets of one pass share no inner node, and a thread writes
// only its own inner nodes, the child fields of X (not X's parent link) and
// the parent links of its treelet leaves, so the threads of a pass are
// independent.  Alternating parities over passes lets changes travel.
struct TBox {
  v3 lo, hi;
};
__device__ __forceinline__ TBox tunion(const TBox& a, const TBox& b) {
  return {vmin(a.lo, b.lo), vmax(a.hi, b.hi)};
}
__device__ __forceinline__ float tarea(const TBox& b) {
  v3 e = vmax(b.hi - b.lo, mk3(0.f, 0.f, 0.f));
  return 2.f * (e.x * e.y + e.y * e.z + e.z * e.x);
}
__device__ __forceinline__ TBox get_box(const BvhNode& n, int slot) {
  const float* fp = (const float*)&n + slot * 6;
  return {mk3(fp[0], fp[1], fp[2]), mk3(fp[3], fp[4], fp[5])};
}

// node i gets children (c0, b0), (c1, b1); with_parent: also its parent link
__device__ __forceinline__ void set_node(BvhNode* nodes, int i, int c0, const TBox& b0, int c1,
                                         const TBox& b1, bool with_parent, int parent) {
  BvhNode* P = &nodes[i];
  put_box(P, 0, b0.lo, b0.hi);
  put_box(P, 1, b1.lo, b1.hi);
  int* pd = (int*)&P->d;
  pd[0] = c0;
  pd[1] = c1;
  if (with_parent) pd[2] = parent;
}

__device__ __forceinline__ void set_parent(BvhNode* nodes, int32_t* leaf_parent, int ref, int parent) {
  if ((uint32_t)ref & DT_LEAF_BIT)
    leaf_parent[(uint32_t)ref & ~DT_LEAF_BIT] = parent;
  else
    ((int*)&nodes[ref].d)[2] = parent;
}

__global__ void k_treelet(int32_t n_int, BvhNode* nodes, int32_t* leaf_parent, const int32_t* even,
                          int want_even) {
  const int X = blockIdx.x * blockDim.x + threadIdx.x;
  if (X >= n_int || (even[X] != 0) != (want_even != 0)) return;
  int ref[4], inner[3];
  TBox box[4];
  int n = 0, m = 1;
  inner[0] = X;
  {
    const BvhNode nx = nodes[X];
    const int* xd = (const int*)&nx.d;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int c = xd[k];
      if ((uint32_t)c & DT_LEAF_BIT) {
        ref[n] = c;
        box[n++] = get_box(nx, k);
      } else {
        inner[m++] = c;
        const BvhNode nc = nodes[c];
        const int* cd = (const int*)&nc.d;
        ref[n] = cd[0];
        box[n++] = get_box(nc, 0);
        ref[n] = cd[1];
        box[n++] = get_box(nc, 1);
      }
    }
  }
  if (n < 3) return;
  // candidate topologies, costs = summed areas of the inner nodes below X
  if (n == 3) {
    // ((a b) c): the pair with the least box area
    int bi = 0, bj = 1, bk = 2;
    float best = tarea(tunion(box[0], box[1]));
    float c02 = tarea(tunion(box[0], box[2])), c12 = tarea(tunion(box[1], box[2]));
    if (c02 < best) { best = c02; bi = 0; bj = 2; bk = 1; }
    if (c12 < best) { best = c12; bi = 1; bj = 2; bk = 0; }
    const int P1 = inner[1];
    // current shape: X's internal child holds the pair
    const TBox pb = tunion(box[bi], box[bj]);
    set_node(nodes, P1, ref[bi], box[bi], ref[bj], box[bj], true, X);
    set_node(nodes, X, P1, pb, ref[bk], box[bk], false, 0);
    set_parent(nodes, leaf_parent, ref[bi], P1);
    set_parent(nodes, leaf_parent, ref[bj], P1);
    set_parent(nodes, leaf_parent, ref[bk], X);
    return;
  }
  // four leaves: 3 balanced trees ((a b)(c d)) and 12 chains (((a b) c) d)
  float pa[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i + 1; j < 4; ++j) pa[i][j] = tarea(tunion(box[i], box[j]));
  // the current tree is balanced with pairs (0 1)(2 3)
  float best = pa[0][1] + pa[2][3];
  int kind = 0, a = 0, b = 1, c = 2, d = 3;
  if (pa[0][2] + pa[1][3] < best) { best = pa[0][2] + pa[1][3]; kind = 0; a = 0; b = 2; c = 1; d = 3; }
  if (pa[0][3] + pa[1][2] < best) { best = pa[0][3] + pa[1][2]; kind = 0; a = 0; b = 3; c = 1; d = 2; }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = i + 1; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k == i || k == j) continue;
        const int l = 6 - i - j - k;
        const float cost = pa[i][j] + tarea(tunion(tunion(box[i], box[j]), box[k]));
        if (cost < best) { best = cost; kind = 1; a = i; b = j; c = k; d = l; }
      }
  if (kind == 0 && a == 0 && b == 1) return;  // already the best
  const int P1 = inner[1], P2 = inner[2];
  const TBox ab = tunion(box[a], box[b]);
  if (kind == 0) {
    const TBox cd = tunion(box[c], box[d]);
    set_node(nodes, P1, ref[a], box[a], ref[b], box[b], true, X);
    set_node(nodes, P2, ref[c], box[c], ref[d], box[d], true, X);
    set_node(nodes, X, P1, ab, P2, cd, false, 0);
    set_parent(nodes, leaf_parent, ref[a], P1);
    set_parent(nodes, leaf_parent, ref[b], P1);
    set_parent(nodes, leaf_parent, ref[c], P2);
    set_parent(nodes, leaf_parent, ref[d], P2);
  } else {
    const TBox abc = tunion(ab, box[c]);
    set_node(nodes, P2, ref[a], box[a], ref[b], box[b], true, P1);
    set_node(nodes, P1, P2, ab, ref[c], box[c], true, X);
    set_node(nodes, X, P1, abc, ref[d], box[d], false, 0);
    set_parent(nodes, leaf_parent, ref[a], P2);
    set_parent(nodes, leaf_parent, ref[b], P2);
    set_parent(nodes, leaf_parent, ref[c], P1);
    set_parent(nodes, leaf_parent, ref[d], X);
  }
}

// Exponent e of the quantization step 2^e of one axis of a node box [lo, hi]:
// 254 steps must span the box (with the origin rounded down to a multiple of
// the step, 255 then reach past hi), and every p + q 2^e, q in [0, 255], must be
// exact in FP32, which holds once 2^(e+22) >= max(|lo|, |hi|).
__device__ __forceinline__ int quant_exponent(float lo, float hi) {
  float m = fmaxf(fabsf(lo), fabsf(hi));
  int e = -126;
  if (m > 0.f) {
    int em = ilogbf(m) + 1 - 22;  // 2^(ilogb + 1) > m
    e = em > e ? em : e;
  }
  float ext = hi - lo;
  if (ext > 0.f) {
    int ee = ilogbf(ext / 254.0f) + 1;  // 2^ee > ext / 254
    e = ee > e ? ee : e;
  }
  // make sure the span fits (the rounded-down origin costs up to one step);
  // p + 255 s is exact, so the comparison is too
  while (e < 127 && floorf(ldexpf(lo, -e)) * ldexpf(1.0f, e) + 255.0f * ldexpf(1.0f, e) < hi) ++e;
  return e;
}

// Writes the 4-wide node of every even-depth internal node i at index idx[i]:
// each leaf child keeps its slot, each internal child hands over its two
// children (their boxes are stored in that child's node).
__global__ void k_collapse(int32_t n_int, const BvhNode* nodes, const int32_t* flag,
                           const int32_t* idx, Bvh4Node* out, int32_t cap4) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_int || !flag[i]) return;
  int j = idx[i];
  if (j < 0 || j >= cap4) return;
  float lo[4][3], hi[4][3];
  uint32_t ch[4];
  int k = 0;
  auto ref = [&](uint32_t c) -> uint32_t {
    if (c & DT_LEAF_BIT) return c;
    return c < (uint32_t)n_int ? (uint32_t)idx[c] : DT_NO_CHILD;
  };
  auto put = [&](const BvhNode& m, int side, uint32_t c) {
    const float4 a = m.a, b = m.b, cc = m.c;
    if (side == 0) {
      lo[k][0] = a.x, lo[k][1] = a.y, lo[k][2] = a.z;
      hi[k][0] = a.w, hi[k][1] = b.x, hi[k][2] = b.y;
    } else {
      lo[k][0] = b.z, lo[k][1] = b.w, lo[k][2] = cc.x;
      hi[k][0] = cc.y, hi[k][1] = cc.z, hi[k][2] = cc.w;
    }
    ch[k] = ref(c);
    ++k;
  };
  const BvhNode n = nodes[i];
  uint32_t cs[2] = {(uint32_t)n.d.x, (uint32_t)n.d.y};
  for (int side = 0; side < 2; ++side) {
    uint32_t c = cs[side];
    if ((c & DT_LEAF_BIT) || c >= (uint32_t)n_int) {
      put(n, side, c);
    } else {
      const BvhNode m = nodes[c];
      put(m, 0, (uint32_t)m.d.x);
      put(m, 1, (uint32_t)m.d.y);
    }
  }
  int cnt = k;
  for (; k < 4; ++k) {
    lo[k][0] = lo[k][1] = lo[k][2] = 0.f;
    hi[k][0] = hi[k][1] = hi[k][2] = 0.f;
    ch[k] = DT_NO_CHILD;
  }
  Bvh4Node q;
  float org[3];
  uint32_t ebits = 0, qlo[3] = {0u, 0u, 0u}, qhi[3] = {0u, 0u, 0u};
  for (int a = 0; a < 3; ++a) {
    float nlo = lo[0][a], nhi = hi[0][a];
    for (int c = 1; c < cnt; ++c) {
      nlo = fminf(nlo, lo[c][a]);
      nhi = fmaxf(nhi, hi[c][a]);
    }
    int e = quant_exponent(nlo, nhi);
    float sc = ldexpf(1.0f, e);
    float p = floorf(ldexpf(nlo, -e)) * sc;  // a multiple of sc, <= nlo
    org[a] = p;
    ebits |= (uint32_t)(uint8_t)(int8_t)e << (8 * a);
    for (int c = 0; c < cnt; ++c) {
      int ql = (int)floorf(ldexpf(lo[c][a] - p, -e));
      ql = ql < 0 ? 0 : (ql > 255 ? 255 : ql);
      while (ql > 0 && p + (float)ql * sc > lo[c][a]) --ql;
      int qh = (int)ceilf(ldexpf(hi[c][a] - p, -e));
      qh = qh < 0 ? 0 : (qh > 255 ? 255 : qh);
      while (qh < 255 && p + (float)qh * sc < hi[c][a]) ++qh;
      qlo[a] |= (uint32_t)ql << (8 * c);
      qhi[a] |= (uint32_t)qh << (8 * c);
    }
  }
  q.org = make_float4(org[0], org[1], org[2], __uint_as_float(ebits | ((uint32_t)cnt << 24)));
  q.qlo = make_uint4(qlo[0], qlo[1], qlo[2], 0u);
  q.qhi = make_uint4(qhi[0], qhi[1], qhi[2], 0u);
  q.child = make_uint4(ch[0], ch[1], ch[2], ch[3]);
  out[j] = q;
}

__global__ void k_header(BvhHeader* hdr, int32_t nv, int32_t nf) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    hdr->nv = nv;
    hdr->nf = nf;
    hdr->depth = nf == 1 ? 1 : 0;  // larger trees: the last depth-parity pass
    hdr->pad0 = 0;
  }
}

__global__ void k_copy_vn(const float4* vn, int32_t nv, float* N) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  float4 a = vn[v];
  N[3 * v] = a.x;
  N[3 * v + 1] = a.y;
  N[3 * v + 2] = a.z;
}

struct BuildWs {
  uint64_t *k0, *k1;
  int32_t *v0, *v1;
  int32_t* hist;
  int32_t* scanp;
  float* bpart;
  int32_t* arrive;
  int* acc;
  int32_t *flag4, *idx4;
  int32_t *vcnt, *cursor;
};

int rs_tiles(int32_t nf) { return (int)((nf + RS_TILE - 1) / RS_TILE); }

size_t carve_build(Carver& c, int32_t nv, int32_t nf, BuildWs* w) {
  int nt = rs_tiles(nf);
  BuildWs x;
  x.k0 = c.take<uint64_t>(nf);
  x.k1 = c.take<uint64_t>(nf);
  x.v0 = c.take<int32_t>(nf);
  x.v1 = c.take<int32_t>(nf);
  x.hist = c.take<int32_t>((size_t)256 * nt);
  x.scanp = c.take<int32_t>(SCAN_NB + 1);
  x.bpart = c.take<float>(NBB * 6);
  x.arrive = c.take<int32_t>(nf > 1 ? nf - 1 : 1);
  x.acc = c.take<int>(6 * (size_t)(nf > 1 ? nf - 1 : 1));
  x.flag4 = c.take<int32_t>(nf);
  x.idx4 = c.take<int32_t>(nf);
  x.vcnt = c.take<int32_t>(nv);
  x.cursor = c.take<int32_t>(nv);
  if (w) *w = x;
  return c.used();
}

}  // namespace

// ------------------------------------------------------------------ shared helpers
dt_status dt_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return DT_OK;
  unsigned nb = dt_blocks(n, 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3(nb), dim3(256), 0, s, p, value, n);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

size_t dt_scan_partials_count() { return SCAN_NB + 1; }

// out[0..n) = exclusive prefix sums of in[0..n); partials[SCAN_NB] = total.
// in == out is allowed.
dt_status dt_scan_exclusive_i32(const int32_t* in, int32_t* out, int32_t n, int32_t* partials,
                                hipStream_t s) {
  if (n <= 0) return DT_OK;
  int32_t chunk = (n + SCAN_NB - 1) / SCAN_NB;
  hipLaunchKernelGGL(k_scan_reduce, dim3(SCAN_NB), dim3(SCAN_T), 0, s, in, n, chunk, partials);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_NB), 0, s, partials, SCAN_NB);
  hipLaunchKernelGGL(k_scan_apply, dim3(SCAN_NB), dim3(SCAN_T), 0, s, in, out, n, chunk, partials);
  DT_CHECK_LAUNCH();
  return DT_OK;
}

// ------------------------------------------------------------------ C ABI
extern "C" dt_status dt_bvh_bytes(int32_t nv, int32_t nf, size_t* bvh_bytes, size_t* ws_bytes) {
  DT_REQUIRE(nv >= 3 && nf >= 1, "dt_bvh_bytes: need nv >= 3 and nf >= 1 (got %d, %d)", nv, nf);
  DT_REQUIRE(nf <= DT_MAX_FACES && nv < (1 << 30), "dt_bvh_bytes: mesh too large (at most 2^26 triangles)");
  DT_REQUIRE(bvh_bytes && ws_bytes, "dt_bvh_bytes: null output pointer");
  *bvh_bytes = bvh_layout(nv, nf).total;
  Carver c(nullptr, 0);
  *ws_bytes = carve_build(c, nv, nf, nullptr);
  return DT_OK;
}

extern "C" dt_status dt_build_bvh(const float* V, int32_t nv, const int32_t* F, int32_t nf,
                                  void* bvh, size_t bvh_bytes, void* ws, size_t ws_bytes,
                                  void* stream) {
  DT_REQUIRE(V && F && bvh && ws, "dt_build_bvh: null pointer argument");
  DT_REQUIRE(nv >= 3 && nf >= 1, "dt_build_bvh: need nv >= 3 and nf >= 1 (got %d, %d)", nv, nf);
  DT_REQUIRE(nf <= DT_MAX_FACES && nv < (1 << 30), "dt_build_bvh: mesh too large (at most 2^26 triangles)");
  BvhLayout L = bvh_layout(nv, nf);
  if (bvh_bytes < L.total) {
    dt_set_error("dt_build_bvh: bvh blob has %zu bytes, needs %zu", bvh_bytes, L.total);
    return DT_ERR_WORKSPACE_TOO_SMALL;
  }
  Carver c(ws, ws_bytes);
  BuildWs w;
  carve_build(c, nv, nf, &w);
  if (c.overflow) {
    dt_set_error("dt_build_bvh: workspace has %zu bytes, needs %zu", ws_bytes, c.used());
    return DT_ERR_WORKSPACE_TOO_SMALL;
  }
  hipStream_t s = (hipStream_t)stream;
  char* b = (char*)bvh;
  BvhHeader* hdr = (BvhHeader*)(b + L.header);
  BvhNode* nodes = (BvhNode*)(b + L.nodes);
  float4* leaves = (float4*)(b + L.leaves);
  float4* vn = (float4*)(b + L.vnormals);
  float4* fn = (float4*)(b + L.fnormals);
  int32_t* off = (int32_t*)(b + L.csr_off);
  int32_t* idx = (int32_t*)(b + L.csr_idx);
  int32_t* lpar = (int32_t*)(b + L.leaf_parent);

  hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, s, hdr, nv, nf);
  // normals (Eq. 12-13)
  hipLaunchKernelGGL(k_face_normals, dim3(dt_blocks(nf, 256)), dim3(256), 0, s, V, F, nf, nv, fn);
  if (dt_status st = dt_fill_u32((uint32_t*)w.vcnt, 0u, nv, s)) return st;
  if (dt_status st = dt_fill_u32((uint32_t*)w.cursor, 0u, nv, s)) return st;
  hipLaunchKernelGGL(k_vcount, dim3(dt_blocks(nf, 256)), dim3(256), 0, s, F, nf, nv, w.vcnt);
  if (dt_status st = dt_scan_exclusive_i32(w.vcnt, off, nv, w.scanp, s)) return st;
  hipLaunchKernelGGL(k_copy_total, dim3(1), dim3(64), 0, s, w.scanp, SCAN_NB, off + nv);
  hipLaunchKernelGGL(k_vfill, dim3(dt_blocks(nf, 256)), dim3(256), 0, s, F, nf, nv, off, w.cursor,
                     idx);
  hipLaunchKernelGGL(k_vsort, dim3(dt_blocks(nv, 256)), dim3(256), 0, s, off, nv, idx);
  hipLaunchKernelGGL(k_vnormals, dim3(dt_blocks(nv, 256)), dim3(256), 0, s, off, idx, fn, nv, vn);
  DT_CHECK_LAUNCH();
  // Morton codes of face centroids
  hipLaunchKernelGGL(k_bounds, dim3(NBB), dim3(256), 0, s, V, F, nf, nv, w.bpart);
  // up to 2^20 triangles the top 32 bits of the code order them finely enough
  // (ties fall back to the face index) and halve the sort
  const int key_bits = nf <= (1 << 20) ? 32 : 64;
  hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(NBB), 0, s, w.bpart, hdr);
  hipLaunchKernelGGL(k_morton, dim3(dt_blocks(nf, 256)), dim3(256), 0, s, V, F, nf, nv,
                     key_bits == 32 ? 31 : 0, hdr, w.k0, w.v0);
  DT_CHECK_LAUNCH();
  // stable LSD radix sort of (key, face), passes of 8 bits
  int nt = rs_tiles(nf);
  uint64_t *ki = w.k0, *ko = w.k1;
  int32_t *vi = w.v0, *vo = w.v1;
  for (int shift = 0; shift < key_bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nt), dim3(RS_T), 0, s, ki, nf, shift, w.hist, nt);
    if (dt_status st = dt_scan_exclusive_i32(w.hist, w.hist, 256 * nt, w.scanp, s)) return st;
    hipLaunchKernelGGL(k_rs_scatter, dim3(nt), dim3(RS_T), 0, s, ki, vi, ko, vo, nf, shift, w.hist,
                       nt);
    DT_CHECK_LAUNCH();
    uint64_t* tk = ki;
    ki = ko;
    ko = tk;
    int32_t* tv = vi;
    vi = vo;
    vo = tv;
  }
  // tree + boxes
  if (nf > 1) {
    hipLaunchKernelGGL(k_karras, dim3(dt_blocks(nf - 1, 256)), dim3(256), 0, s, ki, nf, nodes, lpar);
    if (dt_status st = dt_fill_u32((uint32_t*)w.arrive, 0u, nf - 1, s)) return st;
    hipLaunchKernelGGL(k_fit_init, dim3(dt_blocks(6 * (int64_t)(nf - 1), 256) < 4096 ?
                                        dt_blocks(6 * (int64_t)(nf - 1), 256) : 4096),
                       dim3(256), 0, s, w.acc, nf - 1);
  }
  hipLaunchKernelGGL(k_fit, dim3(dt_blocks(nf, 256)), dim3(256), 0, s, V, F, nv, vi, nf, nodes,
                     lpar, w.arrive, w.acc, leaves);
  // treelet restructuring: even-depth roots, then odd, twice
  if (nf > 2) {
    for (int pass = 0; pass < TREELET_PASSES; ++pass) {
      hipLaunchKernelGGL(k_even, dim3(dt_blocks(nf - 1, 256)), dim3(256), 0, s, nf - 1, nodes, w.flag4,
                         (BvhHeader*)nullptr);
      hipLaunchKernelGGL(k_treelet, dim3(dt_blocks(nf - 1, 256)), dim3(256), 0, s, nf - 1, nodes, lpar,
                         w.flag4, (pass & 1) == 0 ? 1 : 0);
    }
  }
  DT_CHECK_LAUNCH();
  // 4-wide traversal tree
  if (nf > 1) {
    Bvh4Node* nodes4 = (Bvh4Node*)(b + L.nodes4);
    hipLaunchKernelGGL(k_even, dim3(dt_blocks(nf - 1, 256)), dim3(256), 0, s, nf - 1, nodes, w.flag4,
                       hdr);
    if (dt_status st = dt_scan_exclusive_i32(w.flag4, w.idx4, nf - 1, w.scanp, s)) return st;
    hipLaunchKernelGGL(k_collapse, dim3(dt_blocks(nf - 1, 256)), dim3(256), 0, s, nf - 1, nodes,
                       w.flag4, w.idx4, nodes4, bvh4_cap(nf));
    DT_CHECK_LAUNCH();
  }
  return DT_OK;
}

// ------------------------------------------------------------------ build without allocation
// Build workspace held by the library itself, for callers that cannot
// allocate device memory.  Every GPU the library runs on holds its own copy
// from module load until the process ends.  In host code `scratch` only names
// the array: its device address is looked up once per device and kept in
// g_scratch_ptr, which is what the kernels are given.
static __device__ __align__(256) unsigned char scratch[DT_BVH_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

dt_status scratch_address(void** out) {
  int dev = -1;
  DT_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    dt_set_error("dt_build_bvh_noalloc: device ordinal %d out of range", dev);
    return DT_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    // with device `dev` current: this device's copy of the array
    DT_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DT_OK;
}
}  // namespace

extern "C" dt_status dt_build_bvh_noalloc(const float* V, int32_t nv, const int32_t* F, int32_t nf,
                                          void* bvh, size_t bvh_bytes, void* stream) {
  DT_REQUIRE(V && F && bvh, "dt_build_bvh_noalloc: null pointer argument");
  DT_REQUIRE(nv >= 3 && nf >= 1, "dt_build_bvh_noalloc: need nv >= 3 and nf >= 1 (got %d, %d)", nv,
             nf);
  DT_REQUIRE(nf <= DT_MAX_FACES && nv < (1 << 30),
             "dt_build_bvh_noalloc: mesh too large (at most 2^26 triangles)");
  Carver c(nullptr, 0);
  const size_t need = carve_build(c, nv, nf, nullptr);
  if (need > (size_t)DT_BVH_SCRATCH_BYTES) {
    dt_set_error("dt_build_bvh_noalloc: a mesh of %d vertices and %d faces needs %zu bytes of "
                 "build workspace, more than the library's %zu (use dt_build_bvh with a "
                 "caller-owned workspace)", nv, nf, need, (size_t)DT_BVH_SCRATCH_BYTES);
    return DT_ERR_CAPACITY;
  }
  void* ws = nullptr;
  if (dt_status st = scratch_address(&ws)) return st;
  return dt_build_bvh(V, nv, F, nf, bvh, bvh_bytes, ws, (size_t)DT_BVH_SCRATCH_BYTES, stream);
}

extern "C" dt_status dt_bvh_vertex_normals(const void* bvh, int32_t nv, int32_t nf, float* N,
                                           void* stream) {
  DT_REQUIRE(bvh && N, "dt_bvh_vertex_normals: null pointer argument");
  DT_REQUIRE(nv >= 3 && nf >= 1, "dt_bvh_vertex_normals: need nv >= 3 and nf >= 1");
  BvhView v = bvh_view(bvh, nv, nf);
  hipLaunchKernelGGL(k_copy_vn, dim3(dt_blocks(nv, 256)), dim3(256), 0, (hipStream_t)stream, v.vn, nv,
                     N);
  DT_CHECK_LAUNCH();
  return DT_OK;
}
