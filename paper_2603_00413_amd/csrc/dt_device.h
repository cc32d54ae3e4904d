// Device functions of the tracer: closest-hit traversal, environment lookup,
// and the shading step (classification, shading normal, Snell / TIR, Fresnel,
// absorption) shared by the forward kernels and the adjoint.
#pragma once

#include "dt_internal.h"
#include "dt_field.h"

#define DT_PI 3.14159265358979323846f

// ------------------------------------------------------------------ device views
struct EnvDev {
  int kind, W, H;
  const float* tex;
  float* d_tex;  // equirect: dLoss/dtexel target of the backward (may be NULL)
  int n_freq, n_layers, hidden, in_pad;
  const uint16_t* w;
  const float* b;
  float* d_w;    // MLP: dLoss/d(weights, biases) targets of the backward (may be NULL)
  float* d_b;
};

// Spatially varying absorption rate: trilinear RGB grid (mu == NULL: the
// constant rate sigma).  scale = (n - 1) / (hi - lo) grid units per length.
struct AbsorbDev {
  const float* mu;
  float* d_mu;
  int nx, ny, nz, samples;
  float lo[3], scale[3];
};

struct SceneDev {
  const float* V;
  const int32_t* F;
  int nv, nf;
  BvhView bvh;
  const float* ior;
  const float* sigma;
  EnvDev env;
  AbsorbDev ab;
  FieldDev fd;  // volumetric environment field outside the object (fd.grid NULL: none)
  int max_depth, terminal_env;
  float t_eps;
};

// ------------------------------------------------------------------ absorption grid
// Position along one axis in grid units, clamped into [0, n - 1]; the cell
// (at most n - 2), the fraction inside it, and whether the position lies
// strictly inside the box (outside, the clamp is constant: no derivative).
struct GridAxis {
  int i;
  float f;
  bool in;
};

__device__ __forceinline__ GridAxis grid_axis(float x, float lo, float scale, int n) {
  float u = (x - lo) * scale;
  GridAxis a;
  a.in = u > 0.f && u < (float)(n - 1);
  u = fminf(fmaxf(u, 0.f), (float)(n - 1));
  a.i = min((int)u, n - 2);
  a.f = u - (float)a.i;
  return a;
}

// mu_t(x): trilinear blend of the cell's 8 corner nodes
__device__ __forceinline__ v3 grid_mu(const AbsorbDev& G, v3 x) {
  const GridAxis ax = grid_axis(x.x, G.lo[0], G.scale[0], G.nx);
  const GridAxis ay = grid_axis(x.y, G.lo[1], G.scale[1], G.ny);
  const GridAxis az = grid_axis(x.z, G.lo[2], G.scale[2], G.nz);
  const size_t sy = 3 * (size_t)G.nx, sz = sy * (size_t)G.ny;
  const float* b = G.mu + (size_t)az.i * sz + (size_t)ay.i * sy + 3 * (size_t)ax.i;
  v3 acc = mk3(0.f, 0.f, 0.f);
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
    const float w = (dx ? ax.f : 1.f - ax.f) * (dy ? ay.f : 1.f - ay.f) * (dz ? az.f : 1.f - az.f);
    const float* q = b + dz * sz + dy * sy + 3 * dx;
    acc = acc + mk3(q[0], q[1], q[2]) * w;
  }
  return acc;
}

// Optical depth of the segment o + s d, s in [0, t], per channel: the rate at
// the midpoints of samples equal steps, summed, times the step t / samples.
__device__ __forceinline__ v3 absorb_tau(const AbsorbDev& G, v3 o, v3 d, float t) {
  const float h = t / (float)G.samples;
  v3 acc = mk3(0.f, 0.f, 0.f);
  for (int k = 0; k < G.samples; ++k) acc = acc + grid_mu(G, o + d * (h * ((float)k + 0.5f)));
  return acc * h;
}

// ------------------------------------------------------------------ environment (equirect)
// Texel lookup at a direction (normalised here): phi = atan2(x, -z),
// theta = polar angle from +y (computed as atan2(sqrt(x^2+z^2), y), which is
// acos(y) for a unit direction but well conditioned at the poles),
// texel coordinates (uW - 1/2, vH - 1/2) with u = phi/2pi + 1/2, v = theta/pi;
// bilinear, wrap in u, clamp in v.
struct EquirectTap {
  int x0, x1, y0, y1;
  float fx, fy;
  float dphi_dd[3], dth_dd[3];
};

__device__ __forceinline__ void equirect_tap(const EnvDev& e, v3 d, EquirectTap& tp, bool grad) {
  float rho2 = d.x * d.x + d.z * d.z;
  float rho = sqrtf(rho2);
  float phi = atan2f(d.x, -d.z);
  float th = atan2f(rho, d.y);
  float x = (phi * (0.5f / DT_PI) + 0.5f) * (float)e.W - 0.5f;
  float y = th * (1.0f / DT_PI) * (float)e.H - 0.5f;
  if (!(x > -2.0f && x < (float)e.W + 1.0f)) x = 0.0f;  // NaN direction
  if (!(y > -2.0f && y < (float)e.H + 1.0f)) y = 0.0f;
  float xf = floorf(x), yf = floorf(y);
  tp.fx = x - xf;
  tp.fy = y - yf;
  int xi = (int)xf, yi = (int)yf;
  tp.x0 = ((xi % e.W) + e.W) % e.W;
  tp.x1 = (tp.x0 + 1 == e.W) ? 0 : tp.x0 + 1;
  tp.y0 = min(max(yi, 0), e.H - 1);
  tp.y1 = min(max(yi + 1, 0), e.H - 1);
  if (grad) {
    // d phi / d d, d theta / d d (both independent of |d|)
    float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
    float ip = rho2 > 0.f ? 1.0f / rho2 : 0.f;
    tp.dphi_dd[0] = -d.z * ip;
    tp.dphi_dd[1] = 0.f;
    tp.dphi_dd[2] = d.x * ip;
    float ir = rho > 0.f ? 1.0f / (rho * r2) : 0.f;
    tp.dth_dd[0] = d.x * d.y * ir;
    tp.dth_dd[1] = -rho / r2;
    tp.dth_dd[2] = d.z * d.y * ir;
    // clamping in v makes the lookup constant in theta outside the centres
    if (yi < 0 || yi + 1 > e.H - 1) tp.dth_dd[0] = tp.dth_dd[1] = tp.dth_dd[2] = 0.f;
  }
}

__device__ __forceinline__ v3 texel(const EnvDev& e, int y, int x) {
  const float* p = e.tex + ((size_t)y * e.W + x) * 3;
  return mk3(p[0], p[1], p[2]);
}

__device__ __forceinline__ v3 env_equirect(const EnvDev& e, v3 d) {
  EquirectTap tp;
  equirect_tap(e, d, tp, false);
  v3 t00 = texel(e, tp.y0, tp.x0), t01 = texel(e, tp.y0, tp.x1);
  v3 t10 = texel(e, tp.y1, tp.x0), t11 = texel(e, tp.y1, tp.x1);
  float gx = 1.f - tp.fx, gy = 1.f - tp.fy;
  return t00 * (gx * gy) + t01 * (tp.fx * gy) + t10 * (gx * tp.fy) + t11 * (tp.fx * tp.fy);
}

// value and dE/dd^T g (g: upstream adjoint of the RGB value)
__device__ __forceinline__ v3 env_equirect_grad(const EnvDev& e, v3 d, v3 g, v3* dd) {
  EquirectTap tp;
  equirect_tap(e, d, tp, true);
  v3 t00 = texel(e, tp.y0, tp.x0), t01 = texel(e, tp.y0, tp.x1);
  v3 t10 = texel(e, tp.y1, tp.x0), t11 = texel(e, tp.y1, tp.x1);
  float gx = 1.f - tp.fx, gy = 1.f - tp.fy;
  v3 E = t00 * (gx * gy) + t01 * (tp.fx * gy) + t10 * (gx * tp.fy) + t11 * (tp.fx * tp.fy);
  v3 dEdfx = (t01 - t00) * gy + (t11 - t10) * tp.fy;
  v3 dEdfy = (t10 - t00) * gx + (t11 - t01) * tp.fx;
  float sx = dot(g, dEdfx) * ((float)e.W * (0.5f / DT_PI));
  float sy = dot(g, dEdfy) * ((float)e.H / DT_PI);
  *dd = mk3(sx * tp.dphi_dd[0] + sy * tp.dth_dd[0], sx * tp.dphi_dd[1] + sy * tp.dth_dd[1],
            sx * tp.dphi_dd[2] + sy * tp.dth_dd[2]);
  return E;
}

// ------------------------------------------------------------------ closest hit
struct Hit {
  float t, b1, b2;
  int tri;  // original triangle id, -1 = miss
};

struct RayPre {
  v3 o, d;
  v3 inv;  // reciprocal direction (zero components replaced by a tiny value)
  int kx, ky, kz;
  float Sx, Sy, Sz;
};

__device__ __forceinline__ float safe_rcp(float x) {
  const float tiny = 1e-30f;
  float y = fabsf(x) < tiny ? copysignf(tiny, x) : x;
  return 1.0f / y;
}

__device__ __forceinline__ RayPre ray_pre(v3 o, v3 d) {
  RayPre r;
  r.o = o;
  r.d = d;
  r.inv = mk3(safe_rcp(d.x), safe_rcp(d.y), safe_rcp(d.z));
  float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  if (comp(d, kz) < 0.f) {
    int t = kx;
    kx = ky;
    ky = t;
  }
  r.kx = kx;
  r.ky = ky;
  r.kz = kz;
  float dz = comp(d, kz);
  r.Sx = comp(d, kx) / dz;
  r.Sy = comp(d, ky) / dz;
  r.Sz = 1.0f / dz;
  return r;
}

// Watertight ray/triangle test (shear to ray space, signed edge functions,
// FP64 recomputation of edge functions that come out exactly zero); edges
// inclusive, no back-face culling.  Accepts t in (t_eps, tbest]; equal t is
// decided by the triangle id (smaller wins).
__device__ __forceinline__ bool tri_test(const RayPre& r, v3 a, v3 b, v3 c, int tri, float t_eps,
                                         Hit& h) {
  v3 A = a - r.o, B = b - r.o, C = c - r.o;
  float Az = comp(A, r.kz), Bz = comp(B, r.kz), Cz = comp(C, r.kz);
  float Ax = comp(A, r.kx) - r.Sx * Az, Ay = comp(A, r.ky) - r.Sy * Az;
  float Bx = comp(B, r.kx) - r.Sx * Bz, By = comp(B, r.ky) - r.Sy * Bz;
  float Cx = comp(C, r.kx) - r.Sx * Cz, Cy = comp(C, r.ky) - r.Sy * Cz;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.f || V == 0.f || W == 0.f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  if ((U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f)) return false;
  float det = U + V + W;
  if (det == 0.f) return false;
  float T = U * (r.Sz * Az) + V * (r.Sz * Bz) + W * (r.Sz * Cz);
  // one hardware reciprocal (1 ulp) instead of two IEEE divisions: t and the
  // barycentrics carry 2 ulps, the same function on every path (so BVH and
  // brute-force results stay identical), far inside the parity tolerances
  float inv = __builtin_amdgcn_rcpf(det);
  float t = T * inv;
  if (!(t > t_eps) || !(t < INFINITY)) return false;
  if (h.tri >= 0 && (t > h.t || (t == h.t && tri > h.tri))) return false;
  h.t = t;
  h.b1 = V * inv;
  h.b2 = W * inv;
  h.tri = tri;
  return true;
}

#define DT_STACK 64       // total stack entries per lane (LDS part + global overflow part)
#define DT_STACK_LDS 8    // entries kept in LDS by the traversal kernels (4 KB per wave)

// Closest-hit traversal of the 4-wide tree as a resumable per-lane state,
// advanced one node at a time.  The stack holds (node, entry distance) pairs:
// the first SL entries in LDS (stk points at this lane's column, stride
// entries apart), deeper ones in this lane's global overflow area gstk (gcap
// entries; may be NULL when GLOBAL is false).  At a node, the leaf children
// whose boxes the ray enters are handed back for testing; the internal ones
// are ordered by entry distance, the nearest is visited next and the others
// are pushed, farthest first.  A popped subtree whose box is entered beyond
// the closest hit known when it is popped is skipped without fetching its
// node.  overflow is set if the stack would overflow (the result is then
// incomplete and flagged).
struct Trav {
  RayPre r;
  Hit h;
  uint32_t node;
  int sp;
  int skip;
  uint32_t steps;
  bool overflow;
  bool done;
};

__device__ __forceinline__ void trav_init(Trav& s, const BvhView& bv, v3 o, v3 d, int skip,
                                          float t_eps) {
  s.h.tri = -1;
  s.h.t = INFINITY;
  s.h.b1 = s.h.b2 = 0.f;
  s.r = ray_pre(o, d);
  s.node = 0;
  s.sp = 0;
  s.skip = skip;
  s.steps = 0;
  s.overflow = false;
  s.done = false;
  if (bv.nf == 1) {
    const float4* L = bv.leaves;
    int f = __float_as_int(L[0].w);
    if (f != skip) tri_test(s.r, xyz(L[0]), xyz(L[1]), xyz(L[2]), f, t_eps, s.h);
    s.done = true;
  }
}

// One step: visit the current node and choose the next one (or finish).
// Bit k of lm is set for each leaf child k whose box the ray enters, with its
// leaf index in lf[k]; those are left to the caller to test.
template <int SL, bool GLOBAL>
__device__ __forceinline__ void trav_visit(Trav& s, const BvhView& bv, uint2* stk, int stride,
                                           uint2* gstk, int gcap, uint32_t& lm, uint32_t* lf) {
  const uint32_t cap4 = (uint32_t)bvh4_cap(bv.nf);
  const uint32_t lmax = (uint32_t)(bv.nf - 1);
  // a depth-first walk visits each 4-wide node at most once
  if (s.node >= cap4 || ++s.steps > cap4 + 64) {
    s.overflow = true;
    s.done = true;
    return;
  }
  auto push = [&](uint32_t c, float t) {
    uint2 e = make_uint2(c, __float_as_uint(t));
    if (s.sp < SL) {
      stk[s.sp * stride] = e;
      ++s.sp;
    } else if (GLOBAL && s.sp - SL < gcap) {
      if constexpr (GLOBAL) gstk[s.sp - SL] = e;
      ++s.sp;
    } else {
      s.overflow = true;
    }
  };
  const Bvh4Node& n = bv.nodes4[s.node];
  const float4 org = n.org;
  const uint4 ql = n.qlo, qh = n.qhi, cc = n.child;
  // the quantized child boxes: lo = p + qlo s, hi = p + qhi s, s = 2^e per axis
  const uint32_t eb = __float_as_uint(org.w);
  const int ebx = (int)(int8_t)(eb & 0xFFu), eby = (int)(int8_t)((eb >> 8) & 0xFFu);
  const int ebz = (int)(int8_t)((eb >> 16) & 0xFFu);
  // widened like the exit distances (the closest hit's t carries rounding
  // too, and boxes entered at exactly that t must stay in play for ties)
  const float tmaxw = (s.h.tri >= 0 ? s.h.t : INFINITY) * 1.0000008f;
  // Slab distances straight from the codes: the plane p + q s lies at
  // t(q) = (p + q s - o) inv = q a + b with a = s inv (exact, s is a power of
  // two) and b = (p - o) inv, one fused multiply-add per plane.  Against the
  // exact (p + q s - o) / d the computed value is off by at most about
  // 6u (255 |a| + |b|), u = 2^-24 (the roundings of b, of inv, of the fma);
  // each axis's near planes are lowered and far planes raised by
  // 8u (255 |a| + |b|), so near and far distances bound the exact ones from
  // below and above and no box the exact ray enters before the closest hit is
  // rejected.  The near face per axis follows the sign of inv.
  const float ax = ldexpf(s.r.inv.x, ebx), ay = ldexpf(s.r.inv.y, eby), az = ldexpf(s.r.inv.z, ebz);
  const float bx = (org.x - s.r.o.x) * s.r.inv.x;
  const float by = (org.y - s.r.o.y) * s.r.inv.y;
  const float bz = (org.z - s.r.o.z) * s.r.inv.z;
  const float ex = 0x1p-21f * fmaf(255.f, fabsf(ax), fabsf(bx));
  const float ey = 0x1p-21f * fmaf(255.f, fabsf(ay), fabsf(by));
  const float ez = 0x1p-21f * fmaf(255.f, fabsf(az), fabsf(bz));
  const float bnx = bx - ex, bfx = bx + ex, bny = by - ey, bfy = by + ey, bnz = bz - ez, bfz = bz + ez;
  const bool px = s.r.inv.x >= 0.f, py = s.r.inv.y >= 0.f, pz = s.r.inv.z >= 0.f;
  const uint32_t nqx = px ? ql.x : qh.x, fqx = px ? qh.x : ql.x;
  const uint32_t nqy = py ? ql.y : qh.y, fqy = py ? qh.y : ql.y;
  const uint32_t nqz = pz ? ql.z : qh.z, fqz = pz ? qh.z : ql.z;
  float t[4];
  uint32_t c[4] = {cc.x, cc.y, cc.z, cc.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int sh = 8 * k;
    const float tnx = fmaf((float)((nqx >> sh) & 0xFFu), ax, bnx);
    const float tny = fmaf((float)((nqy >> sh) & 0xFFu), ay, bny);
    const float tnz = fmaf((float)((nqz >> sh) & 0xFFu), az, bnz);
    const float tfx = fmaf((float)((fqx >> sh) & 0xFFu), ax, bfx);
    const float tfy = fmaf((float)((fqy >> sh) & 0xFFu), ay, bfy);
    const float tfz = fmaf((float)((fqz >> sh) & 0xFFu), az, bfz);
    const float tn = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, 0.0f));
    const float tf = fminf(fminf(tfx, tfy), fminf(tfz, tmaxw));
    t[k] = tn <= tf ? tn : INFINITY;
  }
  // branch-free split of the entered children into leaves and internal nodes
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool entered = c[k] != DT_NO_CHILD && t[k] != INFINITY;
    const bool is_leaf = entered && (c[k] & DT_LEAF_BIT) != 0u;
    lf[k] = min(c[k] & ~DT_LEAF_BIT, lmax);
    lm |= is_leaf ? (1u << k) : 0u;
    t[k] = entered && !is_leaf ? t[k] : INFINITY;
  }
  // order the entered internal children by entry distance (sorting network)
#define DT_CSWAP(i, j)                 \
  if (t[j] < t[i]) {                   \
    float tt = t[i];                   \
    t[i] = t[j];                       \
    t[j] = tt;                         \
    uint32_t cx = c[i];                \
    c[i] = c[j];                       \
    c[j] = cx;                         \
  }
  DT_CSWAP(0, 1)
  DT_CSWAP(2, 3)
  DT_CSWAP(0, 2)
  DT_CSWAP(1, 3)
  DT_CSWAP(1, 2)
#undef DT_CSWAP
  if (t[0] != INFINITY) {
    if (t[3] != INFINITY) push(c[3], t[3]);
    if (t[2] != INFINITY) push(c[2], t[2]);
    if (t[1] != INFINITY) push(c[1], t[1]);
    s.node = c[0];
    return;
  }
  // pop the nearest pending subtree that can still hold a closer hit
  // (the margin keeps equal-distance ties, decided by triangle id, in play)
  while (s.sp > 0) {
    --s.sp;
    uint2 e = make_uint2(0u, 0u);
    if (s.sp < SL) {
      e = stk[s.sp * stride];
    } else {
      if constexpr (GLOBAL) e = gstk[s.sp - SL];
    }
    if (s.h.tri >= 0 && __uint_as_float(e.y) > s.h.t * 1.000001f) continue;
    s.node = e.x;
    return;
  }
  s.done = true;
}

// Closest hits of a wave's 64 rays, leaf tests batched across the wave.
//
// A lane's ray visits nodes as in trav_visit, but the leaf children it enters
// are not tested in place: a node yields 0-4 of them per lane, so per-child
// tests would run with a handful of the 64 lanes busy.  Instead each candidate
// (leaf index << 6 | lane) goes into a wave-wide LDS queue, and whenever the
// queue holds a full round every lane takes one entry, fetches the owner's
// ray-space constants with cross-lane reads, and runs the triangle test.  A
// hit meets the owner's best so far as the 64-bit key (t bits << 32 | id),
// min-reduced with an LDS atomic: t > 0, so its bit pattern orders like the
// value, and equal t resolves to the smaller id as in tri_test.  The winning
// leaf is noted, and its test is rerun by the owner at the end for the
// barycentrics (the same function on the same operands: bit-identical t).
// Traversal prunes with the best t as of the last round, which is never below
// the final one, so the result is the exact closest hit as before.
//
// Every lane of the wave must call this together (active = false for lanes
// without a ray).  SCENE_PER_LANE: lanes may trace different scenes (the
// owner's leaf array and t_eps travel with the candidate).
#define DT_LQ_CAP 192
struct LeafQueue {
  uint32_t req[DT_LQ_CAP];       // (leaf << 6) | owner lane
  unsigned long long best[64];   // per owner: (t bits << 32) | triangle id
  uint32_t win[64];              // per owner: leaf of the best key
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int SL, bool GLOBAL, bool SCENE_PER_LANE>
__device__ __forceinline__ Hit closest_hit_wave(const BvhView& bv, bool active, v3 o, v3 d,
                                                int skip, float t_eps, uint2* stk, int stride,
                                                uint2* gstk, int gcap, LeafQueue& lq,
                                                bool* overflow) {
  const int lane = (int)(threadIdx.x & 63u);
  const uint64_t lt = (1ull << lane) - 1ull;
  Trav s;
  trav_init(s, bv, o, d, skip, t_eps);
  if (!active) s.done = true;
  lq.best[lane] = ~0ull;
  bool queued = false;  // this lane's best came from the queue
  uint32_t qn = 0;      // queue fill (wave-uniform)
  const int kpack = s.r.kx | (s.r.ky << 2) | (s.r.kz << 4);
  const uint64_t lptr = (uint64_t)(uintptr_t)bv.leaves;

  auto rounds = [&](uint32_t thresh) {
    while (qn >= thresh && qn > 0u) {
      const uint32_t take = qn < 64u ? qn : 64u;
      qn -= take;
      wave_lds_sync();
      const bool has = (uint32_t)lane < take;
      const uint32_t rq = has ? lq.req[qn + (uint32_t)lane] : 0u;
      const int ow = (int)(rq & 63u);
      RayPre r;
      r.o = mk3(__shfl(s.r.o.x, ow), __shfl(s.r.o.y, ow), __shfl(s.r.o.z, ow));
      r.Sx = __shfl(s.r.Sx, ow);
      r.Sy = __shfl(s.r.Sy, ow);
      r.Sz = __shfl(s.r.Sz, ow);
      const int kp = __shfl(kpack, ow);
      r.kx = kp & 3;
      r.ky = (kp >> 2) & 3;
      r.kz = (kp >> 4) & 3;
      const int sk = __shfl(s.skip, ow);
      const float4* L = bv.leaves;
      float te = t_eps;
      if constexpr (SCENE_PER_LANE) {
        const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)lptr, ow);
        const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(lptr >> 32), ow);
        L = (const float4*)(uintptr_t)(((uint64_t)hi << 32) | lo);
        te = __shfl(t_eps, ow);
      }
      if (has) {
        const uint32_t j = rq >> 6;
        const float4 p0 = L[3 * j], p1 = L[3 * j + 1], p2 = L[3 * j + 2];
        const int f = __float_as_int(p0.w);
        Hit h;
        h.tri = -1;
        h.t = INFINITY;
        if (f != sk && tri_test(r, xyz(p0), xyz(p1), xyz(p2), f, te, h)) {
          const unsigned long long key =
              ((unsigned long long)__float_as_uint(h.t) << 32) | (unsigned long long)(uint32_t)f;
          atomicMin(&lq.best[ow], key);
          wave_lds_sync();
          if (lq.best[ow] == key) lq.win[ow] = j;
        }
      }
    }
    wave_lds_sync();
    const unsigned long long kb = lq.best[lane];
    if (kb != ~0ull) {
      s.h.t = __uint_as_float((uint32_t)(kb >> 32));
      s.h.tri = (int)(uint32_t)kb;
      queued = true;
    }
  };

  uint32_t lf[4] = {0u, 0u, 0u, 0u};
  uint32_t lm = 0u;
  auto append = [&](int k) {
    const bool m = (lm >> k) & 1u;
    const uint64_t b = __ballot(m);
    if (m) lq.req[qn + (uint32_t)__popcll(b & lt)] = (lf[k] << 6) | (uint32_t)lane;
    qn += (uint32_t)__popcll(b);
  };

  while (__ballot(!s.done) != 0ull) {
    lm = 0u;
    if (!s.done) trav_visit<SL, GLOBAL>(s, bv, stk, stride, gstk, gcap, lm, lf);
    // at most 63 + 2 * 64 entries are held at any time
    append(0);
    append(1);
    rounds(64u);
    append(2);
    append(3);
    rounds(64u);
  }
  rounds(1u);
  if (s.overflow) *overflow = true;
  Hit h = s.h;
  if (queued) {
    const float4* L = bv.leaves;
    const uint32_t j = lq.win[lane];
    const float4 p0 = L[3 * j];
    Hit r;
    r.tri = -1;
    r.t = INFINITY;
    r.b1 = r.b2 = 0.f;
    tri_test(s.r, xyz(p0), xyz(L[3 * j + 1]), xyz(L[3 * j + 2]), __float_as_int(p0.w), t_eps, r);
    h.b1 = r.b1;
    h.b2 = r.b2;
  }
  return h;
}

// brute force over every triangle with the same predicate
__device__ __forceinline__ Hit closest_brute(const BvhView& bv, v3 o, v3 d, int skip, float t_eps) {
  Hit h;
  h.tri = -1;
  h.t = INFINITY;
  h.b1 = h.b2 = 0.f;
  RayPre r = ray_pre(o, d);
  const float4* L = bv.leaves;
  for (int j = 0; j < bv.nf; ++j) {
    int f = __float_as_int(L[3 * j].w);
    if (f == skip) continue;
    tri_test(r, xyz(L[3 * j]), xyz(L[3 * j + 1]), xyz(L[3 * j + 2]), f, t_eps, h);
  }
  return h;
}

// ------------------------------------------------------------------ shading
// decision bits stored per ray (forward) and re-used by emit / adjoint
#define C_HIT 1u
#define C_ENTER 2u
#define C_TIR 4u
#define C_DEGEN 8u
#define C_TRUNC 16u
#define C_HAS_R 32u
#define C_HAS_T 64u
#define C_GRAZE 128u
#define C_TIRB 256u

struct HitGeo {
  int i0, i1, i2;
  v3 p0, p1, p2;
  v3 n0, n1, n2;
};

__device__ __forceinline__ int vclampi(int i, int nv) { return i < 0 ? 0 : (i >= nv ? nv - 1 : i); }

__device__ __forceinline__ HitGeo load_geo(const SceneDev& sc, int tri) {
  HitGeo g;
  tri = tri < 0 ? 0 : (tri >= sc.nf ? sc.nf - 1 : tri);
  g.i0 = vclampi(sc.F[3 * tri], sc.nv);
  g.i1 = vclampi(sc.F[3 * tri + 1], sc.nv);
  g.i2 = vclampi(sc.F[3 * tri + 2], sc.nv);
  g.p0 = load3(sc.V + 3 * g.i0);
  g.p1 = load3(sc.V + 3 * g.i1);
  g.p2 = load3(sc.V + 3 * g.i2);
  g.n0 = xyz(sc.bvh.vn[g.i0]);
  g.n1 = xyz(sc.bvh.vn[g.i1]);
  g.n2 = xyz(sc.bvh.vn[g.i2]);
  return g;
}

struct Shade {
  v3 x;        // hit point (child origin)
  v3 n;        // oriented unit normal (against the incident ray)
  v3 m;        // unnormalised interpolated normal (smooth case)
  float cos_i;
  float eta, eta_i, eta_t, eta_r;
  float sin2t, cos_t;
  float rs, rp, R, T;
  v3 A;        // attenuation over the segment just travelled
  v3 Cem;      // emission of the field over that segment (exterior segments, FIELD)
  v3 ur, ut;   // unnormalised child directions
  v3 dr, dt;   // unit child directions
  uint32_t code;
};

// Paper Sec. 3.2-3.3.  `code_in` (when nonzero) supplies the discrete
// decisions recorded by the forward pass so that every later recomputation
// takes the same branches.
// GRID: the scene carries an absorption grid; FIELD: a volumetric
// environment field (separate instantiations, so the plain kernels keep their
// register budget)
template <bool GRID = false, bool FIELD = false>
__device__ __forceinline__ Shade shade(const SceneDev& sc, const HitGeo& g, v3 o, v3 d, float t,
                                       float b1, float b2, uint32_t code_in) {
  Shade s;
  s.x = o + d * t;
  v3 ng = cross(g.p1 - g.p0, g.p2 - g.p0);
  bool entering = code_in ? (code_in & C_ENTER) != 0u : dot(d, ng) < 0.f;
  float b0 = 1.f - b1 - b2;
  s.m = g.n0 * b0 + g.n1 * b1 + g.n2 * b2;
  v3 n = normalize3(s.m);
  if (!entering) n = -n;
  float ci = -dot(d, n);
  bool degen = code_in ? (code_in & C_DEGEN) != 0u : !(ci > 0.f);
  if (degen) {
    n = normalize3(ng);
    if (!entering) n = -n;
    ci = -dot(d, n);
  }
  s.n = n;
  s.cos_i = ci;
  s.eta = sc.ior[0];
  s.eta_i = entering ? 1.f : s.eta;
  s.eta_t = entering ? s.eta : 1.f;
  s.eta_r = s.eta_t / s.eta_i;
  s.Cem = mk3(0.f, 0.f, 0.f);
  if (entering) {
    s.A = mk3(1.f, 1.f, 1.f);
    if constexpr (FIELD) {
      // the exterior segment just travelled: its emission, and its
      // transmittance attenuates everything beyond the hit
      float T;
      field_segment(sc.fd, o, d, t, false, s.Cem, T);
      s.A = mk3(T, T, T);
    }
  } else {
    if constexpr (GRID) {
      const v3 tau = absorb_tau(sc.ab, o, d, t);
      s.A = mk3(expf(-tau.x), expf(-tau.y), expf(-tau.z));
    } else {
      s.A = mk3(expf(-sc.sigma[0] * t), expf(-sc.sigma[1] * t), expf(-sc.sigma[2] * t));
    }
  }
  s.sin2t = (1.f - ci * ci) / (s.eta_r * s.eta_r);
  bool tir = code_in ? (code_in & C_TIR) != 0u : s.sin2t > 1.f;
  s.ur = d + n * (2.f * ci);
  s.dr = normalize3(s.ur);
  if (tir) {
    s.cos_t = 0.f;
    s.rs = s.rp = 1.f;
    s.R = 1.f;
    s.T = 0.f;
    s.ut = s.dt = mk3(0.f, 0.f, 0.f);
  } else {
    s.cos_t = sqrtf(fmaxf(1.f - s.sin2t, 0.f));
    float a = s.eta_i * ci, b = s.eta_t * s.cos_t;
    float c = s.eta_i * s.cos_t, e = s.eta_t * ci;
    s.rs = (a - b) / (a + b);
    s.rp = (c - e) / (c + e);
    s.R = 0.5f * (s.rs * s.rs + s.rp * s.rp);
    s.T = 1.f - s.R;
    s.ut = d * (1.f / s.eta_r) + n * (ci / s.eta_r - s.cos_t);
    s.dt = normalize3(s.ut);
  }
  uint32_t code = C_HIT;
  if (entering) code |= C_ENTER;
  if (tir) code |= C_TIR;
  if (degen) code |= C_DEGEN;
  // markers of ill-conditioned hits: cos(theta_i) or cos(theta_t) below 0.1
  if (ci < 0.1f) code |= C_GRAZE;
  if (fabsf(1.f - s.sin2t) < 1e-2f) code |= C_TIRB;
  s.code = code;
  return s;
}
