// Volumetric environment field outside the object: the exterior half of the
// sampling split (Sec. 3.3, "Recursive Ray Tracing"), a radiance field of a
// coarse dense grid plus three planes (Sec. 3.1 "Environment Initialization").
//
// Inside the box [lo, hi] the feature of x is the trilinear interpolant of the
// grid plus the bilinear interpolants of the planes over (x, y), (x, z) and
// (y, z), 4 channels each; channel 0 gives the density softplus(f0), 1-3 the
// colour.  An exterior segment is clipped to the box and sampled at the
// midpoints of S equal steps h: a_k = exp(-sigma_k h), T_0 = 1,
// T_{k+1} = T_k a_k, emission C = sum_k T_k (1 - a_k) c_k, and the segment
// passes T_S of what lies beyond it.  The discrete choices (which box faces
// clip, the cell of each sample) are held fixed, as everywhere else.
#pragma once

#include "dt_internal.h"

struct FieldDev {
  const float* grid;    // [nz][ny][nx][4], NULL: no field
  const float* planes;  // [3][res][res][4]
  float* d_grid;        // gradient targets of the backward (may be NULL)
  float* d_planes;
  int nx, ny, nz, res, samples;
  float lo[3], hi[3];
  float sg[3], sp[3];   // node units per length: grid (n - 1)/(hi - lo), planes (res - 1)/(hi - lo)
};

struct FieldAxis {
  int i;
  float f;
};

__device__ __forceinline__ FieldAxis field_axis(float x, float lo, float scale, int n) {
  float u = (x - lo) * scale;
  u = fminf(fmaxf(u, 0.f), (float)(n - 1));
  FieldAxis a;
  a.i = min((int)u, n - 2);
  a.f = u - (float)a.i;
  return a;
}

// Visit the 20 taps of a point: 8 grid nodes and 4 nodes of each plane, as
// fn(parameter index (grid nodes, then plane nodes), weight, the weight's
// gradient in x).  Taps are produced one at a time, so a caller that ignores
// the gradient does not pay for it.
template <class Fn>
__device__ __forceinline__ void field_for_taps(const FieldDev& F, v3 x, Fn&& fn) {
  const float xs[3] = {x.x, x.y, x.z};
  FieldAxis g[3], p[3];
  const int n[3] = {F.nx, F.ny, F.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g[a] = field_axis(xs[a], F.lo[a], F.sg[a], n[a]);
    p[a] = field_axis(xs[a], F.lo[a], F.sp[a], F.res);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
    const float wx = dx ? g[0].f : 1.f - g[0].f, wy = dy ? g[1].f : 1.f - g[1].f;
    const float wz = dz ? g[2].f : 1.f - g[2].f;
    const float sx = dx ? F.sg[0] : -F.sg[0], sy = dy ? F.sg[1] : -F.sg[1], sz = dz ? F.sg[2] : -F.sg[2];
    const int64_t idx = ((int64_t)(g[2].i + dz) * F.ny + (g[1].i + dy)) * F.nx + (g[0].i + dx);
    fn(idx, wx * wy * wz, mk3(sx * wy * wz, wx * sy * wz, wx * wy * sz));
  }
  const int64_t ng = (int64_t)F.nx * F.ny * F.nz;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int a = q == 2 ? 1 : 0, b = q == 0 ? 1 : 2;  // (x, y), (x, z), (y, z)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int di = k & 1, dj = k >> 1;
      const float wa = di ? p[a].f : 1.f - p[a].f, wb = dj ? p[b].f : 1.f - p[b].f;
      const float sa = di ? F.sp[a] : -F.sp[a], sb = dj ? F.sp[b] : -F.sp[b];
      float dw[3] = {0.f, 0.f, 0.f};
      dw[a] = sa * wb;
      dw[b] = wa * sb;
      fn(ng + ((int64_t)q * F.res + (p[b].i + dj)) * F.res + (p[a].i + di), wa * wb,
         mk3(dw[0], dw[1], dw[2]));
    }
  }
}

__device__ __forceinline__ const float* field_param(const FieldDev& F, int64_t k) {
  const int64_t ng = (int64_t)F.nx * F.ny * F.nz;
  return k < ng ? F.grid + 4 * k : F.planes + 4 * (k - ng);
}

__device__ __forceinline__ float* field_dparam(const FieldDev& F, int64_t k) {
  const int64_t ng = (int64_t)F.nx * F.ny * F.nz;
  return k < ng ? F.d_grid + 4 * k : F.d_planes + 4 * (k - ng);
}

__device__ __forceinline__ void field_feature(const FieldDev& F, v3 x, float f[4]) {
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  field_for_taps(F, x, [&](int64_t k, float w, v3) {
    const float4 v = *(const float4*)field_param(F, k);
    a0 += w * v.x;
    a1 += w * v.y;
    a2 += w * v.z;
    a3 += w * v.w;
  });
  f[0] = a0;
  f[1] = a1;
  f[2] = a2;
  f[3] = a3;
}

__device__ __forceinline__ float softplusf(float x) {
  return x > 0.f ? x + log1pf(expf(-x)) : log1pf(expf(x));
}

// The part [s0, s1] of o + s d, s in [0, t_end] (open: s unbounded), inside
// the box; ea / xa: the axis whose face gives s0 / s1 (-1: s0 = 0, or
// s1 = t_end).  False when the segment misses the box.
struct FieldClip {
  float s0, s1;
  int ea, xa;
};

__device__ __forceinline__ bool field_clip(const FieldDev& F, v3 o, v3 d, float t_end, bool open,
                                           FieldClip& c) {
  c.s0 = 0.f;
  c.s1 = t_end;
  c.ea = -1;
  c.xa = -1;
  bool have1 = !open;
  const float os[3] = {o.x, o.y, o.z}, ds[3] = {d.x, d.y, d.z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (ds[a] == 0.f) {
      if (os[a] < F.lo[a] || os[a] > F.hi[a]) return false;
      continue;
    }
    float ta = (F.lo[a] - os[a]) / ds[a], tb = (F.hi[a] - os[a]) / ds[a];
    if (ta > tb) {
      const float tmp = ta;
      ta = tb;
      tb = tmp;
    }
    if (ta > c.s0) {
      c.s0 = ta;
      c.ea = a;
    }
    if (!have1 || tb < c.s1) {
      c.s1 = tb;
      c.xa = a;
      have1 = true;
    }
  }
  return c.s1 > c.s0;
}

// Emission C and transmittance T of an exterior segment.
__device__ __forceinline__ void field_segment(const FieldDev& F, v3 o, v3 d, float t_end, bool open,
                                              v3& C, float& T) {
  C = mk3(0.f, 0.f, 0.f);
  T = 1.f;
  FieldClip cl;
  if (!field_clip(F, o, d, t_end, open, cl)) return;
  const float h = (cl.s1 - cl.s0) / (float)F.samples;
  for (int k = 0; k < F.samples; ++k) {
    float f[4];
    field_feature(F, o + d * (cl.s0 + h * ((float)k + 0.5f)), f);
    const float a = expf(-softplusf(f[0]) * h);
    const float w = T * (1.f - a);
    C = C + mk3(f[1], f[2], f[3]) * w;
    T *= a;
  }
}

// Backward of L = C + T_S M for the upstream gradient Lbar (M: the radiance
// beyond the segment, its own gradient T_S Lbar is the caller's; Ltot = C +
// T_S M, the segment's radiance, which the caller has from field_segment):
// adds the gradients of the origin, the direction and (closed segments
// ending inside the box) of t_end, and scatters the field parameters'
// gradients (float atomics) when the field has gradient targets.
__device__ __forceinline__ void field_segment_bwd(const FieldDev& F, v3 o, v3 d, float t_end, bool open,
                                                  v3 Ltot, v3 Lbar, v3& obar, v3& dbar, float& tbar) {
  FieldClip cl;
  if (!field_clip(F, o, d, t_end, open, cl)) return;
  const int S = F.samples;
  const float h = (cl.s1 - cl.s0) / (float)S;
  // backward, front to back with the running prefix of the emission
  v3 P = mk3(0.f, 0.f, 0.f);
  float Tk = 1.f, hbar = 0.f, s0bar = 0.f;
  for (int k = 0; k < S; ++k) {
    const float sk = cl.s0 + h * ((float)k + 0.5f);
    const v3 xk = o + d * sk;
    // the feature and, per channel, its gradient in x, from one pass over the
    // taps (the feature's operations are field_feature's, so the same bits)
    float f0 = 0.f, f1 = 0.f, f2 = 0.f, f3 = 0.f;
    v3 G0 = mk3(0.f, 0.f, 0.f), G1 = G0, G2 = G0, G3 = G0;
    field_for_taps(F, xk, [&](int64_t j, float wj, v3 dwj) {
      const float4 v = *(const float4*)field_param(F, j);
      f0 += wj * v.x;
      f1 += wj * v.y;
      f2 += wj * v.z;
      f3 += wj * v.w;
      G0 = G0 + dwj * v.x;
      G1 = G1 + dwj * v.y;
      G2 = G2 + dwj * v.z;
      G3 = G3 + dwj * v.w;
    });
    const float f[4] = {f0, f1, f2, f3};
    const float sig = softplusf(f[0]);
    const float a = expf(-sig * h);
    const v3 c = mk3(f[1], f[2], f[3]);
    const float w = Tk * (1.f - a);
    P = P + c * w;
    const float Tn = Tk * a;
    // everything after sample k, and dL/dsigma_k = h (T_{k+1} c_k - after_k) . Lbar
    const v3 after = Ltot - P;
    const float g = dot(Lbar, c * Tn - after);
    const float sigbar = h * g;
    hbar += sig * g;
    const float fb[4] = {sigbar / (1.f + expf(-f[0])), w * Lbar.x, w * Lbar.y, w * Lbar.z};
    const v3 xbar = G0 * fb[0] + G1 * fb[1] + G2 * fb[2] + G3 * fb[3];
    if (F.d_grid)
      field_for_taps(F, xk, [&](int64_t j, float wj, v3) {
        float* q = field_dparam(F, j);
        atomicAdd(q, wj * fb[0]);
        atomicAdd(q + 1, wj * fb[1]);
        atomicAdd(q + 2, wj * fb[2]);
        atomicAdd(q + 3, wj * fb[3]);
      });
    // x_k = o + (s0 + (k + 1/2) h) d
    obar = obar + xbar;
    dbar = dbar + xbar * sk;
    const float dx = dot(d, xbar);
    s0bar += dx;
    hbar += ((float)k + 0.5f) * dx;
    Tk = Tn;
  }
  // h = (s1 - s0) / S
  const float s1bar = hbar / (float)S;
  s0bar -= hbar / (float)S;
  const float os[3] = {o.x, o.y, o.z}, ds[3] = {d.x, d.y, d.z};
  float ob[3] = {0.f, 0.f, 0.f}, db[3] = {0.f, 0.f, 0.f};
  if (cl.ea >= 0) {  // s0 = (face - o_a) / d_a
    ob[cl.ea] -= s0bar / ds[cl.ea];
    db[cl.ea] -= s0bar * cl.s0 / ds[cl.ea];
  }
  if (cl.xa >= 0) {
    ob[cl.xa] -= s1bar / ds[cl.xa];
    db[cl.xa] -= s1bar * cl.s1 / ds[cl.xa];
  } else {
    tbar += s1bar;  // the segment ends at the hit, inside the box
  }
  obar = obar + mk3(ob[0], ob[1], ob[2]);
  dbar = dbar + mk3(db[0], db[1], db[2]);
  (void)os;
}
