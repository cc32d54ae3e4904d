// Ray-queue records shared by the wavefront kernels and the environment MLP.
#pragma once

#include "dt_device.h"

constexpr uint32_t RAY_INSIDE = 1u;  // ray flag: travelling inside the object

// One generation of rays, structure of arrays.
struct Gen {
  float4 *o, *d, *w, *hit;  // origin+skip, dir+pixel, weight+flags, (t, tri, b1, b2)
  uint32_t* code;
  int2* child;
};

// Device-side counters of a trace (also the tape header).
struct Counters {
  uint32_t count[DT_MAX_DEPTH + 2];  // rays in generation g
  uint32_t nrefl[DT_MAX_DEPTH + 2];  // reflected children emitted by g (refracted follow them)
  uint32_t work[DT_MAX_DEPTH + 2];   // work-queue cursor of the traversal kernel
  uint32_t hits[DT_MAX_DEPTH + 2];   // rays of g that hit the mesh
  uint32_t nmiss[DT_MAX_DEPTH + 2];  // length of the miss list of g (MLP environment)
  uint32_t dropped;
  uint32_t pad[3];
};

// Adjoint records of one generation.
struct Adj {
  float4 *L, *O, *D;  // subtree radiance, d loss / d origin, d loss / d direction
};

// environment MLP launchers (env_mlp.hip)
bool mlp_supported(const EnvDev& e);
dt_status mlp_query(const EnvDev& e, const float* dirs, int64_t n, float* rgb, hipStream_t s);
dt_status mlp_query_backward(const EnvDev& e, const float* dirs, int64_t n, const float* g,
                             float* gd, hipStream_t s);
// forward: E for the rays on the miss list of generation g, rgb[pixel] += W * E
dt_status mlp_trace_forward(const EnvDev& e, Gen q, const uint32_t* list, const Counters* ctr,
                            int g, int64_t cap, float* rgb, hipStream_t s);
// adjoint: for the rays on the list, L = E(d), D = (dE/dd)^T (dLoss/dC * W), O = 0
dt_status mlp_trace_backward(const EnvDev& e, Gen q, const uint32_t* list, const Counters* ctr,
                             int g, int64_t cap, const float* grad_rgb, Adj cur, hipStream_t s);
