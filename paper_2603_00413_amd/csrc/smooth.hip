// The vertex reparameterisation of the mesh optimiser: solves
// (I + lambda L) x = b for the three coordinate columns, L the combinatorial
// Laplacian D - A of the mesh's edge graph, by Chebyshev iteration on the
// device.  The matrix's eigenvalues lie in [1, 1 + lambda m], m = the largest
// d_i + d_j over the edges (i, j) (an upper bound of L's largest eigenvalue,
// Anderson and Morley 1985), and on a known interval the Chebyshev
// recurrence's scalars are fixed numbers, computed on the host: an iteration
// takes no inner product, so it is one kernel (the product with the last
// correction, over an int32 CSR adjacency, and the updates), where conjugate
// gradients need two with a global sum each.  The residual's norm is summed
// every CHECK iterations (block partials, then one block, in a fixed order)
// and read back to stop; the solve is deterministic.
#include "dt_internal.h"

namespace {

constexpr int ST = 256;          // threads per block
constexpr int WAVES = ST / 64;
constexpr int CHECK = 16;        // iterations between residual read-backs

struct SmoothWs {
  double* r;        // [nv][3] residual
  double* d[2];     // [nv][3] corrections: iteration k reads d[k & 1] and writes d[(k + 1) & 1]
  double* part;     // [2][blocks][3] partial b . b and r . r
  int* bmax;        // [blocks] largest d_i + d_j over the block's vertices' edges
  double* sums;     // [8]: b . b, r . r per column; [6] the edge bound m
};

size_t smooth_layout(int32_t nv, SmoothWs* w, char* base) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = dt_align(o + bytes);
    return base ? (double*)(base + at) : nullptr;
  };
  const size_t col = 3 * (size_t)nv * sizeof(double);
  SmoothWs t;
  t.r = take(col);
  t.d[0] = take(col);
  t.d[1] = take(col);
  const size_t nb = dt_blocks(nv, ST);
  t.part = take(6 * nb * sizeof(double));
  t.bmax = (int*)take(nb * sizeof(int));
  t.sums = take(8 * sizeof(double));
  if (w) *w = t;
  return o;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// the block's sums of v[0..2] over its threads, in a fixed order
__device__ __forceinline__ void block_sum3(const double v[3], double out[3]) {
  __shared__ double sh[3][WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double s = wave_sum(v[c]);
    if (lane == 0) sh[c][wv] = s;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) s += sh[c][k];
    out[c] = s;
  }
  __syncthreads();
}

// this block's sums of v[0..2] into part[blockIdx]
__device__ __forceinline__ void block_partial(const double v[3], double* part) {
  double s[3];
  block_sum3(v, s);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) part[3 * blockIdx.x + c] = s[c];
}

// y = (I + lambda L) v at vertex i: (1 + lambda deg) v_i - lambda sum_j v_j
__device__ __forceinline__ void apply_row(const int32_t* off, const int32_t* adj, int i, double lambda,
                                          const double* v, double y[3]) {
  const int a = off[i], e = off[i + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = a; k < e; ++k) {
    const int64_t j = 3 * (int64_t)adj[k];
    s0 += v[j];
    s1 += v[j + 1];
    s2 += v[j + 2];
  }
  const double dg = 1.0 + lambda * (double)(e - a);
  const int64_t i3 = 3 * (int64_t)i;
  y[0] = dg * v[i3] - lambda * s0;
  y[1] = dg * v[i3 + 1] - lambda * s1;
  y[2] = dg * v[i3 + 2] - lambda * s2;
}

// r = b - A x, and a copy of r in d[0] (the first correction is r / theta,
// scaled where it is read); partials of b . b (part[0 .. nb)) and r . r
// (part[nb .. 2 nb))
__global__ void __launch_bounds__(ST) k_sm_init(const int32_t* off, const int32_t* adj, int nv, double lambda,
                                                const double* b, const double* x, SmoothWs w) {
  const int i = blockIdx.x * ST + threadIdx.x;
  double bb[3] = {0.0, 0.0, 0.0}, rr[3] = {0.0, 0.0, 0.0};
  if (i < nv) {
    double ax[3];
    apply_row(off, adj, i, lambda, x, ax);
    for (int c = 0; c < 3; ++c) {
      const int64_t k = 3 * (int64_t)i + c;
      const double r = b[k] - ax[c];
      w.r[k] = r;
      w.d[0][k] = r;
      bb[c] = b[k] * b[k];
      rr[c] = r * r;
    }
  }
  block_partial(bb, w.part);
  block_partial(rr, w.part + 3 * gridDim.x);
}

// per block, the largest d_i + d_j over its vertices' edges (i, j)
__global__ void __launch_bounds__(ST) k_sm_bound(const int32_t* off, const int32_t* adj, int nv, int* bmax) {
  __shared__ int sh[WAVES];
  const int i = blockIdx.x * ST + threadIdx.x;
  int m = 0;
  if (i < nv) {
    const int a = off[i], e = off[i + 1];
    for (int k = a; k < e; ++k) {
      const int j = adj[k];
      m = max(m, (e - a) + (off[j + 1] - off[j]));
    }
  }
  for (int s = 32; s > 0; s >>= 1) m = max(m, __shfl_xor(m, s, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < WAVES; ++k) m = max(m, sh[k]);
    bmax[blockIdx.x] = max(m, sh[0]);
  }
}

// sums[0..3) = sum of part[0 .. nb) (with both), sums[3..6) = sum of
// part[nb .. 2 nb), in block order; with both, sums[6] = the largest bmax
__global__ void __launch_bounds__(ST) k_sm_sums(int nb, int both, SmoothWs w) {
  for (int h = both ? 0 : 1; h < 2; ++h) {
    double a[3] = {0.0, 0.0, 0.0};
    const double* part = w.part + 3 * (size_t)nb * h;
    for (int k = threadIdx.x; k < nb; k += ST)
      for (int c = 0; c < 3; ++c) a[c] += part[3 * k + c];
    double s[3];
    block_sum3(a, s);
    if (threadIdx.x == 0)
      for (int c = 0; c < 3; ++c) w.sums[3 * h + c] = s[c];
  }
  if (both) {
    __shared__ int sh[WAVES];
    int m = 0;
    for (int k = threadIdx.x; k < nb; k += ST) m = max(m, w.bmax[k]);
    for (int s = 32; s > 0; s >>= 1) m = max(m, __shfl_xor(m, s, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = 0; k < WAVES; ++k) m = max(m, sh[k]);
      w.sums[6] = (double)m;
    }
  }
}

// One Chebyshev step: x += d, r -= A d, d' = c1 d + c2 r (the new r); with
// partial, the partials of the new r . r into part[nb .. 2 nb).  first: d
// holds r and the correction is d / theta.
__global__ void __launch_bounds__(ST) k_sm_step(const int32_t* off, const int32_t* adj, int nv, double lambda,
                                                int first, double inv_theta, const double* d, double* dn,
                                                double c1, double c2, double* x, int partial, SmoothWs w) {
  const double* src = d;
  const double sc = first ? inv_theta : 1.0;
  const int i = blockIdx.x * ST + threadIdx.x;
  double rr[3] = {0.0, 0.0, 0.0};
  if (i < nv) {
    double ad[3];
    apply_row(off, adj, i, lambda, src, ad);
    for (int c = 0; c < 3; ++c) {
      const int64_t k = 3 * (int64_t)i + c;
      const double dk = sc * src[k];
      x[k] += dk;
      const double r = w.r[k] - sc * ad[c];
      w.r[k] = r;
      dn[k] = c1 * dk + c2 * r;
      rr[c] = r * r;
    }
  }
  if (partial) block_partial(rr, w.part + 3 * gridDim.x);
}

}  // namespace

extern "C" dt_status dt_smooth_bytes(int32_t nv, size_t* ws_bytes) {
  DT_REQUIRE(ws_bytes, "dt_smooth_bytes: ws_bytes is NULL");
  DT_REQUIRE(nv >= 1 && nv < (1 << 28), "dt_smooth_bytes: nv must be in [1, 2^28) (got %d)", nv);
  *ws_bytes = smooth_layout(nv, nullptr, nullptr);
  return DT_OK;
}

extern "C" dt_status dt_smooth_solve(const int32_t* adj_off, const int32_t* adj, int32_t nv, double lambda,
                                     const double* b, double* x, double tol, int32_t max_iters,
                                     int32_t* iters_out, double* resid_out, void* ws, size_t ws_bytes,
                                     void* stream) {
  DT_REQUIRE(adj_off && adj && b && x && ws, "dt_smooth_solve: a required pointer is NULL");
  DT_REQUIRE(nv >= 1 && nv < (1 << 28), "dt_smooth_solve: nv must be in [1, 2^28) (got %d)", nv);
  DT_REQUIRE(lambda >= 0.0 && tol > 0.0 && max_iters >= 1,
             "dt_smooth_solve: needs lambda >= 0, tol > 0, max_iters >= 1");
  const size_t need = smooth_layout(nv, nullptr, nullptr);
  if (ws_bytes < need) {
    dt_set_error("dt_smooth_solve: workspace has %zu bytes, needs %zu", ws_bytes, need);
    return DT_ERR_WORKSPACE_TOO_SMALL;
  }
  SmoothWs w;
  smooth_layout(nv, &w, (char*)ws);
  hipStream_t s = (hipStream_t)stream;
  const int nb = (int)dt_blocks(nv, ST);
  hipLaunchKernelGGL(k_sm_bound, dim3(nb), dim3(ST), 0, s, adj_off, adj, nv, w.bmax);
  hipLaunchKernelGGL(k_sm_init, dim3(nb), dim3(ST), 0, s, adj_off, adj, nv, lambda, b, x, w);
  hipLaunchKernelGGL(k_sm_sums, dim3(1), dim3(ST), 0, s, nb, 1, w);
  DT_CHECK_LAUNCH();
  double sums[7];
  DT_CHECK_HIP(hipMemcpyAsync(sums, w.sums, sizeof(sums), hipMemcpyDeviceToHost, s));
  DT_CHECK_HIP(hipStreamSynchronize(s));
  // eigenvalues in [1, 1 + lambda m]
  const double lo = 1.0, hi = 1.0 + lambda * sums[6];
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  double b2[3], lim[3];
  for (int c = 0; c < 3; ++c) {
    b2[c] = sums[c] > 1e-300 ? sums[c] : 1e-300;
    lim[c] = tol * tol * b2[c];
  }
  auto within_tol = [&](const double* rr, double& worst) {
    bool ok = true;
    worst = 0.0;
    for (int c = 0; c < 3; ++c) {
      ok = ok && rr[c] <= lim[c];
      worst = fmax(worst, rr[c] / b2[c]);
    }
    return ok;
  };
  double worst = 0.0;
  bool done = within_tol(sums + 3, worst);
  int it = 0;
  // rho_0 = delta / theta, rho_{k+1} = 1 / (2 sigma - rho_k), sigma = theta / delta;
  // d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1} / delta) r_{k+1} (a matrix with
  // one eigenvalue, delta = 0, is solved by the first step alone)
  const bool single = delta <= 1e-12 * theta;
  const double sigma = single ? 0.0 : theta / delta;
  double rho = single ? 0.0 : delta / theta;
  while (!done && it < max_iters) {
    double c1 = 0.0, c2 = 0.0;
    if (!single) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      c1 = rn * rho;
      c2 = 2.0 * rn / delta;
      rho = rn;
    }
    ++it;
    const bool check = it % CHECK == 0 || it == max_iters || single;
    hipLaunchKernelGGL(k_sm_step, dim3(nb), dim3(ST), 0, s, adj_off, adj, nv, lambda, (int)(it == 1),
                       1.0 / theta, w.d[(it - 1) & 1], w.d[it & 1], c1, c2, x, (int)check, w);
    DT_CHECK_LAUNCH();
    if (check) {
      hipLaunchKernelGGL(k_sm_sums, dim3(1), dim3(ST), 0, s, nb, 0, w);
      DT_CHECK_LAUNCH();
      DT_CHECK_HIP(hipMemcpyAsync(sums + 3, w.sums + 3, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
      DT_CHECK_HIP(hipStreamSynchronize(s));
      done = within_tol(sums + 3, worst);
    }
  }
  if (iters_out) *iters_out = it;
  if (resid_out) *resid_out = sqrt(worst);
  if (!done) {
    dt_set_error("dt_smooth_solve: relative residual %.3e above %.1e after %d iterations", sqrt(worst), tol,
                 it);
    return DT_ERR_NOT_CONVERGED;
  }
  return DT_OK;
}
