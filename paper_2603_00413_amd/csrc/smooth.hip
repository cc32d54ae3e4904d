// The vertex reparameterisation of the mesh optimiser: solves
// (I + lambda L) x = b for the three coordinate columns, L the combinatorial
// Laplacian D - A of the mesh's edge graph, by conjugate gradients on the
// device, in the Chronopoulos-Gear arrangement (both inner products of an
// iteration taken in one pass, so an iteration needs one global sum):
// w = A r with the partial sums of r . r and w . r per block; then the
// scalars and the updates of p, s = A p, x and r.  Each kernel first sums the
// previous kernel's block partials in a fixed order (every block the same
// way), so the scalars never leave the device and the whole solve is
// deterministic.  The host reads the verdict back every CHECK iterations to
// stop.  (One cooperative launch with grid barriers in place of the kernel
// boundaries measured ten times slower: each barrier has to make every
// block's writes visible across the chip.)
#include "dt_internal.h"

namespace {

constexpr int ST = 256;          // threads per block
constexpr int WAVES = ST / 64;
constexpr int CHECK = 16;        // iterations between residual read-backs

struct SmoothWs {
  double* r;        // [nv][3] residual
  double* w;        // [nv][3] A r
  double* p;        // [nv][3] direction
  double* s;        // [nv][3] A p
  double* part_a;   // [blocks][3] partial r . r
  double* part_b;   // [blocks][3] partial w . r
  double* part_c;   // [blocks][3] partial b . b
  double* sc;       // [2][6] gamma and alpha of the last two iterations
  double* b2;       // [3] b . b
  double* state;    // [4] done, gamma per column (of the last update)
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
  t.w = take(col);
  t.p = take(col);
  t.s = take(col);
  const size_t nb = dt_blocks(nv, ST);
  t.part_a = take(3 * nb * sizeof(double));
  t.part_b = take(3 * nb * sizeof(double));
  t.part_c = take(3 * nb * sizeof(double));
  t.sc = take(12 * sizeof(double));
  t.b2 = take(3 * sizeof(double));
  t.state = take(4 * sizeof(double));
  if (w) *w = t;
  return o;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// the block's sums of v[0..2] over its threads, in a fixed order, into every
// thread's out[0..2]
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

// the sum over blocks of a [blocks][3] partial array, the same bits in every block
__device__ __forceinline__ void sum_partials(const double* part, int nb, double out[3]) {
  double a[3] = {0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < nb; k += ST) {
    a[0] += part[3 * k];
    a[1] += part[3 * k + 1];
    a[2] += part[3 * k + 2];
  }
  block_sum3(a, out);
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

// r = b - A x; partials of b . b
__global__ void __launch_bounds__(ST) k_sm_init(const int32_t* off, const int32_t* adj, int nv, double lambda,
                                                const double* b, const double* x, SmoothWs w) {
  const int i = blockIdx.x * ST + threadIdx.x;
  double bb[3] = {0.0, 0.0, 0.0};
  if (i < nv) {
    double ax[3];
    apply_row(off, adj, i, lambda, x, ax);
    for (int c = 0; c < 3; ++c) {
      const int64_t k = 3 * (int64_t)i + c;
      w.r[k] = b[k] - ax[c];
      bb[c] = b[k] * b[k];
    }
  }
  block_partial(bb, w.part_c);
}

__global__ void __launch_bounds__(ST) k_sm_init_sums(int nb, SmoothWs w) {
  double bb[3];
  sum_partials(w.part_c, nb, bb);
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) w.b2[c] = bb[c];
}

// w = A r; partials of gamma = r . r and delta = w . r
__global__ void __launch_bounds__(ST) k_sm_apply(const int32_t* off, const int32_t* adj, int nv, double lambda,
                                                 SmoothWs w) {
  const int i = blockIdx.x * ST + threadIdx.x;
  double rr[3] = {0.0, 0.0, 0.0}, wr[3] = {0.0, 0.0, 0.0};
  if (i < nv) {
    double y[3];
    apply_row(off, adj, i, lambda, w.r, y);
    for (int c = 0; c < 3; ++c) {
      const int64_t k = 3 * (int64_t)i + c;
      const double r = w.r[k];
      w.w[k] = y[c];
      rr[c] = r * r;
      wr[c] = y[c] * r;
    }
  }
  block_partial(rr, w.part_a);
  block_partial(wr, w.part_b);
}

// Iteration it: gamma = r . r, delta = w . r from the partials; unless every
// column already meets the tolerance (then nothing changes and block 0 marks
// the solve done), beta = gamma / gamma', alpha = gamma / (delta - beta gamma
// / alpha') (alpha = gamma / delta, beta = 0 at it = 0), p = r + beta p,
// s = w + beta s (= A p), x += alpha p, r -= alpha s.  Block 0 keeps gamma and
// alpha in slot it & 1 (every block reads the other slot's).  report_only:
// only the verdict, nothing updated (the iteration budget is spent).
__global__ void __launch_bounds__(ST) k_sm_update(int nv, int nb, int it, double lim0, double lim1, double lim2,
                                                  int report_only, double* x, SmoothWs w) {
  double ga[3], de[3];
  sum_partials(w.part_a, nb, ga);
  sum_partials(w.part_b, nb, de);
  const bool done = ga[0] <= lim0 && ga[1] <= lim1 && ga[2] <= lim2;
  double al[3], be[3];
  const double* prev = w.sc + 6 * ((it + 1) & 1);  // gamma', alpha'
  for (int c = 0; c < 3; ++c) {
    be[c] = it > 0 && prev[c] > 0.0 ? ga[c] / prev[c] : 0.0;
    const double corr = be[c] > 0.0 && prev[3 + c] > 0.0 ? be[c] * ga[c] / prev[3 + c] : 0.0;
    const double den = de[c] - corr;
    al[c] = den > 0.0 ? ga[c] / den : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* cur = w.sc + 6 * (it & 1);
    for (int c = 0; c < 3; ++c) {
      cur[c] = ga[c];
      cur[3 + c] = al[c];
    }
    w.state[0] = done ? 1.0 : 0.0;
    for (int c = 0; c < 3; ++c) w.state[1 + c] = ga[c];
  }
  if (done || report_only) return;
  const int i = blockIdx.x * ST + threadIdx.x;
  if (i < nv)
    for (int c = 0; c < 3; ++c) {
      const int64_t k = 3 * (int64_t)i + c;
      const double r = w.r[k];
      const double pk = it > 0 ? r + be[c] * w.p[k] : r;
      const double sk = it > 0 ? w.w[k] + be[c] * w.s[k] : w.w[k];
      w.p[k] = pk;
      w.s[k] = sk;
      x[k] += al[c] * pk;
      w.r[k] = r - al[c] * sk;
    }
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
  hipLaunchKernelGGL(k_sm_init, dim3(nb), dim3(ST), 0, s, adj_off, adj, nv, lambda, b, x, w);
  hipLaunchKernelGGL(k_sm_init_sums, dim3(1), dim3(ST), 0, s, nb, w);
  hipLaunchKernelGGL(k_sm_apply, dim3(nb), dim3(ST), 0, s, adj_off, adj, nv, lambda, w);
  DT_CHECK_LAUNCH();
  double b2[3], st[4];
  DT_CHECK_HIP(hipMemcpyAsync(b2, w.b2, sizeof(b2), hipMemcpyDeviceToHost, s));
  DT_CHECK_HIP(hipStreamSynchronize(s));
  double lim[3];
  for (int c = 0; c < 3; ++c) {
    b2[c] = b2[c] > 1e-300 ? b2[c] : 1e-300;
    lim[c] = tol * tol * b2[c];
  }
  int it = 0;
  double worst = 0.0;
  bool done = false;
  while (true) {
    // the update finds the residual of `it` iterations and, if it meets the
    // tolerance, stops there; the host reads its verdict at the first
    // iteration, every CHECK iterations and at max_iters
    const bool last = it == max_iters;
    hipLaunchKernelGGL(k_sm_update, dim3(nb), dim3(ST), 0, s, nv, nb, it, lim[0], lim[1], lim[2], (int)last, x,
                       w);
    DT_CHECK_LAUNCH();
    if (it % CHECK == 0 || last) {
      DT_CHECK_HIP(hipMemcpyAsync(st, w.state, sizeof(st), hipMemcpyDeviceToHost, s));
      DT_CHECK_HIP(hipStreamSynchronize(s));
      done = st[0] != 0.0;
      worst = 0.0;
      for (int c = 0; c < 3; ++c) worst = fmax(worst, st[1 + c] / b2[c]);
      if (done || last) break;
    }
    hipLaunchKernelGGL(k_sm_apply, dim3(nb), dim3(ST), 0, s, adj_off, adj, nv, lambda, w);
    DT_CHECK_LAUNCH();
    ++it;
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
