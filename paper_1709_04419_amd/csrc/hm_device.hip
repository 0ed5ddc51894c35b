// Device kernels for the H-matrix Gaussian log-likelihood on gfx950.
//
//   matern()            Matern covariance entries, eq. (2) (Section 2.2), with
//                       K_nu by Temme's series (x <= 2) or Steed's evaluation of
//                       the second continued fraction (x > 2), then upward
//                       recurrence in the order.
//   k_assemble_dense    dense leaves of the H-matrix (Section 2.1), nugget on the
//                       diagonal (remark in Section 2.4).
//   k_aca               adaptive cross approximation of admissible blocks
//                       (Section 2.1) followed by SVD truncation at relative
//                       accuracy eps or fixed rank k (Remark 2.4, Definition 2.1).
//   k_level             H-Cholesky (Section 3.2) as a task graph, one launch per
//                       dependency level, one work-group per task.
//   k_level_tasks       forward substitution L v = Z (and the backward one with
//                       L^T) as task graphs of cluster solves and row-chunk products;
//   k_reduce            log|C| = 2 sum log L_ii and v^T v, assembled into eq. (4)
//                       of Section 3.1.
//   k_apply             products with L, L^T and the assembled matrix (simulation
//                       of data, refinement, accuracy diagnostics); k_dense_matvec
//                       the product with the exact covariance.
//
// One work-group = 256 threads = 4 wavefronts of 64.  All floating point is FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "hm_device.h"

namespace hm {

// Threads per work-group (4 wavefronts, one per SIMD: one work-group per CU,
// as the executor's LDS arena takes most of the CU's LDS anyway).
#ifndef HM_NT
#define HM_NT 256
#endif
#define NT HM_NT
#define NW (NT / 64)
// Most columns of a matrix that is truncated in explicit form.
#define CMAX (4 * LEAF_MAX)
// Reflectors per block in the compact WY (I - V T V^T) paths for tall panels.
#define QB 8
__device__ __forceinline__ int64_t clk() { return (int64_t)__builtin_amdgcn_s_memrealtime(); }
// LDS arena (doubles) of the executor work-groups: one per CU.
#define LDS_FACTOR 17408

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the work-group in a fixed order; every thread gets the result.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  // pairwise over the wavefronts, fixed order
  double t[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) t[k] = red[k];
#pragma unroll
  for (int h = 1; h < NW; h <<= 1)
#pragma unroll
    for (int k = 0; k + h < NW; k += 2 * h) t[k] += t[k + h];
  return t[0];
}

// Arg-max of val over the work-group; ties go to the lowest index.
__device__ __forceinline__ void amax_merge(double& v, int64_t& i, double v2, int64_t i2) {
  if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

__device__ void block_argmax(double& v, int64_t& idx, double* redv, int64_t* redi) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double v2 = __shfl_xor(v, o, 64);
    int64_t i2 = __shfl_xor(idx, o, 64);
    amax_merge(v, idx, v2, i2);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) { redv[w] = v; redi[w] = idx; }
  __syncthreads();
  v = redv[0];
  idx = redi[0];
  for (int k = 1; k < NW; ++k) amax_merge(v, idx, redv[k], redi[k]);
}

// ------------------------------------------------------------------ Matern

// K_mu(x), K_{mu+1}(x) for |mu| <= 1/2, 0 < x <= 2: Temme's series.
__device__ void bessel_k_temme(double x, const MaternConst& c, double& k0, double& k1) {
  const double mu = c.mu;
  const double h = 0.5 * x;
  const double lg = -log(h);          // ln(2/x)
  const double s = mu * lg;
  const double shs = (fabs(s) < 1e-300) ? 1.0 : sinh(s) / s;
  double f = c.fact * (cosh(s) * c.g1 + shs * lg * c.g2);
  const double e = exp(s);            // (x/2)^(-mu)
  double p = 0.5 * e * c.gp;
  double q = 0.5 / e * c.gm;
  double ck = 1.0;
  const double y = h * h;
  double sum0 = f, sum1 = p;
  for (int k = 1; k < 60; ++k) {
    const double dk = (double)k;
    f = (dk * f + p + q) / (dk * dk - mu * mu);
    p = p / (dk - mu);
    q = q / (dk + mu);
    ck = ck * y / dk;
    const double t0 = ck * f;
    sum0 += t0;
    sum1 += ck * (p - dk * f);
    if (fabs(t0) < 1e-17 * fabs(sum0)) break;
  }
  k0 = sum0;
  k1 = sum1 * 2.0 / x;
}

// x > 2: Steed's algorithm for the continued fraction CF2 (Temme 1975,
// Thompson & Barnett 1987).  Returns K_mu and K_{mu+1} with the factor
// exp(-x) included.
__device__ void bessel_k_cf2(double x, const MaternConst& c, double& k0, double& k1) {
  const double mu = c.mu;
  double b = 2.0 * (1.0 + x);
  double d = 1.0 / b;
  double h = d, dh = d;
  double q1 = 0.0, q2 = 1.0;
  const double a1 = 0.25 - mu * mu;
  double q = a1, cc = a1, a = -a1;
  double s = 1.0 + q * dh;
  for (int i = 1; i < 2000; ++i) {
    const double di = (double)i;
    a -= 2.0 * di;
    cc = -a * cc / (di + 1.0);
    const double qn = (q1 - b * q2) / a;
    q1 = q2;
    q2 = qn;
    q += cc * qn;
    b += 2.0;
    d = 1.0 / (b + a * d);
    dh = (b * d - 1.0) * dh;
    h += dh;
    const double ds = q * dh;
    s += ds;
    if (fabs(ds) < 1e-17 * fabs(s)) break;
  }
  h = a1 * h;
  k0 = sqrt(M_PI / (2.0 * x)) * exp(-x) / s;
  k1 = k0 * (mu + x + 0.5 - h) / x;
}

// sigma^2 * M_nu(x), x = distance / ell  (no nugget)
__device__ double matern(double x, const MaternConst& c) {
  if (x == 0.0) return c.sigma2;
  if (c.half == 1) return c.sigma2 * exp(-x);
  if (c.half == 3) return c.sigma2 * (1.0 + x) * exp(-x);
  if (c.half == 5) return c.sigma2 * (1.0 + x + x * x * (1.0 / 3.0)) * exp(-x);
  double k0, k1;
  if (x <= 2.0) bessel_k_temme(x, c, k0, k1);
  else bessel_k_cf2(x, c, k0, k1);
  double kn;
  if (c.nrec == 0) {
    kn = k0;
  } else {
    // K_{mu+j+1} = K_{mu+j-1} + 2 (mu + j) / x K_{mu+j}
    double km = k0, kc = k1;
    for (int j = 1; j < c.nrec; ++j) {
      const double kp = km + 2.0 * (c.mu + j) / x * kc;
      km = kc;
      kc = kp;
    }
    kn = kc;
  }
  return c.sigma2 * pow(x, c.nu) * kn * c.norm;
}

__device__ __forceinline__ double entry(const DevData& D, int64_t i, int64_t j) {
  const double dx = D.px[i] - D.px[j];
  const double dy = D.py[i] - D.py[j];
  const double r = sqrt(dx * dx + dy * dy);
  double v = matern(r * D.mc.inv_ell, D.mc);
  if (i == j) v += D.mc.nugget;
  return v;
}

__device__ __forceinline__ double* lr_U(const DevData& D, int32_t b) { return D.lr + D.lr_off[b]; }
__device__ __forceinline__ double* lr_V(const DevData& D, int32_t b) { return D.lr + D.lr_voff[b]; }

// Rounds the rows x cols block A (ld) to FP32 values (the storage precision of
// low-rank factors in the mixed form).
__device__ void round_f32(double* A, int64_t rows, int cols, int64_t ld) {
  for (int64_t e = threadIdx.x; e < rows * (int64_t)cols; e += NT) {
    double* p = A + (e % rows) + (e / rows) * ld;
    *p = (double)(float)*p;
  }
  __syncthreads();
}


// ------------------------------------------------------------------ dense leaves

__global__ void __launch_bounds__(NT) k_assemble_dense(DevData D) {
  for (int32_t q = blockIdx.x; q < D.ndense; q += gridDim.x) {
    const int32_t b = D.dense_ids[q];
    const Block bk = D.bk[b];
    double* out = D.dense + D.dense_off[b];
    const int64_t cnt = bk.m * bk.n;
    for (int64_t e = threadIdx.x; e < cnt; e += NT) {
      const int64_t i = e % bk.m, j = e / bk.m;
      out[e] = entry(D, bk.r0 + i, bk.c0 + j);
    }
  }
}

// ------------------------------------------------------------------ QR / SVD

// Term instances of the current task, resolved (factor pointers, leading
// dimensions, rank and the instance's rectangle), a chunk at a time in LDS.
#define TM_CHUNK 24
struct TermMeta {
  const double* X;
  const double* Y;
  int64_t ldx, ldy, xr0, yr0;
  int32_t lr0, lc0, mx, ny, r, dd;
};

struct Smem {
  TermMeta tm[TM_CHUNK];
  int32_t tm_begin, tm_n;  // instance range held in tm (tm_begin = -1: none)
  double red[NW];
  int64_t redi[NW];
  double tau_x[2 * K_MAX];
  double tau_y[2 * K_MAX];
  double sig[CMAX];
  int32_t ord[CMAX];
  double cn[2][CMAX];      // pivoted QR: partial column norms^2 (by column), by step parity
  int32_t pos[2][CMAX];    // pivoted QR: column at each position, by step parity
  double tau_p[CMAX];      // pivoted QR: reflector coefficients
  double tau_g[CMAX];      // QR of the transposed triangular factor (explicit SVD)
  double Tb[QB][QB];       // compact WY factor of a block of reflectors
  double gp[NW][QB * (QB - 1) / 2];   // per-wave partial Gram entries of that block
  int32_t flag;
  int32_t task;
  int32_t ival[4];
  double dval[4];
  double flops;     // algorithmic flop count of the current task (thread 0 accumulates)
  int64_t ph[5];    // per-task phase clocks (QR, SVD, Q application, solve, explicit formation)
};

// Threads per column when `cols` columns are processed side by side: a power
// of two (<= 64, so a group never straddles a wavefront).
__device__ __forceinline__ int group_size(int cols) {
  int g = 64;
  while (g > 1 && g * cols > NT) g >>= 1;
  return g;
}

// Panels with more rows than these take the wave-per-column QR steps and the
// blocked QR (TALL_QR_ROWS), and the blocked application of Q (TALL_ROWS);
// the pivoted QR takes wave-per-column steps while the columns below the pivot
// row have at least CPQR_WAVE_ROWS entries.
#define CPQR_WAVE_ROWS 96
// Rows per thread loaded together in the passes of the row-stored pivoted QR.
#define CPQR_ROWS_BATCH 32
#define TALL_QR_ROWS 512
#define TALL_ROWS 256

// Lane-strided partial dot product sum_{i = i0, i0 + 64, ... < m} x[i] y[i],
// eight rows in flight (combine across the wave with wave_sum).
__device__ __forceinline__ double wave_rows_dot(const double* x, const double* y, int64_t i0, int64_t m) {
  double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
  int64_t i = i0;
  for (; i + 7 * 64 < m; i += 8 * 64) {
    double xv[8], yv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) { xv[u] = x[i + u * 64]; yv[u] = y[i + u * 64]; }
    d0 += xv[0] * yv[0]; d1 += xv[1] * yv[1]; d2 += xv[2] * yv[2]; d3 += xv[3] * yv[3];
    d0 += xv[4] * yv[4]; d1 += xv[5] * yv[5]; d2 += xv[6] * yv[6]; d3 += xv[7] * yv[7];
  }
  for (; i < m; i += 64) d0 += x[i] * y[i];
  return (d0 + d1) + (d2 + d3);
}

// y[i] += alpha x[i] for the lane's rows i = i0, i0 + 64, ... < m.
__device__ __forceinline__ void wave_rows_axpy(double alpha, const double* x, double* y, int64_t i0, int64_t m) {
  int64_t i = i0;
  for (; i + 7 * 64 < m; i += 8 * 64) {
    double xv[8], yv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) { xv[u] = x[i + u * 64]; yv[u] = y[i + u * 64]; }
#pragma unroll
    for (int u = 0; u < 8; ++u) y[i + u * 64] = yv[u] + alpha * xv[u];
  }
  for (; i < m; i += 64) y[i] += alpha * x[i];
}

// Up to four columns at once (nc <= 4; unused slots alias x and are ignored):
// d[q] = sum over the lane's rows of x[i] y_q[i] and, if want_xx, xx = sum
// x[i]^2; eight rows in flight per column.
__device__ __forceinline__ void wave_rows_dot4(const double* x, const double* const (&y)[4], int nc, int64_t i0,
                                               int64_t m, bool want_xx, double (&d)[4], double& xx) {
  double acc[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  double n0 = 0.0, n1 = 0.0;
  int64_t i = i0;
  for (; i + 7 * 64 < m; i += 8 * 64) {
    double xv[8], yv[4][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = x[i + u * 64];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nc) {
#pragma unroll
        for (int u = 0; u < 8; ++u) yv[q][u] = y[q][i + u * 64];
      }
    if (want_xx) {
#pragma unroll
      for (int u = 0; u < 8; u += 2) { n0 += xv[u] * xv[u]; n1 += xv[u + 1] * xv[u + 1]; }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nc) {
#pragma unroll
        for (int u = 0; u < 8; u += 2) { acc[q][0] += xv[u] * yv[q][u]; acc[q][1] += xv[u + 1] * yv[q][u + 1]; }
      }
  }
  for (; i < m; i += 64) {
    const double xv = x[i];
    if (want_xx) n0 += xv * xv;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nc) acc[q][0] += xv * y[q][i];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) d[q] = acc[q][0] + acc[q][1];
  xx = n0 + n1;
}

// y_q[i] += alpha_q x[i] over the lane's rows, for q < nc (<= 4).
__device__ __forceinline__ void wave_rows_axpy4(const double (&alpha)[4], const double* x, double* const (&y)[4],
                                                int nc, int64_t i0, int64_t m) {
  int64_t i = i0;
  for (; i + 7 * 64 < m; i += 8 * 64) {
    double xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = x[i + u * 64];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nc) {
        double yv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) yv[u] = y[q][i + u * 64];
#pragma unroll
        for (int u = 0; u < 8; ++u) y[q][i + u * 64] = yv[u] + alpha[q] * xv[u];
      }
  }
  for (; i < m; i += 64) {
    const double xv = x[i];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nc) y[q][i] += alpha[q] * xv;
  }
}

// In-place Householder QR of A (m x r, column-major, lda); p = min(m, r)
// reflectors H_j = I - tau_j v_j v_j^T, v_j(j) = 1 implicit, stored below the
// diagonal; R on and above it.
//
// One pass and one barrier per step: the trailing columns are processed side
// by side, a group of g threads per column, and every group forms both its
// column's dot product with the (still unscaled) pivot column and, redundantly,
// the pivot column's norm over the same rows, so the reflector is known to
// every group without a block-wide reduction.  The pivot column itself is
// scaled into v_j at the start of the next step (nobody reads it then).
__device__ void wg_qr(double* A, int64_t m, int r, int64_t lda, double* tau, Smem& S) {
  const int p = (int)(m < r ? m : r);
  const int tid = threadIdx.x;
  if (tid == 0)
    for (int j = 0; j < p; ++j) S.flops += 2.0 * (m - j) + 4.0 * (double)(m - j) * (r - j - 1);
  double prev_scale = 0.0, prev_beta = 0.0;
  for (int j = 0; j < p; ++j) {
    if (j > 0) {
      // deferred: column j-1 becomes v_{j-1}, its diagonal R_{j-1,j-1}
      double* ap = A + (int64_t)(j - 1) * lda;
      if (prev_scale != 0.0)
        for (int64_t i = j + tid; i < m; i += NT) ap[i] *= prev_scale;
      if (tid == 0) ap[j - 1] = prev_beta;
    }
    const double* a = A + (int64_t)j * lda;
    const double alpha = a[j];
    const int C = r - j - 1;
    double s = 0.0, t = 0.0, beta = alpha, scale = 0.0;
    if (C > 0 && m - j > TALL_QR_ROWS) {
      // tall panel: one wavefront per trailing column (each load instruction
      // reads 64 consecutive rows), columns dealt round-robin to the waves;
      // every wave forms the pivot norm itself, over the same rows and order
      // (four columns of a wave at a time; the pivot norm rides on the first
      // batch of every wave)
      const int lane = tid & 63, wv = tid >> 6;
      bool first = true;
      for (int c0 = 4 * wv; first || c0 < C; c0 += 4 * NW) {
        const int nc = (c0 < C) ? ((C - c0 < 4) ? C - c0 : 4) : 0;
        double* cols[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) cols[q] = (q < nc) ? A + (int64_t)(j + 1 + c0 + q) * lda : (double*)a;
        double acj[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acj[q] = (q < nc) ? cols[q][j] : 0.0;
        double dots[4], xx;
        wave_rows_dot4(a, cols, nc, j + 1 + lane, m, first, dots, xx);
        if (first) {
          s = wave_sum(xx);
          if (s != 0.0) {
            beta = -copysign(sqrt(alpha * alpha + s), alpha);
            t = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
          }
          first = false;
        }
        if (nc == 0 || s == 0.0) continue;
        double fs[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double dq = wave_sum(dots[q]);
          const double f = t * (acj[q] + scale * dq);
          if (q < nc && lane == 0) cols[q][j] = acj[q] - f;
          fs[q] = -f * scale;
        }
        wave_rows_axpy4(fs, a, cols, nc, j + 1 + lane, m);
      }
    } else if (C > 0) {
      const int g = group_size(C);
      const int c = tid / g, gl = tid % g;
      // the first C groups own a trailing column each; the remaining (idle)
      // groups only form the pivot norm, over the same row partition
      double* ac = A + (int64_t)(j + 1 + (c < C ? c : 0)) * lda;
      double dot = 0.0, nrm = 0.0, acj = 0.0;
      // eight (then four) rows in flight per iteration; the partial sums are
      // combined in a fixed order, identical in every group
      const int64_t i0 = j + 1 + gl;
      const int64_t g4 = 4 * (int64_t)g, g8 = 8 * (int64_t)g;
      double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0;
      if (c < C) {
        acj = ac[j];
        double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
        int64_t i = i0;
        for (; i + 7 * g < m; i += g8) {
          double x[8], y[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) { x[u] = a[i + u * g]; y[u] = ac[i + u * g]; }
          n0 += x[0] * x[0]; n1 += x[1] * x[1]; n2 += x[2] * x[2]; n3 += x[3] * x[3];
          d0 += x[0] * y[0]; d1 += x[1] * y[1]; d2 += x[2] * y[2]; d3 += x[3] * y[3];
          n0 += x[4] * x[4]; n1 += x[5] * x[5]; n2 += x[6] * x[6]; n3 += x[7] * x[7];
          d0 += x[4] * y[4]; d1 += x[5] * y[5]; d2 += x[6] * y[6]; d3 += x[7] * y[7];
        }
        for (; i + 3 * g < m; i += g4) {
          const double x0 = a[i], x1 = a[i + g], x2 = a[i + 2 * g], x3 = a[i + 3 * g];
          const double y0 = ac[i], y1 = ac[i + g], y2 = ac[i + 2 * g], y3 = ac[i + 3 * g];
          n0 += x0 * x0; n1 += x1 * x1; n2 += x2 * x2; n3 += x3 * x3;
          d0 += x0 * y0; d1 += x1 * y1; d2 += x2 * y2; d3 += x3 * y3;
        }
        for (; i < m; i += g) {
          const double x = a[i];
          n0 += x * x;
          d0 += x * ac[i];
        }
        dot = (d0 + d1) + (d2 + d3);
      } else {
        int64_t i = i0;
        for (; i + 7 * g < m; i += g8) {
          double x[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) x[u] = a[i + u * g];
          n0 += x[0] * x[0]; n1 += x[1] * x[1]; n2 += x[2] * x[2]; n3 += x[3] * x[3];
          n0 += x[4] * x[4]; n1 += x[5] * x[5]; n2 += x[6] * x[6]; n3 += x[7] * x[7];
        }
        for (; i + 3 * g < m; i += g4) {
          const double x0 = a[i], x1 = a[i + g], x2 = a[i + 2 * g], x3 = a[i + 3 * g];
          n0 += x0 * x0; n1 += x1 * x1; n2 += x2 * x2; n3 += x3 * x3;
        }
        for (; i < m; i += g) n0 += a[i] * a[i];
      }
      nrm = (n0 + n1) + (n2 + n3);
      for (int o = 1; o < g; o <<= 1) {
        nrm += __shfl_xor(nrm, o, 64);
        dot += __shfl_xor(dot, o, 64);
      }
      s = nrm;
      if (s != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + s), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
        if (c < C) {
          const double f = t * (acj + scale * dot);
          const double fs = f * scale;
          if (gl == 0) ac[j] -= f;
          int64_t i = i0;
          for (; i + 7 * g < m; i += g8) {
            double x[8], y[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) { x[u] = a[i + u * g]; y[u] = ac[i + u * g]; }
#pragma unroll
            for (int u = 0; u < 8; ++u) ac[i + u * g] = y[u] - fs * x[u];
          }
          for (; i + 3 * g < m; i += g4) {
            const double x0 = a[i], x1 = a[i + g], x2 = a[i + 2 * g], x3 = a[i + 3 * g];
            const double y0 = ac[i], y1 = ac[i + g], y2 = ac[i + 2 * g], y3 = ac[i + 3 * g];
            ac[i] = y0 - fs * x0;
            ac[i + g] = y1 - fs * x1;
            ac[i + 2 * g] = y2 - fs * x2;
            ac[i + 3 * g] = y3 - fs * x3;
          }
          for (; i < m; i += g) ac[i] -= fs * a[i];
        }
      }
    } else {
      double part = 0.0;
      for (int64_t i = j + 1 + tid; i < m; i += NT) part += a[i] * a[i];
      s = block_sum(part, S.red);
      if (s != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + s), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
    }
    if (tid == 0) tau[j] = t;
    prev_scale = (s != 0.0) ? scale : 0.0;
    prev_beta = beta;
    __syncthreads();
  }
  if (p > 0) {
    double* ap = A + (int64_t)(p - 1) * lda;
    if (prev_scale != 0.0)
      for (int64_t i = p + tid; i < m; i += NT) ap[i] *= prev_scale;
    if (tid == 0) ap[p - 1] = prev_beta;
  }
  __syncthreads();
}

// Compact WY factor of reflectors j0 .. j0+nb-1 (nb <= QB; reflector j in
// column pos[j] (or j) of A, v_j(j) = 1 implicit, zero above row j):
//   H_{j0} H_{j0+1} ... H_{j0+nb-1} = I - V T V^T,  T upper triangular (S.Tb),
// built from the Gram matrix V^T V column by column (T(l,l) = tau_l,
// T(0:l,l) = -tau_l T(0:l,0:l) (V^T v_l)(0:l)).  Rows are dealt to the threads;
// the partial Gram entries are combined per wave, then over the waves in a
// fixed order.  Ends with a barrier.
__device__ void wg_block_T(const double* A, int64_t m, int j0, int nb, int64_t lda, const int32_t* pos,
                           const double* tau, Smem& S) {
  constexpr int NP = QB * (QB - 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* v[QB];
#pragma unroll
  for (int l = 0; l < QB; ++l) {
    const int jj = j0 + (l < nb ? l : 0);
    v[l] = A + (int64_t)(pos ? pos[jj] : jj) * lda;
  }
  double g[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) g[q] = 0.0;
  // the triangular rows j0 .. j0+nb-1, then the full rows
  if (tid < nb && j0 + tid < m) {
    const int64_t i = j0 + tid;
    double x[QB];
#pragma unroll
    for (int l = 0; l < QB; ++l) x[l] = (l < nb && i >= j0 + l) ? ((i == j0 + l) ? 1.0 : v[l][i]) : 0.0;
    int q = 0;
#pragma unroll
    for (int l = 0; l < QB; ++l)
#pragma unroll
      for (int l2 = l + 1; l2 < QB; ++l2) g[q++] += x[l] * x[l2];
  }
  for (int64_t i = j0 + nb + tid; i < m; i += NT) {
    double x[QB];
#pragma unroll
    for (int l = 0; l < QB; ++l) x[l] = (l < nb) ? v[l][i] : 0.0;
    int q = 0;
#pragma unroll
    for (int l = 0; l < QB; ++l)
#pragma unroll
      for (int l2 = l + 1; l2 < QB; ++l2) g[q++] += x[l] * x[l2];
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const double t = wave_sum(g[q]);
    if (lane == 0) S.gp[wv][q] = t;
  }
  __syncthreads();
  if (tid == 0) {
    double G[QB][QB];
    int q = 0;
    for (int l = 0; l < QB; ++l)
      for (int l2 = l + 1; l2 < QB; ++l2) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += S.gp[w][q];
        G[l][l2] = t;
        ++q;
      }
    for (int l = 0; l < QB; ++l)
      for (int i = 0; i < QB; ++i) S.Tb[i][l] = 0.0;
    for (int l = 0; l < nb; ++l) {
      const double tl = tau[j0 + l];
      S.Tb[l][l] = tl;
      for (int i = 0; i < l; ++i) {
        double t = 0.0;
        for (int p2 = i; p2 < l; ++p2) t += S.Tb[i][p2] * G[p2][l];
        S.Tb[i][l] = -tl * t;
      }
    }
    S.flops += (double)(m - j0) * nb * (nb - 1);
  }
  __syncthreads();
}

// B <- (I - V T V^T) B (trans = false) or (I - V T^T V^T) B (trans = true) for
// the block of reflectors j0 .. j0+nb-1 with T = S.Tb (wg_block_T); B has k
// columns (ldb) and rows j0 .. m-1 change.  One wavefront per four columns of
// B; row i belongs to lane i mod 64, so no value crosses lanes between blocks.
// Two passes over the rows: W = V^T B, then B -= V (T W).
__device__ void wg_block_apply(const double* A, int64_t m, int j0, int nb, int64_t lda, const int32_t* pos,
                               bool trans, double* B, int k, int64_t ldb, Smem& S) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* v[QB];
#pragma unroll
  for (int l = 0; l < QB; ++l) {
    const int jj = j0 + (l < nb ? l : 0);
    v[l] = A + (int64_t)(pos ? pos[jj] : jj) * lda;
  }
  if (tid == 0) S.flops += 4.0 * (double)(m - j0) * nb * k;
  const int64_t ifirst = j0 + ((lane - j0) & 63);
  for (int c0 = 4 * wv; c0 < k; c0 += 4 * NW) {
    const int nc = (k - c0 < 4) ? k - c0 : 4;
    double* cols[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) cols[q] = B + (int64_t)(c0 + (q < nc ? q : 0)) * ldb;
    double w[QB][4];
#pragma unroll
    for (int l = 0; l < QB; ++l)
#pragma unroll
      for (int q = 0; q < 4; ++q) w[l][q] = 0.0;
    int64_t i = ifirst;
    if (i < j0 + nb && i < m) {
      double x[QB];
#pragma unroll
      for (int l = 0; l < QB; ++l) x[l] = (l < nb && i >= j0 + l) ? ((i == j0 + l) ? 1.0 : v[l][i]) : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nc) {
          const double bq = cols[q][i];
#pragma unroll
          for (int l = 0; l < QB; ++l) w[l][q] += x[l] * bq;
        }
      i += 64;
    }
    for (; i + 64 < m; i += 128) {
      double x0[QB], x1[QB], b0[4], b1[4];
#pragma unroll
      for (int l = 0; l < QB; ++l) { x0[l] = (l < nb) ? v[l][i] : 0.0; x1[l] = (l < nb) ? v[l][i + 64] : 0.0; }
#pragma unroll
      for (int q = 0; q < 4; ++q) { b0[q] = (q < nc) ? cols[q][i] : 0.0; b1[q] = (q < nc) ? cols[q][i + 64] : 0.0; }
#pragma unroll
      for (int l = 0; l < QB; ++l)
#pragma unroll
        for (int q = 0; q < 4; ++q) w[l][q] += x0[l] * b0[q] + x1[l] * b1[q];
    }
    if (i < m) {
      double x[QB];
#pragma unroll
      for (int l = 0; l < QB; ++l) x[l] = (l < nb) ? v[l][i] : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nc) {
          const double bq = cols[q][i];
#pragma unroll
          for (int l = 0; l < QB; ++l) w[l][q] += x[l] * bq;
        }
    }
    // W over the wave, then W' = T W (or T^T W)
    double wt[QB][4];
#pragma unroll
    for (int l = 0; l < QB; ++l)
#pragma unroll
      for (int q = 0; q < 4; ++q) wt[l][q] = wave_sum(w[l][q]);
#pragma unroll
    for (int l = 0; l < QB; ++l)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double t = 0.0;
#pragma unroll
        for (int l2 = 0; l2 < QB; ++l2) t += (trans ? S.Tb[l2][l] : S.Tb[l][l2]) * wt[l2][q];
        w[l][q] = t;
      }
    // B -= V W'
    i = ifirst;
    if (i < j0 + nb && i < m) {
      double x[QB];
#pragma unroll
      for (int l = 0; l < QB; ++l) x[l] = (l < nb && i >= j0 + l) ? ((i == j0 + l) ? 1.0 : v[l][i]) : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nc) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < QB; ++l) t += x[l] * w[l][q];
          cols[q][i] -= t;
        }
      i += 64;
    }
    for (; i < m; i += 64) {
      double x[QB];
#pragma unroll
      for (int l = 0; l < QB; ++l) x[l] = (l < nb) ? v[l][i] : 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nc) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < QB; ++l) t += x[l] * w[l][q];
          cols[q][i] -= t;
        }
    }
  }
}

// Householder QR of a tall A (m > TALL_QR_ROWS) by panels of QB columns: each
// panel by wg_qr, then its reflectors applied to the trailing columns in the
// compact WY form.  Same reflectors, tau and R as wg_qr (up to rounding).
__device__ void wg_qr_blocked(double* A, int64_t m, int r, int64_t lda, double* tau, Smem& S) {
  const int p = (int)(m < r ? m : r);
  for (int j0 = 0; j0 < p; j0 += QB) {
    const int nb = (p - j0 < QB) ? p - j0 : QB;
    wg_qr(A + j0 + (int64_t)j0 * lda, m - j0, nb, lda, tau + j0, S);
    const int kt = r - j0 - nb;
    if (kt > 0) {
      wg_block_T(A, m, j0, nb, lda, nullptr, tau, S);
      wg_block_apply(A, m, j0, nb, lda, nullptr, true, A + (int64_t)(j0 + nb) * lda, kt, lda, S);
      __syncthreads();
    }
  }
}

// B <- Q B with Q = H_0 ... H_{p-1} from wg_qr (B is m x k, ldb).  With a
// column map, reflector j is stored in column pos[j] of A (wg_cpqr).
__device__ void wg_apply_q(const double* A, int64_t m, int p, int64_t lda, const double* tau,
                           double* B, int k, int64_t ldb, Smem& S, const int32_t* pos = nullptr) {
  const int tid = threadIdx.x;
  if (k <= 0) return;
  if (m > TALL_ROWS) {
    // tall: blocks of QB reflectors, last block first, each applied in the
    // compact WY form (two passes over B per block)
    for (int j0 = ((p - 1) / QB) * QB; j0 >= 0; j0 -= QB) {
      const int nb = (p - j0 < QB) ? p - j0 : QB;
      wg_block_T(A, m, j0, nb, lda, pos, tau, S);
      wg_block_apply(A, m, j0, nb, lda, pos, false, B, k, ldb, S);
    }
    __syncthreads();
    return;
  }
  const int g = group_size(k);
  const int c0 = tid / g, gl = tid % g;
  const int cstep = NT / g;
  for (int j = p - 1; j >= 0; --j) {
    const double t = tau[j];
    if (t != 0.0) {
      const double* a = A + (int64_t)(pos ? pos[j] : j) * lda;
      for (int c = c0; c < k; c += cstep) {
        double* bc = B + (int64_t)c * ldb;
        const int64_t i0 = j + 1 + gl;
        const int64_t g4 = 4 * (int64_t)g, g8 = 8 * (int64_t)g;
        double d0 = (gl == 0) ? bc[j] : 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
        int64_t i = i0;
        for (; i + 7 * g < m; i += g8) {
          double x[8], y[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) { x[u] = a[i + u * g]; y[u] = bc[i + u * g]; }
          d0 += x[0] * y[0]; d1 += x[1] * y[1]; d2 += x[2] * y[2]; d3 += x[3] * y[3];
          d0 += x[4] * y[4]; d1 += x[5] * y[5]; d2 += x[6] * y[6]; d3 += x[7] * y[7];
        }
        for (; i + 3 * g < m; i += g4) {
          d0 += a[i] * bc[i];
          d1 += a[i + g] * bc[i + g];
          d2 += a[i + 2 * g] * bc[i + 2 * g];
          d3 += a[i + 3 * g] * bc[i + 3 * g];
        }
        for (; i < m; i += g) d0 += a[i] * bc[i];
        double dot = (d0 + d1) + (d2 + d3);
        for (int o = 1; o < g; o <<= 1) dot += __shfl_xor(dot, o, 64);
        const double f = t * dot;
        if (gl == 0) bc[j] -= f;
        i = i0;
        for (; i + 7 * g < m; i += g8) {
          double x[8], y[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) { x[u] = a[i + u * g]; y[u] = bc[i + u * g]; }
#pragma unroll
          for (int u = 0; u < 8; ++u) bc[i + u * g] = y[u] - f * x[u];
        }
        for (; i + 3 * g < m; i += g4) {
          const double x0 = a[i], x1 = a[i + g], x2 = a[i + 2 * g], x3 = a[i + 3 * g];
          const double y0 = bc[i], y1 = bc[i + g], y2 = bc[i + 2 * g], y3 = bc[i + 3 * g];
          bc[i] = y0 - f * x0;
          bc[i + g] = y1 - f * x1;
          bc[i + 2 * g] = y2 - f * x2;
          bc[i + 3 * g] = y3 - f * x3;
        }
        for (; i < m; i += g) bc[i] -= f * a[i];
      }
    }
    __syncthreads();
  }
}

// One-sided Jacobi on the columns of G (px x py, column-major, ld px):
// on exit G = W Sigma (columns mutually orthogonal).  Round-robin ordering,
// p/2 disjoint column pairs per round, a group of g threads per pair.  A pair
// is rotated when its columns are not orthogonal to 2e-15 sqrt(px) relative;
// columns below 4 max(px,py) eps ||G||_F are numerically zero and are left
// alone (they carry no singular value that any truncation keeps).
__device__ void wg_jacobi(double* G, int px, int py, int ldg, Smem& S) {
  const int tid = threadIdx.x;
  const int q = (py + 1) & ~1;
  if (q < 2) return;
  double f2 = 0.0;
  for (int e = tid; e < px * py; e += NT) f2 += G[(e % px) + (e / px) * ldg] * G[(e % px) + (e / px) * ldg];
  f2 = block_sum(f2, S.red);
  const double epsm = 2.220446049250313e-16;
  const double tnorm = 4.0 * (double)(px > py ? px : py) * epsm;
  const double tiny = tnorm * tnorm * f2;
  const double tol = 2e-15 * sqrt((double)px);
  const int npairs = q / 2;
  const int g = group_size(npairs);
  const int pair = tid / g, gl = tid % g;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) S.flag = 0;
    __syncthreads();
    for (int rnd = 0; rnd < q - 1; ++rnd) {
      if (pair < npairs) {
        int i, j;
        if (pair == 0) { i = rnd; j = q - 1; }
        else { i = (rnd + pair) % (q - 1); j = (rnd - pair + q - 1) % (q - 1); }
        const bool act = (i < py && j < py);
        double al = 0.0, be = 0.0, ga = 0.0;
        double* ci = G + (int64_t)(act ? i : 0) * ldg;
        double* cj = G + (int64_t)(act ? j : 0) * ldg;
        if (act) {
          for (int rr = gl; rr < px; rr += g) {
            const double u = ci[rr], v = cj[rr];
            al += u * u;
            be += v * v;
            ga += u * v;
          }
        }
        for (int o = 1; o < g; o <<= 1) {
          al += __shfl_xor(al, o, 64);
          be += __shfl_xor(be, o, 64);
          ga += __shfl_xor(ga, o, 64);
        }
        if (act && al > tiny && be > tiny && fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double az = fabs(zeta);
          const double t = (az < 1e150) ? copysign(1.0, zeta) / (az + sqrt(1.0 + zeta * zeta)) : 0.5 / zeta;
          const double cs = 1.0 / sqrt(1.0 + t * t);
          const double sn = cs * t;
          for (int rr = gl; rr < px; rr += g) {
            const double u = ci[rr], v = cj[rr];
            ci[rr] = cs * u - sn * v;
            cj[rr] = sn * u + cs * v;
          }
          if (gl == 0) S.flag = 1;
        }
      }
      __syncthreads();
    }
    const int f = S.flag;
    if (tid == 0) S.flops += 12.0 * (double)px * npairs * (q - 1);
    __syncthreads();
    if (!f) break;
  }
}

__device__ __forceinline__ int64_t odd_ld(int64_t rows) { return rows | 1; }

// B <- Q B (wg_apply_q) with the reflectors and B staged through LDS when both
// fit (odd leading dimensions against bank conflicts).
__device__ void wg_apply_q_staged(const double* A, int64_t m, int p, const double* tau, double* B, int k,
                                  double* lds, int lds_cap, Smem& S) {
  const int tid = threadIdx.x;
  if (k <= 0) return;
  const int64_t ld = odd_ld(m);
  if (ld * (p + k) <= lds_cap) {
    double* As = lds;
    double* Bs = lds + ld * p;
    for (int64_t e = tid; e < m * p; e += NT) As[(e % m) + (e / m) * ld] = A[e];
    for (int64_t e = tid; e < m * k; e += NT) Bs[(e % m) + (e / m) * ld] = B[e];
    __syncthreads();
    wg_apply_q(As, m, p, ld, tau, Bs, k, ld, S);
    for (int64_t e = tid; e < m * k; e += NT) B[e] = Bs[(e % m) + (e / m) * ld];
    __syncthreads();
  } else {
    wg_apply_q(A, m, p, m, tau, B, k, m, S);
  }
}

// Householder QR with column pivoting of A (m x n, column-major, lda, n <=
// CMAX), in place and without moving columns.  Step j takes, among the columns
// not yet chosen, the one of largest norm below row j (ties: lowest position in
// the current order) and eliminates it below row j.  The factorisation stops
// before step j once that norm is at most tolrel ||A||_F (tolrel = 0: only at
// an exactly zero remainder).  Returns the number of steps r.  On return
// S.pos[r & 1][q] is the column at position q; reflector j (v_j(j) = 1
// implicit) lies below row j of column pos[j], with S.tau_p[j]; and
// R(i, q) = A(i, pos[q]) for i <= q, i < r.  The discarded remainder (rows >= r
// of the columns at positions >= r) has Frobenius norm at most
// sqrt(n - r) tolrel ||A||_F.
//
// One fused pass and one barrier per step, as in wg_qr: a group of g threads
// per trailing column forms its dot product with the pivot column, the pivot
// column's norm (redundantly, same rows and order in every group), applies the
// reflector and forms the column's new norm below row j.  The pivot order and
// the norms are double-buffered by step parity, so that a step only reads the
// copies written before the previous barrier.
__device__ int wg_cpqr(double* A, int m, int n, int64_t lda, double tolrel, Smem& S) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int p = m < n ? m : n;
  for (int c = wv; c < n; c += NW) {
    const double* ac = A + (int64_t)c * lda;
    double v = 0.0;
    for (int i = lane; i < m; i += 64) v += ac[i] * ac[i];
    v = wave_sum(v);
    if (lane == 0) S.cn[0][c] = v;
  }
  for (int c = tid; c < n; c += NT) S.pos[0][c] = c;
  __syncthreads();
  const double f2 = block_sum(tid < n ? S.cn[0][tid] : 0.0, S.red);
  const double thr = tolrel * tolrel * f2;
  double prev_scale = 0.0, prev_beta = 0.0;
  int prev_col = 0;
  int r = p;
  double flops = 0.0;
  for (int j = 0; j < p; ++j) {
    const int cur = j & 1, nxt = cur ^ 1;
    const int32_t* pos = S.pos[cur];
    const double* cn = S.cn[cur];
    // pivot: each wavefront scans positions j..n-1 and reduces the same way
    double best = -1.0;
    int bq = n;
    for (int q = j + lane; q < n; q += 64) {
      const double v = cn[pos[q]];
      if (v > best) { best = v; bq = q; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double b2 = __shfl_xor(best, o, 64);
      const int q2 = __shfl_xor(bq, o, 64);
      if (b2 > best || (b2 == best && q2 < bq)) { best = b2; bq = q2; }
    }
    if (!(best > thr)) { r = j; break; }
    const int pc = pos[bq], pj = pos[j];
    if (j > 0) {
      // deferred: the previous pivot column becomes v_{j-1}, R_{j-1,j-1}
      double* ap = A + (int64_t)prev_col * lda;
      if (prev_scale != 0.0)
        for (int i = j + tid; i < m; i += NT) ap[i] *= prev_scale;
      if (tid == 0) ap[j - 1] = prev_beta;
    }
    for (int q = tid; q < n; q += NT) S.pos[nxt][q] = (q == j) ? pc : (q == bq) ? pj : pos[q];
    const double* a = A + (int64_t)pc * lda;
    const double alpha = a[j];
    const int C = n - j - 1;
    double sp = 0.0, t = 0.0, beta = alpha, scale = 0.0;
    flops += 2.0 * (m - j) + 6.0 * (double)(m - j) * C;
    if (C > 0 && m - j - 1 >= CPQR_WAVE_ROWS) {
      // long columns: one wavefront per trailing column (each load instruction
      // reads 64 consecutive rows), columns dealt round-robin to the waves;
      // every wave forms the pivot column's norm itself, over the same rows in
      // the same order, so all waves hold the same reflector
      double pl = 0.0;
      for (int i = j + 1 + lane; i < m; i += 64) pl += a[i] * a[i];
      sp = wave_sum(pl);
      if (sp != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + sp), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      // four columns of a wave at a time, so that each row step has five
      // independent loads in flight
      for (int c0 = 4 * wv; c0 < C; c0 += 4 * NW) {
        const int nc = (C - c0 < 4) ? C - c0 : 4;
        double* cols[4];
        int cid[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = j + 1 + c0 + (u < nc ? u : 0);
          cid[u] = (q == bq) ? pj : pos[q];
          cols[u] = A + (int64_t)cid[u] * lda;
        }
        double pn[4] = {0.0, 0.0, 0.0, 0.0};
        if (sp != 0.0) {
          double acj[4], dl[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int u = 0; u < 4; ++u) acj[u] = cols[u][j];
          for (int i = j + 1 + lane; i < m; i += 64) {
            const double ai = a[i];
#pragma unroll
            for (int u = 0; u < 4; ++u) dl[u] += ai * cols[u][i];
          }
          double fs[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double dot = wave_sum(dl[u]);
            const double f = t * (acj[u] + scale * dot);
            fs[u] = f * scale;
            if (lane == 0 && u < nc) cols[u][j] = acj[u] - f;
          }
          for (int i = j + 1 + lane; i < m; i += 64) {
            const double ai = a[i];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (u < nc) {
                const double y = cols[u][i] - fs[u] * ai;
                cols[u][i] = y;
                pn[u] += y * y;
              }
          }
        } else {
          for (int i = j + 1 + lane; i < m; i += 64) {
#pragma unroll
            for (int u = 0; u < 4; ++u) pn[u] += cols[u][i] * cols[u][i];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double v = wave_sum(pn[u]);
          if (lane == 0 && u < nc) S.cn[nxt][cid[u]] = v;
        }
      }
    } else if (C > 0) {
      const int g = group_size(C);
      const int c = tid / g, gl = tid % g;
      const int q = j + 1 + (c < C ? c : 0);
      const int col = (q == bq) ? pj : pos[q];
      double* ac = A + (int64_t)col * lda;
      const int64_t i0 = j + 1 + gl;
      const int64_t g4 = 4 * (int64_t)g;
      double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0;
      double dot = 0.0, acj = 0.0;
      if (c < C) {
        acj = ac[j];
        double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
        int64_t i = i0;
        for (; i + 3 * g < m; i += g4) {
          const double x0 = a[i], x1 = a[i + g], x2 = a[i + 2 * g], x3 = a[i + 3 * g];
          const double y0 = ac[i], y1 = ac[i + g], y2 = ac[i + 2 * g], y3 = ac[i + 3 * g];
          n0 += x0 * x0; n1 += x1 * x1; n2 += x2 * x2; n3 += x3 * x3;
          d0 += x0 * y0; d1 += x1 * y1; d2 += x2 * y2; d3 += x3 * y3;
        }
        for (; i < m; i += g) {
          const double x = a[i];
          n0 += x * x;
          d0 += x * ac[i];
        }
        dot = (d0 + d1) + (d2 + d3);
      } else {
        int64_t i = i0;
        for (; i + 3 * g < m; i += g4) {
          const double x0 = a[i], x1 = a[i + g], x2 = a[i + 2 * g], x3 = a[i + 3 * g];
          n0 += x0 * x0; n1 += x1 * x1; n2 += x2 * x2; n3 += x3 * x3;
        }
        for (; i < m; i += g) n0 += a[i] * a[i];
      }
      double nrm = (n0 + n1) + (n2 + n3);
      for (int o = 1; o < g; o <<= 1) {
        nrm += __shfl_xor(nrm, o, 64);
        dot += __shfl_xor(dot, o, 64);
      }
      sp = nrm;
      if (sp != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + sp), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      if (c < C) {
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
        int64_t i = i0;
        if (sp != 0.0) {
          const double f = t * (acj + scale * dot);
          const double fs = f * scale;
          if (gl == 0) ac[j] = acj - f;
          for (; i + 3 * g < m; i += g4) {
            const double x0 = a[i], x1 = a[i + g], x2 = a[i + 2 * g], x3 = a[i + 3 * g];
            const double y0 = ac[i] - fs * x0, y1 = ac[i + g] - fs * x1;
            const double y2 = ac[i + 2 * g] - fs * x2, y3 = ac[i + 3 * g] - fs * x3;
            ac[i] = y0; ac[i + g] = y1; ac[i + 2 * g] = y2; ac[i + 3 * g] = y3;
            p0 += y0 * y0; p1 += y1 * y1; p2 += y2 * y2; p3 += y3 * y3;
          }
          for (; i < m; i += g) {
            const double y = ac[i] - fs * a[i];
            ac[i] = y;
            p0 += y * y;
          }
        } else {
          for (; i < m; i += g) p0 += ac[i] * ac[i];
        }
        double pn = (p0 + p1) + (p2 + p3);
        for (int o = 1; o < g; o <<= 1) pn += __shfl_xor(pn, o, 64);
        if (gl == 0) S.cn[nxt][col] = pn;
      }
    } else {
      double part = 0.0;
      for (int64_t i = j + 1 + tid; i < m; i += NT) part += a[i] * a[i];
      sp = block_sum(part, S.red);
      if (sp != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + sp), alpha);
        t = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
    }
    if (tid == 0) S.tau_p[j] = t;
    prev_scale = (sp != 0.0) ? scale : 0.0;
    prev_beta = beta;
    prev_col = pc;
    __syncthreads();
  }
  if (r > 0) {
    double* ap = A + (int64_t)prev_col * lda;
    if (prev_scale != 0.0)
      for (int i = r + tid; i < m; i += NT) ap[i] *= prev_scale;
    if (tid == 0) ap[r - 1] = prev_beta;
  }
  if (tid == 0) S.flops += flops;
  __syncthreads();
  return r;
}

// Pivoted QR of a matrix stored by rows (At[c + i ldt] = A(i, c); n <= NT):
// the same steps, pivot rule, stopping rule and outputs as wg_cpqr, with the
// entries of column c at At[c + i ldt].  Thread c owns column c for the whole
// factorisation: it forms the column's dot product with the pivot column, its
// update and its new norm by itself, reading one row of 64 consecutive
// columns per wavefront load, so no step needs a cross-lane reduction except
// the pivot column's norm.  The pivot column is staged in sa (LDS, m doubles);
// piv (LDS, n ints) marks the columns already chosen.
__device__ int wg_cpqr_rows(double* At, int m, int n, int64_t ldt, double tolrel, double* sa, int32_t* piv,
                            Smem& S) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int p = m < n ? m : n;
  const int c = tid;
  const bool own = c < n;
  double* col = At + c;
  if (own) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < m; i += CPQR_ROWS_BATCH) {
      double x[CPQR_ROWS_BATCH];
#pragma unroll
      for (int u = 0; u < CPQR_ROWS_BATCH; ++u) x[u] = (i + u < m) ? col[(int64_t)(i + u) * ldt] : 0.0;
#pragma unroll
      for (int u = 0; u < CPQR_ROWS_BATCH; ++u) v[u & 3] += x[u] * x[u];
    }
    S.cn[0][c] = (v[0] + v[1]) + (v[2] + v[3]);
    S.pos[0][c] = c;
    piv[c] = 0;
  }
  __syncthreads();
  const double f2 = block_sum(own ? S.cn[0][c] : 0.0, S.red);
  const double thr = tolrel * tolrel * f2;
  int r = p;
  double flops = 0.0;
  for (int j = 0; j < p; ++j) {
    const int cur = j & 1, nxt = cur ^ 1;
    const int32_t* pos = S.pos[cur];
    const double* cn = S.cn[cur];
    double best = -1.0;
    int bq = n;
    for (int q = j + lane; q < n; q += 64) {
      const double v = cn[pos[q]];
      if (v > best) { best = v; bq = q; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double b2 = __shfl_xor(best, o, 64);
      const int q2 = __shfl_xor(bq, o, 64);
      if (b2 > best || (b2 == best && q2 < bq)) { best = b2; bq = q2; }
    }
    if (!(best > thr)) { r = j; break; }
    const int pc = pos[bq], pj = pos[j];
    for (int q = tid; q < n; q += NT) S.pos[nxt][q] = (q == j) ? pc : (q == bq) ? pj : pos[q];
    for (int i = j + tid; i < m; i += NT) sa[i] = At[pc + (int64_t)i * ldt];
    __syncthreads();
    const double alpha = sa[j];
    double pl = 0.0;
    for (int i = j + 1 + lane; i < m; i += 64) pl += sa[i] * sa[i];
    const double sp = wave_sum(pl);
    double t = 0.0, beta = alpha, scale = 0.0;
    if (sp != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + sp), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    flops += 2.0 * (m - j) + 6.0 * (double)(m - j) * (n - j - 1);
    if (own && c != pc && !piv[c]) {
      double pn0 = 0.0, pn1 = 0.0, pn2 = 0.0, pn3 = 0.0;
      if (sp != 0.0) {
        const double acj = col[(int64_t)j * ldt];
        // CPQR_ROWS_BATCH rows in flight per thread (a wavefront keeps as many
        // loads of 512 consecutive bytes outstanding)
        // rows past the end of the column load as zero (the batch stays whole)
        double d[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = j + 1; i < m; i += CPQR_ROWS_BATCH) {
          double x[CPQR_ROWS_BATCH];
#pragma unroll
          for (int u = 0; u < CPQR_ROWS_BATCH; ++u) x[u] = (i + u < m) ? col[(int64_t)(i + u) * ldt] : 0.0;
#pragma unroll
          for (int u = 0; u < CPQR_ROWS_BATCH; ++u)
            if (i + u < m) d[u & 3] += sa[i + u] * x[u];
        }
        const double dot = (d[0] + d[1]) + (d[2] + d[3]);
        const double f = t * (acj + scale * dot);
        col[(int64_t)j * ldt] = acj - f;
        const double fs = f * scale;
        for (int i = j + 1; i < m; i += CPQR_ROWS_BATCH) {
          double y[CPQR_ROWS_BATCH];
#pragma unroll
          for (int u = 0; u < CPQR_ROWS_BATCH; ++u) y[u] = (i + u < m) ? col[(int64_t)(i + u) * ldt] : 0.0;
#pragma unroll
          for (int u = 0; u < CPQR_ROWS_BATCH; ++u)
            if (i + u < m) {
              y[u] -= fs * sa[i + u];
              col[(int64_t)(i + u) * ldt] = y[u];
            }
#pragma unroll
          for (int u = 0; u < CPQR_ROWS_BATCH; u += 4) {
            pn0 += y[u] * y[u]; pn1 += y[u + 1] * y[u + 1]; pn2 += y[u + 2] * y[u + 2]; pn3 += y[u + 3] * y[u + 3];
          }
        }
      } else {
        for (int i = j + 1; i < m; i += CPQR_ROWS_BATCH) {
          double y[CPQR_ROWS_BATCH];
#pragma unroll
          for (int u = 0; u < CPQR_ROWS_BATCH; ++u) y[u] = (i + u < m) ? col[(int64_t)(i + u) * ldt] : 0.0;
#pragma unroll
          for (int u = 0; u < CPQR_ROWS_BATCH; u += 4) {
            pn0 += y[u] * y[u]; pn1 += y[u + 1] * y[u + 1]; pn2 += y[u + 2] * y[u + 2]; pn3 += y[u + 3] * y[u + 3];
          }
        }
      }
      S.cn[nxt][c] = (pn0 + pn1) + (pn2 + pn3);
    }
    // the pivot column becomes R(j, j) and, below it, the reflector
    if (tid == 0) {
      At[pc + (int64_t)j * ldt] = beta;
      S.tau_p[j] = t;
      piv[pc] = 1;
    }
    if (sp != 0.0)
      for (int i = j + 1 + tid; i < m; i += NT) At[pc + (int64_t)i * ldt] = sa[i] * scale;
    __syncthreads();
  }
  if (tid == 0) S.flops += flops;
  __syncthreads();
  return r;
}

// Best approximation of an explicit m x n matrix A (lda; destroyed; n <= CMAX)
// at the accuracy of D (relative eps, or the fixed rank), capped at D.kmax.
// Pivoted QR A P = Q R (wg_cpqr; in the accuracy mode stopped at a remainder
// below min(2 max(m,n) u, eps / 1000) ||A||_F, far under what any truncation
// keeps), then one-sided Jacobi on the columns of R^T (n x r): R^T J = W Sigma
// with W orthonormal, so that A = Q [J Sigma; 0] (P W)^T up to the discarded
// remainder.  The Jacobi iteration on the transposed triangular factor of a
// pivoted QR needs a few sweeps where it needs many on A itself.  Writes
//   U (mU x k, ldu):  Q [R W ; 0]            (the singular values ride on U)
//   V (nV x k, ldv):  P W Sigma^{-1}         (orthonormal columns)
// with rows m..mU-1 of U and n..nV-1 of V set to zero; returns k.
// gws: global workspace of at least odd_ld(n) * min(m, n) doubles, used for
// R^T when it does not fit in lds (lds_cap doubles).
__device__ int wg_svd_explicit(const DevData& D, double* A, int m, int n, int64_t lda, double* U, int64_t mU,
                               int64_t ldu, double* V, int64_t nV, int64_t ldv, double* gws, double* lds,
                               int lds_cap, Smem& S, bool timed = false, double* a_spill = nullptr,
                               bool by_rows = false) {
  const int tid = threadIdx.x;
  int64_t c0 = (timed && tid == 0) ? clk() : 0;
  const double u = 2.220446049250313e-16;
  double tolrel = 0.0;
  if (D.kfix <= 0) {
    tolrel = 2.0 * (double)(m > n ? m : n) * u;
    if (1e-3 * D.eps < tolrel) tolrel = 1e-3 * D.eps;
  }
  if (D.mixed) {
    // FP32-valued inputs: below 4 u_32 ||A||_F the remainder is rounding of the
    // inputs (kept under 1e-2 eps, so no singular value that eps keeps is lost)
    double t32 = 4.0 * 5.9604644775390625e-8;
    if (D.kfix <= 0 && 1e-2 * D.eps < t32) t32 = 1e-2 * D.eps;
    if (t32 > tolrel) tolrel = t32;
  }
  const int r = by_rows ? wg_cpqr_rows(A, m, n, lda, tolrel, lds, (int32_t*)(lds + m), S)
                        : wg_cpqr(A, m, n, lda, tolrel, S);
  if (timed && tid == 0) { const int64_t c1 = clk(); S.ph[0] += c1 - c0; c0 = c1; }
  // entry (i, c) of the factored A
  const int64_t si = by_rows ? lda : 1, sc = by_rows ? 1 : lda;
  if (r == 0) return 0;
  const int32_t* pos = S.pos[r & 1];
  const int ldg = (int)odd_ld(n);
  if (a_spill && (int64_t)ldg * r > lds_cap && (int64_t)ldg * r <= lds_cap + lda * n) {
    // A sits in LDS just below `lds`: move it to global memory so that the
    // Jacobi iteration gets the whole arena
    double* src = A;
    for (int64_t e = tid; e < lda * n; e += NT) a_spill[e] = src[e];
    __syncthreads();
    A = a_spill;
    lds = src;
    lds_cap += (int)(lda * n);
  }
  double* G = ((int64_t)ldg * r <= lds_cap) ? lds : gws;
  for (int e = tid; e < n * r; e += NT) {
    const int q = e % n, i = e / n;
    G[q + i * ldg] = (i <= q) ? A[i * si + (int64_t)pos[q] * sc] : 0.0;
  }
  __syncthreads();
  // With r well below n: QR of R^T = Q2 [R2; 0] first, and the Jacobi
  // iteration on the r x r factor R2 (R2 J = X Sigma, so that R^T J = Q2 [X; 0]
  // Sigma): the same rotations (R2 has the Gram matrix of R^T), on r rows
  // instead of n.  R2 and the reflectors go to gws (odd_ld(n) r doubles, within
  // its stated size).
  const int ldm = (int)odd_ld(r);
  const bool precond = n >= 2 * r && r >= 8 && (int64_t)ldm * r + odd_ld(n) <= lds_cap;
  double* M = lds;
  double* Gq = G;
  if (precond) {
    wg_qr(G, n, r, ldg, S.tau_g, S);
    if (G != gws) {
      // R2 and the reflectors to global memory: LDS is for the r x r iteration
      for (int e = tid; e < ldg * r; e += NT) gws[e] = G[e];
      __syncthreads();
      Gq = gws;
    }
    for (int e = tid; e < r * r; e += NT) {
      const int i = e % r, j = e / r;
      M[i + j * ldm] = (i <= j) ? Gq[i + (int64_t)j * ldg] : 0.0;
    }
    __syncthreads();
    wg_jacobi(M, r, r, ldm, S);
    for (int l = tid; l < r; l += NT) {
      double sq = 0.0;
      for (int q = 0; q < r; ++q) sq += M[q + l * ldm] * M[q + l * ldm];
      S.sig[l] = sqrt(sq);
    }
  } else {
    wg_jacobi(G, n, r, ldg, S);
    for (int l = tid; l < r; l += NT) {
      double sq = 0.0;
      for (int q = 0; q < n; ++q) sq += G[q + l * ldg] * G[q + l * ldg];
      S.sig[l] = sqrt(sq);
    }
  }
  __syncthreads();
  for (int l = tid; l < r; l += NT) {
    int rk = 0;
    const double sl = S.sig[l];
    for (int i = 0; i < r; ++i) {
      const double si = S.sig[i];
      if (si > sl || (si == sl && i < l)) ++rk;
    }
    S.ord[rk] = l;
  }
  __syncthreads();
  if (timed && tid == 0) { const int64_t c1 = clk(); S.ph[1] += c1 - c0; c0 = c1; }
  const double s1 = S.sig[S.ord[0]];
  int k = 0;
  if (s1 > 0.0) {
    if (D.kfix > 0) {
      for (int l = 0; l < r; ++l) if (S.sig[S.ord[l]] > 0.0) ++k;
      if (k > D.kfix) k = D.kfix;
    } else {
      for (int l = 0; l < r; ++l) if (S.sig[S.ord[l]] > D.eps * s1) ++k;
      if (k > D.kmax && tid == 0) atomicAdd(D.capped, 1);   // the cap binds: this block misses eps
    }
    if (k > D.kmax) k = D.kmax;
  }
  // V(pos[q], l) = G(q, o_l) / sigma_l
  for (int64_t e = tid; e < nV * k; e += NT) {
    const int64_t c = e % nV;
    const int l = (int)(e / nV);
    V[c + l * ldv] = 0.0;
  }
  __syncthreads();
  if (precond) {
    // V(pos[q], l) = (Q2 [X(:, o_l); 0])(q), in column chunks staged in LDS
    const int ldb = (int)odd_ld(n);
    double* Bc = M + (int64_t)ldm * r;
    int kc = (lds_cap - ldm * r) / ldb;
    if (kc > k) kc = k;
    for (int l0 = 0; l0 < k; l0 += kc) {
      const int nb = (k - l0 < kc) ? k - l0 : kc;
      for (int e = tid; e < n * nb; e += NT) {
        const int q = e % n, l = e / n;
        const int o = S.ord[l0 + l];
        Bc[q + l * ldb] = (q < r) ? M[q + o * ldm] / S.sig[o] : 0.0;
      }
      __syncthreads();
      wg_apply_q(Gq, n, r, ldg, S.tau_g, Bc, nb, ldb, S);
      for (int e = tid; e < n * nb; e += NT) {
        const int q = e % n, l = e / n;
        V[pos[q] + (int64_t)(l0 + l) * ldv] = Bc[q + l * ldb];
      }
      __syncthreads();
    }
    // U(:, l) = R W(:, l) = R2^T X(:, o_l), zero below row r
    for (int64_t e = tid; e < mU * k; e += NT) {
      const int64_t i = e % mU;
      const int l = (int)(e / mU);
      double acc = 0.0;
      if (i < r) {
        const int o = S.ord[l];
        for (int j = 0; j <= (int)i; ++j) acc += Gq[j + i * ldg] * M[j + o * ldm];
        acc /= S.sig[o];
      }
      U[i + l * ldu] = acc;
    }
  } else {
    for (int e = tid; e < n * k; e += NT) {
      const int q = e % n, l = e / n;
      const int o = S.ord[l];
      V[pos[q] + l * ldv] = G[q + o * ldg] / S.sig[o];
    }
    // U(i, l) = (R G(:, o_l))_i / sigma_l for i < r, zero below
    for (int64_t e = tid; e < mU * k; e += NT) {
      const int64_t i = e % mU;
      const int l = (int)(e / mU);
      double acc = 0.0;
      if (i < r) {
        const int o = S.ord[l];
        for (int q = (int)i; q < n; ++q) acc += A[i * si + (int64_t)pos[q] * sc] * G[q + o * ldg];
        acc /= S.sig[o];
      }
      U[i + l * ldu] = acc;
    }
  }
  __syncthreads();
  if (tid == 0) {
    double f = 2.0 * (double)r * n * k;
    for (int j = 0; j < r; ++j) f += 4.0 * (double)(m - j) * k;
    S.flops += f;
  }
  if (by_rows) {
    // reflector j lies in column pos[j] below row j: gather the reflectors
    // into columns (LDS when they fit; G is no longer needed)
    const int64_t ldr = odd_ld(m);
    double* Vr = (ldr * r <= lds_cap) ? lds : gws;
    for (int e = tid; e < m * r; e += NT) {
      const int i = e % m, j = e / m;
      Vr[i + j * ldr] = (i > j) ? A[(int64_t)i * lda + pos[j]] : 0.0;
    }
    __syncthreads();
    wg_apply_q(Vr, m, r, ldr, S.tau_p, U, k, ldu, S);
  } else {
    wg_apply_q(A, m, r, lda, S.tau_p, U, k, ldu, S, pos);
  }
  if (timed && tid == 0) S.ph[2] += clk() - c0;
  return k;
}

// Best approximation of X Y^T (X: m x r, Y: n x r, in workspace, destroyed) at
// relative accuracy eps (kfix == 0) or rank kfix, capped at kmax: Householder
// QR of both factors, the small core Rx Ry^T truncated by wg_svd_explicit, and
// its factors mapped back through the reflectors.  Writes U (m x k, ldu = m)
// and V (n x k, ldv = n); returns k.
// work: at least 2 (r + 1) r doubles of global workspace.
__device__ int wg_truncate(const DevData& D, double* X, int64_t m, double* Y, int64_t n, int r,
                           double* U, double* V, double* work, double* lds_g, int lds_cap, Smem& S) {
  const int tid = threadIdx.x;
  if (r == 0) return 0;
  int64_t c0 = (tid == 0) ? clk() : 0;
  // QR of each factor, staged through LDS when it fits (copy in, factor, copy back)
  for (int side = 0; side < 2; ++side) {
    double* A = side ? Y : X;
    const int64_t rows = side ? n : m;
    double* tau = side ? S.tau_y : S.tau_x;
    const int64_t ld = odd_ld(rows);
    if (ld * (int64_t)r <= lds_cap) {
      for (int64_t e = tid; e < rows * r; e += NT) lds_g[(e % rows) + (e / rows) * ld] = A[e];
      __syncthreads();
      wg_qr(lds_g, rows, r, ld, tau, S);
      for (int64_t e = tid; e < rows * r; e += NT) A[e] = lds_g[(e % rows) + (e / rows) * ld];
      __syncthreads();
    } else if (rows > TALL_QR_ROWS) {
      wg_qr_blocked(A, rows, r, rows, tau, S);
    } else {
      wg_qr(A, rows, r, rows, tau, S);
    }
  }
  const int px = (int)(m < r ? m : r), py = (int)(n < r ? n : r);
  // M = Rx Ry^T (px x py), in LDS when it fits
  const int ldm = (int)odd_ld(px);
  const bool m_lds = (int64_t)ldm * py <= lds_cap;
  double* M = m_lds ? lds_g : work;
  for (int e = tid; e < px * py; e += NT) {
    const int i = e % px, j = e / px;
    const int l0 = i > j ? i : j;
    double acc = 0.0;
    for (int l = l0; l < r; ++l) acc += X[i + (int64_t)l * m] * Y[j + (int64_t)l * n];
    M[i + j * ldm] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    S.flops += 2.0 * px * py * r;
    const int64_t c1 = clk();
    S.ph[0] += c1 - c0;
    c0 = c1;
  }
  // core: U = [Uc ; 0], V = [Vc ; 0] with Uc Vc^T the best approximation of M
  double* gl_lds = m_lds ? lds_g + (int64_t)ldm * py : lds_g;
  const int gl_cap = m_lds ? lds_cap - ldm * py : lds_cap;
  double* gws = m_lds ? work : work + (int64_t)ldm * py;
  const int k = wg_svd_explicit(D, M, px, py, ldm, U, m, m, V, n, n, gws, gl_lds, gl_cap, S);
  if (tid == 0) { const int64_t c1 = clk(); S.ph[1] += c1 - c0; c0 = c1; }
  __syncthreads();
  if (tid == 0) {
    double f = 0.0;
    for (int j = 0; j < px; ++j) f += 4.0 * (double)(m - j) * k;
    for (int j = 0; j < py; ++j) f += 4.0 * (double)(n - j) * k;
    S.flops += f;
  }
  wg_apply_q_staged(X, m, px, S.tau_x, U, k, lds_g, lds_cap, S);
  wg_apply_q_staged(Y, n, py, S.tau_y, V, k, lds_g, lds_cap, S);
  __syncthreads();
  if (tid == 0) S.ph[2] += clk() - c0;
  return k;
}

// ------------------------------------------------------------------ ACA

// ACA factors Ua (m x kmax), Va (n x kmax): in the workspace slot, or for a
// big block (storage of 2 K_MAX columns) in the upper half of its own storage,
// so that the truncation writes U, V into the lower half.  Then used flags (m
// as doubles) and work for the truncation in the slot.
__global__ void __launch_bounds__(NT) k_aca(DevData D) {
  extern __shared__ double dyn[];
  __shared__ Smem S;
  const int tid = threadIdx.x;
  double* slot = D.ws + (int64_t)blockIdx.x * D.ws_stride;
  for (int32_t q = blockIdx.x; q < D.nlr; q += gridDim.x) {
    const int32_t b = D.lr_ids[q];
    const Block bk = D.bk[b];
    const int64_t m = bk.m, n = bk.n;
    const int kcap = (int)((D.kmax < m) ? ((D.kmax < n) ? D.kmax : n) : ((m < n) ? m : n));
    const bool big = D.lr_cap[b] == 2 * K_MAX;
    double* Ua = big ? lr_U(D, b) + m * K_MAX : slot;
    double* Va = big ? lr_V(D, b) + n * K_MAX : Ua + m * K_MAX;
    double* used = big ? slot : Va + n * K_MAX;
    double* work = used + m;
    for (int64_t i = tid; i < m; i += NT) used[i] = 0.0;
    __syncthreads();
    int k = 0;
    int64_t istar = 0;
    double S2 = 0.0;
    int64_t nused = 0;
    bool converged = false;
    while (k < kcap) {
      // residual row -> Va[:, k]
      double* v = Va + (int64_t)k * n;
      double best = -1.0;
      int64_t bj = 0;
      for (int64_t j = tid; j < n; j += NT) {
        double r = entry(D, bk.r0 + istar, bk.c0 + j);
        for (int l = 0; l < k; ++l) r -= Ua[istar + (int64_t)l * m] * Va[j + (int64_t)l * n];
        v[j] = r;
        const double a = fabs(r);
        if (a > best || (a == best && j < bj)) { best = a; bj = j; }
      }
      block_argmax(best, bj, S.red, S.redi);
      if (tid == 0) used[istar] = 1.0;
      ++nused;
      __syncthreads();
      const double piv = v[bj];
      __syncthreads();   // every thread has the pivot before its owner rescales it
      if (piv == 0.0) {
        if (nused >= m) { converged = true; break; }
        // lowest unused row
        int64_t lo = m;
        for (int64_t i = tid; i < m; i += NT) if (used[i] == 0.0 && i < lo) lo = i;
        double dv = -(double)lo;
        block_argmax(dv, lo, S.red, S.redi);
        istar = (int64_t)(-dv);
        __syncthreads();
        continue;
      }
      const double inv = 1.0 / piv;
      for (int64_t j = tid; j < n; j += NT) v[j] = v[j] * inv;
      double* u = Ua + (int64_t)k * m;
      __syncthreads();
      for (int64_t i = tid; i < m; i += NT) {
        double r = entry(D, bk.r0 + i, bk.c0 + bj);
        for (int l = 0; l < k; ++l) r -= Va[bj + (int64_t)l * n] * Ua[i + (int64_t)l * m];
        u[i] = r;
      }
      __syncthreads();
      // norms and cross terms
      double pu = 0.0, pv = 0.0;
      for (int64_t i = tid; i < m; i += NT) pu += u[i] * u[i];
      for (int64_t j = tid; j < n; j += NT) pv += v[j] * v[j];
      const double nu2 = block_sum(pu, S.red);
      const double nv2 = block_sum(pv, S.red);
      double cross = 0.0;
      for (int l = 0; l < k; ++l) {
        double a = 0.0, c = 0.0;
        for (int64_t i = tid; i < m; i += NT) a += Ua[i + (int64_t)l * m] * u[i];
        for (int64_t j = tid; j < n; j += NT) c += Va[j + (int64_t)l * n] * v[j];
        a = block_sum(a, S.red);
        c = block_sum(c, S.red);
        cross += a * c;
      }
      S2 = S2 + 2.0 * cross + nu2 * nv2;
      ++k;
      if (sqrt(nu2) * sqrt(nv2) <= D.eps * sqrt(S2)) { converged = true; break; }
      if (nused >= m) { converged = true; break; }
      // next row: largest |u_i| among unused rows
      double bv = -1.0;
      int64_t bi = 0;
      for (int64_t i = tid; i < m; i += NT) {
        const double a = (used[i] != 0.0) ? -1.0 : fabs(u[i]);
        if (a > bv || (a == bv && i < bi)) { bv = a; bi = i; }
      }
      block_argmax(bv, bi, S.red, S.redi);
      istar = bi;
      __syncthreads();
    }
    __syncthreads();
    // the rank cap stopped the iteration before its accuracy test was met
    const int64_t mn = m < n ? m : n;
    if (tid == 0 && D.kfix <= 0 && D.kmax < mn && k == kcap && !converged) atomicAdd(D.capped, 1);
    double* U = lr_U(D, b);
    double* V = lr_V(D, b);
    const int kt = wg_truncate(D, Ua, m, Va, n, k, U, V, work, dyn, 4096, S);
    if (tid == 0) D.rank[b] = kt;
    __syncthreads();
    if (D.mixed) {
      round_f32(U, m, kt, m);
      round_f32(V, n, kt, n);
    }
  }
}

// ------------------------------------------------------------------ tasks

__device__ __forceinline__ int term_rank(const DevData& D, const TermDef& t) {
  if (t.kind == TK_DD) return (int)D.bk[t.A].n;
  if (t.kind == TK_LRA) return D.rank[t.A];
  return D.rank[t.B];
}

// Pointers/leading dimensions of the factors of a term.
__device__ __forceinline__ void term_factors(const DevData& D, const TermDef& t, const double*& X,
                                             int64_t& ldx, const double*& Y, int64_t& ldy) {
  const Block A = D.bk[t.A], B = D.bk[t.B];
  if (t.kind == TK_DD) {
    X = D.dense + D.dense_off[t.A]; ldx = A.m;
    Y = D.dense + D.dense_off[t.B]; ldy = B.m;
  } else if (t.kind == TK_LRA) {
    X = lr_U(D, t.A); ldx = A.m;
    Y = D.termbuf + t.buf; ldy = t.rows;
  } else {
    X = D.termbuf + t.buf; ldx = t.rows;
    Y = lr_U(D, t.B); ldy = B.m;
  }
}

// Y(i0:i1, :) += sign L_blk(i0:i1, :) W for one leaf of the factor (rows
// local to the leaf): W (ncols(blk) x k, ldw), Y (ldy, row 0 = the leaf's
// first row).  tmp: k_blk x k doubles (global or shared).
__device__ void leaf_matvec_rows_f32(const DevData& D, int32_t blk, const double* W, int64_t ldw, int k, double* Y,
                                     int64_t ldy, float sign, double* tmp, Smem& S, int64_t i0, int64_t i1);

__device__ void leaf_matvec_rows(const DevData& D, int32_t blk, const double* W, int64_t ldw, int k, double* Y,
                                 int64_t ldy, double sign, double* tmp, Smem& S, int64_t i0, int64_t i1,
                                 bool f32 = false) {
  if (f32) {
    leaf_matvec_rows_f32(D, blk, W, ldw, k, Y, ldy, (float)sign, tmp, S, i0, i1);
    return;
  }
  const Block L = D.bk[blk];
  const int tid = threadIdx.x;
  const int64_t mr = i1 - i0;
  if (tid == 0)
    S.flops += (L.kind == BK_DENSE) ? 2.0 * mr * L.n * k
                                    : 2.0 * (double)(mr + L.n) * D.rank[blk] * k;
  if (L.kind == BK_DENSE) {
    const double* A = D.dense + D.dense_off[blk];
    for (int64_t e = tid; e < mr * (int64_t)k; e += NT) {
      const int64_t i = i0 + e % mr;
      const int c = (int)(e / mr);
      double acc = 0.0;
      for (int64_t l = 0; l < L.n; ++l) acc += A[i + l * L.m] * W[l + c * ldw];
      Y[i + c * ldy] += sign * acc;
    }
  } else {
    const double* U = lr_U(D, blk);
    const double* V = lr_V(D, blk);
    const int kb = D.rank[blk];
    // tmp = V^T W  (kb x k)
    const int w = tid >> 6, lane = tid & 63;
    for (int e = w; e < kb * k; e += NW) {
      const int a = e % kb, c = e / kb;
      double acc = 0.0;
      for (int64_t l = lane; l < L.n; l += 64) acc += V[l + a * L.n] * W[l + c * ldw];
      acc = wave_sum(acc);
      if (lane == 0) tmp[e] = acc;
    }
    __syncthreads();
    for (int64_t e = tid; e < mr * (int64_t)k; e += NT) {
      const int64_t i = i0 + e % mr;
      const int c = (int)(e / mr);
      double acc = 0.0;
      for (int a = 0; a < kb; ++a) acc += U[i + (int64_t)a * L.m] * tmp[a + c * kb];
      Y[i + c * ldy] += sign * acc;
    }
  }
  __syncthreads();
}

// FP32 arithmetic form of leaf_matvec_rows (the mixed-precision term
// products): operands rounded to FP32, products and sums in FP32, Y kept
// FP32-valued.
__device__ void leaf_matvec_rows_f32(const DevData& D, int32_t blk, const double* W, int64_t ldw, int k, double* Y,
                                     int64_t ldy, float sign, double* tmp, Smem& S, int64_t i0, int64_t i1) {
  const Block L = D.bk[blk];
  const int tid = threadIdx.x;
  const int64_t mr = i1 - i0;
  if (tid == 0)
    S.flops += (L.kind == BK_DENSE) ? 2.0 * mr * L.n * k : 2.0 * (double)(mr + L.n) * D.rank[blk] * k;
  if (L.kind == BK_DENSE) {
    const double* A = D.dense + D.dense_off[blk];
    for (int64_t e = tid; e < mr * (int64_t)k; e += NT) {
      const int64_t i = i0 + e % mr;
      const int c = (int)(e / mr);
      float acc = 0.0f;
      for (int64_t l = 0; l < L.n; ++l) acc += (float)A[i + l * L.m] * (float)W[l + c * ldw];
      Y[i + c * ldy] = (double)((float)Y[i + c * ldy] + sign * acc);
    }
  } else {
    const double* U = lr_U(D, blk);
    const double* V = lr_V(D, blk);
    const int kb = D.rank[blk];
    const int w = tid >> 6, lane = tid & 63;
    for (int e = w; e < kb * k; e += NW) {
      const int a = e % kb, c = e / kb;
      float acc = 0.0f;
      for (int64_t l = lane; l < L.n; l += 64) acc += (float)V[l + a * L.n] * (float)W[l + c * ldw];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (lane == 0) tmp[e] = (double)acc;
    }
    __syncthreads();
    for (int64_t e = tid; e < mr * (int64_t)k; e += NT) {
      const int64_t i = i0 + e % mr;
      const int c = (int)(e / mr);
      float acc = 0.0f;
      for (int a = 0; a < kb; ++a) acc += (float)U[i + (int64_t)a * L.m] * (float)tmp[a + c * kb];
      Y[i + c * ldy] = (double)((float)Y[i + c * ldy] + sign * acc);
    }
  }
  __syncthreads();
}

// Y(j0:j1, :) += sign L_blk(:, j0:j1)^T W for one leaf (columns local to the
// leaf): W (nrows(blk) x k, ldw, row 0 = the leaf's first row), Y (ldy, row 0
// = the leaf's first column).  tmp: k_blk x k doubles.
__device__ void leaf_matvec_t_rows(const DevData& D, int32_t blk, const double* W, int64_t ldw, int k, double* Y,
                                   int64_t ldy, double sign, double* tmp, Smem& S, int64_t j0, int64_t j1) {
  const Block L = D.bk[blk];
  const int tid = threadIdx.x;
  const int64_t nc = j1 - j0;
  if (tid == 0)
    S.flops += (L.kind == BK_DENSE) ? 2.0 * nc * L.m * k : 2.0 * (double)(nc + L.m) * D.rank[blk] * k;
  if (L.kind == BK_DENSE) {
    const double* A = D.dense + D.dense_off[blk];
    for (int64_t e = tid; e < nc * (int64_t)k; e += NT) {
      const int64_t j = j0 + e % nc;
      const int c = (int)(e / nc);
      double acc = 0.0;
      for (int64_t i = 0; i < L.m; ++i) acc += A[i + j * L.m] * W[i + c * ldw];
      Y[j + c * ldy] += sign * acc;
    }
  } else {
    const double* U = lr_U(D, blk);
    const double* V = lr_V(D, blk);
    const int kb = D.rank[blk];
    // tmp = U^T W  (kb x k)
    const int w = tid >> 6, lane = tid & 63;
    for (int e = w; e < kb * k; e += NW) {
      const int a = e % kb, c = e / kb;
      double acc = 0.0;
      for (int64_t i = lane; i < L.m; i += 64) acc += U[i + a * L.m] * W[i + c * ldw];
      acc = wave_sum(acc);
      if (lane == 0) tmp[e] = acc;
    }
    __syncthreads();
    for (int64_t e = tid; e < nc * (int64_t)k; e += NT) {
      const int64_t j = j0 + e % nc;
      const int c = (int)(e / nc);
      double acc = 0.0;
      for (int a = 0; a < kb; ++a) acc += V[j + (int64_t)a * L.n] * tmp[a + c * kb];
      Y[j + c * ldy] += sign * acc;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void leaf_matvec(const DevData& D, int32_t blk, const double* W, int64_t ldw, int k,
                                            double* Y, int64_t ldy, double sign, double* tmp, Smem& S) {
  leaf_matvec_rows(D, blk, W, ldw, k, Y, ldy, sign, tmp, S, 0, D.bk[blk].m);
}

// W <- L_cc^{-1} W over cluster c (W: |c| x k, ldw) by the solve program.
__device__ void run_solve(const DevData& D, int32_t c, double* W, int64_t ldw, int k, double* tmp,
                          double* lds, Smem& S) {
  const int tid = threadIdx.x;
  for (int32_t o = D.sop_begin[c]; o < D.sop_begin[c + 1]; ++o) {
    const SolveOp op = D.sops[o];
    const Block L = D.bk[op.blk];
    if (op.kind == SOP_TRSV) {
      // dense lower-triangular solve of the leaf's rows, staged in LDS; one
      // thread per right-hand side column
      const double* A = D.dense + D.dense_off[op.blk];
      const int mm = (int)L.m;
      double* Ls = lds;
      double* Ws = lds + LEAF_MAX * LEAF_MAX;   // mm x k, leading dimension LEAF_MAX + 1
      const int ldl = LEAF_MAX + 1;
      double* w = W + op.off;
      if (tid == 0) S.flops += (double)mm * mm * k;
      for (int e = tid; e < mm * mm; e += NT) Ls[e] = A[e];
      for (int e = tid; e < mm * k; e += NT) Ws[(e % mm) + (e / mm) * ldl] = w[(e % mm) + (int64_t)(e / mm) * ldw];
      __syncthreads();
      for (int c = tid; c < k; c += NT) {
        double* wc = Ws + c * ldl;
        for (int i = 0; i < mm; ++i) {
          double sum = wc[i];
          for (int l = 0; l < i; ++l) sum -= Ls[i + l * mm] * wc[l];
          wc[i] = sum / Ls[i + i * mm];
        }
      }
      __syncthreads();
      for (int e = tid; e < mm * k; e += NT) w[(e % mm) + (int64_t)(e / mm) * ldw] = Ws[(e % mm) + (e / mm) * ldl];
      __syncthreads();
    } else {
      leaf_matvec(D, op.blk, W + op.off2, ldw, k, W + op.off, ldw, -1.0, tmp, S);
    }
  }
}

// W <- L_cc^{-T} W over cluster c: the cluster's solve program backwards with
// every operation transposed (upper triangular leaf solves, W(cols) -= L^T W(rows)).
__device__ void run_solve_t(const DevData& D, int32_t c, double* W, int64_t ldw, int k, double* tmp, double* lds,
                            Smem& S) {
  const int tid = threadIdx.x;
  for (int32_t o = D.sop_begin[c + 1] - 1; o >= D.sop_begin[c]; --o) {
    const SolveOp op = D.sops[o];
    const Block L = D.bk[op.blk];
    if (op.kind == SOP_TRSV) {
      const double* A = D.dense + D.dense_off[op.blk];
      const int mm = (int)L.m;
      double* Ls = lds;
      double* Ws = lds + LEAF_MAX * LEAF_MAX;
      const int ldl = LEAF_MAX + 1;
      double* w = W + op.off;
      if (tid == 0) S.flops += (double)mm * mm * k;
      for (int e = tid; e < mm * mm; e += NT) Ls[e] = A[e];
      for (int e = tid; e < mm * k; e += NT) Ws[(e % mm) + (e / mm) * ldl] = w[(e % mm) + (int64_t)(e / mm) * ldw];
      __syncthreads();
      for (int cc = tid; cc < k; cc += NT) {
        double* wc = Ws + cc * ldl;
        for (int i = mm - 1; i >= 0; --i) {
          double sum = wc[i];
          for (int l = i + 1; l < mm; ++l) sum -= Ls[l + i * mm] * wc[l];
          wc[i] = sum / Ls[i + i * mm];
        }
      }
      __syncthreads();
      for (int e = tid; e < mm * k; e += NT) w[(e % mm) + (int64_t)(e / mm) * ldw] = Ws[(e % mm) + (e / mm) * ldl];
      __syncthreads();
    } else {
      leaf_matvec_t_rows(D, op.blk, W + op.off, ldw, k, W + op.off2, ldw, -1.0, tmp, S, 0, L.n);
    }
  }
}

// Term product: Y = L_B V_A (TK_LRA) or X = L_A V_B (TK_LRB).
__device__ void task_term(const DevData& D, int32_t tid_term, double* tmp, Smem& S) {
  const TermDef t = D.terms[tid_term];
  const int32_t H = (t.kind == TK_LRA) ? t.B : t.A;      // H-block applied
  const int32_t R = (t.kind == TK_LRA) ? t.A : t.B;      // low-rank block providing V
  const Block HB = D.bk[H], RB = D.bk[R];
  const int k = D.rank[R];
  const double* Vr = lr_V(D, R);   // n(R) x k, ld n(R)
  double* out = D.termbuf + t.buf;                        // rows x k, ld rows
  for (int64_t e = threadIdx.x; e < t.rows * (int64_t)k; e += NT) out[e] = 0.0;
  __syncthreads();
  for (int32_t q = D.sub_begin[H]; q < D.sub_end[H]; ++q) {
    const int32_t lf = D.sub_leaves[q];
    const Block L = D.bk[lf];
    leaf_matvec_rows(D, lf, Vr + (L.c0 - HB.c0), RB.n, k, out + (L.r0 - HB.r0), t.rows, 1.0, tmp, S, 0, L.m,
                     D.mixed != 0);
  }
}

// Rows of chunk cluster q (tk.a1) of a term product (see task_term): the
// leaves of the H-block in pre-order, each restricted to those rows.
__device__ void task_term_rows(const DevData& D, const Task& tk, double* tmp, Smem& S) {
  const TermDef t = D.terms[tk.obj];
  const int32_t H = (t.kind == TK_LRA) ? t.B : t.A;
  const int32_t R = (t.kind == TK_LRA) ? t.A : t.B;
  const Block HB = D.bk[H], RB = D.bk[R];
  const Cluster q = D.cl[tk.a1];
  const int k = D.rank[R];
  const double* Vr = lr_V(D, R);
  double* out = D.termbuf + t.buf;
  const int64_t q0 = q.begin - HB.r0, q1 = q.end - HB.r0;
  for (int64_t e = threadIdx.x; e < (q1 - q0) * (int64_t)k; e += NT) {
    const int64_t i = q0 + e % (q1 - q0);
    out[i + (e / (q1 - q0)) * t.rows] = 0.0;
  }
  __syncthreads();
  for (int32_t s = D.sub_begin[H]; s < D.sub_end[H]; ++s) {
    const int32_t lf = D.sub_leaves[s];
    const Block L = D.bk[lf];
    const int64_t a = (q.begin > L.r0 ? q.begin : L.r0), b = (q.end < L.r0 + L.m ? q.end : L.r0 + L.m);
    if (a >= b) continue;
    leaf_matvec_rows(D, lf, Vr + (L.c0 - HB.c0), RB.n, k, out + (L.r0 - HB.r0), t.rows, 1.0, tmp, S,
                     a - L.r0, b - L.r0, D.mixed != 0);
  }
}

// Target of a solve task: a low-rank block's V (rows relative to its column
// cluster, rank columns) or the permuted data W of the final solve.
__device__ __forceinline__ void solve_target(const DevData& D, int32_t obj, double*& W, int64_t& ld, int& k,
                                             int64_t& base) {
  if (obj >= 0) {
    const Block b = D.bk[obj];
    W = lr_V(D, obj);
    ld = b.n;
    k = D.rank[obj];
    base = b.c0;
  } else {
    W = D.W;
    ld = D.n;
    k = D.r;
    base = 0;
  }
}

// W(rows of cluster tk.a0) <- L^{-1} W(same rows): the cluster's solve program.
__device__ void task_solve_seq(const DevData& D, const Task& tk, double* slot, double* lds, Smem& S) {
  double* W;
  int64_t ld, base;
  int k;
  solve_target(D, tk.obj, W, ld, k, base);
  if (k <= 0) return;
  const Cluster c = D.cl[tk.a0];
  run_solve(D, tk.a0, W + (c.begin - base), ld, k, slot, lds, S);
  // rows of c are final: a low-rank factor's V is stored FP32-valued in the mixed form
  if (D.mixed && tk.obj >= 0) round_f32(W + (c.begin - base), c.end - c.begin, k, ld);
}

// W(rows of cluster q = tk.a1) -= L_blk(those rows, :) W(cols of blk), blk =
// tk.a0, over blk's leaves in pre-order (the order of the solve program).
__device__ void task_solve_mv(const DevData& D, const Task& tk, double* tmp, Smem& S) {
  double* W;
  int64_t ld, base;
  int k;
  solve_target(D, tk.obj, W, ld, k, base);
  if (k <= 0) return;
  const int32_t blk = tk.a0;
  const Cluster q = D.cl[tk.a1];
  for (int32_t s = D.sub_begin[blk]; s < D.sub_end[blk]; ++s) {
    const int32_t lf = D.sub_leaves[s];
    const Block L = D.bk[lf];
    const int64_t a = (q.begin > L.r0 ? q.begin : L.r0), b = (q.end < L.r0 + L.m ? q.end : L.r0 + L.m);
    if (a >= b) continue;
    leaf_matvec_rows(D, lf, W + (L.c0 - base), ld, k, W + (L.r0 - base), ld, -1.0, tmp, S, a - L.r0, b - L.r0);
  }
}

// W(rows of cluster tk.a0) <- L^{-T} W(same rows) of the data.
__device__ void task_solve_seq_t(const DevData& D, const Task& tk, double* slot, double* lds, Smem& S) {
  if (D.r <= 0) return;
  run_solve_t(D, tk.a0, D.W + D.cl[tk.a0].begin, D.n, D.r, slot, lds, S);
}

// W(rows of cluster q = tk.a1) -= L_blk(:, those rows)^T W(rows of blk), blk =
// tk.a0, over blk's leaves in pre-order.
__device__ void task_solve_mv_t(const DevData& D, const Task& tk, double* tmp, Smem& S) {
  if (D.r <= 0) return;
  const int32_t blk = tk.a0;
  const Cluster q = D.cl[tk.a1];
  for (int32_t s = D.sub_begin[blk]; s < D.sub_end[blk]; ++s) {
    const int32_t lf = D.sub_leaves[s];
    const Block L = D.bk[lf];
    const int64_t a = (q.begin > L.c0 ? q.begin : L.c0), b = (q.end < L.c0 + L.n ? q.end : L.c0 + L.n);
    if (a >= b) continue;
    leaf_matvec_t_rows(D, lf, D.W + L.r0, D.n, D.r, D.W + L.c0, D.n, -1.0, tmp, S, a - L.c0, b - L.c0);
  }
}

// Y(rows of cluster q = tk.a1) = M W for the leaves of the whole partition:
// M = L (tk.a0 = 0: each leaf's own product), L^T (1: each leaf transposed) or
// the symmetric matrix whose lower blocks are stored (2: both, the diagonal
// leaves once).  Y, W: D.Y, D.W (n x D.r, leading dimension n).
__device__ void task_apply(const DevData& D, const Task& tk, double* tmp, Smem& S) {
  const int k = D.r;
  if (k <= 0) return;
  const Cluster q = D.cl[tk.a1];
  const int64_t len = q.end - q.begin;
  for (int64_t e = threadIdx.x; e < len * (int64_t)k; e += NT) D.Y[q.begin + e % len + (e / len) * D.n] = 0.0;
  __syncthreads();
  for (int32_t s = D.sub_begin[0]; s < D.sub_end[0]; ++s) {
    const int32_t lf = D.sub_leaves[s];
    const Block L = D.bk[lf];
    if (tk.a0 != 1) {
      const int64_t a = (q.begin > L.r0 ? q.begin : L.r0), b = (q.end < L.r0 + L.m ? q.end : L.r0 + L.m);
      if (a < b) leaf_matvec_rows(D, lf, D.W + L.c0, D.n, k, D.Y + L.r0, D.n, 1.0, tmp, S, a - L.r0, b - L.r0);
    }
    if (tk.a0 == 1 || (tk.a0 == 2 && L.r0 != L.c0)) {
      const int64_t a = (q.begin > L.c0 ? q.begin : L.c0), b = (q.end < L.c0 + L.n ? q.end : L.c0 + L.n);
      if (a < b) leaf_matvec_t_rows(D, lf, D.W + L.r0, D.n, k, D.Y + L.c0, D.n, 1.0, tmp, S, a - L.c0, b - L.c0);
    }
  }
}

// ------------------------------------------------------------------ MFMA tiles
//
// A dense tile of at most 64 x 64 entries lives in the accumulators of the
// FP64 matrix instruction v_mfma_f64_16x16x4f64 (D = A B + C, A 16 x 4,
// B 4 x 16): wavefront w owns tile rows 16 w .. 16 w + 15 and holds them as
// four 16 x 16 sub-tiles acc[c] (tile columns 16 c .. 16 c + 15).  Lane l of
// wavefront w holds, in acc[c][q], the entry (16 w + mrow(l, q), 16 c + (l & 15));
// as an operand, lane l supplies A(l & 15, l >> 4) and B(l >> 4, l & 15).
// (Accumulator rows (l >> 4) + 4 q: measured on gfx950 with known operands.)
typedef double dvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int mrow(int lane, int q) { return (lane >> 4) + 4 * q; }

struct Tile {
  dvec4 acc[4];
};

// acc = src (tm x tn, column-major, ld), zero outside.
__device__ __forceinline__ void tile_load(Tile& T, const double* src, int64_t ld, int tm, int tn) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * w + mrow(lane, q), j = 16 * c + (lane & 15);
      T.acc[c][q] = (i < tm && j < tn) ? src[i + (int64_t)j * ld] : 0.0;
    }
}

__device__ __forceinline__ void tile_zero(Tile& T) {
#pragma unroll
  for (int c = 0; c < 4; ++c) T.acc[c] = dvec4{0.0, 0.0, 0.0, 0.0};
}

__device__ __forceinline__ void tile_store(const Tile& T, double* dst, int64_t ld, int tm, int tn) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * w + mrow(lane, q), j = 16 * c + (lane & 15);
      if (i < tm && j < tn) dst[i + (int64_t)j * ld] = T.acc[c][q];
    }
}

// tile_store into a matrix stored by rows: entry (i, j) at dst[j + i ld].
__device__ __forceinline__ void tile_store_t(const Tile& T, double* dst, int64_t ld, int tm, int tn) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * w + mrow(lane, q), j = 16 * c + (lane & 15);
      if (i < tm && j < tn) dst[j + (int64_t)i * ld] = T.acc[c][q];
    }
}

// Tile += sign X Y^T over tile rows [i0, i1) and columns [j0, j1): row i uses
// X row xr + (i - i0), column j uses Y row yr + (j - j0), r columns each.
// Entries outside the rectangle are left exactly as they are (their products
// are formed from zero operands).
__device__ __forceinline__ void tile_xyT(Tile& T, double sign, const double* X, int64_t ldx, int64_t xr,
                                         const double* Y, int64_t ldy, int64_t yr, int r, int i0, int i1, int j0,
                                         int j1) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr0 = 16 * w;
  if (wr0 >= i1 || wr0 + 16 <= i0) return;          // no row of this wavefront is touched
  const int i = wr0 + (lane & 15);
  const bool rowin = i >= i0 && i < i1;
  const double* xp = X + xr + (rowin ? i - i0 : 0);
  const int kl = lane >> 4;
  bool colin[4];
  const double* yp[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = 16 * c + (lane & 15);
    colin[c] = j >= j0 && j < j1;
    yp[c] = Y + yr + (colin[c] ? j - j0 : 0);
  }
  const bool cact[4] = {16 * 0 < j1 && 16 * 0 + 16 > j0, 16 * 1 < j1 && 16 * 1 + 16 > j0,
                        16 * 2 < j1 && 16 * 2 + 16 > j0, 16 * 3 < j1 && 16 * 3 + 16 > j0};
  // four steps (16 columns of the factors) at a time, every operand load
  // issued before the first product; columns past r load as zero
  for (int k0 = 0; k0 < r; k0 += 16) {
    const int ns = (r - k0 + 3) >> 2;          // steps with at least one column (wave-uniform)
    double a[4], bv[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = k0 + 4 * s + kl;
      const bool kin = k < r;
      a[s] = (kin && rowin) ? sign * xp[k * ldx] : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[s][c] = (kin && cact[c] && colin[c]) ? yp[c][k * ldy] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (s < ns)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (cact[c]) T.acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bv[s][c], T.acc[c], 0, 0, 0);
  }
}

// FP32 form of tile_xyT (mixed precision): operands rounded to FP32, the
// product formed and accumulated by v_mfma_f32_16x16x4f32 in FP32, then added
// to the FP64 tile.  That instruction holds accumulator row 4 (l >> 4) + q in
// lane l, register q, against (l >> 4) + 4 q for the FP64 one, so the A
// operand's rows are fed permuted (row 4 a + q carries tile row a + 4 q) to
// land every product in the lane and register of the FP64 tile's entry.
typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void tile_xyT_f32(Tile& T, double sign, const double* X, int64_t ldx, int64_t xr,
                                             const double* Y, int64_t ldy, int64_t yr, int r, int i0, int i1, int j0,
                                             int j1) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr0 = 16 * w;
  if (wr0 >= i1 || wr0 + 16 <= i0) return;
  const int ar = lane & 15;
  const int i = wr0 + (ar >> 2) + 4 * (ar & 3);     // the permuted A row
  const bool rowin = i >= i0 && i < i1;
  const double* xp = X + xr + (rowin ? i - i0 : 0);
  const int kl = lane >> 4;
  bool colin[4];
  const double* yp[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int j = 16 * c + (lane & 15);
    colin[c] = j >= j0 && j < j1;
    yp[c] = Y + yr + (colin[c] ? j - j0 : 0);
  }
  const bool cact[4] = {16 * 0 < j1 && 16 * 0 + 16 > j0, 16 * 1 < j1 && 16 * 1 + 16 > j0,
                        16 * 2 < j1 && 16 * 2 + 16 > j0, 16 * 3 < j1 && 16 * 3 + 16 > j0};
  fvec4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = fvec4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < r; k0 += 16) {
    const int ns = (r - k0 + 3) >> 2;
    float a[4], bv[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = k0 + 4 * s + kl;
      const bool kin = k < r;
      a[s] = (kin && rowin) ? (float)xp[k * ldx] : 0.0f;
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[s][c] = (kin && cact[c] && colin[c]) ? (float)yp[c][k * ldy] : 0.0f;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (s < ns)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          if (cact[c]) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bv[s][c], acc[c], 0, 0, 0);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) T.acc[c][q] += sign * (double)acc[c][q];
}

// Subtracts a leaf's restricted update terms, in order, from the tm x tn tile
// at (ti0, tj0) of the block (FP64 matrix instructions, factors read from
// global memory).  The instances are resolved TM_CHUNK at a time into LDS by
// one thread each (instance, term, rank and factor offsets are a chain of
// dependent loads), and a chunk stays there for the next tile of the same task.
__device__ void apply_terms(const DevData& D, const Task& tk, int ti0, int tj0, int tm, int tn, Tile& T, Smem& S) {
  const int tid = threadIdx.x;
  for (int32_t c0 = 0; c0 < tk.ninst; c0 += TM_CHUNK) {
    const int nc = (tk.ninst - c0 < TM_CHUNK) ? tk.ninst - c0 : TM_CHUNK;
    if (!(S.tm_begin == tk.inst_begin + c0 && S.tm_n == nc)) {
      __syncthreads();   // the previous chunk's readers are done
      if (tid < nc) {
        const TermInst in = D.insts[tk.inst_begin + c0 + tid];
        const TermDef t = D.terms[in.term];
        TermMeta mt;
        term_factors(D, t, mt.X, mt.ldx, mt.Y, mt.ldy);
        mt.r = term_rank(D, t);
        mt.dd = t.kind == TK_DD;
        mt.xr0 = in.xr0;
        mt.yr0 = in.yr0;
        mt.lr0 = in.lr0;
        mt.lc0 = in.lc0;
        mt.mx = in.mx;
        mt.ny = in.ny;
        S.tm[tid] = mt;
      }
      if (tid == 0) {
        S.tm_begin = tk.inst_begin + c0;
        S.tm_n = nc;
      }
      __syncthreads();
    }
    for (int q = 0; q < nc; ++q) {
      const TermMeta& mt = S.tm[q];
      // the term's rectangle, clipped to the tile (block coordinates)
      const int r0 = mt.lr0 > ti0 ? mt.lr0 : ti0;
      const int r1 = (mt.lr0 + mt.mx < ti0 + tm) ? mt.lr0 + mt.mx : ti0 + tm;
      const int cc0 = mt.lc0 > tj0 ? mt.lc0 : tj0;
      const int cc1 = (mt.lc0 + mt.ny < tj0 + tn) ? mt.lc0 + mt.ny : tj0 + tn;
      if (r0 >= r1 || cc0 >= cc1 || mt.r == 0) continue;
      if (tid == 0) S.flops += 2.0 * (r1 - r0) * (cc1 - cc0) * mt.r;
      // products of dense leaves stay FP64; products with low-rank factors are
      // FP32 in the mixed form
      if (D.mixed && !mt.dd)
        tile_xyT_f32(T, -1.0, mt.X, mt.ldx, mt.xr0 + (r0 - mt.lr0), mt.Y, mt.ldy, mt.yr0 + (cc0 - mt.lc0), mt.r,
                     r0 - ti0, r1 - ti0, cc0 - tj0, cc1 - tj0);
      else
        tile_xyT(T, -1.0, mt.X, mt.ldx, mt.xr0 + (r0 - mt.lr0), mt.Y, mt.ldy, mt.yr0 + (cc0 - mt.lc0), mt.r,
                 r0 - ti0, r1 - ti0, cc0 - tj0, cc1 - tj0);
    }
  }
}

// Dense leaf: flush its terms, then Cholesky (diagonal) or triangular solve.
__device__ void task_dense(const DevData& D, const Task& tk, int32_t prog, double* lds, Smem& S) {
  const int tid = threadIdx.x;
  const int32_t b = tk.obj;
  const Block bk = D.bk[b];
  const int m = (int)bk.m, n = (int)bk.n;
  double* Dg = D.dense + D.dense_off[b];
  const int cnt = m * n;
  Tile T;
  tile_load(T, Dg, m, m, n);
  apply_terms(D, tk, 0, 0, m, n, T, S);
  double* A = lds;                  // m x n tile, column-major
  tile_store(T, A, m, m, n);
  __syncthreads();
  if (tid == 0) S.flops += (tk.kind == TASK_DIAG) ? (double)m * m * m / 3.0 : (double)m * n * n;
  if (tk.kind == TASK_DIAG) {
    // right-looking Cholesky in LDS (lower)
    for (int j = 0; j < n; ++j) {
      const double djj = A[j + j * m];
      const bool bad = !(djj > 0.0);
      if (bad && tid == 0) {
        const unsigned long long key = ((unsigned long long)prog << 8) | (unsigned long long)j;
        atomicMin(D.fail_key, key);
      }
      const double ljj = bad ? NAN : sqrt(djj);
      __syncthreads();
      for (int i = j + tid; i < m; i += NT) A[i + j * m] = (i == j) ? ljj : A[i + j * m] / ljj;
      __syncthreads();
      const int rem = m - j - 1;
      for (int e = tid; e < rem * rem; e += NT) {
        const int i = j + 1 + e % rem, c = j + 1 + e / rem;
        if (c <= i) A[i + c * m] -= A[i + j * m] * A[c + j * m];
      }
      __syncthreads();
    }
    double s = 0.0;
    for (int i = tid; i < m; i += NT) s += log(A[i + i * m]);
    s = block_sum(s, S.red);
    if (tid == 0) D.logdet_part[b] = s;
    for (int e = tid; e < cnt; e += NT) {
      const int i = e % m, j = e / m;
      Dg[e] = (j <= i) ? A[e] : 0.0;
    }
  } else {
    // X L^T = A, L the factored diagonal leaf of the column cluster (n x n)
    const double* Lg = D.dense + D.dense_off[tk.diag];
    double* Ls = lds + 64 * 64;
    for (int e = tid; e < n * n; e += NT) Ls[e] = Lg[e];
    __syncthreads();
    for (int i = tid; i < m; i += NT) {
      for (int j = 0; j < n; ++j) {
        double s = A[i + j * m];
        for (int l = 0; l < j; ++l) s -= A[i + l * m] * Ls[j + l * n];
        A[i + j * m] = s / Ls[j + j * n];
      }
    }
    __syncthreads();
    for (int e = tid; e < cnt; e += NT) Dg[e] = A[e];
  }
  __syncthreads();
}

// Low-rank leaf whose row and column clusters both hold at most D.dflush
// points (<= CMAX): the updated block U V^T - sum X Y^T is formed exactly, one
// LEAF_MAX x LEAF_MAX tile at a time in registers, and replaced by its best
// approximation (wg_svd_explicit).  The explicit block lives in LDS when it
// fits (up to 128 x 128), else in the work-group's global workspace slot.  Returns the
// new rank (also written to D.rank).
__device__ int lr_dense_flush(const DevData& D, const Task& tk, double* slot, double* lds, Smem& S) {
  const int tid = threadIdx.x;
  const int32_t b = tk.obj;
  const Block bk = D.bk[b];
  const int m = (int)bk.m, n = (int)bk.n;
  double* U = lr_U(D, b);
  double* V = lr_V(D, b);
  const int k0 = D.rank[b];
  const int64_t c0 = (tid == 0) ? clk() : 0;
  const bool small = (int64_t)(m | 1) * n <= LDS_FACTOR;   // the explicit block fits in LDS
  // in LDS by columns; else in the slot by rows (row length n)
  const int lda = small ? (m | 1) : n;
  double* A = small ? lds : slot;
  for (int tj0 = 0; tj0 < n; tj0 += LEAF_MAX) {
    for (int ti0 = 0; ti0 < m; ti0 += LEAF_MAX) {
      const int tm = (m - ti0 < LEAF_MAX) ? m - ti0 : LEAF_MAX;
      const int tn = (n - tj0 < LEAF_MAX) ? n - tj0 : LEAF_MAX;
      Tile T;
      tile_zero(T);
      if (k0 > 0) {
        if (D.mixed) tile_xyT_f32(T, 1.0, U, m, ti0, V, n, tj0, k0, 0, tm, 0, tn);
        else tile_xyT(T, 1.0, U, m, ti0, V, n, tj0, k0, 0, tm, 0, tn);
      }
      apply_terms(D, tk, ti0, tj0, tm, tn, T, S);
      if (small) tile_store(T, A + ti0 + (int64_t)tj0 * lda, lda, tm, tn);
      else tile_store_t(T, A + tj0 + (int64_t)ti0 * lda, lda, tm, tn);
    }
  }
  __syncthreads();
  if (tid == 0) {
    S.flops += 2.0 * m * n * k0;
    S.ph[4] += clk() - c0;     // explicit formation
  }
  __syncthreads();
  // R^T of the pivoted QR: after the block in LDS, else from the start of LDS
  double* glds = small ? lds + lda * n : lds;
  const int gcap = small ? LDS_FACTOR - lda * n : LDS_FACTOR;
  double* gws = slot + (small ? (int64_t)lda * n : (int64_t)m * n);
  const int k = wg_svd_explicit(D, A, m, n, lda, U, m, m, V, n, n, gws, glds, gcap, S, true, small ? slot : nullptr,
                                !small);
  if (tid == 0) D.rank[b] = k;
  __syncthreads();
  if (D.mixed) {
    round_f32(U, m, k, m);
    round_f32(V, n, k, n);
  }
  return k;
}

// Low-rank leaf: flush its terms (explicitly for blocks of at most D.dflush x
// D.dflush, else in factored form, truncating whenever the accumulated rank
// would exceed R_ACC), then V <- L_{sigma sigma}^{-1} V.
__device__ void task_lr(const DevData& D, const Task& tk, double* slot, double* lds, Smem& S) {
  const int tid = threadIdx.x;
  const int32_t b = tk.obj;
  const Block bk = D.bk[b];
  const int64_t m = bk.m, n = bk.n;
  const int RW = 2 * K_MAX;
  double* U = lr_U(D, b);
  double* V = lr_V(D, b);
  const bool explicit_sum = m <= D.dflush && n <= D.dflush;
  if (tk.ninst > 0 && explicit_sum) {
    const int kk = lr_dense_flush(D, tk, slot, lds, S);
    if (tid == 0) S.ival[0] = kk;
    __syncthreads();
  } else if (tk.ninst > 0) {
    double* Xa = slot;
    double* Ya = Xa + m * RW;
    double* work = Ya + n * RW;
    int rank = D.rank[b];
    for (int64_t e = tid; e < m * rank; e += NT) Xa[e] = U[e];
    for (int64_t e = tid; e < n * rank; e += NT) Ya[e] = V[e];
    __syncthreads();
    for (int32_t ii = 0; ii < tk.ninst; ++ii) {
      const TermInst in = D.insts[tk.inst_begin + ii];
      const TermDef t = D.terms[in.term];
      const int r = term_rank(D, t);
      if (rank > 0 && rank + r > R_ACC) {
        const int kk = wg_truncate(D, Xa, m, Ya, n, rank, U, V, work, lds, LDS_FACTOR, S);
        for (int64_t e = tid; e < m * kk; e += NT) Xa[e] = U[e];
        for (int64_t e = tid; e < n * kk; e += NT) Ya[e] = V[e];
        rank = kk;
        __syncthreads();
      }
      const double *X, *Y;
      int64_t ldx, ldy;
      term_factors(D, t, X, ldx, Y, ldy);
      for (int64_t e = tid; e < m * r; e += NT) {
        const int64_t i = e % m;
        const int l = (int)(e / m);
        const int64_t li = i - in.lr0;
        Xa[(rank + l) * m + i] = (li >= 0 && li < in.mx) ? -X[in.xr0 + li + l * ldx] : 0.0;
      }
      for (int64_t e = tid; e < n * r; e += NT) {
        const int64_t j = e % n;
        const int l = (int)(e / n);
        const int64_t lj = j - in.lc0;
        Ya[(rank + l) * n + j] = (lj >= 0 && lj < in.ny) ? Y[in.yr0 + lj + l * ldy] : 0.0;
      }
      rank += r;
      __syncthreads();
    }
    const int kk = wg_truncate(D, Xa, m, Ya, n, rank, U, V, work, lds, LDS_FACTOR, S);
    if (tid == 0) D.rank[b] = kk;
    if (tid == 0) S.ival[0] = kk;
    __syncthreads();
    if (D.mixed) {
      round_f32(U, m, kk, m);
      round_f32(V, n, kk, n);
    }
  } else {
    if (tid == 0) S.ival[0] = D.rank[b];
    __syncthreads();
  }
  const int k = S.ival[0];
  __syncthreads();
  if (tk.a0 == 0) return;   // the solve runs as tasks of its own
  int64_t c0 = (tid == 0) ? clk() : 0;
  if (k > 0) run_solve(D, tk.diag, V, n, k, slot, lds, S);
  if (D.mixed && k > 0) round_f32(V, n, k, n);
  if (tid == 0) S.ph[3] += clk() - c0;
}

// ------------------------------------------------------------------ big blocks
//
// The factored flush of a big low-rank block (storage of 2 K_MAX columns, the
// accumulation [U, -X_1, ...] / [V, Y_1, ...] in place) as steps i = 1 .. T+1:
// if step i truncates (rank > 0 and rank + rank(term i) > R_ACC, or i = T + 1),
// each row block of both factors is Householder-factorised by its own task
// (TS_A), one task factorises the stacked R factors, truncates the core and
// maps the kept singular vectors back through the stacked Q (TS_B), and each
// row block applies its own Q to its part of them (TS_C); TS_C then appends
// term i's columns.  Same reflector algebra as a single QR of the whole factor
// (tall-skinny QR), so the truncation is that of the oracle up to rounding.

// Row block q of a big block: side 0 = U (m rows), 1 = V (n rows); its rows
// [r0, r1) and the number gs of row blocks of that side.  Same formula as the
// planner's ts_blocks / ts_rows.
__device__ __forceinline__ int ts_nblk(int64_t rows) {
  int64_t g = (rows + TS_MINROWS - 1) / TS_MINROWS;
  if (g > TS_GMAX) g = TS_GMAX;
  return g < 1 ? 1 : (int)g;
}

__device__ __forceinline__ void ts_geom(const Block& bk, int q, int& side, int& g, int& gs, int64_t& r0,
                                        int64_t& r1) {
  const int gx = ts_nblk(bk.m);
  side = q < gx ? 0 : 1;
  g = side ? q - gx : q;
  const int64_t rows = side ? bk.n : bk.m;
  gs = ts_nblk(rows);
  const int64_t h = (rows + gs - 1) / gs;
  r0 = g * h;
  r1 = (r0 + h < rows) ? r0 + h : rows;
}

// Whether step tk.a0 truncates, given the accumulated rank; r_i = the rank of
// the step's term (0 for the final step).
__device__ __forceinline__ bool ts_truncates(const DevData& D, const Task& tk, int rank, int& r_i) {
  if (tk.a0 > tk.ninst) {
    r_i = 0;
    return true;
  }
  const TermInst in = D.insts[tk.inst_begin + tk.a0 - 1];
  r_i = term_rank(D, D.terms[in.term]);
  return rank > 0 && rank + r_i > R_ACC;
}

// Householder QR of A (rows x p, ld) in place, through LDS when it fits.
__device__ void qr_any(double* A, int64_t rows, int p, int64_t ld, double* tau, double* lds, int lds_cap, Smem& S) {
  const int tid = threadIdx.x;
  const int64_t lo = odd_ld(rows);
  if (lo * (int64_t)p <= lds_cap) {
    for (int64_t e = tid; e < rows * p; e += NT) lds[(e % rows) + (e / rows) * lo] = A[(e % rows) + (e / rows) * ld];
    __syncthreads();
    wg_qr(lds, rows, p, lo, tau, S);
    for (int64_t e = tid; e < rows * p; e += NT) A[(e % rows) + (e / rows) * ld] = lds[(e % rows) + (e / rows) * lo];
    __syncthreads();
  } else if (rows > TALL_QR_ROWS) {
    wg_qr_blocked(A, rows, p, ld, tau, S);
  } else {
    wg_qr(A, rows, p, ld, tau, S);
  }
}

__device__ void task_ts_a(const DevData& D, const Task& tk, double* lds, Smem& S) {
  const int32_t b = tk.obj;
  const Block bk = D.bk[b];
  const int rank = D.rank[b];
  int ri;
  if (!ts_truncates(D, tk, rank, ri) || rank == 0) return;
  int side, g, gs;
  int64_t r0, r1;
  ts_geom(bk, tk.a1, side, g, gs, r0, r1);
  const int64_t ld = side ? bk.n : bk.m;
  double* A = (side ? lr_V(D, b) : lr_U(D, b)) + r0;
  double* tau = D.stage + D.stage_off[b] + (int64_t)tk.a1 * 2 * K_MAX;
  qr_any(A, r1 - r0, rank, ld, tau, lds, LDS_FACTOR, S);
}

__device__ void task_ts_b(const DevData& D, const Task& tk, double* slot, double* lds, Smem& S) {
  const int tid = threadIdx.x;
  const int32_t b = tk.obj;
  const Block bk = D.bk[b];
  const int p = D.rank[b];
  int ri;
  const bool trunc = ts_truncates(D, tk, p, ri);
  if (!trunc || p == 0) {
    // no truncation: the term is appended after the current columns
    if (tid == 0) {
      D.ts_app[2 * b] = p;
      D.ts_app[2 * b + 1] = 0;
      D.rank[b] = p + ri;
    }
    return;
  }
  int64_t c0 = (tid == 0) ? clk() : 0;
  const int gx = ts_nblk(bk.m), gy = ts_nblk(bk.n);
  const int64_t mx = (int64_t)gx * p, my = (int64_t)gy * p;
  double* Xs = slot;                     // stacked R factors of the U side (mx x p)
  double* Ys = Xs + mx * p;              // and of the V side (my x p)
  double* work = Ys + my * p;
  for (int side = 0; side < 2; ++side) {
    const int gs = side ? gy : gx;
    const int64_t ms = side ? my : mx;
    double* St = side ? Ys : Xs;
    const int64_t rows = side ? bk.n : bk.m;
    const int64_t h = (rows + gs - 1) / gs;
    const double* F = side ? lr_V(D, b) : lr_U(D, b);
    for (int64_t e = tid; e < ms * p; e += NT) {
      const int64_t i = e % ms;
      const int j = (int)(e / ms);
      const int g = (int)(i / p), ii = (int)(i % p);
      St[e] = (ii <= j) ? F[g * h + ii + (int64_t)j * rows] : 0.0;
    }
  }
  __syncthreads();
  qr_any(Xs, mx, p, mx, S.tau_x, lds, LDS_FACTOR, S);
  qr_any(Ys, my, p, my, S.tau_y, lds, LDS_FACTOR, S);
  if (tid == 0) { const int64_t c1 = clk(); S.ph[0] += c1 - c0; c0 = c1; }
  // core M = Rx Ry^T (p x p), in LDS
  const int ldm = (int)odd_ld(p);
  double* M = lds;
  for (int e = tid; e < p * p; e += NT) {
    const int i = e % p, j = e / p;
    const int l0 = i > j ? i : j;
    double acc = 0.0;
    for (int l = l0; l < p; ++l) acc += Xs[i + (int64_t)l * mx] * Ys[j + (int64_t)l * my];
    M[i + j * ldm] = acc;
  }
  __syncthreads();
  if (tid == 0) S.flops += 2.0 * p * p * p / 3.0;
  double* Wx = D.stage + D.stage_off[b] + (int64_t)(gx + gy) * 2 * K_MAX;
  double* Wy = Wx + (int64_t)gx * 2 * K_MAX * K_MAX;
  const int k = wg_svd_explicit(D, M, p, p, ldm, Wx, mx, mx, Wy, my, my, work, lds + ldm * p,
                                LDS_FACTOR - ldm * p, S);
  __syncthreads();
  if (tid == 0) { const int64_t c1 = clk(); S.ph[1] += c1 - c0; c0 = c1; }
  wg_apply_q(Xs, mx, p, mx, S.tau_x, Wx, k, mx, S);
  wg_apply_q(Ys, my, p, my, S.tau_y, Wy, k, my, S);
  if (tid == 0) S.ph[2] += clk() - c0;
  if (tid == 0) {
    D.ts_app[2 * b] = k;
    D.ts_app[2 * b + 1] = p;
    D.rank[b] = k + ri;
  }
}

__device__ void task_ts_c(const DevData& D, const Task& tk, double* slot, Smem& S) {
  const int tid = threadIdx.x;
  const int32_t b = tk.obj;
  const Block bk = D.bk[b];
  const int app = D.ts_app[2 * b], p = D.ts_app[2 * b + 1];
  int side, g, gs;
  int64_t r0, r1;
  ts_geom(bk, tk.a1, side, g, gs, r0, r1);
  const int64_t ld = side ? bk.n : bk.m, rows = r1 - r0;
  double* A = (side ? lr_V(D, b) : lr_U(D, b)) + r0;
  if (p > 0 && app > 0) {
    // rows of the truncated factor: Q_g [W_g; 0], W_g = rows g p .. g p + p - 1 of the small factor
    const int gx = ts_nblk(bk.m);
    const int64_t ms = (int64_t)gs * p;
    const double* W = D.stage + D.stage_off[b] + (int64_t)(gx + ts_nblk(bk.n)) * 2 * K_MAX +
                      (side ? (int64_t)gx * 2 * K_MAX * K_MAX : 0) + (int64_t)g * p;
    const double* tau = D.stage + D.stage_off[b] + (int64_t)tk.a1 * 2 * K_MAX;
    double* tmp = slot;                 // rows x app
    for (int64_t e = tid; e < rows * app; e += NT) {
      const int64_t i = e % rows;
      const int c = (int)(e / rows);
      tmp[e] = (i < p) ? W[i + (int64_t)c * ms] : 0.0;
    }
    __syncthreads();
    wg_apply_q(A, rows, p, ld, tau, tmp, app, rows, S);
    __syncthreads();
    const bool fin = tk.a0 > tk.ninst;
    for (int64_t e = tid; e < rows * app; e += NT)
      A[(e % rows) + (e / rows) * ld] = (fin && D.mixed) ? (double)(float)tmp[e] : tmp[e];
    __syncthreads();
  }
  if (tk.a0 > tk.ninst) return;        // the final step appends nothing
  const TermInst in = D.insts[tk.inst_begin + tk.a0 - 1];
  const TermDef t = D.terms[in.term];
  const int r = term_rank(D, t);
  const double *X, *Y;
  int64_t ldx, ldy;
  term_factors(D, t, X, ldx, Y, ldy);
  const int64_t lo = side ? in.lc0 : in.lr0, len = side ? in.ny : in.mx, f0 = side ? in.yr0 : in.xr0;
  const double* F = side ? Y : X;
  const int64_t ldf = side ? ldy : ldx;
  const double sg = side ? 1.0 : -1.0;
  for (int64_t e = tid; e < rows * r; e += NT) {
    const int64_t i = e % rows;
    const int l = (int)(e / rows);
    const int64_t li = r0 + i - lo;
    A[i + (int64_t)(app + l) * ld] = (li >= 0 && li < len) ? sg * F[f0 + li + l * ldf] : 0.0;
  }
}

// ------------------------------------------------------------------ executor

// One task of the factorisation (shared by the level executors).
__device__ void dispatch(const DevData& D, const Task& tk, int32_t prog, double* slot, double* dyn, Smem& S) {
  switch (tk.kind) {
    case TASK_TERM: task_term(D, tk.obj, slot, S); break;
    case TASK_TERM_ROWS: task_term_rows(D, tk, slot, S); break;
    case TASK_LR: task_lr(D, tk, slot, dyn, S); break;
    case TASK_SOLVE_SEQ: task_solve_seq(D, tk, slot, dyn, S); break;
    case TASK_SOLVE_MV: task_solve_mv(D, tk, slot, S); break;
    case TASK_TS_A: task_ts_a(D, tk, dyn, S); break;
    case TASK_TS_B: task_ts_b(D, tk, slot, dyn, S); break;
    case TASK_TS_C: task_ts_c(D, tk, slot, S); break;
    case TASK_SOLVE_SEQ_T: task_solve_seq_t(D, tk, slot, dyn, S); break;
    case TASK_SOLVE_MV_T: task_solve_mv_t(D, tk, slot, S); break;
    case TASK_APPLY: task_apply(D, tk, slot, S); break;
    default: task_dense(D, tk, prog, dyn, S); break;
  }
}

__device__ void run_task(const DevData& D, int32_t t, double* slot, double* dyn, Smem& S) {
  const Task tk = D.tasks[t];
  const int32_t prog = D.task_prog[t];
  int64_t ts = 0;
  if (threadIdx.x == 0) { S.flops = 0.0; S.ph[0] = S.ph[1] = S.ph[2] = S.ph[3] = S.ph[4] = 0; }
  // per-task records exist for the factorisation's tasks only (ids below
  // D.ntasks; the stream program's data-solve tasks follow them)
  const bool rec = t < D.ntasks;
  if (rec && D.task_times && threadIdx.x == 0) ts = (int64_t)__builtin_amdgcn_s_memrealtime();
  dispatch(D, tk, prog, slot, dyn, S);
  __syncthreads();
  if (rec && D.task_times && threadIdx.x == 0) {
    D.task_times[7 * t] = ts;
    D.task_times[7 * t + 1] = (int64_t)__builtin_amdgcn_s_memrealtime();
    for (int q = 0; q < 5; ++q) D.task_times[7 * t + 2 + q] = S.ph[q];
  }
  if (rec && D.task_flops && threadIdx.x == 0) D.task_flops[t] = S.flops;
}

// Level-synchronous executor: the tasks of one level have no dependencies
// among themselves, and all their predecessors belong to earlier levels,
// completed by earlier launches.  Work-group w takes tasks order[t0 + w],
// order[t0 + w + gridDim.x], ... of the level; it uses workspace slot
// slot_base + w (launches that may run at the same time on different streams
// use disjoint slot ranges).
// The term-metadata cache of apply_terms starts empty in every launch (LDS
// holds no defined value at kernel start); within a launch a task's instance
// range identifies its chunks (ranges of different tasks are disjoint).
__device__ __forceinline__ void term_cache_init(Smem& S) {
  if (threadIdx.x == 0) {
    S.tm_begin = -1;
    S.tm_n = 0;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(NT) k_level(DevData D, int32_t t0, int32_t t1, int32_t slot_base) {
  extern __shared__ double dyn[];
  __shared__ Smem S;
  double* slot = D.ws + (int64_t)(slot_base + blockIdx.x) * D.ws_stride;
  term_cache_init(S);
  for (int32_t q = t0 + blockIdx.x; q < t1; q += gridDim.x) run_task(D, D.order[q], slot, dyn, S);
}

__global__ void k_eval_init(unsigned long long* fail_key, int32_t* capped) {
  if (threadIdx.x == 0) {
    *fail_key = ~0ull;
    *capped = 0;
  }
}

// ------------------------------------------------------------------ solve

// One level [t0, t1) of an operator task graph (level order).
__global__ void __launch_bounds__(NT) k_level_tasks(DevData D, const Task* tasks, int32_t t0, int32_t t1) {
  extern __shared__ double dyn[];
  __shared__ Smem S;
  double* slot = D.ws + (int64_t)blockIdx.x * D.ws_stride;
  term_cache_init(S);
  for (int32_t q = t0 + blockIdx.x; q < t1; q += gridDim.x) {
    const Task tk = tasks[q];
    dispatch(D, tk, -1, slot, dyn, S);
    __syncthreads();
  }
}

// Row-chunk operator product (TASK_APPLY) over all chunks.
__global__ void __launch_bounds__(NT) k_apply(DevData D, int mode, const int32_t* chunks, int32_t nchunks) {
  __shared__ Smem S;
  double* slot = D.ws + (int64_t)blockIdx.x * D.ws_stride;
  for (int32_t q = blockIdx.x; q < nchunks; q += gridDim.x) {
    Task tk{};
    tk.kind = TASK_APPLY;
    tk.obj = -1;
    tk.a0 = mode;
    tk.a1 = chunks[q];
    task_apply(D, tk, slot, S);
    __syncthreads();
  }
}

// Y = C W with the exact covariance (eq. 2 plus the nugget on the diagonal),
// entries formed on the fly; one thread per row, W read in column order
// (every wavefront reads the same entries).  D.r <= 4.
__global__ void __launch_bounds__(NT) k_dense_matvec(DevData D) {
  const int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (i >= D.n) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t j = 0; j < D.n; ++j) {
    const double c = entry(D, i, j);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < D.r) acc[q] += c * D.W[j + q * D.n];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (q < D.r) D.Y[i + q * D.n] = acc[q];
}

// out(a, b) = C(i0 + a, j0 + b) of the exact covariance (eq. 2 plus the nugget
// on the diagonal) in input order: iperm maps an input index to its position
// in the tree order of the coordinates.
__global__ void __launch_bounds__(NT) k_exact_block(DevData D, const int64_t* iperm, int64_t i0, int64_t ni,
                                                    int64_t j0, int64_t nj, double* out, int64_t ldo) {
  const int64_t total = ni * nj;
  for (int64_t e = blockIdx.x * (int64_t)NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
    const int64_t a = e % ni, b = e / ni;
    out[a + b * ldo] = entry(D, iperm[i0 + a], iperm[j0 + b]);
  }
}

// R = Z - Y and per-work-group partial sums of R^2 and Z^2 per column, each
// work-group over a contiguous range of rows, in a fixed order.
__global__ void __launch_bounds__(NT) k_refine_resid(const double* Z, const double* Y, double* R, int64_t n, int r,
                                                     double* part) {
  __shared__ double red[NW];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = blockIdx.x * per, i1 = (i0 + per < n) ? i0 + per : n;
  for (int c = 0; c < r; ++c) {
    double sr = 0.0, sz = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += NT) {
      const double z = Z[i + c * n], v = z - Y[i + c * n];
      R[i + c * n] = v;
      sr += v * v;
      sz += z * z;
    }
    sr = block_sum(sr, red);
    sz = block_sum(sz, red);
    if (threadIdx.x == 0) {
      part[blockIdx.x * 2 * r + c] = sr;
      part[blockIdx.x * 2 * r + r + c] = sz;
    }
  }
}

// X += Dx (Dx may be null: no update) and per-work-group partial sums of Z X
// per column.
__global__ void __launch_bounds__(NT) k_refine_update(double* X, const double* Dx, const double* Z, int64_t n, int r,
                                                      double* part) {
  __shared__ double red[NW];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = blockIdx.x * per, i1 = (i0 + per < n) ? i0 + per : n;
  for (int c = 0; c < r; ++c) {
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += NT) {
      double x = X[i + c * n];
      if (Dx) {
        x += Dx[i + c * n];
        X[i + c * n] = x;
      }
      s += Z[i + c * n] * x;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x * 2 * r + c] = s;
  }
}

__global__ void k_unpermute(const double* W, const int64_t* perm, int64_t n, int r, double* Z) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * r; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    Z[perm[i] + c * n] = W[e];
  }
}

// Gather Z into permuted order: W[i, c] = Z[perm[i], c].
__global__ void k_permute(const double* Z, const int64_t* perm, int64_t n, int r, double* W) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * r; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, c = e / n;
    W[e] = Z[perm[i] + c * n];
  }
}

// out[0] = log|C| (2 sum over diagonal leaves in order), out[1 + c] = v_c^T v_c.
__global__ void __launch_bounds__(NT) k_reduce(DevData D, const int32_t* diag_ids, int32_t ndiag,
                                               const double* W, int r, double* out) {
  __shared__ double red[NW];
  const int tid = threadIdx.x;
  // log-determinant: per-thread contiguous chunks of leaves, fixed order
  double s = 0.0;
  const int32_t per = (ndiag + NT - 1) / NT;
  for (int32_t q = tid * per; q < ndiag && q < (tid + 1) * per; ++q) s += D.logdet_part[diag_ids[q]];
  s = block_sum(s, red);
  if (tid == 0) out[0] = 2.0 * s;
  for (int c = 0; c < r; ++c) {
    const double* w = W + (int64_t)c * D.n;
    double a = 0.0;
    const int64_t per2 = (D.n + NT - 1) / NT;
    for (int64_t i = tid * per2; i < D.n && i < (tid + 1) * per2; ++i) a += w[i] * w[i];
    a = block_sum(a, red);
    if (tid == 0) out[1 + c] = a;
  }
}

// ------------------------------------------------------------------ test hook

// One work-group truncates X Y^T (X: m x r, Y: n x r, copied into workspace
// slot 0) into U (m x k), V (n x k); k written to *kout.
__global__ void __launch_bounds__(NT) k_truncate_test(DevData D, const double* X, int64_t m,
                                                      const double* Y, int64_t n, int r, double* U,
                                                      double* V, int32_t* kout, int64_t* phases) {
  extern __shared__ double dyn[];
  __shared__ Smem S;
  if (threadIdx.x == 0) S.ph[0] = S.ph[1] = S.ph[2] = S.ph[3] = S.ph[4] = 0;
  int k;
  if (Y == nullptr) {
    // explicit m x n matrix (n <= CMAX): the path of the explicit flush
    double* A = D.ws;
    for (int64_t e = threadIdx.x; e < m * n; e += NT) A[e] = X[e];
    __syncthreads();
    k = wg_svd_explicit(D, A, (int)m, (int)n, m, U, m, m, V, n, n, A + m * n, dyn, LDS_FACTOR, S, true);
  } else {
    double* Xa = D.ws;
    double* Ya = Xa + m * r;
    double* work = Ya + n * r;
    for (int64_t e = threadIdx.x; e < m * r; e += NT) Xa[e] = X[e];
    for (int64_t e = threadIdx.x; e < n * r; e += NT) Ya[e] = Y[e];
    __syncthreads();
    k = wg_truncate(D, Xa, m, Ya, n, r, U, V, work, dyn, LDS_FACTOR, S);
  }
  if (threadIdx.x == 0) {
    *kout = k;
    for (int q = 0; q < 3; ++q) phases[q] = S.ph[q];
  }
}

// ------------------------------------------------------------------ allocation-free truncation
//
// Workspace of the allocation-free truncation entry point: one copy per GPU,
// held until the process ends.  Layout: 64 doubles of counters (the rank-cap
// count, then four phase clocks), then the truncation's workspace.  In host
// code `scratch` names a host-side stand-in: only the address returned by
// hipGetSymbolAddress (noalloc_scratch) may be handed to kernels.
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

__global__ void k_clear_counters(double* base) {
  if (threadIdx.x < 64) base[threadIdx.x] = 0.0;
}

hipError_t launch_truncate_noalloc(DevData D, double* base, const double* X, int64_t m, const double* Y, int64_t n,
                                   int r, double* U, double* V, int32_t* kout, hipStream_t st) {
  // counters first (the array keeps the previous call's contents)
  hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, st, base);
  D.capped = reinterpret_cast<int32_t*>(base);
  D.ws = base + 64;
  D.ws_stride = NOALLOC_DOUBLES - 64;
  return launch_truncate_test(D, X, m, Y, n, r, U, V, kout, reinterpret_cast<int64_t*>(base + 8), st);
}

hipError_t launch_truncate_test(const DevData& D, const double* X, int64_t m, const double* Y, int64_t n,
                                int r, double* U, double* V, int32_t* kout, int64_t* phases, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute((const void*)k_truncate_test, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     LDS_FACTOR * sizeof(double));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_truncate_test, dim3(1), dim3(NT), LDS_FACTOR * sizeof(double), st, D, X, m, Y, n, r, U, V,
                     kout, phases);
  return hipGetLastError();
}

// ------------------------------------------------------------------ launchers

hipError_t launch_assemble(const DevData& D, hipStream_t st) {
  if (D.ndense > 0) {
    int g = D.ndense < 4096 ? D.ndense : 4096;
    hipLaunchKernelGGL(k_assemble_dense, dim3(g), dim3(NT), 0, st, D);
  }
  return hipGetLastError();
}

hipError_t launch_aca(const DevData& D, int grid, hipStream_t st) {
  if (D.nlr > 0) {
    int g = D.nlr < grid ? D.nlr : grid;
    hipLaunchKernelGGL(k_aca, dim3(g), dim3(NT), 4096 * sizeof(double), st, D);
  }
  return hipGetLastError();
}

hipError_t launch_eval_init(const DevData& D, hipStream_t st) {
  hipLaunchKernelGGL(k_eval_init, dim3(1), dim3(64), 0, st, D.fail_key, D.capped);
  return hipGetLastError();
}

hipError_t launch_factor_levels(const DevData& D, const int32_t* level_begin, int32_t l0, int32_t l1, int max_grid,
                                hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_level, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       LDS_FACTOR * sizeof(double));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  for (int32_t l = l0; l < l1; ++l) {
    const int32_t t0 = level_begin[l], t1 = level_begin[l + 1];
    const int g = (t1 - t0) < max_grid ? (t1 - t0) : max_grid;
    if (g > 0) hipLaunchKernelGGL(k_level, dim3(g), dim3(NT), LDS_FACTOR * sizeof(double), st, D, t0, t1, 0);
  }
  return hipGetLastError();
}

hipError_t launch_factor_range(const DevData& D, int32_t t0, int32_t t1, int max_grid, int32_t slot_base,
                               hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_level, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       LDS_FACTOR * sizeof(double));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int g = (t1 - t0) < max_grid ? (t1 - t0) : max_grid;
  if (g > 0) hipLaunchKernelGGL(k_level, dim3(g), dim3(NT), LDS_FACTOR * sizeof(double), st, D, t0, t1, slot_base);
  return hipGetLastError();
}

static hipError_t set_dyn_lds(const void* f, bool& done) {
  if (done) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, LDS_FACTOR * sizeof(double));
  if (e == hipSuccess) done = true;
  return e;
}

hipError_t launch_task_levels(const DevData& D, const Task* tasks, const int32_t* level_begin, int32_t nlev,
                              int max_grid, hipStream_t st) {
  static bool attr = false;
  hipError_t e = set_dyn_lds((const void*)k_level_tasks, attr);
  if (e != hipSuccess) return e;
  for (int32_t l = 0; l < nlev; ++l) {
    const int32_t t0 = level_begin[l], t1 = level_begin[l + 1];
    const int g = (t1 - t0) < max_grid ? (t1 - t0) : max_grid;
    if (g > 0) hipLaunchKernelGGL(k_level_tasks, dim3(g), dim3(NT), LDS_FACTOR * sizeof(double), st, D, tasks, t0, t1);
  }
  return hipGetLastError();
}

hipError_t launch_apply(const DevData& D, int mode, const int32_t* chunks, int32_t nchunks, int max_grid,
                        hipStream_t st) {
  const int g = nchunks < max_grid ? nchunks : max_grid;
  if (g > 0) hipLaunchKernelGGL(k_apply, dim3(g), dim3(NT), 0, st, D, mode, chunks, nchunks);
  return hipGetLastError();
}

hipError_t launch_exact_block(const DevData& D, const int64_t* iperm, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                              double* out, int64_t ldo, hipStream_t st) {
  const int64_t total = ni * nj;
  if (total <= 0) return hipSuccess;
  int64_t g = (total + NT - 1) / NT;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_exact_block, dim3((unsigned)g), dim3(NT), 0, st, D, iperm, i0, ni, j0, nj, out, ldo);
  return hipGetLastError();
}

hipError_t launch_dense_matvec(const DevData& D, hipStream_t st) {
  const int64_t g = (D.n + NT - 1) / NT;
  hipLaunchKernelGGL(k_dense_matvec, dim3((unsigned)g), dim3(NT), 0, st, D);
  return hipGetLastError();
}

hipError_t launch_refine_resid(const double* Z, const double* Y, double* R, int64_t n, int r, double* part, int grid,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_refine_resid, dim3(grid), dim3(NT), 0, st, Z, Y, R, n, r, part);
  return hipGetLastError();
}

hipError_t launch_refine_update(double* X, const double* Dx, const double* Z, int64_t n, int r, double* part,
                                int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_update, dim3(grid), dim3(NT), 0, st, X, Dx, Z, n, r, part);
  return hipGetLastError();
}

hipError_t launch_permute(const double* Z, const int64_t* perm, int64_t n, int r, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_permute, dim3(1024), dim3(NT), 0, st, Z, perm, n, r, W);
  return hipGetLastError();
}

hipError_t launch_unpermute(const double* W, const int64_t* perm, int64_t n, int r, double* Z, hipStream_t st) {
  hipLaunchKernelGGL(k_unpermute, dim3(1024), dim3(NT), 0, st, W, perm, n, r, Z);
  return hipGetLastError();
}

hipError_t launch_solve_reduce(const DevData& D, const int32_t* diag_ids, int32_t ndiag, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(NT), 0, st, D, diag_ids, ndiag, D.W, D.r, out);
  return hipGetLastError();
}

hipError_t launch_solve(const DevData& D, const double* Z, const int64_t* perm, const int32_t* slevel_begin,
                        int32_t nslev, int max_grid, const int32_t* diag_ids, int32_t ndiag, double* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_permute, dim3(1024), dim3(NT), 0, st, Z, perm, D.n, D.r, D.W);
  const hipError_t e = launch_task_levels(D, D.stasks, slevel_begin, nslev, max_grid, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(NT), 0, st, D, diag_ids, ndiag, D.W, D.r, out);
  return hipGetLastError();
}

}  // namespace hm
