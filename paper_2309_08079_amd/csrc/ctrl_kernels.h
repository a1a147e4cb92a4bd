// The control step around the solve: linearisation of the nonlinear problem into the LQ
// problem (MPCGPU Section III-A, Step 1) and the parallel line search with the L1 merit
// (Section III-A, Step 3; Section IV-C).
//
// Model: a chain of NQ = NX / 2 pendulum joints with torsional springs between neighbours,
// one torque per joint, stepped by explicit Euler with timestep h,
//   q+ = q + h v,   v+ = v + h acc,
//   acc_i = u_i - g_i sin q_i - d v_i + kappa (sin(q_{i+1} - q_i) - sin(q_i - q_{i-1}))
// (spring terms that would reach past either end of the chain are absent).
// Cost: J = sum_k 1/2 (x_k - xref_k)^T Q_k (x_k - xref_k) + sum_k 1/2 u_k^T R_k u_k.
// Constraints: c = [x_0 - x_s, x_1 - f(x_0, u_0), ..., x_{N-1} - f(x_{N-2}, u_{N-2})].
//
// Work mapping: a batch is cut into chunks of up to kMaxChunk knots of one problem (the host
// takes 8 when the batch is small, for latency, and 32 when it fills the device); one
// 256-thread workgroup per chunk, one thread per (knot, row) item.  There are no atomics and no
// memory clears: the line search writes per-chunk partial sums, and every chunk of a
// problem then reduces the same partials in the same order, so all of them take the same
// decision without synchronising.  Arithmetic is FP64 on the FP32 inputs; FP32 results
// are rounded once.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mpc {
namespace ctrl {

constexpr int kMaxChunk = 32;  // knots per workgroup: 8 for small batches, 32 for large ones
constexpr int kThreads = 256;
constexpr int kAlphas = 9;    // alpha = 2^-j, j = 0..8
constexpr int kParts = 2 * kAlphas + 1;  // cost(alpha), ||c(alpha)||_1, max |lambda|

struct Chunk {
  int64_t pk0;     // first knot of the problem (packed knot index)
  int32_t b;       // problem
  int32_t N;       // its horizon
  int32_t lk0;     // local knots [lk0, lk1) of this chunk
  int32_t lk1;
  int32_t c0;      // the problem's first chunk
  int32_t nch;     // and its number of chunks
};

struct CtrlArgs {
  // trajectory and model
  const float *X, *U, *xs, *xref, *Q, *R, *grav;
  float h, damp, kap, mu;
  const Chunk *chunks;
  int32_t nchunks;
  // line search
  const float *dX, *dU, *lam;
  double *part;          // [nchunks][kParts]
  float *X_out, *U_out;
  double *merit;         // [batch][kAlphas]
  int32_t *choice;       // [batch]
  // linearisation
  float *A, *B, *q, *r, *x0, *e;
};

__device__ __forceinline__ double alpha_of(int j) { return ldexp(1.0, -j); }

// acc_i of the chain at joint i from positions q (stride 1), velocity v_i and torque u_i
template <int NQ>
__device__ __forceinline__ double chain_acc(const double *q, int i, double v, double u, double g, double d,
                                            double kap) {
  double spring = 0.0;
  if (i + 1 < NQ) spring += sin(q[i + 1] - q[i]);
  if (i > 0) spring -= sin(q[i] - q[i - 1]);
  return u - g * sin(q[i]) - d * v + kap * spring;
}

// ---- Step 1: linearisation ------------------------------------------------------------
// item (k, i): row i of A_k, B_k, e_k and q_k; rows i < NU also r_k; knot 0 also x0.
template <int NX>
__global__ void __launch_bounds__(kThreads) linearize_kernel(const CtrlArgs a) {
  constexpr int NQ = NX / 2, NU = NQ;
  const Chunk C = a.chunks[blockIdx.x];
  const int nk = C.lk1 - C.lk0;
  const int64_t cbase = C.pk0 - C.b;  // control rows of this problem start here
  for (int t = threadIdx.x; t < nk * NX; t += kThreads) {
    const int lk = C.lk0 + t / NX, i = t % NX;
    const int64_t kg = C.pk0 + lk;
    const float *x = a.X + kg * NX;
    // cost gradient q_k = Q_k (x_k - xref_k)
    const float *qrow = a.Q + (kg * NX + i) * NX;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NX; ++j) s += (double)qrow[j] * ((double)x[j] - (double)a.xref[kg * NX + j]);
    a.q[kg * NX + i] = (float)s;
    if (lk == 0) a.x0[(int64_t)C.b * NX + i] = (float)((double)a.xs[(int64_t)C.b * NX + i] - (double)x[i]);
    if (lk >= C.N - 1) continue;
    const int64_t kc = cbase + lk;
    const float *u = a.U + kc * NU;
    const float *xn = x + NX;
    float *arow = a.A + (kc * NX + i) * NX;
    float *brow = a.B + (kc * NX + i) * NU;
    if (i < NQ) {  // q+ = q + h v
#pragma unroll
      for (int j = 0; j < NX; ++j) arow[j] = (j == i) ? 1.0f : (j == NQ + i ? a.h : 0.0f);
#pragma unroll
      for (int j = 0; j < NU; ++j) brow[j] = 0.0f;
      const double f = (double)x[i] + (double)a.h * (double)x[NQ + i];
      a.e[kc * NX + i] = (float)((double)xn[i] - f);
    } else {       // v+ = v + h acc
      const int p = i - NQ;
      double qd[NQ];
#pragma unroll
      for (int j = 0; j < NQ; ++j) qd[j] = (double)x[j];
      const double h = a.h, d = a.damp, kap = a.kap, g = a.grav[p];
      const double cr = (p + 1 < NQ) ? cos(qd[p + 1 < NQ ? p + 1 : p] - qd[p]) : 0.0;
      const double cl = (p > 0) ? cos(qd[p] - qd[p > 0 ? p - 1 : p]) : 0.0;
      const double diag = -g * cos(qd[p]) - kap * (cr + cl);
#pragma unroll
      for (int j = 0; j < NQ; ++j) {
        double dq = (j == p) ? diag : (j == p + 1 ? kap * cr : (j == p - 1 ? kap * cl : 0.0));
        arow[j] = (float)(h * dq);
        arow[NQ + j] = (j == p) ? (float)(1.0 - h * d) : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < NU; ++j) brow[j] = (j == p) ? a.h : 0.0f;
      const double v = x[NQ + p];
      const double acc = chain_acc<NQ>(qd, p, v, (double)u[p], g, d, kap);
      a.e[kc * NX + i] = (float)((double)xn[i] - (v + h * acc));
    }
    if (i < NU) {  // r_k = R_k u_k
      const float *rrow = a.R + (kc * NU + i) * NU;
      double sr = 0.0;
#pragma unroll
      for (int j = 0; j < NU; ++j) sr += (double)rrow[j] * (double)u[j];
      a.r[kc * NU + i] = (float)sr;
    }
  }
}

// ---- Step 3: merit of every trial step, per chunk -------------------------------------
template <int NX>
__global__ void __launch_bounds__(kThreads) merit_kernel(const CtrlArgs a) {
  constexpr int NQ = NX / 2, NU = NQ;
  const Chunk C = a.chunks[blockIdx.x];
  const int nk = C.lk1 - C.lk0;
  const int64_t cbase = C.pk0 - C.b;
  double cost[kAlphas], viol[kAlphas], lmax = 0.0;
#pragma unroll
  for (int j = 0; j < kAlphas; ++j) { cost[j] = 0.0; viol[j] = 0.0; }

  // state rows: 1/2 e_i (Q e)_i with e = x + alpha dx - xref, linear in alpha per row
  for (int t = threadIdx.x; t < nk * NX; t += kThreads) {
    const int lk = C.lk0 + t / NX, i = t % NX;
    const int64_t kg = C.pk0 + lk;
    const float *qrow = a.Q + (kg * NX + i) * NX;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double qj = qrow[j];
      s0 += qj * ((double)a.X[kg * NX + j] - (double)a.xref[kg * NX + j]);
      s1 += qj * (double)a.dX[kg * NX + j];
    }
    const double e0 = (double)a.X[kg * NX + i] - (double)a.xref[kg * NX + i];
    const double de = a.dX[kg * NX + i];
#pragma unroll
    for (int j = 0; j < kAlphas; ++j) {
      const double al = alpha_of(j);
      cost[j] += 0.5 * (e0 + al * de) * (s0 + al * s1);
    }
    if (lk == 0) {  // c_0 = x_0 - x_s
      const double x = a.X[kg * NX + i], xs = a.xs[(int64_t)C.b * NX + i];
#pragma unroll
      for (int j = 0; j < kAlphas; ++j) viol[j] += fabs(x + alpha_of(j) * de - xs);
    }
    if (a.lam) lmax = fmax(lmax, fabs((double)a.lam[kg * NX + i]));
  }

  // control rows: 1/2 u_i (R u)_i
  const int nkc = (C.lk1 < C.N - 1 ? C.lk1 : C.N - 1) - C.lk0;
  for (int t = threadIdx.x; t < nkc * NU; t += kThreads) {
    const int lk = C.lk0 + t / NU, i = t % NU;
    const int64_t kc = cbase + lk;
    const float *rrow = a.R + (kc * NU + i) * NU;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double rj = rrow[j];
      s0 += rj * (double)a.U[kc * NU + j];
      s1 += rj * (double)a.dU[kc * NU + j];
    }
    const double u0 = a.U[kc * NU + i], du = a.dU[kc * NU + i];
#pragma unroll
    for (int j = 0; j < kAlphas; ++j) {
      const double al = alpha_of(j);
      cost[j] += 0.5 * (u0 + al * du) * (s0 + al * s1);
    }
  }

  // dynamics rows: |q+ - (q + h v)| + |v+ - (v + h acc)| of joint i, knot k -> k + 1, one
  // item per (step length, knot, joint): the sines dominate, so the items of a chunk are
  // spread over all its threads.  The terms are summed per step length in item order
  // below, the same order for every step length, so equal trial points give equal merits.
  __shared__ double dyn[kAlphas][kMaxChunk * NQ];
  const int ndyn = nkc * NQ;
  for (int t = threadIdx.x; t < ndyn * kAlphas; t += kThreads) {
    const int j = t / ndyn, rest = t % ndyn;
    const int lk = C.lk0 + rest / NQ, i = rest % NQ;
    const int64_t kg = C.pk0 + lk, kc = cbase + lk;
    const float *x = a.X + kg * NX, *dx = a.dX + kg * NX;
    const double h = a.h, d = a.damp, kap = a.kap, g = a.grav[i];
    const double al = alpha_of(j);
    double qa[NQ];
#pragma unroll
    for (int m = 0; m < NQ; ++m) qa[m] = (double)x[m] + al * (double)dx[m];
    const double v = (double)x[NQ + i] + al * (double)dx[NQ + i];
    const double u = (double)a.U[kc * NU + i] + al * (double)a.dU[kc * NU + i];
    const double qn = (double)x[NX + i] + al * (double)dx[NX + i];
    const double vn = (double)x[NX + NQ + i] + al * (double)dx[NX + NQ + i];
    const double acc = chain_acc<NQ>(qa, i, v, u, g, d, kap);
    dyn[j][rest] = fabs(qn - (qa[i] + h * v)) + fabs(vn - (v + h * acc));
  }

  // workgroup reduction in a fixed order
  __shared__ double red[kThreads / 64][kParts];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kAlphas; ++j) {
    double c = cost[j], v = viol[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      c += __shfl_xor(c, o);
      v += __shfl_xor(v, o);
    }
    if (lane == 0) { red[w][j] = c; red[w][kAlphas + j] = v; }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, o));
  if (lane == 0) red[w][2 * kAlphas] = lmax;
  __syncthreads();
  if (threadIdx.x < kParts) {
    const int j = threadIdx.x;
    double s = red[0][j];
    for (int ww = 1; ww < kThreads / 64; ++ww) s = (j == 2 * kAlphas) ? fmax(s, red[ww][j]) : s + red[ww][j];
    if (j >= kAlphas && j < 2 * kAlphas)
      for (int t = 0; t < ndyn; ++t) s += dyn[j - kAlphas][t];
    a.part[(int64_t)blockIdx.x * kParts + j] = s;
  }
}

// ---- Step 3: selection and update, per chunk ------------------------------------------
template <int NX>
__global__ void __launch_bounds__(kThreads) ls_update_kernel(const CtrlArgs a) {
  constexpr int NQ = NX / 2, NU = NQ;
  const Chunk C = a.chunks[blockIdx.x];
  // The problem's partials, reduced in a fixed order (the same in every chunk): member m of
  // the group of value j sums chunks m, m + kLanes, ... in order, then the group's sums
  // are added in member order.
  constexpr int kLanes = kThreads / kParts;  // 13 members per value
  __shared__ double sub[kParts][kLanes];
  __shared__ double tot[kParts];
  __shared__ int pick;
  if (threadIdx.x < kParts * kLanes) {
    const int j = threadIdx.x / kLanes, m = threadIdx.x % kLanes;
    double s = 0.0;
    for (int c = m; c < C.nch; c += kLanes) {
      const double v = a.part[(int64_t)(C.c0 + c) * kParts + j];
      s = (j == 2 * kAlphas) ? fmax(s, v) : s + v;
    }
    sub[j][m] = s;
  }
  __syncthreads();
  if (threadIdx.x < kParts) {
    const int j = threadIdx.x;
    double s = sub[j][0];
    for (int m = 1; m < kLanes; ++m) s = (j == 2 * kAlphas) ? fmax(s, sub[j][m]) : s + sub[j][m];
    tot[j] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double mu = (double)a.mu + (a.lam ? tot[2 * kAlphas] : 0.0);
    int best = 0;
    double bphi = tot[0] + mu * tot[kAlphas];
    for (int j = 1; j < kAlphas; ++j) {
      const double phi = tot[j] + mu * tot[kAlphas + j];
      if (phi < bphi) { bphi = phi; best = j; }
    }
    pick = best;
    if (C.lk0 == 0) {
      for (int j = 0; j < kAlphas; ++j) a.merit[(int64_t)C.b * kAlphas + j] = tot[j] + mu * tot[kAlphas + j];
      a.choice[C.b] = best;
    }
  }
  __syncthreads();
  const double al = alpha_of(pick);
  const int nk = C.lk1 - C.lk0;
  for (int t = threadIdx.x; t < nk * NX; t += kThreads) {
    const int64_t o = (C.pk0 + C.lk0) * NX + t;
    a.X_out[o] = (float)((double)a.X[o] + al * (double)a.dX[o]);
  }
  const int nkc = (C.lk1 < C.N - 1 ? C.lk1 : C.N - 1) - C.lk0;
  for (int t = threadIdx.x; t < nkc * NU; t += kThreads) {
    const int64_t o = (C.pk0 - C.b + C.lk0) * NU + t;
    a.U_out[o] = (float)((double)a.U[o] + al * (double)a.dU[o]);
  }
}

}  // namespace ctrl
}  // namespace mpc
