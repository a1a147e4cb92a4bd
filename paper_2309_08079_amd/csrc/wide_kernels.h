// Generic-size path (any nx <= 32, nu <= nx; built for the 28-state / 14-control shape).
//
// The 14-state kernel keeps each knot's rows of S and Phi^-1 in registers, one 16-lane
// DPP row per knot.  A 28-row block does not fit that mapping (a row of S is 84 FP64
// values), so this path stages the blocks in a device workspace instead:
//   wide_form    one workgroup per knot: Q^-1, R^-1, the S row blocks, gamma (or the
//                adjoint right-hand side) and D^-1, in FP64, matrices in LDS;
//   wide_precond one workgroup per knot: Phi^-1 row blocks -D_b^-1 S_{b,b+-1} D_{b+-1}^-1
//                (FP32) once every D^-1 exists (the one cross-knot dependency);
//   wide_pcg     one workgroup per problem: PCG (Algorithm 1) with one matrix row per
//                thread, S and Phi^-1 streamed from the workspace every iteration and
//                the vectors broadcast from LDS; then the primal step, or in adjoint mode
//                nu_1 and the block-sparse gradients.
// Precision matches the 14-state kernel: FP64 formation, S, vectors and reductions; FP32
// Phi^-1.  Method references: S, gamma (Section III-B, sign-flipped so S is positive
// definite), Phi^-1 (Section IV-A), PCG (Algorithm 1), dZ = -G^-1 (g - C^T lambda).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpcpcg.h"

namespace mpc {
namespace wide {

struct KnotDesc {    // one per knot of the packed batch
  int64_t k0;        // first knot row of the problem
  int32_t N;         // horizon of the problem
  int32_t b;         // knot index within the problem
  int32_t id;        // problem index
  int32_t pad;
};

struct ProbDescW {
  int64_t k0;
  int32_t N;
  int32_t id;
};

struct WArgs {
  const float *Q, *R, *A, *B, *q, *r, *x0, *e;
  const float *lam_in, *dx_in, *du_in, *gl, *gx, *gu;
  float *lam, *dx, *du;
  mpcpcg_stats *stats;
  float *dQ, *dR, *dA, *dB, *dq, *dr, *dx0, *de, *dgamma;
  float *S_out, *P_out, *gam_out;
  const KnotDesc *knots;
  const ProbDescW *probs;
  int32_t nknots, nprobs;
  // workspace (FP64 unless noted)
  double *S;      // [K][3][NX][NX]
  double *Dinv;   // [K][NX][NX]
  float *P;       // [K][3][NX][NX]
  double *rhs;    // [K][NX]
  double *Qinv;   // [K][NX][NX]
  double *RW;     // [controls][NU][NU + NX]: R^-1 rows then (R^-1 B^T) rows
  float eps;
  int32_t max_iter;
  int32_t warm;
  int32_t adjoint;
  int32_t stop_abs;   // 1: eta < eps; 0: sqrt(eta / eta_ref) < eps
  int32_t from_ws;    // 1: wide_pcg skips PCG and takes lambda from lamw (factorisation path)
  double *lamw;       // [K][NX] lambda of the factorisation path
};

// ---------------------------------------------------------------- LDS dense helpers
// In-place Gauss-Jordan inverse of an n x n SPD matrix in LDS (row stride ld); SPD needs
// no pivoting.  All threads of the block participate.
// `nonpositive` (optional, shared): set to 1 when a pivot is not > 0, i.e. the matrix is not
// positive definite.
template <int NT>
__device__ void lds_gj_inverse(double *a, int n, int ld, int *nonpositive = nullptr) {
  __shared__ double piv_row[64];
  __shared__ double col[64];
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    for (int t = threadIdx.x; t < n; t += NT) {
      piv_row[t] = a[k * ld + t];
      col[t] = a[t * ld + k];
    }
    __syncthreads();
    if (nonpositive && threadIdx.x == 0 && !(piv_row[k] > 0.0)) *nonpositive = 1;
    const double d = 1.0 / piv_row[k];
    for (int t = threadIdx.x; t < n * n; t += NT) {
      const int i = t / n, j = t % n;
      double v;
      if (i == k)
        v = (j == k) ? d : piv_row[j] * d;
      else
        v = (j == k) ? -col[i] * d : a[i * ld + j] - col[i] * d * piv_row[j];
      a[i * ld + j] = v;
    }
  }
  __syncthreads();
}

// C (m x n, ld n) = op(X) (m x k) * op(Y) (k x n); tx/ty transpose the stored operands.
template <int NT>
__device__ void lds_gemm(double *C, const double *X, bool tx, int ldx, const double *Y, bool ty,
                         int ldy, int m, int k, int n, double alpha, bool accumulate) {
  __syncthreads();
  for (int t = threadIdx.x; t < m * n; t += NT) {
    const int i = t / n, j = t % n;
    double s = 0.0;
    for (int p = 0; p < k; ++p) {
      const double xv = tx ? X[p * ldx + i] : X[i * ldx + p];
      const double yv = ty ? Y[j * ldy + p] : Y[p * ldy + j];
      s = __builtin_fma(xv, yv, s);
    }
    C[i * n + j] = accumulate ? __builtin_fma(alpha, s, C[i * n + j]) : alpha * s;
  }
  __syncthreads();
}

template <int NT>
__device__ void lds_load(double *dst, const float *src, int count, bool valid) {
  for (int t = threadIdx.x; t < count; t += NT) dst[t] = valid ? (double)src[t] : 0.0;
}

template <int NT>
__device__ void lds_identity(double *dst, int n) {
  for (int t = threadIdx.x; t < n * n; t += NT) dst[t] = (t / n == t % n) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------- formation
// Knot b of its problem: S row blocks (b,b-1), (b,b), (b,b+1), rhs_b and D_b^-1.
template <int NX, int NU>
__global__ void __launch_bounds__(256) wide_form(const WArgs a) {
  constexpr int NT = 256;
  constexpr int MM = NX * NX;
  __shared__ double Qm[MM], Am[MM], T[MM], Th[MM], Qi[MM], X[MM];
  __shared__ double Rm[NU * NU], Bm[NX * NU], U[NX * NU];
  __shared__ double v0[NX], v1[NX], v2[NX];
  const KnotDesc kd = a.knots[blockIdx.x];
  const int b = kd.b, N = kd.N;
  const int64_t kb = kd.k0 + b;
  const int64_t cb = kd.k0 - kd.id + b;  // packed control row of control b
  const bool hasPrev = b >= 1, hasNext = b + 1 < N;
  const bool adj = a.adjoint != 0;
  const float *qv = adj ? a.gx : a.q;
  const float *rv = adj ? a.gu : a.r;
  const int tid = threadIdx.x;
  double *Sb = a.S + kb * 3 * MM;

  // (1) previous knot: T = A_{b-1} Q_{b-1}^-1, S_{b,b-1} = -T, theta = T A^T + ...
  if (hasPrev) {
    lds_load<NT>(Qm, a.Q + (kb - 1) * MM, MM, true);
    lds_load<NT>(Am, a.A + (cb - 1) * MM, MM, true);
  } else {
    lds_identity<NT>(Qm, NX);
    lds_load<NT>(Am, nullptr, MM, false);
  }
  lds_gj_inverse<NT>(Qm, NX, NX);
  lds_gemm<NT>(T, Am, false, NX, Qm, false, NX, NX, NX, NX, 1.0, false);
  lds_gemm<NT>(Th, T, false, NX, Am, true, NX, NX, NX, NX, 1.0, false);
  for (int t = tid; t < MM; t += NT) Sb[t] = -T[t];
  for (int t = tid; t < NX; t += NT) v0[t] = (hasPrev && qv) ? (double)qv[(kb - 1) * NX + t] : 0.0;
  __syncthreads();
  // (2) control b-1: R^-1, U = B R^-1, theta += U B^T, W = R^-1 B^T
  if (hasPrev) {
    lds_load<NT>(Rm, a.R + (cb - 1) * NU * NU, NU * NU, true);
    lds_load<NT>(Bm, a.B + (cb - 1) * NX * NU, NX * NU, true);
  } else {
    lds_identity<NT>(Rm, NU);
    lds_load<NT>(Bm, nullptr, NX * NU, false);
  }
  for (int t = tid; t < NU; t += NT) v1[t] = (hasPrev && rv) ? (double)rv[(cb - 1) * NU + t] : 0.0;
  lds_gj_inverse<NT>(Rm, NU, NU);
  lds_gemm<NT>(U, Bm, false, NU, Rm, false, NU, NX, NU, NU, 1.0, false);
  lds_gemm<NT>(Th, U, false, NU, Bm, true, NU, NX, NU, NX, 1.0, true);
  if (hasPrev) {
    double *rw = a.RW + (cb - 1) * NU * (NU + NX);
    for (int t = tid; t < NU * NU; t += NT) rw[(t / NU) * (NU + NX) + t % NU] = Rm[t];
    for (int t = tid; t < NU * NX; t += NT) {  // W = R^-1 B^T, row i, column j
      const int i = t / NX, j = t % NX;
      double s = 0.0;
      for (int m = 0; m < NU; ++m) s = __builtin_fma(Rm[i * NU + m], Bm[j * NU + m], s);
      rw[i * (NU + NX) + NU + j] = s;
    }
  }
  // rhs_b = -T q_{b-1} - U r_{b-1} + Q_b^-1 q_b + add
  // (3) own knot
  lds_load<NT>(Qi, a.Q + kb * MM, MM, true);
  for (int t = tid; t < NX; t += NT) v2[t] = qv ? (double)qv[kb * NX + t] : 0.0;
  __syncthreads();
  // keep Q_b itself for D_0^-1 = Q_0
  for (int t = tid; t < MM; t += NT) X[t] = Qi[t];
  lds_gj_inverse<NT>(Qi, NX, NX);
  for (int t = tid; t < MM; t += NT) {
    a.Qinv[kb * MM + t] = Qi[t];
    Th[t] += Qi[t];
  }
  __syncthreads();
  for (int i = tid; i < NX; i += NT) {
    double s = 0.0;
    for (int m = 0; m < NX; ++m) s -= T[i * NX + m] * v0[m];
    for (int m = 0; m < NU; ++m) s -= U[i * NU + m] * v1[m];
    for (int m = 0; m < NX; ++m) s += Qi[i * NX + m] * v2[m];
    double add;
    if (adj) add = (double)a.gl[kb * NX + i];
    else if (b == 0) add = (double)a.x0[(int64_t)kd.id * NX + i];
    else add = a.e ? -(double)a.e[(cb - 1) * NX + i] : 0.0;
    a.rhs[kb * NX + i] = s + add;
  }
  // (4) S_{b,b+1} = -Q_b^-1 A_b^T
  if (hasNext) lds_load<NT>(Am, a.A + cb * MM, MM, true);
  else lds_load<NT>(Am, nullptr, MM, false);
  lds_gemm<NT>(T, Qi, false, NX, Am, true, NX, NX, NX, NX, -1.0, false);
  for (int t = tid; t < MM; t += NT) {
    Sb[2 * MM + t] = T[t];
    Sb[MM + t] = Th[t];
  }
  // (5) D_b^-1 = theta^-1, D_0^-1 = Q_0
  if (b == 0) {
    for (int t = tid; t < MM; t += NT) a.Dinv[kb * MM + t] = X[t];
  } else {
    __syncthreads();
    lds_gj_inverse<NT>(Th, NX, NX);
    for (int t = tid; t < MM; t += NT) a.Dinv[kb * MM + t] = Th[t];
  }
}

// Phi^-1 blocks of knot b (needs D^-1 of b-1, b, b+1) and optional FP32 export of S/gamma.
template <int NX, int NU>
__global__ void __launch_bounds__(256) wide_precond(const WArgs a) {
  constexpr int NT = 256;
  constexpr int MM = NX * NX;
  __shared__ double Db[MM], Dn[MM], Sx[MM], X[MM], Y[MM];
  const KnotDesc kd = a.knots[blockIdx.x];
  const int b = kd.b, N = kd.N;
  const int64_t kb = kd.k0 + b;
  const int tid = threadIdx.x;
  for (int t = tid; t < MM; t += NT) Db[t] = a.Dinv[kb * MM + t];
  float *Pb = a.P + kb * 3 * MM;
  for (int t = tid; t < MM; t += NT) Pb[MM + t] = (float)Db[t];
  for (int side = 0; side < 2; ++side) {
    const bool has = side == 0 ? b >= 1 : b + 1 < N;
    const int slot = side == 0 ? 0 : 2;
    if (!has) {
      for (int t = tid; t < MM; t += NT) Pb[slot * MM + t] = 0.0f;
      continue;
    }
    const int64_t kn = side == 0 ? kb - 1 : kb + 1;
    __syncthreads();
    for (int t = tid; t < MM; t += NT) {
      Dn[t] = a.Dinv[kn * MM + t];
      Sx[t] = a.S[kb * 3 * MM + slot * MM + t];
    }
    lds_gemm<NT>(X, Db, false, NX, Sx, false, NX, NX, NX, NX, 1.0, false);
    lds_gemm<NT>(Y, X, false, NX, Dn, false, NX, NX, NX, NX, -1.0, false);
    for (int t = tid; t < MM; t += NT) Pb[slot * MM + t] = (float)Y[t];
  }
  if (a.S_out) {
    for (int t = tid; t < 3 * MM; t += NT) {
      a.S_out[kb * 3 * MM + t] = (float)a.S[kb * 3 * MM + t];
      a.P_out[kb * 3 * MM + t] = Pb[t];
    }
    for (int t = tid; t < NX; t += NT) a.gam_out[kb * NX + t] = (float)a.rhs[kb * NX + t];
  }
}

// ---------------------------------------------------------------- factorisation
// Block LDL^T of the block-tridiagonal S of one problem per workgroup (the factorisation
// path; the same recurrence as the 14-state sweep, with 28 x 28 blocks in LDS):
//   D_0 = S_00, D_k = S_kk - S_{k,k-1} D_{k-1}^-1 S_{k-1,k}, y_k = rhs_k - S_{k,k-1} D_{k-1}^-1 y_{k-1},
//   lambda_k = D_k^-1 (y_k - S_{k,k+1} lambda_{k+1}).
// Reads the S blocks and rhs written by wide_form; overwrites Dinv with D_k^-1 and rhs with
// y_k; writes lambda to lamw and the problem's stats (BREAKDOWN on a pivot <= 0 or a
// non-finite lambda).
template <int NX>
__global__ void __launch_bounds__(256) wide_sweep(const WArgs a) {
  constexpr int NT = 256;
  constexpr int MM = NX * NX;
  __shared__ double Sm[MM], D[MM], Sp[MM], Dp[MM], Spp[MM], L[MM], T[MM];
  __shared__ double y[NX], yp[NX], lv[NX], tv[NX];
  __shared__ int bad;
  const ProbDescW pd = a.probs[blockIdx.x];
  const int N = pd.N;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int k = 0; k < N; ++k) {
    const int64_t kb = pd.k0 + k;
    __syncthreads();
    for (int t = tid; t < MM; t += NT) {
      Sm[t] = a.S[kb * 3 * MM + t];
      D[t] = a.S[kb * 3 * MM + MM + t];
      Sp[t] = a.S[kb * 3 * MM + 2 * MM + t];
    }
    for (int t = tid; t < NX; t += NT) y[t] = a.rhs[kb * NX + t];
    __syncthreads();
    if (k > 0) {
      lds_gemm<NT>(L, Sm, false, NX, Dp, false, NX, NX, NX, NX, 1.0, false);   // S_{k,k-1} D_{k-1}^-1
      lds_gemm<NT>(T, L, false, NX, Spp, false, NX, NX, NX, NX, 1.0, false);  // ... S_{k-1,k}
      for (int t = tid; t < MM; t += NT) D[t] -= T[t];
      for (int i = tid; i < NX; i += NT) {
        double s = y[i];
        for (int m = 0; m < NX; ++m) s = __builtin_fma(-L[i * NX + m], yp[m], s);
        tv[i] = s;
      }
      __syncthreads();
      for (int i = tid; i < NX; i += NT) y[i] = tv[i];
    }
    lds_gj_inverse<NT>(D, NX, NX, &bad);  // D_k^-1
    __syncthreads();
    for (int t = tid; t < MM; t += NT) {
      a.Dinv[kb * MM + t] = D[t];
      Dp[t] = D[t];
      Spp[t] = Sp[t];
    }
    for (int t = tid; t < NX; t += NT) {
      a.rhs[kb * NX + t] = y[t];
      yp[t] = y[t];
    }
  }
  __syncthreads();
  for (int t = tid; t < NX; t += NT) lv[t] = 0.0;
  bool finite = true;
  for (int k = N - 1; k >= 0; --k) {
    const int64_t kb = pd.k0 + k;
    __syncthreads();
    for (int i = tid; i < NX; i += NT) {
      double s = a.rhs[kb * NX + i];
      const double *sp = a.S + kb * 3 * MM + 2 * MM + i * NX;
      for (int j = 0; j < NX; ++j) s = __builtin_fma(-sp[j], lv[j], s);
      tv[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < NX; i += NT) {
      double s = 0.0;
      const double *dr = a.Dinv + kb * MM + i * NX;
      for (int j = 0; j < NX; ++j) s = __builtin_fma(dr[j], tv[j], s);
      finite = finite && (s == s) && !__builtin_isinf(s);
      a.lamw[kb * NX + i] = s;
      lv[i] = s;
    }
  }
  if (!finite) bad = 1;
  __syncthreads();
  if (tid == 0) {
    mpcpcg_stats st;
    st.iters = 0;
    st.status = bad ? MPCPCG_BREAKDOWN : MPCPCG_OK;
    st.final_ratio = 0.0f;
    st.reserved = 0;
    a.stats[pd.id] = st;
  }
}

// ---------------------------------------------------------------- PCG per problem
constexpr int kWideThreads = 1024;
constexpr int kWideRows = 8;  // rows per thread: N * NX <= 8192

__device__ __forceinline__ double block_sum(double v, double *red) {
  // fixed-shape reduction: butterfly within each wave, then waves in order
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// Dynamic LDS: vd [N+2][NX] FP64, vf [N+2][NX] FP32, vu [N][NU] FP64 (row 0 and N+1 of the
// vectors are zero halos).
template <int NX, int NU>
__global__ void __launch_bounds__(kWideThreads) wide_pcg(const WArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[kWideThreads / 64];
  constexpr int MM = NX * NX;
  const ProbDescW pd = a.probs[blockIdx.x];
  const int N = pd.N;
  const int64_t k0 = pd.k0, c0 = pd.k0 - pd.id;
  const int rows = N * NX;
  double *vd = lds;                                   // [N+2][NX]
  float *vf = reinterpret_cast<float *>(vd + (N + 2) * NX);  // [N+2][NX]
  double *vu = reinterpret_cast<double *>(vf + ((N + 2) * NX + 1) / 2 * 2);  // [N][NU]
  const int tid = threadIdx.x;
  const bool adj = a.adjoint != 0;
  for (int t = tid; t < NX; t += kWideThreads) {
    vd[t] = 0.0; vd[(N + 1) * NX + t] = 0.0;
    vf[t] = 0.0f; vf[(N + 1) * NX + t] = 0.0f;
  }
  // row ownership: thread t owns rows g = t + s * kWideThreads
  double lam[kWideRows], r[kWideRows], p[kWideRows], Y[kWideRows], g0[kWideRows];
  float rt[kWideRows];
#pragma unroll
  for (int s = 0; s < kWideRows; ++s) {
    const int g = tid + s * kWideThreads;
    const bool ok = g < rows;
    lam[s] = (ok && a.warm && !adj) ? (double)a.lam[k0 * NX + g] : 0.0;
    g0[s] = ok ? a.rhs[k0 * NX + g] : 0.0;
  }
  // matvec with the S (FP64) or Phi^-1 (FP32) row of global row g against an LDS vector
  auto s_row = [&](int g, const double *v) {
    const int b = g / NX, i = g % NX;
    const double *Srow = a.S + (k0 + b) * 3 * MM + i * NX;
    double acc = 0.0;
    for (int slot = 0; slot < 3; ++slot) {
      const double *x = v + (b + slot) * NX;  // halo-shifted: row b-1 of the vector is b
      const double *m = Srow + slot * MM;
      for (int j = 0; j < NX; ++j) acc = __builtin_fma(m[j], x[j], acc);
    }
    return acc;
  };
  auto p_row = [&](int g, const float *v) {
    const int b = g / NX, i = g % NX;
    const float *Prow = a.P + (k0 + b) * 3 * MM + i * NX;
    float acc = 0.0f;
    for (int slot = 0; slot < 3; ++slot) {
      const float *x = v + (b + slot) * NX;
      const float *m = Prow + slot * MM;
      for (int j = 0; j < NX; ++j) acc = __builtin_fmaf(m[j], x[j], acc);
    }
    return acc;
  };
  auto put_d = [&](const double *src) {
#pragma unroll
    for (int s = 0; s < kWideRows; ++s) {
      const int g = tid + s * kWideThreads;
      if (g < rows) vd[NX + g] = src[s];
    }
  };
  auto put_f = [&](const double *src) {
#pragma unroll
    for (int s = 0; s < kWideRows; ++s) {
      const int g = tid + s * kWideThreads;
      if (g < rows) vf[NX + g] = (float)src[s];
    }
  };

  int status = MPCPCG_OK, it = 0;
  double eta_ref = 0.0, eta_new = 0.0;
  if (a.from_ws) {
#pragma unroll
    for (int s = 0; s < kWideRows; ++s) {
      const int g = tid + s * kWideThreads;
      lam[s] = g < rows ? a.lamw[k0 * NX + g] : 0.0;
    }
  } else {
  // eta_ref = rhs^T Phi^-1 rhs; r = rhs - S lambda_0
  put_f(g0);
  put_d(lam);
  __syncthreads();
  double pr = 0.0, pe = 0.0;
  float gt[kWideRows];
#pragma unroll
  for (int s = 0; s < kWideRows; ++s) {
    const int g = tid + s * kWideThreads;
    gt[s] = 0.0f;
    r[s] = g0[s];
    if (g < rows) {
      gt[s] = p_row(g, vf);
      if (a.warm && !adj) r[s] = g0[s] - s_row(g, vd);
    }
  }
  __syncthreads();
  put_f(r);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kWideRows; ++s) {
    const int g = tid + s * kWideThreads;
    rt[s] = g < rows ? p_row(g, vf) : 0.0f;
    pr += r[s] * (double)rt[s];
    pe += g0[s] * (double)gt[s];
    p[s] = (double)rt[s];
  }
  double eta = block_sum(pr, red);
  eta_ref = block_sum(pe, red);
  const double tau = a.stop_abs ? (double)a.eps : (double)a.eps * (double)a.eps * eta_ref;
  const int max_iter = a.max_iter > 0 ? a.max_iter : N * NX;
  status = MPCPCG_NOT_CONVERGED;
  eta_new = eta;
  if (!(eta == eta) || !(eta_ref == eta_ref) || __builtin_isinf(eta) || __builtin_isinf(eta_ref)) {
    status = MPCPCG_BREAKDOWN;
  } else if (eta <= tau) {
    status = MPCPCG_OK;
  } else {
    for (it = 1; it <= max_iter; ++it) {
      __syncthreads();
      put_d(p);
      __syncthreads();
      double pu = 0.0;
#pragma unroll
      for (int s = 0; s < kWideRows; ++s) {
        const int g = tid + s * kWideThreads;
        Y[s] = g < rows ? s_row(g, vd) : 0.0;
        pu += p[s] * Y[s];
      }
      const double ups = block_sum(pu, red);
      if (!(ups > 0.0) || __builtin_isinf(ups)) { status = MPCPCG_BREAKDOWN; break; }
      const double alpha = eta / ups;
#pragma unroll
      for (int s = 0; s < kWideRows; ++s) {
        lam[s] = __builtin_fma(alpha, p[s], lam[s]);
        r[s] = __builtin_fma(-alpha, Y[s], r[s]);
      }
      put_f(r);
      __syncthreads();
      double pn = 0.0;
#pragma unroll
      for (int s = 0; s < kWideRows; ++s) {
        const int g = tid + s * kWideThreads;
        rt[s] = g < rows ? p_row(g, vf) : 0.0f;
        pn += r[s] * (double)rt[s];
      }
      eta_new = block_sum(pn, red);
      if (!(eta_new == eta_new) || __builtin_isinf(eta_new)) { status = MPCPCG_BREAKDOWN; break; }
      if (eta_new < tau) { status = MPCPCG_OK; break; }
      const double beta = eta_new / eta;
#pragma unroll
      for (int s = 0; s < kWideRows; ++s) p[s] = __builtin_fma(beta, p[s], (double)rt[s]);
      eta = eta_new;
    }
    if (it > max_iter) it = max_iter;
  }
  }  // PCG (not the factorisation path)

  // ---------------------------------------------------------------- epilogue
  // x rows: dZx_b = -Q_b^-1 (q_b - lambda_b) + S_{b,b+1} lambda_{b+1};
  // u rows of control b-1: -R^-1 r_{b-1} - (R^-1 B^T) lambda_b  (mu and gradients in adjoint)
  const float *qv = adj ? a.gx : a.q;
  const float *rv = adj ? a.gu : a.r;
  __syncthreads();
  put_d(lam);
  __syncthreads();
  double xrow[kWideRows];
#pragma unroll
  for (int s = 0; s < kWideRows; ++s) {
    const int g = tid + s * kWideThreads;
    xrow[s] = 0.0;
    if (g < rows) {
      const int b = g / NX, i = g % NX;
      const double *Qi = a.Qinv + (k0 + b) * MM + i * NX;
      const double *Sp = a.S + (k0 + b) * 3 * MM + 2 * MM + i * NX;
      const double *lb = vd + (b + 1) * NX, *ln = vd + (b + 2) * NX;
      double acc = 0.0;
      for (int j = 0; j < NX; ++j) {
        const double qj = qv ? (double)qv[(k0 + b) * NX + j] : 0.0;
        acc = __builtin_fma(-Qi[j], qj - lb[j], acc);
        acc = __builtin_fma(Sp[j], ln[j], acc);
      }
      xrow[s] = acc;
    }
  }
  // u rows: thread t handles (control c = b-1 for b = 1..N-1, row i < NU)
  for (int g = tid; g < (N - 1) * NU; g += kWideThreads) {
    const int c = g / NU, i = g % NU;  // control c belongs to block row b = c + 1
    const double *rw = a.RW + (c0 + c) * NU * (NU + NX) + i * (NU + NX);
    const double *lb = vd + (c + 2) * NX;  // lambda_{c+1}
    double acc = 0.0;
    for (int m = 0; m < NU; ++m) acc -= rw[m] * (rv ? (double)rv[(c0 + c) * NU + m] : 0.0);
    for (int j = 0; j < NX; ++j) acc -= rw[NU + j] * lb[j];
    vu[c * NU + i] = acc;
  }
  if (!adj) {
#pragma unroll
    for (int s = 0; s < kWideRows; ++s) {
      const int g = tid + s * kWideThreads;
      if (g < rows) {
        a.lam[k0 * NX + g] = (float)lam[s];
        a.dx[k0 * NX + g] = (float)xrow[s];
      }
    }
    __syncthreads();
    for (int g = tid; g < (N - 1) * NU; g += kWideThreads) a.du[c0 * NU + g] = (float)vu[g];
  } else {
    // lam holds mu; xrow = nu1x; vu = nu1u.  vd (mu) is reused for nu1x after a barrier.
#pragma unroll
    for (int s = 0; s < kWideRows; ++s) {
      const int g = tid + s * kWideThreads;
      if (g < rows) {
        if (a.dgamma) a.dgamma[k0 * NX + g] = (float)lam[s];
        a.dq[k0 * NX + g] = (float)xrow[s];
        const int b = g / NX, i = g % NX;
        if (b == 0) a.dx0[(int64_t)pd.id * NX + i] = (float)lam[s];
        if (b >= 1 && a.de) a.de[(c0 + b - 1) * NX + i] = (float)(-lam[s]);
      }
    }
    // nu1x replaces mu in the LDS vector; mu (FP64) is staged in the right-hand-side
    // workspace, which PCG no longer needs
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kWideRows; ++s) {
      const int g = tid + s * kWideThreads;
      if (g < rows) a.rhs[k0 * NX + g] = lam[s];
    }
    put_d(xrow);
    __syncthreads();
    for (int g = tid; g < (N - 1) * NU; g += kWideThreads) a.dr[c0 * NU + g] = (float)vu[g];
    // dQ_b = sym(nu1x_b dx_b^T)
    for (int t = tid; t < N * MM; t += kWideThreads) {
      const int b = t / MM, i = (t / NX) % NX, j = t % NX;
      const double nx_i = vd[(b + 1) * NX + i], nx_j = vd[(b + 1) * NX + j];
      const double dx_i = (double)a.dx_in[(k0 + b) * NX + i], dx_j = (double)a.dx_in[(k0 + b) * NX + j];
      a.dQ[(k0 + b) * MM + i * NX + j] = (float)(0.5 * (nx_i * dx_j + nx_j * dx_i));
    }
    // control c of block row b = c + 1: dA_c = lambda_b nu1x_c^T + mu_b dx_c^T,
    // dB_c = lambda_b nu1u_c^T + mu_b du_c^T, dR_c = sym(nu1u_c du_c^T)
    for (int t = tid; t < (N - 1) * MM; t += kWideThreads) {
      const int c = t / MM, i = (t / NX) % NX, j = t % NX;
      const double lb_i = (double)a.lam_in[(k0 + c + 1) * NX + i];
      const double mu_i = a.rhs[(k0 + c + 1) * NX + i];
      const double n1x_j = vd[(c + 1) * NX + j];
      const double dx_j = (double)a.dx_in[(k0 + c) * NX + j];
      a.dA[(c0 + c) * MM + i * NX + j] = (float)(lb_i * n1x_j + mu_i * dx_j);
    }
    for (int t = tid; t < (N - 1) * NX * NU; t += kWideThreads) {
      const int c = t / (NX * NU), i = (t / NU) % NX, j = t % NU;
      const double lb_i = (double)a.lam_in[(k0 + c + 1) * NX + i];
      const double mu_i = a.rhs[(k0 + c + 1) * NX + i];
      const double n1u_j = vu[c * NU + j];
      const double du_j = (double)a.du_in[(c0 + c) * NU + j];
      a.dB[(c0 + c) * NX * NU + i * NU + j] = (float)(lb_i * n1u_j + mu_i * du_j);
    }
    for (int t = tid; t < (N - 1) * NU * NU; t += kWideThreads) {
      const int c = t / (NU * NU), i = (t / NU) % NU, j = t % NU;
      const double ni = vu[c * NU + i], nj = vu[c * NU + j];
      const double di = (double)a.du_in[(c0 + c) * NU + i], dj = (double)a.du_in[(c0 + c) * NU + j];
      a.dR[(c0 + c) * NU * NU + i * NU + j] = (float)(0.5 * (ni * dj + nj * di));
    }
  }
  if (tid == 0 && !a.from_ws) {
    mpcpcg_stats st;
    st.iters = it;
    st.status = status;
    st.final_ratio = eta_ref > 0.0 ? (float)__builtin_sqrt(eta_new > 0.0 ? eta_new / eta_ref : 0.0) : 0.0f;
    st.reserved = 0;
    a.stats[pd.id] = st;
  }
}

}  // namespace wide
}  // namespace mpc
