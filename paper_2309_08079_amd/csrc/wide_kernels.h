// Generic-size path (any nx <= 32, nu <= nx; built for the 28-state / 14-control shape).
//
// The 14-state kernel keeps each knot's rows of S and Phi^-1 in registers, one 16-lane
// DPP row per knot.  A 28-row block does not fit that mapping (a row of S is 84 FP64
// values), so this path stages the blocks in a device workspace instead:
//   wide_form_inv, wide_form_theta   one wave per knot (and per control): Q^-1, R^-1, the
//                S row blocks, gamma (or the adjoint right-hand side) and D^-1, in FP64,
//                rows in registers;
//   wide_precond one workgroup per knot: Phi^-1 row blocks -D_b^-1 S_{b,b+-1} D_{b+-1}^-1
//                (FP32) once every D^-1 exists (the one cross-knot dependency);
//   wide_pcg_gang (wide_pcg.h) PCG (Algorithm 1) on gangs of workgroups, rows of S and
//                Phi^-1 in registers; then wide_epilogue: the primal step, or in adjoint
//                mode nu_1 and the block-sparse gradients.
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
  int32_t no_dinv;    // 1: wide_form_theta skips D^-1 (only the preconditioner needs it)
  double *lamw;       // [K][NX] lambda of the factorisation path
};

// ---------------------------------------------------------------- LDS dense helpers
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

// ---------------------------------------------------------------- formation
// Two launches, one wave per task, lane r < n owning row r of an n x n block in registers.
//   wide_form_inv    task t < K: knot t inverts Q_t (Gauss-Jordan in registers), writes
//                    Q_t^-1 and S_{t,t+1} = -Q_t^-1 A_t^T, and its transpose as
//                    S_{t+1,t} (S is symmetric, Section III-B); task K + t: control t of
//                    knot t inverts R_t and writes (R_t^-1 | R_t^-1 B_t^T);
//   wide_form_theta  knot b: theta_b = A_{b-1} Q_{b-1}^-1 A_{b-1}^T + B_{b-1} R_{b-1}^-1
//                    B_{b-1}^T + Q_b^-1 = S_{b,b}, the right-hand side gamma_b (or the
//                    adjoint's) and, for the preconditioner, D_b^-1 = theta_b^-1.
// Each Q and R is inverted once (not once per neighbouring knot), and no step needs a
// workgroup barrier.  Products take the left operand's row from the lane's registers and
// the right operand's row from the wave's own LDS block, the same address for every lane
// (a broadcast read).
constexpr int kFormWaves = 4;

__device__ __forceinline__ double lane_value(double v, int m) {  // v of lane m (m uniform)
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), m);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), m);
  return __hiloint2double(hi, lo);
}

// order this wave's LDS accesses: its earlier writes complete before its later reads
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// In-place Gauss-Jordan inverse of an SPD N x N matrix (no pivoting), rows in the lanes'
// registers: the pivot row k is read from lane k with readlane.  `row` is the row a lane
// holds (lane k must hold row k; other lanes may hold copies of rows, or zeros under a row
// id >= N, and keep them consistent).  `pd` ends false if a pivot is not > 0.
template <int N>
__device__ __forceinline__ void reg_gj_inverse(double (&a)[N], int row, bool &pd) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double pk[N];
#pragma unroll
    for (int j = 0; j < N; ++j) pk[j] = lane_value(a[j], k);
    const double piv = pk[k];
    pd = pd && (piv > 0.0);
    const double d = 1.0 / piv;
    // pivot row: a_kj d; other rows: a_ij - f a_kj (f = a_ik d); column k: d / -f,
    // as c a_kj + s a_ij with (s, c) = (0, d) on the pivot lane and (1, -f) elsewhere
    const bool me = row == k;
    const double f = a[k] * d;
    const double sc = me ? 0.0 : 1.0, c = me ? d : -f;
#pragma unroll
    for (int j = 0; j < N; ++j) a[j] = (j == k) ? c : __builtin_fma(c, pk[j], sc * a[j]);
  }
}

// acc_j += sum_{m < M} x_m Y[m][j] for j < NX (Y in LDS, rows of NX)
template <int NX, int M>
__device__ __forceinline__ void row_times(const double (&x)[M], const double *Y, double (&acc)[NX]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double *y = Y + m * NX;
#pragma unroll
    for (int j = 0; j < NX; ++j) acc[j] = __builtin_fma(x[m], y[j], acc[j]);
  }
}

template <int NX, int NU>
__global__ void __launch_bounds__(kFormWaves * 64) wide_form_inv(const WArgs a) {
  constexpr int MM = NX * NX;
  __shared__ __attribute__((aligned(16))) double stage[kFormWaves][MM];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = blockIdx.x * kFormWaves + w;
  if (t >= 2 * a.nknots) return;  // whole waves leave; no workgroup barrier follows
  const bool ctrl = t >= a.nknots;
  const KnotDesc kd = a.knots[ctrl ? t - a.nknots : t];
  const int b = kd.b;
  const int64_t kb = kd.k0 + b;
  const int64_t cb = kd.k0 - kd.id + b;  // packed control row of control b
  const bool hasNext = b + 1 < kd.N;
  double *buf = stage[w];
  bool pd = true;
  if (!ctrl) {
    const bool rowv = lane < NX;
    const int r = rowv ? lane : 0;
    double q[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double v = (double)a.Q[kb * MM + r * NX + j];
      q[j] = rowv ? v : 0.0;
    }
    reg_gj_inverse<NX>(q, lane, pd);
    if (rowv)
#pragma unroll
      for (int j = 0; j < NX; ++j) a.Qinv[kb * MM + r * NX + j] = q[j];
    double *S = a.S + kb * 3 * MM;
    if (b == 0 && rowv)
#pragma unroll
      for (int j = 0; j < NX; ++j) S[r * NX + j] = 0.0;  // no S_{0,-1}
    double acc[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) acc[j] = 0.0;
    if (hasNext) {
      // stage A_b^T: lane j writes row j of A_b as column j
      if (rowv)
#pragma unroll
        for (int m = 0; m < NX; ++m) buf[m * NX + r] = (double)a.A[cb * MM + r * NX + m];
      wave_lds_order();
      row_times<NX, NX>(q, buf, acc);  // (Q_b^-1 A_b^T)_r
    }
    if (rowv) {
#pragma unroll
      for (int j = 0; j < NX; ++j) S[2 * MM + r * NX + j] = -acc[j];
      if (hasNext)
#pragma unroll
        for (int j = 0; j < NX; ++j) S[3 * MM + j * NX + r] = -acc[j];  // S_{b+1,b}, column r
    }
  } else {
    if (!hasNext) return;
    const bool rowv = lane < NU;
    const int r = rowv ? lane : 0;
    double ri[NU];
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double v = (double)a.R[cb * NU * NU + r * NU + j];
      ri[j] = rowv ? v : 0.0;
    }
    reg_gj_inverse<NU>(ri, lane, pd);
    // stage B_b^T (NU rows of NX): lane j writes row j of B_b as column j
    if (lane < NX)
#pragma unroll
      for (int m = 0; m < NU; ++m) buf[m * NX + lane] = (double)a.B[cb * NX * NU + lane * NU + m];
    wave_lds_order();
    double wr[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) wr[j] = 0.0;
    row_times<NX, NU>(ri, buf, wr);  // (R_b^-1 B_b^T)_r
    if (rowv) {
      double *rw = a.RW + cb * NU * (NU + NX) + r * (NU + NX);
#pragma unroll
      for (int j = 0; j < NU; ++j) rw[j] = ri[j];
#pragma unroll
      for (int j = 0; j < NX; ++j) rw[NU + j] = wr[j];
    }
  }
}

template <int NX, int NU>
__global__ void __launch_bounds__(kFormWaves * 64) wide_form_theta(const WArgs a) {
  constexpr int MM = NX * NX;
  __shared__ __attribute__((aligned(16))) double stage[kFormWaves][2][MM];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = blockIdx.x * kFormWaves + w;
  if (t >= a.nknots) return;
  const KnotDesc kd = a.knots[t];
  const int b = kd.b;
  const int64_t kb = kd.k0 + b;
  const int64_t cb = kd.k0 - kd.id + b;
  const bool hasPrev = b >= 1;
  const bool adj = a.adjoint != 0;
  const float *qv = adj ? a.gx : a.q;
  const float *rv = adj ? a.gu : a.r;
  const bool rowv = lane < NX;
  const int r = rowv ? lane : 0;
  double *P = stage[w][0], *W = stage[w][1];
  double th[NX];
  double g = 0.0;  // gamma_b, row r
  {
    double qi[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double v = a.Qinv[kb * MM + r * NX + j];
      qi[j] = rowv ? v : 0.0;
      th[j] = qi[j];
    }
    if (qv)
#pragma unroll
      for (int m = 0; m < NX; ++m) g = __builtin_fma(qi[m], (double)qv[kb * NX + m], g);
  }
  if (hasPrev) {
    // P = -S_{b-1,b} = Q_{b-1}^-1 A_{b-1}^T; W = R_{b-1}^-1 B_{b-1}^T
    const double *Sp = a.S + ((kb - 1) * 3 + 2) * MM;
    const double *rw = a.RW + (cb - 1) * NU * (NU + NX);
    if (rowv) {
#pragma unroll
      for (int m = 0; m < NX; ++m) P[m * NX + r] = -Sp[m * NX + r];
#pragma unroll
      for (int m = 0; m < NU; ++m) W[m * NX + r] = rw[m * (NU + NX) + NU + r];
    }
    double x[NX], y[NU];
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double v = (double)a.A[(cb - 1) * MM + r * NX + j];
      x[j] = rowv ? v : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const double v = (double)a.B[(cb - 1) * NX * NU + r * NU + j];
      y[j] = rowv ? v : 0.0;
    }
    wave_lds_order();
    // gamma_b -= (A Q^-1)_r q_{b-1} + (B R^-1)_r r_{b-1}; (A Q^-1)_{rm} = P_{mr},
    // (B R^-1)_{rm} = W_{mr}
    if (qv)
#pragma unroll
      for (int m = 0; m < NX; ++m) g = __builtin_fma(-P[m * NX + r], (double)qv[(kb - 1) * NX + m], g);
    if (rv)
#pragma unroll
      for (int m = 0; m < NU; ++m) g = __builtin_fma(-W[m * NX + r], (double)rv[(cb - 1) * NU + m], g);
    row_times<NX, NX>(x, P, th);  // + (A Q^-1 A^T)_r
    row_times<NX, NU>(y, W, th);  // + (B R^-1 B^T)_r
  }
  if (rowv) {
    double add;
    if (adj) add = (double)a.gl[kb * NX + r];
    else if (b == 0) add = (double)a.x0[(int64_t)kd.id * NX + r];
    else add = a.e ? -(double)a.e[(cb - 1) * NX + r] : 0.0;
    a.rhs[kb * NX + r] = g + add;
    double *S1 = a.S + (kb * 3 + 1) * MM + r * NX;
#pragma unroll
    for (int j = 0; j < NX; ++j) S1[j] = th[j];
  }
  // D_b^-1 = theta_b^-1 (only the preconditioner needs it); D_0^-1 = Q_0
  if (a.no_dinv) return;
  double *D = a.Dinv + kb * MM + r * NX;
  if (b == 0) {
    if (rowv)
#pragma unroll
      for (int j = 0; j < NX; ++j) D[j] = (double)a.Q[kb * MM + r * NX + j];
    return;
  }
  bool pd = true;
  reg_gj_inverse<NX>(th, lane, pd);
  if (rowv)
#pragma unroll
    for (int j = 0; j < NX; ++j) D[j] = th[j];
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

// ---------------------------------------------------------------- cyclic reduction
// Block cyclic reduction of the block-tridiagonal S of every problem of a batch, the same
// recurrences as the 14-state kernel (tri_kernel.h): with stride s the odd multiples j are
// eliminated (V_j = D_j^-1 L_j, U_j = D_j^-1 L_{j+s}^T, z_j = D_j^-1 y_j), the even
// multiples i absorb them (D_i -= L_i U_{i-s} + L_{i+s}^T V_{i+s}, y_i -= L_i z_{i-s} +
// L_{i+s}^T z_{i+s}, L_i <- -L_i V_{i-s}), then x_0 = D_0^-1 y_0 and the levels are undone,
// x_j = z_j - V_j x_{j-s} - U_j x_{j+s}.  The reduced systems are Schur complements of S,
// so a pivot <= 0 means S is not positive definite (BREAKDOWN).
// Work mapping: one launch per sub-step of a level, over the block tasks of all problems
// (so a level spreads over the whole device), one wave per task, lanes r and r + 32 own
// row r < NX in registers (each computing half of the row's product columns); the
// launches on one stream order the levels.  The Gauss-Jordan inverse
// takes the pivot row from its lane with readlane; a matrix product takes the left
// operand's row from registers and the right operand's rows from the wave's own LDS
// staging block (the same address for every lane: a broadcast read); matrix-vector
// products broadcast the vector from its owner lanes.  A wave only ever reads LDS it
// wrote itself, in program order.
// Storage: S blocks (b,b-1), (b,b) hold L and D (V once the knot is eliminated), block
// (b,b+1) is kept for the primal step; Dinv holds U, rhs holds y then z, lamw the solution.
constexpr int kCrWaves = 8;


// Two lanes per row: lane l holds row l & 31 (valid below NX) and computes the output
// columns [h H, h H + H) of it, h = l >> 5; both lanes of a row hold the whole left-operand
// row, so inverses and matrix-vector products run on full rows in both halves.
template <int NX>
struct WaveBlocks {
  static_assert(NX % 2 == 0 && NX <= 32, "two lanes per row of an even NX <= 32");
  static constexpr int H = NX / 2;  // output columns per lane
  int lane, h, row;  // row: this lane's row (>= NX for a lane without one)
  bool rowv;
  int r;             // row clamped to 0 for loads (results of such lanes are never stored)
  __device__ __forceinline__ WaveBlocks(int l)
      : lane(l), h(l >> 5), row(l & 31), rowv((l & 31) < NX), r((l & 31) < NX ? (l & 31) : 0) {}
  // a global block into the staging block by rows (lane (h, c) copies column c of its
  // half of the rows: coalesced)
  __device__ __forceinline__ void stage_rows(double *buf, const double *B) const {
    if (rowv)
#pragma unroll 2
      for (int mm = 0; mm < H; ++mm) buf[(h * H + mm) * NX + r] = B[(h * H + mm) * NX + r];
  }
  // the transpose of a global block into the staging block (lane (h, c) writes its half
  // of row c as its half of column c)
  __device__ __forceinline__ void stage_cols(double *buf, const double *B) const {
    if (rowv)
#pragma unroll 2
      for (int mm = 0; mm < H; ++mm) buf[(h * H + mm) * NX + r] = B[r * NX + h * H + mm];
  }
  // unconditional loads from the clamped row, then masked: straight-line code
  __device__ __forceinline__ void load(const double *B, double (&o)[NX]) const {
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double v = B[r * NX + j];
      o[j] = rowv ? v : 0.0;
    }
  }
  // row r of the transpose of a global block (column r of the block)
  __device__ __forceinline__ void load_t(const double *B, double (&o)[NX]) const {
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const double v = B[j * NX + r];
      o[j] = rowv ? v : 0.0;
    }
  }
  // this lane's half of row r
  __device__ __forceinline__ void load_half(const double *B, double (&o)[H]) const {
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double v = B[r * NX + h * H + j];
      o[j] = rowv ? v : 0.0;
    }
  }
  __device__ __forceinline__ void store_half(double *B, const double (&v)[H]) const {
    if (rowv)
#pragma unroll
      for (int j = 0; j < H; ++j) B[r * NX + h * H + j] = v[j];
  }
  // this lane's half of row r of C = X Y (rows of X in registers, Y staged)
  __device__ __forceinline__ void mm(const double (&X)[NX], const double *Y, double (&C)[H]) const {
#pragma unroll
    for (int j = 0; j < H; ++j) C[j] = 0.0;
    mm_sub_signed<1>(X, Y, C);
  }
  // C -= X Y on this lane's half
  __device__ __forceinline__ void mm_sub(const double (&X)[NX], const double *Y, double (&C)[H]) const {
    mm_sub_signed<-1>(X, Y, C);
  }
  template <int SIGN>
  __device__ __forceinline__ void mm_sub_signed(const double (&X)[NX], const double *Y, double (&C)[H]) const {
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      const double x = SIGN > 0 ? X[m] : -X[m];
      const double *y = Y + m * NX + h * H;
#pragma unroll
      for (int j = 0; j < H; ++j) C[j] = __builtin_fma(x, y[j], C[j]);
    }
  }
  // (X v)_r with v distributed over the lanes (lane m < NX holds v_m)
  __device__ __forceinline__ double mv(const double (&X)[NX], double v) const {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < NX; ++m) acc = __builtin_fma(X[m], lane_value(v, m), acc);
    return acc;
  }
};

// One block task of the reduction (see the recurrences above).  The stride s is the same
// for every problem of a launch; a problem whose horizon is <= s has no task at that level.
struct CrTask {
  int32_t prob;  // index into WArgs::probs
  int32_t j;     // block of the task
};

enum CrStep { kCrOdd = 0, kCrEven = 1, kCrRoot = 2, kCrBack = 3 };

// One sub-step of one level for every problem of the batch: wave w of workgroup g runs
// task g * kCrWaves + w.  `flag` is set for a problem whose reduced blocks lose positive
// definiteness.
template <int NX, int STEP>
__global__ void __launch_bounds__(kCrWaves * 64) wide_cr_step(const WArgs a, const CrTask *tasks, int ntasks,
                                                                int s, int *flag) {
  constexpr int MM = NX * NX;
  // staged right operands: the elimination loads both of its own before the inverse so
  // that their global round trips overlap it (at its register count one workgroup fills a
  // CU, so the LDS is there); the other sub-steps stage one block at a time
  constexpr int kBufs = STEP == kCrOdd ? 2 : 1;
  __shared__ __attribute__((aligned(16))) double stage[kCrWaves][kBufs][MM];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = blockIdx.x * kCrWaves + w;
  if (t >= ntasks) return;  // whole waves leave; no workgroup barrier follows
  const CrTask tk = tasks[t];
  const ProbDescW pd = a.probs[tk.prob];
  const int N = pd.N, j = tk.j;
  const int64_t k0 = pd.k0;
  const WaveBlocks<NX> W(lane);
  double *b0 = stage[w][0], *b1 = stage[w][kBufs - 1];
  auto blk = [&](int k, int t2) { return a.S + ((k0 + k) * 3 + t2) * MM; };
  auto ublk = [&](int k) { return a.Dinv + (k0 + k) * MM; };
  auto vld = [&](const double *v, int k) {
    const double x = v[(k0 + k) * NX + W.r];
    return W.rowv ? x : 0.0;
  };
  bool ok = true;
  constexpr int H = WaveBlocks<NX>::H;
  const bool out = W.rowv && W.h == 0;  // one writer per row of a vector
  if constexpr (STEP == kCrOdd) {  // eliminate j = s(2m+1)
    const bool up = j + s < N;
    W.stage_rows(b0, blk(j, 0));             // L_j
    if (up) W.stage_cols(b1, blk(j + s, 0)); // L_{j+s}^T
    double D[NX], C[H];
    W.load(blk(j, 1), D);
    const double y = vld(a.rhs, j);
    reg_gj_inverse<NX>(D, W.row, ok);        // D_j^-1, rows in D
    const double z = W.mv(D, y);
    wave_lds_order();
    W.mm(D, b0, C);                          // V_j
    W.store_half(blk(j, 1), C);              // over D_j (read above)
    if (up) {
      W.mm(D, b1, C);                        // U_j
      W.store_half(ublk(j), C);
    }
    if (out) a.rhs[(k0 + j) * NX + W.r] = z;
  } else if constexpr (STEP == kCrEven) {  // i = 2sm absorbs i - s and i + s
    const int i = j;
    double D[H], X[NX];
    double y = vld(a.rhs, i);
    if (i >= s) {
      double C[H];
      W.load(blk(i, 0), X);                  // L_i
      y -= W.mv(X, vld(a.rhs, i - s));
      W.stage_rows(b0, blk(i - s, 1));       // V_{i-s}
      wave_lds_order();
      W.mm(X, b0, C);
#pragma unroll
      for (int c = 0; c < H; ++c) C[c] = -C[c];
      W.store_half(blk(i, 0), C);            // coupling to i - 2s (L_i is in X)
      wave_lds_order();
      W.stage_rows(b0, ublk(i - s));         // U_{i-s}
      W.load_half(blk(i, 1), D);
      wave_lds_order();
      W.mm_sub(X, b0, D);                    // D_i -= L_i U_{i-s}
    } else {
      W.load_half(blk(i, 1), D);
    }
    if (i + s < N) {
      W.load_t(blk(i + s, 0), X);            // L_{i+s}^T
      y -= W.mv(X, vld(a.rhs, i + s));
      wave_lds_order();
      W.stage_rows(b0, blk(i + s, 1));       // V_{i+s}
      wave_lds_order();
      W.mm_sub(X, b0, D);                    // D_i -= L_{i+s}^T V_{i+s}
    }
    W.store_half(blk(i, 1), D);
    if (out) a.rhs[(k0 + i) * NX + W.r] = y;
  } else if constexpr (STEP == kCrRoot) {  // x_0 = D_0^-1 y_0
    double D[NX];
    W.load(blk(0, 1), D);
    reg_gj_inverse<NX>(D, W.row, ok);
    const double x = W.mv(D, vld(a.rhs, 0));
    if (out) a.lamw[k0 * NX + W.r] = x;
  } else {  // x_j = z_j - V_j x_{j-s} - U_j x_{j+s}
    double T[NX];
    W.load(blk(j, 1), T);
    double x = vld(a.rhs, j) - W.mv(T, vld(a.lamw, j - s));
    if (j + s < N) {
      W.load(ublk(j), T);
      x -= W.mv(T, vld(a.lamw, j + s));
    }
    if (out) a.lamw[(k0 + j) * NX + W.r] = x;
  }
  if (!ok && lane == 0) flag[tk.prob] = 1;  // every writer stores the same value
}

// Clears the breakdown flags before the first level (a kernel, so the sequence can be
// captured in a graph).
__global__ void wide_cr_init(int *flag, int nprobs) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nprobs) flag[p] = 0;
}

// Stats of every problem: BREAKDOWN on a non-positive pivot or a non-finite solution.
template <int NX>
__global__ void __launch_bounds__(256) wide_cr_finish(const WArgs a, const int *flag) {
  const ProbDescW pd = a.probs[blockIdx.x];
  bool fin = true;
  for (int t = threadIdx.x; t < pd.N * NX; t += 256) {
    const double v = a.lamw[pd.k0 * NX + t];
    fin = fin && (v == v) && !__builtin_isinf(v);
  }
  const bool bad = __syncthreads_or(!fin) || flag[blockIdx.x] != 0;
  if (threadIdx.x == 0) {
    mpcpcg_stats st;
    st.iters = 0;
    st.status = bad ? MPCPCG_BREAKDOWN : MPCPCG_OK;
    st.final_ratio = 0.0f;
    st.reserved = 0;
    a.stats[pd.id] = st;
  }
}


// ---------------------------------------------------------------- factorisation epilogue
// The primal step of every knot from the multipliers lamw (dZ = -G^-1 (g - C^T lambda)),
// or in adjoint mode nu_1 and the block-sparse gradients (the same expressions as the
// PCG kernel's epilogue).  One wave per knot b; lane r < NX owns row r of the knot's
// state block and lane r < NU row r of control b, which couples to lambda_{b+1}:
//   x_b = -Q_b^-1 (q_b - lambda_b) + S_{b,b+1} lambda_{b+1}
//   u_b = -R_b^-1 r_b - (R_b^-1 B_b^T) lambda_{b+1}
template <int NX, int NU>
__global__ void __launch_bounds__(kFormWaves * 64) wide_epilogue(const WArgs a) {
  constexpr int MM = NX * NX;
  __shared__ double vx[kFormWaves][NX], vu[kFormWaves][NU];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int t = blockIdx.x * kFormWaves + w;
  if (t >= a.nknots) return;  // whole waves leave; no workgroup barrier follows
  const KnotDesc kd = a.knots[t];
  const int b = kd.b;
  const int64_t kb = kd.k0 + b;
  const int64_t cb = kd.k0 - kd.id + b;  // control b
  const bool hasNext = b + 1 < kd.N;
  const bool adj = a.adjoint != 0;
  const float *qv = adj ? a.gx : a.q;
  const float *rv = adj ? a.gu : a.r;
  const double *lam = a.lamw;  // lambda, or mu in adjoint mode
  const bool rowv = lane < NX, urow = lane < NU && hasNext;
  const int r = rowv ? lane : 0, ru = lane < NU ? lane : 0;
  double x = 0.0, u = 0.0;
  {
    const double *Qi = a.Qinv + kb * MM + r * NX;
    const double *Sp = a.S + (kb * 3 + 2) * MM + r * NX;
#pragma unroll 4
    for (int j = 0; j < NX; ++j) {
      const double qj = qv ? (double)qv[kb * NX + j] : 0.0;
      const double ln = hasNext ? lam[(kb + 1) * NX + j] : 0.0;
      x = __builtin_fma(-Qi[j], qj - lam[kb * NX + j], x);
      x = __builtin_fma(Sp[j], ln, x);
    }
  }
  if (hasNext) {
    const double *rw = a.RW + cb * NU * (NU + NX) + ru * (NU + NX);
#pragma unroll
    for (int m = 0; m < NU; ++m) u -= rw[m] * (rv ? (double)rv[cb * NU + m] : 0.0);
#pragma unroll 4
    for (int j = 0; j < NX; ++j) u -= rw[NU + j] * lam[(kb + 1) * NX + j];
  }
  const double mu = rowv ? lam[kb * NX + r] : 0.0;
  if (!adj) {
    if (rowv) {
      a.lam[kb * NX + r] = (float)mu;
      a.dx[kb * NX + r] = (float)x;
    }
    if (urow) a.du[cb * NU + lane] = (float)u;
    return;
  }
  // adjoint: lam holds mu, x = nu_1 of the state rows, u = nu_1 of the control rows
  if (rowv) {
    if (a.dgamma) a.dgamma[kb * NX + r] = (float)mu;
    a.dq[kb * NX + r] = (float)x;
    if (b == 0) a.dx0[(int64_t)kd.id * NX + r] = (float)mu;
    if (b >= 1 && a.de) a.de[(cb - 1) * NX + r] = (float)(-mu);
    vx[w][r] = x;
  }
  if (urow) {
    a.dr[cb * NU + lane] = (float)u;
    vu[w][lane] = u;
  }
  wave_lds_order();
  // dQ_b = sym(nu1x_b dx_b^T)
  const float *dxb = a.dx_in + kb * NX;
  for (int o = lane; o < MM; o += 64) {
    const int i = o / NX, j = o % NX;
    const double nx_i = vx[w][i], nx_j = vx[w][j];
    const double dx_i = (double)dxb[i], dx_j = (double)dxb[j];
    a.dQ[kb * MM + o] = (float)(0.5 * (nx_i * dx_j + nx_j * dx_i));
  }
  if (!hasNext) return;
  // control b of block row b + 1: dA_b = lambda_{b+1} nu1x_b^T + mu_{b+1} dx_b^T,
  // dB_b = lambda_{b+1} nu1u_b^T + mu_{b+1} du_b^T, dR_b = sym(nu1u_b du_b^T)
  const float *lin = a.lam_in + (kb + 1) * NX;
  const double *mun = lam + (kb + 1) * NX;
  const float *dub = a.du_in + cb * NU;
  for (int o = lane; o < MM; o += 64) {
    const int i = o / NX, j = o % NX;
    a.dA[cb * MM + o] = (float)((double)lin[i] * vx[w][j] + mun[i] * (double)dxb[j]);
  }
  for (int o = lane; o < NX * NU; o += 64) {
    const int i = o / NU, j = o % NU;
    a.dB[cb * NX * NU + o] = (float)((double)lin[i] * vu[w][j] + mun[i] * (double)dub[j]);
  }
  for (int o = lane; o < NU * NU; o += 64) {
    const int i = o / NU, j = o % NU;
    const double ni = vu[w][i], nj = vu[w][j];
    const double di = (double)dub[i], dj = (double)dub[j];
    a.dR[cb * NU * NU + o] = (float)(0.5 * (ni * dj + nj * di));
  }
}

}  // namespace wide
}  // namespace mpc
