// Block-tridiagonal factorisation and solve of S lambda = rhs, one problem per 16-lane group.
//
// S is symmetric positive definite and block tridiagonal (N block rows of NX x NX), so its
// block LDL^T factorisation needs no pivoting:
//   D_0 = S_00,   L_k = S_{k,k-1} D_{k-1}^-1,   D_k = S_kk - L_k S_{k-1,k}      (k >= 1)
//   y_0 = rhs_0,  y_k = rhs_k - L_k y_{k-1}
//   lambda_{N-1} = D_{N-1}^-1 y_{N-1},   lambda_k = D_k^-1 (y_k - S_{k,k+1} lambda_{k+1}).
// S is positive definite exactly when every D_k is; a pivot <= 0 in the inversion of some
// D_k (or a non-finite result) is reported as MPCPCG_BREAKDOWN.
// This is the direct alternative to PCG for the Schur system of MPCGPU (Section III-B):
// it reaches the exact solution up to rounding in a fixed number of steps, with no
// synchronisation between workgroups, at the price of a sequential sweep over the knots.
// The forward sweep keeps D_k^-1 and y_k in the workspace for the back substitution.
//
// Work mapping: lane i of a group owns row i of every block, as in the PCG kernel; the
// block products run on the fused DPP row broadcasts of lane_ops.h.  A workgroup is one
// wave of four problems, so a batch spreads over the CUs; problems arrive longest-first so
// the groups of a wave sweep similar lengths.
// Arithmetic is FP64 throughout.
#pragma once
#include "lane_ops.h"
#include "mpcpcg.h"
#include "pcg_kernel.h"

namespace mpc {

struct TriArgs {
  const double *s_ws;     // [knots][NX][3 NX]: rows of S_{b,b-1}, S_bb, S_{b,b+1}
  double *rhs_ws;         // [knots][NX]: right-hand side in, y out
  double *dinv_ws;        // [knots][NX][NX]: rows of D_b^-1
  double *lam_ws;         // [knots][NX]: the solution
  const ProbDesc *probs;  // [nprobs] longest first, or nullptr for `single`
  ProbDesc single;
  int32_t nprobs;
  int32_t pad;
  mpcpcg_stats *stats;    // indexed by ProbDesc::id
};

constexpr int kTriThreads = 64;  // one wave, four problems, per workgroup: problems spread over CUs

template <int NX>
__global__ void __launch_bounds__(kTriThreads) tri_sweep(const TriArgs a) {
  const int lane = threadIdx.x & (kGroup - 1);
  const int g = blockIdx.x * (kTriThreads / kGroup) + (threadIdx.x >> 4);
  if (g >= a.nprobs) return;  // whole groups leave together
  const ProbDesc P = a.probs ? a.probs[g] : a.single;
  const bool rowv = lane < NX;
  const int rl = rowv ? lane : 0;
  // each step depends on the previous one, so the next knot's rows are loaded while the
  // current knot is processed
  auto load_s = [&](int64_t kb, double (&Sm)[NX], double (&Sd)[NX], double (&Sp)[NX], double &r) {
    const double *srow = a.s_ws + (kb * NX + rl) * (3 * NX);
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      Sm[j] = rowv ? srow[j] : 0.0;
      Sd[j] = rowv ? srow[NX + j] : 0.0;
      Sp[j] = rowv ? srow[2 * NX + j] : 0.0;
    }
    r = rowv ? a.rhs_ws[kb * NX + lane] : 0.0;
  };

  // forward sweep
  double Dinv[NX], Spp[NX], yp = 0.0;
  bool pd = true;
#pragma unroll
  for (int j = 0; j < NX; ++j) { Dinv[j] = 0.0; Spp[j] = 0.0; }
  double Sm[NX], D[NX], Sp[NX], y;
  load_s(P.k0, Sm, D, Sp, y);
  for (int k = 0; k < P.N; ++k) {
    const int64_t kb = P.k0 + k;
    double nSm[NX], nSd[NX], nSp[NX], ny;
    load_s(P.k0 + (k + 1 < P.N ? k + 1 : k), nSm, nSd, nSp, ny);
    if (k > 0) {
      double L[NX], T[NX];
      mm_nn<NX, NX>(Sm, Dinv, L);  // L_k = S_{k,k-1} D_{k-1}^-1
      mm_nn<NX, NX>(L, Spp, T);    // L_k S_{k-1,k}
#pragma unroll
      for (int j = 0; j < NX; ++j) D[j] -= T[j];
      y -= row_dot<NX>(L, yp);
    }
    gj_inverse<NX>(D, lane, &pd);  // D_k^-1; S is SPD iff every D_k is
    if (rowv) {
      double *drow = a.dinv_ws + (kb * NX + lane) * NX;
#pragma unroll
      for (int j = 0; j < NX; ++j) drow[j] = D[j];
      a.rhs_ws[kb * NX + lane] = y;
    }
#pragma unroll
    for (int j = 0; j < NX; ++j) { Dinv[j] = D[j]; Spp[j] = Sp[j]; }
    yp = y;
#pragma unroll
    for (int j = 0; j < NX; ++j) { Sm[j] = nSm[j]; D[j] = nSd[j]; Sp[j] = nSp[j]; }
    y = ny;
  }

  // back substitution (the rows of knot k - 1 are loaded while knot k is solved)
  auto load_b = [&](int64_t kb, double (&Spr)[NX], double (&Dr)[NX], double &yv) {
    const double *srow = a.s_ws + (kb * NX + rl) * (3 * NX);
    const double *drow = a.dinv_ws + (kb * NX + rl) * NX;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      Spr[j] = rowv ? srow[2 * NX + j] : 0.0;
      Dr[j] = rowv ? drow[j] : 0.0;
    }
    yv = rowv ? a.rhs_ws[kb * NX + lane] : 0.0;
  };
  double lnext = 0.0;
  bool finite = true;
  double Spb[NX], Dr[NX], yb;
  load_b(P.k0 + P.N - 1, Spb, Dr, yb);
  for (int k = P.N - 1; k >= 0; --k) {
    const int64_t kb = P.k0 + k;
    double nSp[NX], nDr[NX], nyb;
    load_b(P.k0 + (k > 0 ? k - 1 : 0), nSp, nDr, nyb);
    const double t = yb - row_dot<NX>(Spb, lnext);
    double lam = row_dot<NX>(Dr, t);
    if (!rowv) lam = 0.0;
    finite = finite && (lam == lam) && !__builtin_isinf(lam);
    if (rowv) a.lam_ws[kb * NX + lane] = lam;
    lnext = lam;
#pragma unroll
    for (int j = 0; j < NX; ++j) { Spb[j] = nSp[j]; Dr[j] = nDr[j]; }
    yb = nyb;
  }
  const uint64_t bad = __ballot(!finite || !pd);
  const bool group_bad = ((bad >> (threadIdx.x & 48)) & 0xffffull) != 0;
  if (lane == 0) {
    mpcpcg_stats st;
    st.iters = 0;
    st.status = group_bad ? MPCPCG_BREAKDOWN : MPCPCG_OK;
    st.final_ratio = 0.0f;
    st.reserved = 0;
    a.stats[P.id] = st;
  }
}

}  // namespace mpc
