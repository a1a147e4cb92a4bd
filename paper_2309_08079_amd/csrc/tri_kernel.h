// Direct solve of the block-tridiagonal Schur system S lambda = rhs by block cyclic
// reduction (the alternative to PCG for the Schur system of MPCGPU, Section III-B; the
// paper names a direct block-tridiagonal solve as future work, Section VI).  It reaches
// the exact solution up to rounding in a fixed number of parallel steps, log2 N levels
// per problem, with no synchronisation between workgroups.
#pragma once
#include "lane_ops.h"
#include "mpcpcg.h"
#include "pcg_kernel.h"

namespace mpc {

struct TriArgs {
  double *s_ws;           // [knots][3][NX][kGroup]: S_{b,b-1}, S_bb, S_{b,b+1} by columns (fws_index; overwritten)
  double *rhs_ws;         // [knots][NX]: right-hand side in (overwritten)
  double *dinv_ws;        // [knots][NX][kGroup]: elimination workspace, by columns
  double *lam_ws;         // [knots][NX]: the solution
  const ProbDesc *probs;  // [nprobs] longest first, or nullptr for `single`
  ProbDesc single;
  int32_t nprobs;
  int32_t pad;
  mpcpcg_stats *stats;    // indexed by ProbDesc::id
};

// S is symmetric positive definite and block tridiagonal.  With stride s (1, 2, 4, ...), the active blocks are the
// multiples of s; write L_i for the coupling of active block i to the active block before
// it (S_{i,i-1} at s = 1) and D_i for its diagonal block.  One level:
//   (a) every odd multiple j = s(2m+1) is eliminated:
//         V_j = D_j^-1 L_j,   U_j = D_j^-1 L_{j+s}^T,   z_j = D_j^-1 y_j;
//   (b) every even multiple i = 2sm absorbs its eliminated neighbours j = i -+ s:
//         D_i -= L_i U_{i-s} + L_{i+s}^T V_{i+s},   y_i -= L_i z_{i-s} + L_{i+s}^T z_{i+s},
//         L_i <- -L_i V_{i-s}  (the coupling to i - 2s).
// The reduced systems are Schur complements of S, so they stay symmetric positive definite
// (a pivot <= 0 in some D_j^-1 means S is not).  When block 0 is the last one active,
// x_0 = D_0^-1 y_0, and the levels are undone in reverse order:
//   x_j = z_j - V_j x_{j-s} - U_j x_{j+s}   (no U term when j + s >= N).
// Work mapping: one workgroup per problem, one 16-lane group per block task, lane r owns
// row r as in the other kernels; a workgroup barrier separates the sub-steps.  Storage is
// the factorisation workspace: each knot's first two S blocks hold L and D (V once the
// knot is eliminated: D_j is inverted in registers first), its third keeps S_{b,b+1} for
// the primal step; dinv_ws holds U, rhs_ws holds y and then z, lam_ws the solution.  FP64
// throughout.
constexpr int kCrThreads = 512;

template <int NX>
__global__ void __launch_bounds__(kCrThreads) cr_solve(const TriArgs a) {
  constexpr int G = kCrThreads / kGroup;  // block tasks in flight per workgroup
  const int lane = threadIdx.x & (kGroup - 1);
  const int grp = threadIdx.x / kGroup;
  const ProbDesc P = a.probs ? a.probs[blockIdx.x] : a.single;
  const int N = P.N;
  const bool rowv = lane < NX;
  const int rl = rowv ? lane : 0;
  // Blocks are stored by columns (fws_index): entry (r, c) of block t of knot k at
  // blk(k, t)[c * kGroup] for lane r, so a 16-lane group moves whole 128-byte lines.
  // Rows >= NX are zero in every block, so all 16 lanes store.
  auto blk = [&](int k, int t) { return a.s_ws + fws_index<NX>(P.k0 + k, t, 0, lane); };
  auto ublk = [&](int k) { return a.dinv_ws + ((P.k0 + k) * NX) * kGroup + lane; };
  auto vec = [&](double *v, int k) { return v + (P.k0 + k) * NX + rl; };
  // Loads are unconditional (a lane past the block's rows reads an in-bounds address) and
  // then masked, so they compile to straight-line code.
  // row r of L_k^T, i.e. column r of L_k: one contiguous column per lane
  auto load_lt = [&](int k, double (&out)[NX]) {
    const double *col = a.s_ws + fws_index<NX>(P.k0 + k, 0, rl, 0);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      const double v = col[c];
      out[c] = rowv ? v : 0.0;
    }
  };
  // a row of a stored block (rows >= NX are stored zeros)
  auto load_row = [&](const double *src, double (&out)[NX]) {
#pragma unroll
    for (int c = 0; c < NX; ++c) out[c] = src[c * kGroup];
  };
  auto store_row = [&](double *dst, const double (&v)[NX]) {
#pragma unroll
    for (int c = 0; c < NX; ++c) dst[c * kGroup] = v[c];
  };
  auto load_v = [&](double *v, int k) {
    const double x = *vec(v, k);
    return rowv ? x : 0.0;
  };

  bool pd = true;
  int s = 1;
  for (; s < N; s *= 2) {
    const int nodd = (N - s + 2 * s - 1) / (2 * s);  // j = s(2m+1) < N
    for (int m = grp; m < nodd; m += G) {
      const int j = s * (2 * m + 1);
      double D[NX], T[NX], C[NX];
      load_row(blk(j, 1), D);
      gj_inverse<NX>(D, lane, &pd);                        // D_j^-1
      load_row(blk(j, 0), T);                              // L_j (rows by lane)
      mm_nn<NX, NX>(D, T, C);                              // V_j
      store_row(blk(j, 1), C);                             // (over D_j, consumed above)
      const double z = row_dot<NX>(D, load_v(a.rhs_ws, j));
      if (j + s < N) {
        load_lt(j + s, T);                                 // L_{j+s}^T (rows by lane)
        mm_nn<NX, NX>(D, T, C);                            // U_j
        store_row(ublk(j), C);
      }
      if (rowv) *vec(a.rhs_ws, j) = z;
    }
    __syncthreads();
    const int neven = (N - 1) / (2 * s) + 1;  // i = 2sm < N
    for (int m = grp; m < neven; m += G) {
      const int i = 2 * s * m;
      double D[NX], L[NX], T[NX], C[NX];
      load_row(blk(i, 1), D);
      double y = load_v(a.rhs_ws, i);
      if (i >= s) {  // left neighbour i - s
        load_row(blk(i, 0), L);
        load_row(ublk(i - s), T);
        mm_nn<NX, NX>(L, T, C);                            // L_i U_{i-s}
#pragma unroll
        for (int c = 0; c < NX; ++c) D[c] -= C[c];
        y -= row_dot<NX>(L, load_v(a.rhs_ws, i - s));
        load_row(blk(i - s, 1), T);
        mm_nn<NX, NX>(L, T, C);                            // L_i V_{i-s}
#pragma unroll
        for (int c = 0; c < NX; ++c) C[c] = -C[c];
        store_row(blk(i, 0), C);
      }
      if (i + s < N) {  // right neighbour i + s
        load_lt(i + s, L);                                 // row r of L_{i+s}^T
        load_row(blk(i + s, 1), T);
        mm_nn<NX, NX>(L, T, C);                            // L_{i+s}^T V_{i+s}
#pragma unroll
        for (int c = 0; c < NX; ++c) D[c] -= C[c];
        y -= row_dot<NX>(L, load_v(a.rhs_ws, i + s));
      }
      store_row(blk(i, 1), D);
      if (rowv) *vec(a.rhs_ws, i) = y;
    }
    __syncthreads();
  }
  if (grp == 0) {  // the last active block
    double D[NX];
    load_row(blk(0, 1), D);
    gj_inverse<NX>(D, lane, &pd);
    const double x = row_dot<NX>(D, load_v(a.rhs_ws, 0));
    if (rowv) *vec(a.lam_ws, 0) = x;
  }
  __syncthreads();
  for (s /= 2; s >= 1; s /= 2) {
    const int nodd = (N - s + 2 * s - 1) / (2 * s);
    for (int m = grp; m < nodd; m += G) {
      const int j = s * (2 * m + 1);
      double T[NX];
      load_row(blk(j, 1), T);
      double x = load_v(a.rhs_ws, j) - row_dot<NX>(T, load_v(a.lam_ws, j - s));
      if (j + s < N) {
        load_row(ublk(j), T);
        x -= row_dot<NX>(T, load_v(a.lam_ws, j + s));
      }
      if (rowv) *vec(a.lam_ws, j) = x;
    }
    __syncthreads();
  }
  // breakdown: a non-positive pivot anywhere, or a non-finite solution entry
  bool bad = !pd;
  for (int t = threadIdx.x; t < N * NX; t += kCrThreads) {
    const double v = a.lam_ws[P.k0 * NX + t];
    bad = bad || !(v == v) || __builtin_isinf(v);
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    mpcpcg_stats st;
    st.iters = 0;
    st.status = bad ? MPCPCG_BREAKDOWN : MPCPCG_OK;
    st.final_ratio = 0.0f;
    st.reserved = 0;
    a.stats[P.id] = st;
  }
}

}  // namespace mpc
