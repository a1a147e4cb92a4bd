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
  int32_t s0;             // cr_solve starts at stride s0 (1: the whole reduction)
  mpcpcg_stats *stats;    // indexed by ProbDesc::id
  int *flag;              // split single solve: set on a non-positive pivot (cr_finish clears it)
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
// row r as in the other kernels; a workgroup barrier separates the sub-steps.  A single
// problem runs its levels with more tasks than a workgroup holds as one launch per
// sub-step over the device (cr_level), the rest in one workgroup (cr_solve).  Storage is
// the factorisation workspace: each knot's first two S blocks hold L and D (V once the
// knot is eliminated: D_j is inverted in registers first), its third keeps S_{b,b+1} for
// the primal step; dinv_ws holds U, rhs_ws holds y and then z, lam_ws the solution.  FP64
// throughout.
constexpr int kCrThreads = 512;
constexpr int kCrGroups = kCrThreads / kGroup;  // block tasks in flight per workgroup

// The block tasks of one problem, executed by one 16-lane group (lane r owns row r).
// Blocks are stored by columns (fws_index): entry (r, c) of block t of knot k at
// blk(k, t)[c * kGroup] for lane r, so a 16-lane group moves whole 128-byte lines.  Rows
// >= NX are zero in every block, so all 16 lanes store.  Loads are unconditional (a lane
// past the block's rows reads an in-bounds address) and then masked, so they compile to
// straight-line code.
template <int NX>
struct CrOps {
  const TriArgs &a;
  const ProbDesc P;
  const int N, lane, rl;
  const bool rowv;
  __device__ __forceinline__ CrOps(const TriArgs &a_, const ProbDesc &p, int l)
      : a(a_), P(p), N(p.N), lane(l), rl(l < NX ? l : 0), rowv(l < NX) {}
  __device__ __forceinline__ double *blk(int k, int t) const { return a.s_ws + fws_index<NX>(P.k0 + k, t, 0, lane); }
  __device__ __forceinline__ double *ublk(int k) const { return a.dinv_ws + ((P.k0 + k) * NX) * kGroup + lane; }
  __device__ __forceinline__ double *vec(double *v, int k) const { return v + (P.k0 + k) * NX + rl; }
  // row r of L_k^T, i.e. column r of L_k: one contiguous column per lane
  __device__ __forceinline__ void load_lt(int k, double (&out)[NX]) const {
    const double *col = a.s_ws + fws_index<NX>(P.k0 + k, 0, rl, 0);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      const double v = col[c];
      out[c] = rowv ? v : 0.0;
    }
  }
  // a row of a stored block (rows >= NX are stored zeros)
  __device__ __forceinline__ void load_row(const double *src, double (&out)[NX]) const {
#pragma unroll
    for (int c = 0; c < NX; ++c) out[c] = src[c * kGroup];
  }
  __device__ __forceinline__ void store_row(double *dst, const double (&v)[NX]) const {
#pragma unroll
    for (int c = 0; c < NX; ++c) dst[c * kGroup] = v[c];
  }
  __device__ __forceinline__ double load_v(double *v, int k) const {
    const double x = *vec(v, k);
    return rowv ? x : 0.0;
  }
  __device__ __forceinline__ static int n_odd(int N, int s) { return (N - s + 2 * s - 1) / (2 * s); }  // j = s(2m+1) < N
  __device__ __forceinline__ static int n_even(int N, int s) { return (N - 1) / (2 * s) + 1; }  // i = 2sm < N

  // (a) eliminate j = s(2m+1)
  __device__ __forceinline__ void odd(int j, int s, bool &pd) const {
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
  // (b) i = 2sm absorbs i - s and i + s
  __device__ __forceinline__ void even(int i, int s) const {
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
  // x_0 = D_0^-1 y_0 (block 0 is the last one active)
  __device__ __forceinline__ void root(bool &pd) const {
    double D[NX];
    load_row(blk(0, 1), D);
    gj_inverse<NX>(D, lane, &pd);
    const double x = row_dot<NX>(D, load_v(a.rhs_ws, 0));
    if (rowv) *vec(a.lam_ws, 0) = x;
  }
  // x_j = z_j - V_j x_{j-s} - U_j x_{j+s}
  __device__ __forceinline__ void back(int j, int s) const {
    double T[NX];
    load_row(blk(j, 1), T);
    double x = load_v(a.rhs_ws, j) - row_dot<NX>(T, load_v(a.lam_ws, j - s));
    if (j + s < N) {
      load_row(ublk(j), T);
      x -= row_dot<NX>(T, load_v(a.lam_ws, j + s));
    }
    if (rowv) *vec(a.lam_ws, j) = x;
  }
};

// One workgroup per problem: the levels from stride a.s0 up, the root, and the levels
// back down to a.s0, a workgroup barrier between sub-steps.  With a.s0 = 1 this is the
// whole solve and it writes the problem's stats; otherwise (a single problem whose first
// levels ran as cr_level launches) it records a non-positive pivot in a.flag and cr_finish
// writes the stats after the last level.
template <int NX>
__global__ void __launch_bounds__(kCrThreads) cr_solve(const TriArgs a) {
  const int lane = threadIdx.x & (kGroup - 1);
  const int grp = threadIdx.x / kGroup;
  const ProbDesc P = a.probs ? a.probs[blockIdx.x] : a.single;
  const CrOps<NX> op(a, P, lane);
  const int N = P.N;
  bool pd = true;
  int s = a.s0;
  for (; s < N; s *= 2) {
    for (int m = grp; m < op.n_odd(N, s); m += kCrGroups) op.odd(s * (2 * m + 1), s, pd);
    __syncthreads();
    for (int m = grp; m < op.n_even(N, s); m += kCrGroups) op.even(2 * s * m, s);
    __syncthreads();
  }
  if (grp == 0) op.root(pd);
  __syncthreads();
  for (s /= 2; s >= a.s0; s /= 2) {
    for (int m = grp; m < op.n_odd(N, s); m += kCrGroups) op.back(s * (2 * m + 1), s);
    __syncthreads();
  }
  if (a.s0 > 1) {
    if (!pd) *a.flag = 1;  // every writer stores the same value
    return;
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

// One sub-step of one level of a single problem (a.single) spread over the device: group
// g of the grid runs task g.  Used for the levels with more tasks than one workgroup
// holds, so that a lone problem's first levels take one round each.
enum CrLevelStep { kLvlOdd = 0, kLvlEven = 1, kLvlBack = 2 };

template <int NX, int STEP>
__global__ void __launch_bounds__(kCrThreads) cr_level(const TriArgs a, int s) {
  const int lane = threadIdx.x & (kGroup - 1);
  const int m = blockIdx.x * kCrGroups + threadIdx.x / kGroup;
  const CrOps<NX> op(a, a.single, lane);
  const int N = a.single.N;
  bool pd = true;
  if constexpr (STEP == kLvlOdd) {
    if (m < op.n_odd(N, s)) op.odd(s * (2 * m + 1), s, pd);
    if (!pd) *a.flag = 1;
  } else if constexpr (STEP == kLvlEven) {
    if (m < op.n_even(N, s)) op.even(2 * s * m, s);
  } else {
    if (m < op.n_odd(N, s)) op.back(s * (2 * m + 1), s);
  }
}

// Stats of a split single solve: BREAKDOWN on a recorded non-positive pivot or a
// non-finite solution entry.  Clears the flag for the next solve.
template <int NX>
__global__ void __launch_bounds__(kCrThreads) cr_finish(const TriArgs a) {
  const ProbDesc P = a.single;
  bool bad = false;
  for (int t = threadIdx.x; t < P.N * NX; t += kCrThreads) {
    const double v = a.lam_ws[P.k0 * NX + t];
    bad = bad || !(v == v) || __builtin_isinf(v);
  }
  bad = __syncthreads_or(bad) || *a.flag != 0;
  __syncthreads();  // every thread has read the flag
  if (threadIdx.x == 0) {
    *a.flag = 0;
    mpcpcg_stats st;
    st.iters = 0;
    st.status = bad ? MPCPCG_BREAKDOWN : MPCPCG_OK;
    st.final_ratio = 0.0f;
    st.reserved = 0;
    a.stats[P.id] = st;
  }
}

}  // namespace mpc
