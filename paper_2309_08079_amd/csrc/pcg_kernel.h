// Fused Schur-complement formation + PCG + reconstruction kernel for gfx950.
//
// Work decomposition
//   * One knot (block row b of S) per 16-lane group; lane i owns row i of the block row.
//   * A workgroup holds KPW consecutive knots ("a part").  A problem of N knots needs
//     ceil(N / KPW) parts; the parts of one problem form a gang that meets at gang
//     barriers (tagged words in global memory) whenever data crosses a part boundary.
//   * For the whole solve each lane keeps the FP64 row of S (three nx-blocks: (b,b-1),
//     (b,b), (b,b+1)) in registers and its FP32 row of Phi^-1 (same three blocks) in LDS,
//     plus the PCG vectors lambda, r, p, s = S p and copies of r and s for knots b-1, b+1.
//
// Method (MPCGPU): S, gamma follow Section III-B (theta_k, phi_k, zeta_k; S and gamma
// negated so S is positive definite), Phi^-1 follows Section IV-A (symmetric stair:
// D_b^-1 on the diagonal, -D_b^-1 S_{b,b+-1} D_{b+-1}^-1 beside it), the loop computes
// the iterates of Algorithm 1 per block row as Algorithm 2 distributes it, with its two
// inner products gathered at one barrier per iteration, and the primal step is
// dZ = -G^-1 (g - C^T lambda).  Stopping rule: sqrt(eta/eta_ref) < eps with
// eta_ref = gamma^T Phi^-1 gamma, or eta < eps as Algorithm 1 prints it.
//
// Precision: inputs/outputs FP32; formation, S, the PCG vectors and all reductions in
// FP64; Phi^-1 stored and applied in FP32 (a preconditioner only changes the Krylov
// path, not the system being solved).
#pragma once
#include "lane_ops.h"
#include "mpcpcg.h"

namespace mpc {

enum Mode : int { kForm = 0, kForward = 1, kAdjoint = 2 };

constexpr int kMaxWaves = 12;   // waves per workgroup (48 knots x 16 lanes / 64)

struct ProbDesc {
  int64_t k0;       // first knot row of the problem in the packed arrays
  int32_t N;        // knots
  int32_t t0;       // index of the problem's first task (part 0)
  int32_t nparts;   // ceil(N / KPW)
  int32_t id;       // problem index b (x0 row, stats slot, control offset k0 - b)
};

struct Task {
  int32_t prob;
  int32_t part;
};

// Per-problem gang state, zero between launches (reset by the last part out), on its
// own 256-byte block so that gangs never share a cache line.
struct alignas(256) Gang {
  int done;        // parts finished with the problem
  int abort;       // set when a part gave up waiting
  int timed_out;   // factorisation path: set by the formation launch when a part gave up,
                   // read and cleared by the primal-step launch (reports TIMEOUT)
  int pad[61];
};

// Tagged words of the loop barriers, per task: (tag << 32) | 32-bit payload with tag =
// barrier index + 1; a double is two words (low half, high half).  Zero = never written.
struct TagWS {
  uint64_t red[2][2][2];              // [parity][value][half] this part's partial sums
  uint64_t hv[2][2][2][kGroup][2];    // [parity][channel][side][lane][half] double halos
};

template <int NX>
struct TaskWS {       // per task; read by the other parts of the same gang
  TagWS tg;
  // formation barrier: (launch generation << 32) | 1 once the hm rows below are complete
  uint64_t flag;
  uint64_t pad[7];
  double hm[2][NX][kGroup];      // [side][row][col] D^-1 rows of the two boundary knots
  // setup exchange (flag stage 2, once Phi^-1 exists): the boundary knots' Phi^-1 rows and
  // two halo channels (gamma at depths 1 and 2, or gamma and lambda_0 at depth 1); a row is
  // padded to 3 NX + 2 floats, a whole number of 16-byte words and the row stride in LDS
  float hp[2][NX][3 * NX + 2];   // [side][row][col]
  double hs[2][2][kGroup];       // [side][channel][lane]
};

// Debug build (MPC_LDS_POISON=1, libmpcpcg_poison.so): every workgroup fills its LDS with a
// NaN pattern at the start of each task, so that a read of LDS the task has not written
// turns the outputs into NaN instead of silently reusing an earlier task's values.
#ifndef MPC_LDS_POISON
#define MPC_LDS_POISON 0
#endif
__device__ __forceinline__ void lds_poison(void *p, size_t bytes, int tid, int nt) {
  uint32_t *w = reinterpret_cast<uint32_t *>(p);
  for (size_t i = tid; i < bytes / 4; i += nt) w[i] = 0x7fc00000u;  // a quiet NaN, as float and as double
}

// Integral constant for the compile-time shape of a barrier.
template <int V>
struct IC {
  static constexpr int value = V;
};

// The two tagged words of a double move as one 16-byte device-scope (sc1) buffer access:
// one memory request instead of two.  Each aligned 8-byte word inside it is still read and
// written whole, so the per-word tags keep validating every word.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kDeviceScope = 16;  // cache-policy bit sc1
__device__ __forceinline__ __amdgpu_buffer_rsrc_t ws_rsrc(void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ void store_pair(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t tag, double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const u32x4 d = {(uint32_t)u, tag, (uint32_t)(u >> 32), tag};
  __builtin_amdgcn_raw_buffer_store_b128(d, rs, off, 0, kDeviceScope);
}
__device__ __forceinline__ u32x4 load_pair(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kDeviceScope);
}
__device__ __forceinline__ bool pair_has(u32x4 w, uint32_t tag) { return w.y == tag && w.w == tag; }
// The same exchange inside one XCD, for a gang whose parts all run on it: stores go to the
// XCD's L2 (the per-CU L1 is write-through) and loads carry the non-temporal bit, which
// makes them miss the CU's L1 and read the L2 (a load with only sc0 set is served from the
// CU's L1 and would keep returning a stale line).  Measured on MI355X: ~0.4 us per
// barrier round of 32 parts, against ~1.0 us for the device-scope words.
constexpr int kL2Load = 2;  // cache-policy bit nt
__device__ __forceinline__ void store_pair_l2(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t tag, double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const u32x4 d = {(uint32_t)u, tag, (uint32_t)(u >> 32), tag};
  __builtin_amdgcn_raw_buffer_store_b128(d, rs, off, 0, 0);
}
__device__ __forceinline__ u32x4 load_pair_l2(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kL2Load);
}
// 8 and 16 bytes of plain data for the formation and setup exchanges (data, a completion
// wait, then a flag): at device scope, or through the XCD's L2 (plain stores, non-temporal
// loads) for a gang whose parts all run on one XCD.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store16_x(__amdgpu_buffer_rsrc_t rs, uint32_t off, u32x4 d, bool l2) {
  if (l2)
    __builtin_amdgcn_raw_buffer_store_b128(d, rs, off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b128(d, rs, off, 0, kDeviceScope);
}
__device__ __forceinline__ u32x4 load16_x(__amdgpu_buffer_rsrc_t rs, uint32_t off, bool l2) {
  return l2 ? __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kL2Load)
            : __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kDeviceScope);
}
__device__ __forceinline__ void store8_x(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint64_t v, bool l2) {
  const u32x2 d = {(uint32_t)v, (uint32_t)(v >> 32)};
  if (l2)
    __builtin_amdgcn_raw_buffer_store_b64(d, rs, off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(d, rs, off, 0, kDeviceScope);
}
__device__ __forceinline__ uint64_t load8_x(__amdgpu_buffer_rsrc_t rs, uint32_t off, bool l2) {
  const u32x2 d = l2 ? __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, kL2Load)
                     : __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, kDeviceScope);
  return ((uint64_t)d.y << 32) | d.x;
}
__device__ __forceinline__ u32x4 pack_d2(double x, double y) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x), v = __builtin_bit_cast(uint64_t, y);
  return u32x4{(uint32_t)u, (uint32_t)(u >> 32), (uint32_t)v, (uint32_t)(v >> 32)};
}
__device__ __forceinline__ u32x4 pack_f4(float x, float y, float z, float w) {
  return u32x4{__builtin_bit_cast(uint32_t, x), __builtin_bit_cast(uint32_t, y), __builtin_bit_cast(uint32_t, z),
               __builtin_bit_cast(uint32_t, w)};
}
// Tag of loop barrier n of a launch: (launch generation mod 256) << 24 | (n + 1), so that a
// word left by an earlier launch never carries a live tag, whichever cache still holds it.
__device__ __forceinline__ uint32_t loop_tag(uint64_t gen, int n) {
  return ((uint32_t)(gen & 0xffu) << 24) | ((uint32_t)(n + 1) & 0xffffffu);
}
__device__ __forceinline__ double pair_value(u32x4 w) {
  return __builtin_bit_cast(double, ((uint64_t)w.z << 32) | w.x);
}

struct KArgs {
  // problem data (packed)
  const float *Q, *R, *A, *B, *q, *r, *x0, *e;
  // adjoint inputs: saved forward solution and loss gradients
  const float *lam_in, *dx_in, *du_in, *gl, *gx, *gu;
  // outputs
  float *lam, *dx, *du;
  mpcpcg_stats *stats;
  float *dQ, *dR, *dA, *dB, *dq, *dr, *dx0, *de, *dgamma;
  float *S_out, *P_out, *gam_out;
  // schedule
  const ProbDesc *probs;
  const Task *tasks;
  ProbDesc single;       // used when probs == nullptr (one problem, task = blockIdx.x)
  int32_t ntasks;
  int32_t persistent;    // 1: workgroups pop tasks from queue[0] (or their XCD's queue)
  const int32_t *xoff;   // [9] or nullptr: the tasks of XCD x are [xoff[x], xoff[x+1]), popped
                         // from queue[4 + x] by the workgroups running on XCD x only, so all
                         // parts of a gang run on one XCD
  int32_t one_xcd;       // non-persistent: the grid holds 8 workgroups per part; those running
                         // on XCD 0 (HW_REG_XCC_ID) take the parts from queue[4], the rest exit
  int32_t l2x;           // 1: every gang's parts run on one XCD (per-XCD lists or one_xcd), so
                         // the loop barriers exchange through that XCD's L2
  // workspace
  void *tws;             // TaskWS<NX>[ntasks]
  Gang *gang;            // [nprobs]
  int *queue;            // [0] head, [1] workgroups finished, [2] launch generation,
                         // [4 + x] head of XCD x
  double *qinv_ws;       // [knots][NX][kGroup]   Q_b^-1 by columns (row r at r)
  double *rinv_ws;       // [controls][NU + NX][kURows]  (R^-1 | R^-1 B^T) by columns
  // factorisation path: S rows [knots][NX][3 NX] and rhs [knots][NX] written by phase 1,
  // lambda [knots][NX] read by phase 2
  double *s_ws, *rhs_ws, *lam_ws;  // factorisation workspace (layout: fws_index)
  // factor record of a forward solve (written when fac_mode = 1): Phi^-1 (FP32) by columns
  // (layout: fws_index), read back by its adjoint (PHASE 3) instead of inverting S_bb,
  // exchanging D^-1 between parts and forming the off-diagonal blocks again; qinv_ws and
  // rinv_ws then point into the same record, and the adjoint reads Q^-1 and R^-1 there
  // instead of inverting Q and R
  float *fac_p;
  int32_t fac_mode;
  int32_t pad_fac;
  // options
  float eps;
  int32_t max_iter;
  int32_t warm;
  int32_t stop_abs;      // 1: eta < eps; 0: sqrt(eta / eta_ref) < eps
  // every cross-workgroup wait gives up after this many wall-clock ticks (the host sets
  // 2 s); a part that gives up raises its gang's abort flag and the problem reports TIMEOUT
  int64_t spin_limit;
  int32_t stall;         // test hook: the formation barrier waits for a flag never written
  int32_t pad_opts;
};

// Writes one problem's stats with device-scope stores, so that a later override of the
// status by another part of the gang (TIMEOUT) is ordered after it through the gang counter.
__device__ __forceinline__ void put_stats(mpcpcg_stats *s, int iters, int status, float ratio) {
  int *w = reinterpret_cast<int *>(s);
  __hip_atomic_store(w + 0, iters, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 1, status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 2, __builtin_bit_cast(int, ratio), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 3, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-uniform copies (kept in SGPRs): values every lane of the workgroup shares.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}


// Register budget: the FP64 S row (84 VGPRs) stays resident for the whole solve and the
// FP32 Phi^-1 row lives in LDS; the occupancy target sets how many knots stay resident.
// A 32-knot workgroup (8 waves) fits only two waves per SIMD anyway, so it keeps the full
// 256-VGPR budget; the other shapes target three (a 24-knot workgroup has 6 waves, two
// per compute unit; a 48-knot one has 12 waves, one per compute unit).
template <int KPW>
constexpr int waves_per_eu() { return KPW == 32 ? 2 : 3; }
// The formation-only and epilogue-only kernels of the factorisation path hold no PCG state:
// two waves per SIMD give them the registers of the formation without spills.
template <int KPW, int PHASE>
constexpr int phase_waves_per_eu() { return (PHASE == 1 || PHASE == 2) ? 2 : waves_per_eu<KPW>(); }
// Rows of a control block as stored by columns (NU = 7 rows padded to 8: half a line).
constexpr int kURows = 8;

// Factorisation workspace: element (r, c) of block t (0: S_{b,b-1}, 1: S_bb, 2: S_{b,b+1})
// of packed knot k.  Blocks are stored by columns padded to kGroup rows, so one column is
// one 128-byte line and the 16 lanes of a knot group (lane = row) read or write it whole.
template <int NX>
__device__ __forceinline__ int64_t fws_index(int64_t k, int t, int c, int r) {
  return ((k * 3 + t) * NX + c) * kGroup + r;
}

// PHASE 0: formation, PCG and epilogue fused (a forward solve with fac_mode 1 also writes
// its factor record).  PHASE 1 (factorisation path): formation only, S rows and the
// right-hand side written to s_ws / rhs_ws.  PHASE 2: formation, lambda read from lam_ws
// (the block-tridiagonal solve), then the epilogue.  PHASE 3 (adjoint): S formed as in
// PHASE 0 from the inverses of Q and R read from the forward's factor record, Phi^-1 read
// from it as well, then PCG and epilogue.
template <int NX, int NU, int KPW, int MODE, int PHASE = 0>
__global__ void __launch_bounds__(KPW * kGroup) __attribute__((amdgpu_waves_per_eu(phase_waves_per_eu<KPW, PHASE>(), phase_waves_per_eu<KPW, PHASE>())))
    pcg_kernel(const KArgs a) {
  static_assert(NX == 14 && NU <= NX, "the fused row kernels are written for 14-row blocks");
  constexpr int NT = KPW * kGroup;
  constexpr int NW = NT / 64;
  static_assert(NT % 64 == 0 && NW <= kMaxWaves, "whole waves, at most kMaxWaves");

  __shared__ double ex_d[2][KPW + 2][kGroup];  // vector exchange, slot s+1 is knot s
  __shared__ float ex_f[KPW + 2][kGroup];
  // One LDS region serves two phases: the D^-1 row exchange of the formation, then the
  // FP32 Phi^-1 rows for the rest of the solve (row r of knot slot s at
  // pl[(s * NX + r) * kPRow], blocks (b,b-1), (b,b), (b,b+1) at offsets 0, 14, 28; slots
  // KPW and KPW + 1 hold the rows of the neighbouring parts' boundary knots b0 - 1 and
  // b_last + 1, the "ghost" knots whose preconditioned residual this part recomputes).
  constexpr int kPRow = 44;
  constexpr size_t kExBytes = sizeof(double) * (KPW + 2) * NX * kGroup;
  constexpr size_t kPlBytes = sizeof(float) * (KPW + 2) * NX * kPRow;
  __shared__ __attribute__((aligned(16))) unsigned char big[kExBytes > kPlBytes ? kExBytes : kPlBytes];
  auto ex_m = reinterpret_cast<double (*)[NX][kGroup]>(big);
  float *const pl = reinterpret_cast<float *>(big);
  __shared__ __attribute__((aligned(16))) double red_g[2][KPW][2];  // [phase][knot slot][value]
  __shared__ double tot[2];
  __shared__ double rcp_sh[2];  // 1 / gamma_prev, 1 / alpha_prev of the PCG loop
  __shared__ int sh_task;
  __shared__ int sh_abort;

  // Lane indices are re-derived through an opaque copy of threadIdx.x at every phase
  // boundary (refresh below).  Otherwise the compiler computes every per-lane address of
  // the formation and epilogue once, up front, and keeps them live through the PCG loop,
  // which costs the registers the loop needs for S and Phi^-1.
  int tid = threadIdx.x;
  int lane = tid & (kGroup - 1);  // row within the knot block
  int slot = tid >> 4;            // knot slot within the workgroup
  int wave = tid >> 6;
  int wl = tid & 63;
  TaskWS<NX> *tws = reinterpret_cast<TaskWS<NX> *>(a.tws);
  const __amdgpu_buffer_rsrc_t wsr = ws_rsrc(a.tws);
  auto ws_off = [&](const void *p) { return (uint32_t)((const char *)p - (const char *)a.tws); };
  // launch generation: advanced by the last workgroup of every launch, so flags written
  // by earlier launches are always older than any epoch of this one
  const uint64_t gen = (uint64_t)(uint32_t)uni(__hip_atomic_load(&a.queue[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));

  for (int iter_task = 0;; ++iter_task) {
    // ------------------------------------------------------------- task selection
    int task;
    if (a.persistent) {
      __syncthreads();
      if (tid == 0) {
        if (a.xoff) {
          unsigned x;
          asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
          x &= 7u;
          const int t = a.xoff[x] + atomicAdd(&a.queue[4 + x], 1);
          sh_task = t < a.xoff[x + 1] ? t : a.ntasks;  // this XCD's queue is empty
        } else {
          sh_task = atomicAdd(&a.queue[0], 1);
        }
      }
      __syncthreads();
      task = uni(sh_task);
      if (task >= a.ntasks) break;
    } else {
      if (iter_task > 0) break;
      if (a.one_xcd) {
        if (tid == 0) {
          unsigned x;
          asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
          sh_task = (x & 7u) ? a.ntasks : atomicAdd(&a.queue[4], 1);
        }
        __syncthreads();
        task = uni(sh_task);
        if (task >= a.ntasks) break;
      } else {
        task = (int)blockIdx.x;
      }
    }
    if constexpr (MPC_LDS_POISON) {
      __syncthreads();
      lds_poison(big, sizeof big, tid, NT);
      lds_poison(ex_d, sizeof ex_d, tid, NT);
      lds_poison(ex_f, sizeof ex_f, tid, NT);
      lds_poison(red_g, sizeof red_g, tid, NT);
      lds_poison(tot, sizeof tot, tid, NT);
      lds_poison(rcp_sh, sizeof rcp_sh, tid, NT);
      __syncthreads();
    }
    const Task tk = a.probs ? a.tasks[task] : Task{0, task};
    const ProbDesc pd = a.probs ? a.probs[tk.prob] : a.single;
    const int part = tk.part;
    const int G = pd.nparts;
    const bool multi = G > 1;
    const int N = pd.N;
    int b;             // knot (block row) of this group
    bool act, rowv, hasPrev, hasNext;  // knot exists / row < nx / control b-1 / control b
    int64_t kb, cb;    // packed knot row of knot b, packed control row of control b
    auto refresh = [&]() {
      asm volatile("" : "+v"(tid));
      lane = tid & (kGroup - 1);
      slot = tid >> 4;
      wave = tid >> 6;
      wl = tid & 63;
      b = part * KPW + slot;
      act = b < N;
      rowv = lane < NX;
      hasPrev = act && b >= 1;
      hasNext = act && b + 1 < N;
      kb = pd.k0 + b;
      cb = pd.k0 - pd.id + b;
    };
    refresh();
    Gang *gang = a.gang + (a.probs ? tk.prob : 0);
    const int my_t = a.probs ? pd.t0 + part : part;
    // halo slots 0 and KPW+1 are zero unless a neighbouring part fills them
    for (int t = tid; t < 2 * kGroup; t += NT) {
      const int side = t / kGroup, l = t % kGroup;
      const int s = side ? KPW + 1 : 0;
      ex_d[0][s][l] = 0.0;
      ex_d[1][s][l] = 0.0;
      ex_f[s][l] = 0.0f;
    }
    if constexpr (PHASE == 0) {
      for (int t = tid; t < 2 * NX * kGroup; t += NT) {
        const int side = t / (NX * kGroup), rem = t % (NX * kGroup);
        ex_m[side ? KPW + 1 : 0][rem / kGroup][rem % kGroup] = 0.0;
      }
    }
    int nsync = 0;   // gang barrier counter (identical sequence in every part)
    bool aborted = false;
    if (tid == 0) sh_abort = 0;

    // Gang barriers.  Every value that crosses a part boundary (halo rows of the vectors,
    // the part's partial sums) is published as 64-bit words (tag << 32) | payload, where
    // the tag is the barrier index + 1 and a double takes two words.  A 64-bit store is seen
    // whole or not at all, so a reader that finds the expected tag in a word also has its
    // payload: waiting and loading are the same round trip, and a writer never waits for
    // its stores to complete.  Lane g of wave 0 polls the partial sums of part g, lanes
    // 0..31 poll the left / right halos.  A part publishes one sum per value (its waves'
    // partials added in order after the workgroup barrier), which keeps the polled words,
    // and so the traffic at the coherence point, at 2 * NR per part: per-wave words made
    // the polling itself the bottleneck once hundreds of workgroups wait at once.  Stale
    // words from earlier solves never carry a live tag: the last part out of a gang zeroes
    // the tagged words of every part.
    auto poll_spin = [&](int &polls, long long t_start) -> int {
      __builtin_amdgcn_s_sleep(1);
      if ((++polls & 63) == 0) {
        if (__hip_atomic_load(&gang->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 1;
        if (wall_clock64() - t_start > a.spin_limit) {
          __hip_atomic_store(&gang->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return 1;
        }
      }
      return 0;
    };
    // this part's totals of its NR per-knot partials (wave 0, after a workgroup barrier):
    // lanes 0..31 add value 0 of knot slots wl, wl + 32, ..., lanes 32..63 value 1, then one
    // packed reduction (fixed shape) gives both, uniform
    auto part_sums = [&](int ph, int nr, double &s0, double &s1) {
      const int vi = wl >> 5;
      double v = 0.0;
      if (vi < nr) {
#pragma unroll
        for (int k = 0; k < KPW; k += 32)
          if (k + (wl & 31) < KPW) v += red_g[ph][k + (wl & 31)][vi];
      }
      half_sums(v, s0, s1);
    };
    // the tagged words of the loop barriers: through one XCD's L2 when the gang runs there
    const bool l2x = a.l2x != 0;
    auto put_pair = [&](uint32_t off, uint32_t tag, double v) {
      if (l2x)
        store_pair_l2(wsr, off, tag, v);
      else
        store_pair(wsr, off, tag, v);
    };
    auto get_pair = [&](uint32_t off) -> u32x4 {
      u32x4 w;
      if (l2x)
        w = load_pair_l2(wsr, off);
      else
        w = load_pair(wsr, off);
      return w;
    };
    // Loop barrier: ND double channels of halos, NR partial sums
    // (read from red_g[ph] when the problem has one part); totals land in tot[].  `after`
    // runs in every wave right after the closing workgroup barrier, before the abort flag is
    // read, so that the LDS reads it issues share one round trip with that read.
    auto sync_point = [&](auto nd_c, auto nr_c, int ph, auto &&after) {
      constexpr int ND = decltype(nd_c)::value, NR = decltype(nr_c)::value;
      __syncthreads();
      if (multi && aborted) {
        // the gang has given up: no part waits any more (outputs are undefined)
        ++nsync;
        after();
      } else if (multi) {
        if (wave == 0) {
          // the whole workgroup waits for this wave until the totals are out: it issues
          // ahead of the co-resident workgroups' waves meanwhile
          __builtin_amdgcn_s_setprio(2);
          const int par = nsync & 1;
          const uint32_t tag = loop_tag(gen, nsync);
          // test hook: the launch's first wait expects a tag that no part writes
          const uint32_t want_tag = (a.stall && nsync == 0) ? 0xffffffffu : tag;
          if (NR > 0) {  // this part's sums over its knots
            double ps0, ps1;
            part_sums(ph, NR, ps0, ps1);
            if (wl < NR) put_pair(ws_off(tws[my_t].tg.red[par][wl]), tag, wl == 0 ? ps0 : ps1);
          }
          const int side = wl >> 4, l = wl & 15;
          const int nb = side == 0 ? part - 1 : part + 1;
          const bool has = wl < 2 * kGroup && nb >= 0 && nb < G;
          const TagWS *hsrc = &tws[has ? my_t + (side == 0 ? -1 : 1) : my_t].tg;
          const int srcside = side == 0 ? 1 : 0;  // left neighbour's last knot / right's first
          u32x4 hq[ND > 0 ? ND : 1];
          // lanes 0..31 read value 0 of 32 parts at a time, lanes 32..63 value 1 (when there
          // is one), so one packed reduction below gives both totals
          const int vi = wl >> 5;
          double v = 0.0;
          int ab = 0, polls = 0;
          const long long t_start = wall_clock64();
          // Device scope: the last part's words land ~1 us after the first part arrives, so
          // an immediate poll almost always fails and only adds traffic at the coherence
          // point, which every other gang's polls share: waiting ~1,500 cycles first
          // measured 10% faster on 256 x N=512 (and no slower for one problem).  Through
          // one XCD's L2 a round takes ~0.4 us, and polling at once measured fastest.
          if (!l2x) __builtin_amdgcn_s_sleep(24);
          for (int g0 = 0; g0 < G && !ab; g0 += 32) {
            const int g = g0 + (wl & 31);
            const bool mine = vi < NR && g < G;
            const bool halo = g0 == 0 && has;
            const TagWS *rsrc = &tws[pd.t0 + (mine ? g : 0)].tg;
            u32x4 rw = {0u, 0u, 0u, 0u};
            while (true) {
              bool ok = true;
              if (mine) {
                rw = get_pair(ws_off(rsrc->red[par][vi]));
                ok &= pair_has(rw, want_tag);
              }
              if (halo) {
#pragma unroll
                for (int c = 0; c < ND; ++c) {
                  hq[c] = get_pair(ws_off(hsrc->hv[par][c][srcside][l]));
                  ok &= pair_has(hq[c], want_tag);
                }
              }
              if (__ballot(ok) == ~0ull) break;
              if ((ab = poll_spin(polls, t_start))) break;
            }
            // totals over parts in a fixed order and a fixed-shape reduction, so every part
            // computes bit-identical totals
            if (mine && !ab) v += pair_value(rw);
          }
          if (wl < 2 * kGroup && !ab) {
            const int dst = side == 0 ? 0 : KPW + 1;
#pragma unroll
            for (int c = 0; c < ND; ++c) ex_d[c][dst][l] = has ? pair_value(hq[c]) : 0.0;
          }
          double w0, w1;
          half_sums(v, w0, w1);
          if (wl == 0) {
            tot[0] = w0;
            tot[1] = w1;
            sh_abort = ab;
          }
          __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        ++nsync;
        after();
        aborted = aborted || uni(sh_abort) != 0;
      } else {
        if (wave == 0) {
          double s0, s1;
          part_sums(ph, NR, s0, s1);
          if (wl == 0) {
            tot[0] = s0;
            tot[1] = s1;
          }
        }
        __syncthreads();
        after();
      }
    };
    auto nothing = [] {};
    // Formation barrier (barrier 0): the D^-1 rows of the two boundary knots (NX doubles
    // per lane) go through plain stores, then a completion wait and a flag
    // (launch generation << 32) | 1.  It runs once per solve, so it keeps the simpler
    // protocol and leaves no tagged words behind.
    auto sync_form = [&]() {
      if (multi) __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (multi) {
        const uint64_t epoch = (gen << 32) | 1u;
        // test hook: wait for an epoch that no part ever writes, so every wait gives up
        const uint64_t need = a.stall ? ~0ull : epoch;
        if (wave == 0) {
          if (wl == 0) store8_x(wsr, ws_off(&tws[my_t].flag), epoch, l2x);
          const long long t_start = wall_clock64();
          int ab = 0, polls = 0;
          // only the two neighbours' rows are needed
          const int nb = wl == 0 ? part - 1 : part + 1;
          const bool want = wl < 2 && nb >= 0 && nb < G;
          while (true) {
            const bool seen = !want || load8_x(wsr, ws_off(&tws[pd.t0 + (want ? nb : 0)].flag), l2x) >= need;
            if (__ballot(seen) == ~0ull) break;
            if ((ab = poll_spin(polls, t_start))) break;
          }
          // lane l of each half copies row l of the neighbour's boundary D^-1 (its 16-byte
          // words all in flight at once)
          if (wl < 2 * kGroup && (wl & 15) < NX && !ab) {
            const int side = wl >> 4, l = wl & 15;
            const int nbh = side == 0 ? part - 1 : part + 1;
            const bool has = nbh >= 0 && nbh < G;
            const TaskWS<NX> *src = &tws[has ? my_t + (side == 0 ? -1 : 1) : my_t];
            const int dst = side == 0 ? 0 : KPW + 1;
            const int srcside = side == 0 ? 1 : 0;
            const uint32_t o = ws_off(&src->hm[srcside][l][0]);
            u32x4 q[kGroup / 2];
#pragma unroll
            for (int k = 0; k < kGroup / 2; ++k) q[k] = has ? load16_x(wsr, o + 16 * k, l2x) : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int k = 0; k < kGroup / 2; ++k) *reinterpret_cast<u32x4 *>(&ex_m[dst][l][2 * k]) = q[k];
          }
          if (wl == 0) sh_abort = ab;
        }
        __syncthreads();
        ++nsync;
        aborted = aborted || uni(sh_abort) != 0;
      }
    };

    // Setup barrier (barrier 1, flag stage 2): the neighbours' boundary Phi^-1 rows go to the
    // ghost slots of pl, and two double halo channels to the halo slots of ex_d.
    auto sync_setup = [&]() {
      if (multi) __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (!multi) {
        for (int t = tid; t < 2 * NX * kPRow; t += NT) pl[KPW * NX * kPRow + t] = 0.0f;
        __syncthreads();
        return;
      }
      if (aborted) {  // the gang has given up: no part waits any more
        ++nsync;
        return;
      }
      const uint64_t epoch = (gen << 32) | 2u;
      if (wave == 0) {
        if (wl == 0) store8_x(wsr, ws_off(&tws[my_t].flag), epoch, l2x);
        const long long t_start = wall_clock64();
        int ab = 0, polls = 0;
        const int nb = wl == 0 ? part - 1 : part + 1;
        const bool want = wl < 2 && nb >= 0 && nb < G;
        while (true) {
          const bool seen = !want || load8_x(wsr, ws_off(&tws[pd.t0 + (want ? nb : 0)].flag), l2x) >= epoch;
          if (__ballot(seen) == ~0ull) break;
          if ((ab = poll_spin(polls, t_start))) break;
        }
        if (!ab) {
          // the neighbours' boundary rows, 16-byte words copied flat (the rows of hp and of
          // pl have the same padded layout), then the two halo channels; every load of a
          // lane is issued before any of them is used
          static_assert(3 * NX + 2 == kPRow, "hp rows and Phi^-1 rows in LDS share a layout");
          constexpr int kW = NX * kPRow / 4;                  // 16-byte words per side
          constexpr int kPer = (2 * kW + 63) / 64;
          u32x4 q[kPer];
#pragma unroll
          for (int i = 0; i < kPer; ++i) {
            const int t = wl + 64 * i;
            const int side = t < kW ? 0 : 1;
            const int nbh = side == 0 ? part - 1 : part + 1;
            const bool has = t < 2 * kW && nbh >= 0 && nbh < G;
            const TaskWS<NX> *src = &tws[has ? my_t + (side == 0 ? -1 : 1) : my_t];
            q[i] = has ? load16_x(wsr, ws_off(&src->hp[side == 0 ? 1 : 0][0][0]) + 16 * (t - side * kW), l2x)
                       : u32x4{0u, 0u, 0u, 0u};
          }
          double hv[2] = {0.0, 0.0};
          if (wl < 2 * kGroup) {
            const int side = wl >> 4, l = wl & 15;
            const int nbh = side == 0 ? part - 1 : part + 1;
            const bool has = nbh >= 0 && nbh < G;
            const TaskWS<NX> *src = &tws[has ? my_t + (side == 0 ? -1 : 1) : my_t];
#pragma unroll
            for (int c = 0; c < 2; ++c)
              hv[c] = has ? __builtin_bit_cast(double, load8_x(wsr, ws_off(&src->hs[side == 0 ? 1 : 0][c][l]), l2x)) : 0.0;
          }
#pragma unroll
          for (int i = 0; i < kPer; ++i) {
            const int t = wl + 64 * i;
            if (t < 2 * kW) *reinterpret_cast<u32x4 *>(pl + KPW * NX * kPRow + 4 * t) = q[i];
          }
          if (wl < 2 * kGroup) {
            const int dst = (wl >> 4) == 0 ? 0 : KPW + 1;
#pragma unroll
            for (int c = 0; c < 2; ++c) ex_d[c][dst][wl & 15] = hv[c];
          }
        }
        if (wl == 0) sh_abort = ab;
      }
      __syncthreads();
      ++nsync;
      aborted = aborted || uni(sh_abort) != 0;
    };

    // publish this group's value of a double vector channel (LDS + boundary halo)
    auto put_d = [&](int c, double v) {
      ex_d[c][slot + 1][lane] = v;
      if (multi && (slot == 0 || slot == KPW - 1)) {
        put_pair(ws_off(tws[my_t].tg.hv[nsync & 1][c][slot == 0 ? 0 : 1][lane]), loop_tag(gen, nsync), v);
      }
    };
    // publish a double vector whose neighbours need two knots deep: LDS channel 0, and to the
    // gang channel 0 (boundary knots) / channel 1 (second knots in from each end)
    auto put_d2 = [&](double v) {
      ex_d[0][slot + 1][lane] = v;
      if (multi && (slot <= 1 || slot >= KPW - 2)) {
        const int side = slot <= 1 ? 0 : 1;
        const int c = (slot == 0 || slot == KPW - 1) ? 0 : 1;
        put_pair(ws_off(tws[my_t].tg.hv[nsync & 1][c][side][lane]), loop_tag(gen, nsync), v);
      }
    };
    // per-knot partial of a lane value (fixed-shape sum over the knot group), written to
    // red_g[ph][slot][v] by the group's last lane
    auto put_red = [&](int ph, int v, double x) {
      const double g = group_sum_to_last(x);
      if (lane == kGroup - 1) red_g[ph][slot][v] = g;
    };
    // both values at once (the two reduction chains interleave; one 16-byte LDS write)
    auto put_red2 = [&](int ph, double x0, double x1) {
      group_sums2(x0, x1);
      if (lane == kGroup - 1) *reinterpret_cast<double2 *>(&red_g[ph][slot][0]) = make_double2(x0, x1);
    };

    // ================================================================== formation
    refresh();
    // Blocks that do not exist (no previous control at b = 0, no next one at b = N-1,
    // slots past the end of the horizon) are loaded as zeros, and missing Q blocks as the
    // identity, so every group runs the same instruction stream.

    double Sm[NX], Sd[NX], Sp[NX];
    double rhs;  // gamma_b (forward) or the adjoint right-hand side y_b
    const float *qv = (MODE == kAdjoint) ? a.gx : a.q;
    const float *rv = (MODE == kAdjoint) ? a.gu : a.r;
    double Dd[NX];
    float Pm[NX], Pd[NX], Pp[NX];
    if constexpr (PHASE == 2) {
      // the epilogue needs only S_{b,b+1} (the rest of its inputs are in the workspace)
      const double *sp = a.s_ws + fws_index<NX>(act ? kb : 0, 2, 0, lane);
#pragma unroll
      for (int j = 0; j < NX; ++j) { Sm[j] = 0.0; Sd[j] = 0.0; Dd[j] = 0.0; Sp[j] = (act && rowv) ? sp[j * kGroup] : 0.0; }
      rhs = 0.0;
    } else {
    {
      // (1) previous-knot terms: T = A_{b-1} Q_{b-1}^-1 -> S_{b,b-1} = -T,
      //     theta = T A_{b-1}^T + ..., zeta = -T q_{b-1} - ...
      double Qm[NX], Ar[NX], T[NX];
#pragma unroll
      for (int j = 0; j < NX; ++j) { Qm[j] = 0.0; Ar[j] = 0.0; }
      if (hasPrev && rowv) {
        const float *pq = a.Q + ((kb - 1) * NX + lane) * NX;
        const float *pa = a.A + ((cb - 1) * NX + lane) * NX;
#pragma unroll
        for (int j = 0; j < NX; ++j) { Qm[j] = (double)pq[j]; Ar[j] = (double)pa[j]; }
      } else if (rowv) {
#pragma unroll
        for (int j = 0; j < NX; ++j) Qm[j] = (j == lane) ? 1.0 : 0.0;
      }
      if constexpr (PHASE == 3) {
        // Q_{b-1}^-1 as knot b-1 inverted it in the forward (the same inputs and steps)
        if (hasPrev) {
          const double *w = a.qinv_ws + (kb - 1) * NX * kGroup + lane;
#pragma unroll
          for (int j = 0; j < NX; ++j) Qm[j] = w[j * kGroup];
        }
      } else {
        gj_inverse<NX>(Qm, lane);
      }
      mm_nn<NX, NX>(Ar, Qm, T);
#pragma unroll
      for (int j = 0; j < NX; ++j) Sm[j] = -T[j];
      mm_nt<NX, NX>(T, Ar, Sd);
      double qprev = 0.0;
      if (hasPrev && rowv && qv) qprev = (double)qv[(kb - 1) * NX + lane];
      rhs = -row_dot<NX>(T, qprev);
    }
    {
      // (2) control b-1: R^-1, U = B R^-1, theta += U B^T, zeta -= U r,
      //     W = R^-1 B^T kept for the primal step
      double Rr[NX], Br[NX], U[NX], th2[NX], W[NX];
#pragma unroll
      for (int j = 0; j < NX; ++j) { Rr[j] = 0.0; Br[j] = 0.0; }
      if (hasPrev && lane < NU) {
        const float *pr = a.R + ((cb - 1) * NU + lane) * NU;
#pragma unroll
        for (int j = 0; j < NU; ++j) Rr[j] = (double)pr[j];
      } else if (lane < NU) {
#pragma unroll
        for (int j = 0; j < NU; ++j) Rr[j] = (j == lane) ? 1.0 : 0.0;
      }
      if (hasPrev && rowv) {
        const float *pb = a.B + ((cb - 1) * NX + lane) * NU;
#pragma unroll
        for (int j = 0; j < NU; ++j) Br[j] = (double)pb[j];
      }
      if constexpr (PHASE == 3) {
        // R_{b-1}^-1 (and R^-1 B^T for the epilogue) as the forward formed them
        if (hasPrev && lane < kURows) {
          const double *w = a.rinv_ws + (cb - 1) * (NU + NX) * kURows + lane;
#pragma unroll
          for (int j = 0; j < NU; ++j) Rr[j] = w[j * kURows];
        }
      } else {
        gj_inverse<NU>(Rr, lane);
        // W first, stored at once, so that it is not live beside U and theta's update
        mm_nt<NU, NX>(Rr, Br, W);
        if (MODE != kForm && hasPrev && lane < kURows) {  // lane NU stores the zero pad row
          double *w = a.rinv_ws + (cb - 1) * (NU + NX) * kURows + lane;
#pragma unroll
          for (int j = 0; j < NU; ++j) w[j * kURows] = Rr[j];
#pragma unroll
          for (int j = 0; j < NX; ++j) w[(NU + j) * kURows] = W[j];
        }
      }
      mm_nn<NU, NU>(Br, Rr, U);
      mm_nt<NU, NX>(U, Br, th2);
#pragma unroll
      for (int j = 0; j < NX; ++j) Sd[j] += th2[j];
      double rprev = 0.0;
      if (hasPrev && lane < NU && rv) rprev = (double)rv[(cb - 1) * NU + lane];
      rhs -= row_dot<NU>(U, rprev);
    }
    {
      // (3) own knot: Q_b^-1 enters theta and gamma; (4) S_{b,b+1} = -Q_b^-1 A_b^T
      double Qi[NX], An[NX], Sx[NX];
#pragma unroll
      for (int j = 0; j < NX; ++j) { Qi[j] = 0.0; An[j] = 0.0; }
      if (act && rowv) {
        const float *pq = a.Q + (kb * NX + lane) * NX;
#pragma unroll
        for (int j = 0; j < NX; ++j) Qi[j] = (double)pq[j];
      } else if (rowv) {
#pragma unroll
        for (int j = 0; j < NX; ++j) Qi[j] = (j == lane) ? 1.0 : 0.0;
      }
      if constexpr (PHASE == 3) {
        if (act) {  // Q_b^-1 as the forward formed it
          const double *w = a.qinv_ws + kb * NX * kGroup + lane;
#pragma unroll
          for (int j = 0; j < NX; ++j) Qi[j] = w[j * kGroup];
        }
      } else {
        gj_inverse<NX>(Qi, lane);
        if (MODE != kForm && act) {  // all 16 lanes: rows >= NX are zero, columns are whole lines
          double *w = a.qinv_ws + kb * NX * kGroup + lane;
#pragma unroll
          for (int j = 0; j < NX; ++j) w[j * kGroup] = Qi[j];
        }
      }
#pragma unroll
      for (int j = 0; j < NX; ++j) Sd[j] += Qi[j];
      double qb = 0.0, add = 0.0;
      if (act && rowv) {
        if (qv) qb = (double)qv[kb * NX + lane];
        if (MODE == kAdjoint) {
          add = (double)a.gl[kb * NX + lane];
        } else if (b == 0) {
          add = (double)a.x0[(int64_t)pd.id * NX + lane];
        } else if (a.e) {
          add = -(double)a.e[(cb - 1) * NX + lane];
        }
      }
      rhs += row_dot<NX>(Qi, qb) + add;
      if (hasNext && rowv) {
        const float *pa = a.A + (cb * NX + lane) * NX;
#pragma unroll
        for (int j = 0; j < NX; ++j) An[j] = (double)pa[j];
      }
      mm_nt<NX, NX>(Qi, An, Sx);
#pragma unroll
      for (int j = 0; j < NX; ++j) Sp[j] = -Sx[j];
    }
    // (5) D_b^-1 = S_bb^-1 (theta_{b-1}^-1 for b >= 1, Q_0 up to rounding for b = 0).  Knot
    //     slots past the horizon have S_bb = I, so their D^-1 = I stays finite.  Only the
    //     preconditioner needs it (not the factorisation path).
    if constexpr (PHASE == 0) {
#pragma unroll
      for (int j = 0; j < NX; ++j) Dd[j] = Sd[j];
      gj_inverse<NX>(Dd, lane);
    }
    }  // PHASE != 2 (formation)
    if constexpr (PHASE == 0) {
    // (6) exchange D^-1 rows with the neighbouring knots (the one cross-knot dependency of
    //     the formation; section IV-A, Symmetric Stair preconditioner: of the whole
    //     preconditioner, only the neighbours' inverted diagonal blocks cross knots)
    if (rowv) {
#pragma unroll
      for (int j = 0; j < NX; ++j) ex_m[slot + 1][lane][j] = Dd[j];
    }
    if (multi && rowv && (slot == 0 || slot == KPW - 1)) {
      const uint32_t o = ws_off(&tws[my_t].hm[slot == 0 ? 0 : 1][lane][0]);
#pragma unroll
      for (int k = 0; k < NX / 2; ++k) store16_x(wsr, o + 16 * k, pack_d2(Dd[2 * k], Dd[2 * k + 1]), l2x);
    }
    sync_form();
    // (7) Phi^-1_{b,b-1} = -D_b^-1 S_{b,b-1} D_{b-1}^-1, Phi^-1_{b,b+1} likewise.  X = D_b^-1
    //     S_{b,b-1} is this lane's row; lane m reads row m of the neighbour's D^-1 from LDS
    //     (two columns at a time) and each column's product broadcasts it across the knot
    //     group, the terms added in row order
    {
      const int dr = rowv ? lane : 0;
      double X[NX];
      auto times_neighbour = [&](int ns, float (&P)[NX]) {
#pragma unroll
        for (int j = 0; j < NX; j += 2) {
          const double2 d = *reinterpret_cast<const double2 *>(&ex_m[ns][dr][j]);
          double c0 = 0.0, c1 = 0.0;
          row_fma14_f64(c0, d.x, X);
          row_fma14_f64(c1, d.y, X);
          P[j] = (float)(-c0);
          P[j + 1] = (float)(-c1);
        }
      };
      mm_nn<NX, NX>(Dd, Sm, X);
      times_neighbour(slot, Pm);
      mm_nn<NX, NX>(Dd, Sp, X);
      times_neighbour(slot + 2, Pp);
#pragma unroll
      for (int j = 0; j < NX; ++j) Pd[j] = (float)Dd[j];
    }
    } else if constexpr (PHASE == 3) {
      // (5)-(7) replaced: Phi^-1 as the forward formed it (knot slots past the horizon: the
      // blocks the formation gives them, D_b^-1 = I and zero off-diagonal blocks)
      if (act) {
        const float *fp = a.fac_p + fws_index<NX>(kb, 0, 0, lane);
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          Pm[j] = __builtin_nontemporal_load(fp + j * kGroup);
          Pd[j] = __builtin_nontemporal_load(fp + (NX + j) * kGroup);
          Pp[j] = __builtin_nontemporal_load(fp + (2 * NX + j) * kGroup);
        }
      } else {
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          Pm[j] = 0.0f;
          Pd[j] = (j == lane) ? 1.0f : 0.0f;
          Pp[j] = 0.0f;
        }
      }
    }  // PHASE 0 forms Phi^-1, PHASE 3 reads it
    if (!rowv) {
#pragma unroll
      for (int j = 0; j < NX; ++j) { Sm[j] = 0.0; Sd[j] = 0.0; Sp[j] = 0.0; Pm[j] = 0.f; Pd[j] = 0.f; Pp[j] = 0.f; }
      rhs = 0.0;
    }
    if constexpr (MODE == kForward && PHASE == 0) {
      if (a.fac_mode == 1 && act) {
        // the factor record (Phi^-1): all 16 lanes store (rows >= NX hold zeros), whole
        // lines, streamed past the caches (the adjoint reads it once)
        float *fp = a.fac_p + fws_index<NX>(kb, 0, 0, lane);
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          __builtin_nontemporal_store(Pm[j], fp + j * kGroup);
          __builtin_nontemporal_store(Pd[j], fp + (NX + j) * kGroup);
          __builtin_nontemporal_store(Pp[j], fp + (2 * NX + j) * kGroup);
        }
      }
    }
    if constexpr (PHASE == 1) {
      if (act) {
        // all 16 lanes store (rows >= NX hold zeros), so every column is one whole line
        double *col = a.s_ws + fws_index<NX>(kb, 0, 0, lane);
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          col[j * kGroup] = Sm[j];
          col[(NX + j) * kGroup] = Sd[j];
          col[(2 * NX + j) * kGroup] = Sp[j];
        }
        if (rowv) a.rhs_ws[kb * NX + lane] = rhs;
      }
    }

    if constexpr (MODE == kForm) {
      if (act && rowv) {
        const int64_t o = kb * 3 * NX * NX + (int64_t)lane * NX;
        if (a.S_out)
          for (int j = 0; j < NX; ++j) {
            a.S_out[o + j] = (float)Sm[j];
            a.S_out[o + NX * NX + j] = (float)Sd[j];
            a.S_out[o + 2 * NX * NX + j] = (float)Sp[j];
          }
        if (a.P_out)
          for (int j = 0; j < NX; ++j) {
            a.P_out[o + j] = Pm[j];
            a.P_out[o + NX * NX + j] = Pd[j];
            a.P_out[o + 2 * NX * NX + j] = Pp[j];
          }
        if (a.gam_out) a.gam_out[kb * NX + lane] = (float)rhs;
      }
    } else if constexpr (PHASE != 1) {
      double lam = 0.0, eta_ref = 0.0, eta_new = 0.0;
      int status = MPCPCG_NOT_CONVERGED, it = 0;
      if constexpr (PHASE == 2) {
        if (act && rowv) lam = a.lam_ws[kb * NX + lane];
        status = MPCPCG_OK;
      } else {
      // Phi^-1 rows move to LDS for the solve (the D^-1 exchange above used the same bytes)
      __syncthreads();
      if (rowv) {
        float *row = pl + (slot * NX + lane) * kPRow;
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          row[j] = Pm[j];
          row[NX + j] = Pd[j];
          row[2 * NX + j] = Pp[j];
        }
      }
      // ================================================================== PCG
      refresh();
      // r~ row = Phi^-1 row . [x(b-1), x(b), x(b+1)] for the rows of knot slot ps (a ghost
      // slot for the recomputed neighbour knots): two blocks are read from LDS up front and
      // the third while the first product runs, so that at most 28 of its values occupy
      // registers and only two LDS round trips are exposed
      auto phi_row = [&](int ps) { return pl + (ps * NX + (rowv ? lane : 0)) * kPRow; };
      auto load_m01 = [&](const float *row, float (&m0)[NX], float (&m1)[NX]) {
#pragma unroll
        for (int j = 0; j < NX; ++j) {
          m0[j] = row[j];
          m1[j] = row[NX + j];
        }
      };
      // the product with the first two blocks already in registers
      auto precond_m01 = [&](const float *row, const float (&m0)[NX], const float (&m1)[NX], float xm, float x0v,
                             float xp) {
        float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
        float m2[NX];
        row_fma14_f32(acc0, xm, m0);
#pragma unroll
        for (int j = 0; j < NX; ++j) m2[j] = row[2 * NX + j];
        row_fma14_f32(acc1, x0v, m1);
        row_fma14_f32(acc2, xp, m2);
        return rowv ? (acc0 + acc1) + acc2 : 0.0f;
      };
      auto precond_row = [&](int ps, float xm, float x0v, float xp) {
        const float *row = phi_row(ps);
        float m0[NX], m1[NX];
        load_m01(row, m0, m1);
        return precond_m01(row, m0, m1, xm, x0v, xp);
      };
      // one barrier per iteration; the cap keeps barrier indices within the 24 bits the tags give them
      const int max_iter = (int)min((int64_t)(a.max_iter > 0 ? a.max_iter : (int64_t)N * NX), (int64_t)1 << 23);
      const bool warm = (MODE == kForward) && a.warm;
      if (warm && act && rowv) lam = (double)a.lam[kb * NX + lane];
      // setup exchange: boundary Phi^-1 rows; gamma at depths 1 and 2 (cold) or gamma and
      // lambda_0 at depth 1 (warm); device-scope stores, completed before the stage flag
      if (multi && (slot <= 1 || slot >= KPW - 2)) {
        TaskWS<NX> &w = tws[my_t];
        const int side = slot <= 1 ? 0 : 1;
        if (slot == 0 || slot == KPW - 1) {
          if (rowv) {
            float row[kPRow];
#pragma unroll
            for (int j = 0; j < NX; ++j) {
              row[j] = Pm[j];
              row[NX + j] = Pd[j];
              row[2 * NX + j] = Pp[j];
            }
            row[3 * NX] = 0.0f;
            row[3 * NX + 1] = 0.0f;
            const uint32_t o = ws_off(&w.hp[side][lane][0]);
#pragma unroll
            for (int k = 0; k < kPRow / 4; ++k)
              store16_x(wsr, o + 16 * k, pack_f4(row[4 * k], row[4 * k + 1], row[4 * k + 2], row[4 * k + 3]), l2x);
          }
          store8_x(wsr, ws_off(&w.hs[side][0][lane]), __builtin_bit_cast(uint64_t, rhs), l2x);
          if (warm) store8_x(wsr, ws_off(&w.hs[side][1][lane]), __builtin_bit_cast(uint64_t, lam), l2x);
        } else if (!warm) {
          store8_x(wsr, ws_off(&w.hs[side][1][lane]), __builtin_bit_cast(uint64_t, rhs), l2x);
        }
      }
      ex_d[0][slot + 1][lane] = rhs;
      ex_d[1][slot + 1][lane] = warm ? lam : 0.0;
      sync_setup();
      double r = rhs, rm = ex_d[0][slot][lane], rp = ex_d[0][slot + 2][lane];
      // r and s of the knot two beyond this part's end, kept in the registers of the edge
      // slots' lanes (the only lanes that use them)
      double r2 = 0.0, s2 = 0.0;
      if (slot == 0) r2 = ex_d[1][0][lane];
      if (slot == KPW - 1) r2 = ex_d[1][KPW + 1][lane];
      if (warm) {
        // r = gamma - S lambda_0; eta_ref = gamma^T Phi^-1 gamma; then r's halos two deep
        const double lm = ex_d[1][slot][lane], lp = ex_d[1][slot + 2][lane];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        row_fma14_f64(a0, lm, Sm);
        row_fma14_f64(a1, lam, Sd);
        row_fma14_f64(a2, lp, Sp);
        r = rhs - ((a0 + a1) + a2);
        const float gt = precond_row(slot, (float)rm, (float)rhs, (float)rp);
        put_red(0, 0, rhs * (double)gt);
        __syncthreads();  // every halo read of the setup channels is done
        put_d2(r);
        sync_point(IC<2>{}, IC<1>{}, 0, nothing);
        eta_ref = uni(tot[0]);
        rm = ex_d[0][slot][lane];
        rp = ex_d[0][slot + 2][lane];
        if (slot == 0) r2 = ex_d[1][0][lane];
        if (slot == KPW - 1) r2 = ex_d[1][KPW + 1][lane];
      }
      // Algorithm 1 with its two inner products gathered at one barrier per iteration
      // (Chronopoulos-Gear form): u = Phi^-1 r and w = S u, then gam = r^T u (= eta') and
      // delta = w^T u meet at the barrier; p^T S p = delta - beta gam / alpha_prev, and the
      // recurrences p = u + beta p, s = w + beta s (s = S p), lambda += alpha p,
      // r -= alpha s give the iterates of Algorithm 1.  Each part keeps r and s of the
      // two knots beyond each of its ends (bit-identical copies, updated from the
      // neighbours' w), and recomputes u of the adjacent knot itself from a copy of that
      // knot's Phi^-1 row, so no second exchange is needed inside an iteration.
      double p = 0.0, sv = 0.0, sm = 0.0, sp = 0.0;
      double gam_prev = 1.0, alpha_prev = 1.0, tau = 0.0;
      const bool edge_wave = multi && (wave == 0 || wave == NW - 1);
      // the reciprocals of the previous iteration's gamma and alpha are formed before the
      // iteration's first workgroup barrier by a wave that does no ghost product (it waits
      // there anyway), so only one division remains after the gang barrier
      const int rcp_wave = NW > 2 ? 1 : 0;
      for (it = 0;; ++it) {
        if (aborted) break;
        // (1) u = Phi^-1 r on this knot, and on the ghost knot beyond each end
        const float u = precond_row(slot, (float)rm, (float)r, (float)rp);
        ex_f[slot + 1][lane] = u;
        if (edge_wave) {
          // (the rest of the workgroup waits for the edge waves' second product)
          __builtin_amdgcn_s_setprio(1);
          const bool left = slot == 0;
          const float ug = precond_row(left ? KPW : KPW + 1, (float)(left ? r2 : r), (float)(left ? rm : rp),
                                       (float)(left ? r : r2));
          if (slot == 0) ex_f[0][lane] = ug;
          if (slot == KPW - 1) ex_f[KPW + 1][lane] = ug;
          __builtin_amdgcn_s_setprio(0);
        }
        if (wave == rcp_wave) {
          const double rg = 1.0 / gam_prev, ra = 1.0 / alpha_prev;
          if (wl == 0) {
            rcp_sh[0] = rg;
            rcp_sh[1] = ra;
          }
        }
        __syncthreads();
        const double rg = uni(rcp_sh[0]), ra = uni(rcp_sh[1]);
        // (2) w = S u
        // (the own block first: it needs no LDS value, so it runs while u of the
        // neighbouring knots is read)
        const double um = (double)ex_f[slot][lane], up = (double)ex_f[slot + 2][lane];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        row_fma14_f64(a1, (double)u, Sd);
        row_fma14_f64(a0, um, Sm);
        row_fma14_f64(a2, up, Sp);
        const double w = (a0 + a1) + a2;
        // (3) gam = r^T u, delta = w^T u; w two knots deep to the neighbours
        put_red2(0, r * (double)u, w * (double)u);
        put_d2(w);
        // after the barrier, one LDS round trip: the totals, w of the neighbouring knots
        // (the halo copies at the part's ends) and w two knots out for the edge slots
        double tg, td, wm, wp, wh2;
        sync_point(IC<2>{}, IC<2>{}, 0, [&] {
          tg = tot[0];
          td = tot[1];
          wm = ex_d[0][slot][lane];
          wp = ex_d[0][slot + 2][lane];
          wh2 = ex_d[1][slot == 0 ? 0 : KPW + 1][lane];
        });
        const double gam = uni(tg), del = uni(td);
        eta_new = gam;
        if (it == 0) {
          if (!warm) eta_ref = gam;  // lambda_0 = 0: r = gamma, so gam = gamma^T Phi^-1 gamma
          tau = a.stop_abs ? (double)a.eps : (double)a.eps * (double)a.eps * eta_ref;
          if (!(eta_ref == eta_ref) || __builtin_isinf(eta_ref)) {
            status = MPCPCG_BREAKDOWN;
            break;
          }
        }
        if (!(gam == gam) || __builtin_isinf(gam)) {
          status = MPCPCG_BREAKDOWN;
          break;
        }
        if (it == 0 ? gam <= tau : gam < tau) {
          status = MPCPCG_OK;
          break;
        }
        if (it >= max_iter) break;
        const double beta = it == 0 ? 0.0 : gam * rg;
        const double pSp = it == 0 ? del : del - beta * gam * ra;
        if (!(pSp > 0.0) || __builtin_isinf(pSp)) {
          status = MPCPCG_BREAKDOWN;
          break;
        }
        const double alpha = gam / pSp;
        // (4) recurrences on this knot and on the halo copies (depth 1 everywhere, depth 2
        //     at the part's ends)
        p = __builtin_fma(beta, p, (double)u);
        sv = __builtin_fma(beta, sv, w);
        sm = __builtin_fma(beta, sm, wm);
        sp = __builtin_fma(beta, sp, wp);
        lam = __builtin_fma(alpha, p, lam);
        r = __builtin_fma(-alpha, sv, r);
        rm = __builtin_fma(-alpha, sm, rm);
        rp = __builtin_fma(-alpha, sp, rp);
        if (multi && (slot == 0 || slot == KPW - 1)) {
          s2 = __builtin_fma(beta, s2, wh2);
          r2 = __builtin_fma(-alpha, s2, r2);
        }
        gam_prev = gam;
        alpha_prev = alpha;
      }
      if (it > max_iter) it = max_iter;
      }  // PHASE == 0 (PCG)
      if (aborted) status = MPCPCG_TIMEOUT;
      if (!rowv || !act) lam = 0.0;

      // ================================================================== epilogue
      refresh();
      // primal step dZ = -G^-1 (g - C^T lambda) (with mu and the loss gradients in the
      // adjoint): x rows use Q_b^-1 and S_{b,b+1} = -Q_b^-1 A_b^T; u rows of control b-1
      // use R_{b-1}^-1 and W = R_{b-1}^-1 B_{b-1}^T (both written during formation).
      put_d(0, lam);
      sync_point(IC<1>{}, IC<0>{}, 0, nothing);
      const double lp = ex_d[0][slot + 2][lane];
      double qmin = 0.0;   // q_b - lambda_b  (or gx_b - mu_b)
      if (act && rowv) {
        const double qb = qv ? (double)qv[kb * NX + lane] : 0.0;
        qmin = qb - lam;
      }
      double Qi[NX];
#pragma unroll
      for (int j = 0; j < NX; ++j) Qi[j] = 0.0;
      if (act && rowv) {
        const double *w = a.qinv_ws + kb * NX * kGroup + lane;
#pragma unroll
        for (int j = 0; j < NX; ++j) Qi[j] = w[j * kGroup];
      }
      const double xrow = -row_dot<NX>(Qi, qmin) + row_dot<NX>(Sp, lp);
      double Rr[NX], W[NX];
#pragma unroll
      for (int j = 0; j < NX; ++j) { Rr[j] = 0.0; W[j] = 0.0; }
      double rprev = 0.0;
      if (hasPrev && lane < NU) {
        const double *w = a.rinv_ws + (cb - 1) * (NU + NX) * kURows + lane;
#pragma unroll
        for (int j = 0; j < NU; ++j) Rr[j] = w[j * kURows];
#pragma unroll
        for (int j = 0; j < NX; ++j) W[j] = w[(NU + j) * kURows];
        if (rv) rprev = (double)rv[(cb - 1) * NU + lane];
      }
      const double urow = -row_dot<NU>(Rr, rprev) - row_dot<NX>(W, lam);
      if constexpr (MODE == kForward) {
        if (act && rowv) {
          a.lam[kb * NX + lane] = (float)lam;
          a.dx[kb * NX + lane] = (float)xrow;
        }
        if (hasPrev && lane < NU) a.du[(cb - 1) * NU + lane] = (float)urow;
      } else {
        // adjoint: lam holds mu, xrow = nu1x_b, urow = nu1u_{b-1}
        const double mu = lam, n1x = xrow, n1u = urow;
        put_d(0, n1x);
          sync_point(IC<1>{}, IC<0>{}, 1, nothing);
        const double n1xm = ex_d[0][slot][lane];  // nu1x_{b-1}
        double dxb = 0.0, dxm = 0.0, lb = 0.0, dum = 0.0;
        if (act && rowv) {
          dxb = (double)a.dx_in[kb * NX + lane];
          lb = (double)a.lam_in[kb * NX + lane];
        }
        if (hasPrev && rowv) dxm = (double)a.dx_in[(kb - 1) * NX + lane];
        if (hasPrev && lane < NU) dum = (double)a.du_in[(cb - 1) * NU + lane];
        // dQ_b = sym(nu1x_b dx_b^T); row i = (nu1x_i dx^T + dx_i nu1x^T) / 2
        double dQrow[NX], tmp[NX];
        outer_row<NX>(dQrow, dxb, 0.5 * n1x);
        outer_row<NX>(tmp, n1x, 0.5 * dxb);
#pragma unroll
        for (int j = 0; j < NX; ++j) dQrow[j] += tmp[j];
        if (act && rowv) {
          float *dq = a.dQ + (kb * NX + lane) * NX;
#pragma unroll
          for (int j = 0; j < NX; ++j) dq[j] = (float)dQrow[j];
          a.dq[kb * NX + lane] = (float)n1x;
          if (a.dgamma) a.dgamma[kb * NX + lane] = (float)mu;
          if (b == 0) a.dx0[(int64_t)pd.id * NX + lane] = (float)mu;
        }
        // control b-1 (owned by this group): dA, dB, dR, dr, de
        double dArow[NX], dBrow[NX], dRrow[NX];
        outer_row<NX>(dArow, n1xm, lb);
        outer_row<NX>(tmp, dxm, mu);
#pragma unroll
        for (int j = 0; j < NX; ++j) dArow[j] += tmp[j];
        outer_row<NU>(dBrow, n1u, lb);
        outer_row<NU>(tmp, dum, mu);
#pragma unroll
        for (int j = 0; j < NU; ++j) dBrow[j] += tmp[j];
        outer_row<NU>(dRrow, dum, 0.5 * n1u);
        outer_row<NU>(tmp, n1u, 0.5 * dum);
#pragma unroll
        for (int j = 0; j < NU; ++j) dRrow[j] += tmp[j];
        if (hasPrev && rowv) {
          float *pa = a.dA + ((cb - 1) * NX + lane) * NX;
#pragma unroll
          for (int j = 0; j < NX; ++j) pa[j] = (float)dArow[j];
          float *pb = a.dB + ((cb - 1) * NX + lane) * NU;
#pragma unroll
          for (int j = 0; j < NU; ++j) pb[j] = (float)dBrow[j];
          if (a.de) a.de[(cb - 1) * NX + lane] = (float)(-mu);
        }
        if (hasPrev && lane < NU) {
          float *pr = a.dR + ((cb - 1) * NU + lane) * NU;
#pragma unroll
          for (int j = 0; j < NU; ++j) pr[j] = (float)dRrow[j];
          a.dr[(cb - 1) * NU + lane] = (float)n1u;
        }
      }
      if ((PHASE == 0 || PHASE == 3) && tid == 0 && part == 0)
        put_stats(a.stats + pd.id, it, status,
                  eta_ref > 0.0 ? (float)__builtin_sqrt(eta_new > 0.0 ? eta_new / eta_ref : 0.0) : 0.0f);
    }

    // ------------------------------------------------------------- gang teardown
    // Every part has read all it needs once all G have arrived here, so the last one out
    // zeroes the gang's tagged words (no stale tag survives into a later solve) and resets
    // the gang state.  The arrival is a relaxed count after a wait for this wave's stores:
    // the only values another part reads after it (part 0's stats, the abort flag) are
    // device-scope stores of this wave, so they have landed before the count moves, and an
    // acquire-release count would also write back the whole L2 at every task's end.
    if (multi) {
      __syncthreads();
      if (tid == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        const int d = __hip_atomic_fetch_add(&gang->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sh_task = d == G - 1;
      }
      __syncthreads();
      if (uni(sh_task)) {
        constexpr int kWords = sizeof(TagWS) / sizeof(uint64_t);
        for (int i = tid; i < G * kWords; i += NT) {
          uint64_t *w = reinterpret_cast<uint64_t *>(&tws[pd.t0 + i / kWords].tg) + i % kWords;
          __hip_atomic_store(w, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid == 0) {
          // a part that gave up raised the abort flag: the problem reports TIMEOUT (part 0
          // wrote its stats before its arrival was counted, so this store comes later)
          const int ab = __hip_atomic_load(&gang->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          int *status_word = a.stats ? reinterpret_cast<int *>(a.stats + pd.id) + 1 : nullptr;
          if constexpr (PHASE == 1) {
            if (ab) __hip_atomic_store(&gang->timed_out, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else if constexpr (PHASE == 2) {
            const int t1 = __hip_atomic_load(&gang->timed_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((ab || t1) && status_word)
              __hip_atomic_store(status_word, (int)MPCPCG_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&gang->timed_out, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else if constexpr (MODE != kForm) {
            if (ab && status_word)
              __hip_atomic_store(status_word, (int)MPCPCG_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          __hip_atomic_store(&gang->abort, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          // (the next solve of this gang record is in a later launch)
          __hip_atomic_store(&gang->done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }

  // ------------------------------------------------------------- launch teardown
  // The last workgroup out resets the queue and advances the launch generation.  With
  // per-XCD lists it first checks that every list was drained: a list whose XCD ran no
  // workgroup of this launch (a placement the host did not expect) leaves its problems
  // unsolved, and those report TIMEOUT instead of stale stats.
  __syncthreads();
  if (tid == 0) {
    // relaxed, as the gang count: the queue counters are atomics, the stats device-scope
    // stores of this wave, and the next launch starts after this one's end
    __builtin_amdgcn_s_waitcnt(0);
    const int d = __hip_atomic_fetch_add(&a.queue[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (d == (int)gridDim.x - 1) {
      if (a.persistent && a.xoff && a.stats) {
        for (int x = 0; x < 8; ++x) {
          const int popped = __hip_atomic_load(&a.queue[4 + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          for (int t = a.xoff[x] + max(popped, 0); t < a.xoff[x + 1]; ++t) {
            const Task tk = a.tasks[t];
            if (tk.part == 0) put_stats(a.stats + a.probs[tk.prob].id, 0, MPCPCG_TIMEOUT, 0.0f);
          }
        }
      }
      __hip_atomic_store(&a.queue[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int x = 0; x < 8; ++x) __hip_atomic_store(&a.queue[4 + x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&a.queue[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.queue[1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace mpc
