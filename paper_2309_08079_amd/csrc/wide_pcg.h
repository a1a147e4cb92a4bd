// PCG of the 28-state path (nx = 28, nu = 14) on gangs of workgroups.
//
// A problem of N knots is cut into parts of KW consecutive knots, one workgroup per part
// and one wave per knot; the parts of a problem form a gang that meets at gang barriers,
// as in the 14-state kernel.  Lanes r and r + 32 of a knot's wave both own row r (< 28)
// of the knot's block row and each keeps half of its columns of S (FP64) and of Phi^-1
// (FP32) in registers for the whole solve: 3 x 14 doubles and 3 x 14 floats per lane.  A
// product takes the vector entries of its half from LDS (the same address for every lane
// of a half: a broadcast read) and the two halves add their partial sums across the wave.
//
// The loop is Algorithm 1 as printed, with its two inner products each met at a gang
// barrier.  Values that cross a part boundary travel with those barriers as 16-byte tagged
// words (the 14-state kernel's protocol): each part publishes its partial sum and the rows
// of its first and last knot of the vector just formed (S p at the first barrier,
// Phi^-1 r at the second); every part then updates its copies of r and p of the two
// neighbouring knots with the same fused operations the neighbour applies to its own, so
// the copies stay bit-identical and no other exchange is needed.  Partial sums are added
// in a fixed order, so every part takes the same decisions.
//
// Inputs are the workspace blocks the formation and preconditioner launches write (S, Phi^-1,
// the right-hand side); the output is lambda (or mu in adjoint mode) in FP64 in lamw and
// the stats; the primal step / gradients follow in wide_epilogue.  Stopping rule, status
// codes and precision are those of the 14-state kernel: FP64 S, vectors and reductions,
// FP32 Phi^-1 applied with FP32 accumulation.
#pragma once
#include "pcg_kernel.h"
#include "wide_kernels.h"

namespace mpc {
namespace wide {

constexpr int kGangKnots = 4;  // knots (waves) per workgroup

// Tagged words of one part (read by its gang): [parity][value] partial sums and
// [parity][channel][side][row] boundary rows, each a 16-byte pair (payload halves tagged).
struct WTag {
  uint64_t red[2][2][2];
  uint64_t rows[2][2][2][32][2];
};

struct GangArgs {
  void *tws;              // WTag[ntasks]
  Gang *gang;             // [problems]
  int *queue;             // [0] head, [1] workgroups finished, [2] launch generation,
                          // [4 + x] head of XCD x's list
  const ProbDesc *probs;  // per problem: k0, N, t0 (first task), nparts, id
  const Task *tasks;      // longest problem first, the parts of a problem adjacent
  const int32_t *xoff;    // [9] or nullptr: the tasks of XCD x are [xoff[x], xoff[x+1]),
                          // popped by the workgroups running on XCD x only, so that every
                          // gang runs on one XCD and its barriers use that XCD's L2
  int32_t ntasks;
  int32_t l2x;            // 1 with xoff: barrier words through the XCD's L2
  int64_t spin_limit;     // wall-clock ticks before a wait gives up
};

template <int NX, int KW>
__global__ void __launch_bounds__(KW * 64) __attribute__((amdgpu_waves_per_eu(3, 3)))
    wide_pcg_gang(const WArgs a, const GangArgs g) {
  static_assert(NX % 2 == 0 && NX <= 32, "two lanes per row of an even NX <= 32");
  constexpr int H = NX / 2;
  constexpr int MM = NX * NX;
  constexpr int NT = KW * 64;
  __shared__ __attribute__((aligned(16))) double vx[KW + 2][32];  // slot s + 1 = knot s of the part
  __shared__ __attribute__((aligned(16))) float vf[KW + 2][32];
  __shared__ double hr[2][32], hp[2][32], hg[2][32];  // neighbours' r, p, rhs [side][row]
  __shared__ double hin[2][2][32];                    // received rows [channel][side][row]
  __shared__ double red_w[2][KW];                     // [value][wave]
  __shared__ double tot[2];
  __shared__ int sh_task, sh_abort;

  // Lane indices are re-derived through an opaque copy of threadIdx.x at the top of every
  // PCG iteration (refresh below), so that the compiler recomputes the LDS addresses of the
  // products instead of keeping them live across the loop, where the registers hold S and
  // Phi^-1.
  int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  int h = lane >> 5, row = lane & 31;
  bool rowv = row < NX;
  int r = rowv ? row : 0;
  auto refresh = [&]() {
    asm volatile("" : "+v"(tid));
    wave = tid >> 6;
    lane = tid & 63;
    h = lane >> 5;
    row = lane & 31;
    rowv = row < NX;
    r = rowv ? row : 0;
  };
  WTag *tws = reinterpret_cast<WTag *>(g.tws);
  const __amdgpu_buffer_rsrc_t wsr = ws_rsrc(g.tws);
  auto ws_off = [&](const void *p) { return (uint32_t)((const char *)p - (const char *)g.tws); };
  // launch generation (advanced by the last workgroup of every launch), part of every tag
  const uint64_t gen = (uint64_t)(uint32_t)uni(__hip_atomic_load(&g.queue[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  const bool l2x = g.l2x != 0;
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

  for (;;) {
    __syncthreads();
    if (tid == 0) {
      if (g.xoff) {
        unsigned x;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
        x &= 7u;
        const int t = g.xoff[x] + atomicAdd(&g.queue[4 + x], 1);
        sh_task = t < g.xoff[x + 1] ? t : g.ntasks;  // this XCD's list is empty
      } else {
        sh_task = atomicAdd(&g.queue[0], 1);
      }
    }
    __syncthreads();
    const int task = uni(sh_task);
    if (task >= g.ntasks) break;
    const Task tk = g.tasks[task];
    const ProbDesc pd = g.probs[tk.prob];
    const int part = tk.part, G = pd.nparts, N = pd.N;
    const bool multi = G > 1;
    const int b = part * KW + wave;
    const bool act = b < N;
    const bool mine = act && rowv;  // this lane holds a row of an existing knot
    const int64_t kb = pd.k0 + (act ? b : 0);
    const int my_t = pd.t0 + part;
    Gang *gang = g.gang + tk.prob;
    int nsync = 0;
    bool aborted = false;
    if (tid == 0) sh_abort = 0;
    for (int t = tid; t < 2 * 32; t += NT) {
      const int s = t >> 5, l = t & 31;
      vx[s ? KW + 1 : 0][l] = 0.0;
      vf[s ? KW + 1 : 0][l] = 0.0f;
      hr[s][l] = 0.0; hp[s][l] = 0.0; hg[s][l] = 0.0;
    }

    // rows of S and Phi^-1: this lane's half of the columns of blocks (b,b-1), (b,b), (b,b+1)
    double S[3][H];
    float P[3][H];
    {
      const double *sb = a.S + kb * 3 * MM + (int64_t)r * NX + h * H;
      const float *pb = a.P + kb * 3 * MM + (int64_t)r * NX + h * H;
#pragma unroll
      for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int j = 0; j < H; ++j) {
          const double sv = sb[s * MM + j];
          const float pv = pb[s * MM + j];
          S[s][j] = mine ? sv : 0.0;
          P[s][j] = mine ? pv : 0.0f;
        }
    }
    const bool adj = a.adjoint != 0;
    const bool warm = !adj && a.warm;
    const double rhs = mine ? a.rhs[kb * NX + r] : 0.0;
    double lam = (warm && mine) ? (double)a.lam[kb * NX + r] : 0.0;

    // ---- products with the vector in vx / vf (slots wave, wave+1, wave+2 = b-1, b, b+1)
    // (one block's vector entries at a time in registers: the loads of a block are not
    // hoisted above the previous block's products)
    auto s_prod = [&]() {
      double acc = 0.0;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const double *x = &vx[wave + s][h * H];
#pragma unroll
        for (int j = 0; j < H; ++j) acc = __builtin_fma(S[s][j], x[j], acc);
        __builtin_amdgcn_sched_barrier(0);
      }
      const double other = __shfl_xor(acc, 32);
      return h == 0 ? acc + other : other + acc;
    };
    auto p_prod = [&]() {
      float acc = 0.0f;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const float *x = &vf[wave + s][h * H];
#pragma unroll
        for (int j = 0; j < H; ++j) acc = __builtin_fmaf(P[s][j], x[j], acc);
        __builtin_amdgcn_sched_barrier(0);
      }
      const float other = __shfl_xor(acc, 32);
      return h == 0 ? acc + other : other + acc;
    };
    // this wave's knot's share of an inner product, summed over its rows in a fixed order
    // (the rows live in lanes 0..31)
    auto put_red = [&](int v, double x) {
      const double s = sum_rows01((h == 0 && mine) ? x : 0.0);
      if (lane == 0) red_w[v][wave] = s;
    };
    // a boundary row of channel c (first knot: side 0, last knot: side 1) to the gang
    auto put_row = [&](int c, double x) {
      if (multi && h == 0 && rowv) {
        const uint32_t tag = loop_tag(gen, nsync);
        if (wave == 0) put_pair(ws_off(tws[my_t].rows[nsync & 1][c][0][row]), tag, x);
        if (wave == KW - 1) put_pair(ws_off(tws[my_t].rows[nsync & 1][c][1][row]), tag, x);
      }
    };
    auto poll_spin = [&](int &polls, long long t_start) -> bool {
      __builtin_amdgcn_s_sleep(1);
      if ((++polls & 63) == 0) {
        if (__hip_atomic_load(&gang->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return true;
        if (wall_clock64() - t_start > g.spin_limit) {
          __hip_atomic_store(&gang->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          return true;
        }
      }
      return false;
    };
    // Gang barrier: NV partial sums (totals in tot[]) and NC channels of boundary rows
    // (the neighbours' rows land in hin[c][side][row]; zeros where no neighbour exists).
    auto sync = [&](int nv, int nc) {
      __syncthreads();
      if (!multi || aborted) {
        if (tid == 0)
          for (int v = 0; v < nv; ++v) {
            double s = 0.0;
            for (int w = 0; w < KW; ++w) s += red_w[v][w];
            tot[v] = s;
          }
        for (int t = tid; t < 2 * 2 * 32; t += NT) (&hin[0][0][0])[t] = 0.0;
        ++nsync;
        __syncthreads();
        return;
      }
      const int par = nsync & 1;
      const uint32_t tag = loop_tag(gen, nsync);
      if (wave == 0 && lane < nv) {  // this part's sums, its waves in order
        double ps = 0.0;
        for (int w = 0; w < KW; ++w) ps += red_w[lane][w];
        put_pair(ws_off(tws[my_t].red[par][lane]), tag, ps);
      }
      // device scope: the last part's words land ~1 us after the first part arrives; through
      // one XCD's L2 a round takes ~0.4 us and polling at once is fastest
      if (!l2x) __builtin_amdgcn_s_sleep(24);
      const long long t_start = wall_clock64();
      int polls = 0;
      bool ab = false;
      // halo rows: thread t < nc * 2 * NX waits for (channel, side, row)
      const bool hw = tid < nc * 2 * NX;
      const int hc = tid / (2 * NX), hs = (tid / NX) & 1, hrow = tid % NX;
      const int nb = hs == 0 ? part - 1 : part + 1;
      const bool has = hw && nb >= 0 && nb < G;
      const uint32_t hoff = ws_off(tws[has ? my_t + (hs == 0 ? -1 : 1) : my_t].rows[par][hc & 1][hs ^ 1][hrow]);
      u32x4 hq = {0u, 0u, 0u, 0u};
      double v0 = 0.0, v1 = 0.0;
      for (int g0 = 0; g0 < (wave == 0 ? G : 1) && !ab; g0 += 64) {
        const int gp = g0 + lane;
        const bool want_red = wave == 0 && nv > 0 && gp < G;
        const bool want_halo = g0 == 0 && has;
        u32x4 rw0 = {0u, 0u, 0u, 0u}, rw1 = {0u, 0u, 0u, 0u};
        while (true) {
          bool ok = true;
          if (want_red) {
            rw0 = get_pair(ws_off(tws[pd.t0 + gp].red[par][0]));
            ok &= pair_has(rw0, tag);
            if (nv > 1) {
              rw1 = get_pair(ws_off(tws[pd.t0 + gp].red[par][1]));
              ok &= pair_has(rw1, tag);
            }
          }
          if (want_halo) {
            hq = get_pair(hoff);
            ok &= pair_has(hq, tag);
          }
          if (__ballot(ok) == ~0ull) break;
          if ((ab = poll_spin(polls, t_start))) break;
        }
        if (want_red && !ab) {
          v0 += pair_value(rw0);
          if (nv > 1) v1 += pair_value(rw1);
        }
      }
      if (hw) hin[hc][hs][hrow] = (has && !ab) ? pair_value(hq) : 0.0;
      if (wave == 0) {
        const double w0 = wave_sum(v0), w1 = nv > 1 ? wave_sum(v1) : 0.0;
        if (lane == 0) {
          tot[0] = w0;
          tot[1] = w1;
        }
      }
      if (ab) sh_abort = 1;
      __syncthreads();
      ++nsync;
      aborted = aborted || uni(sh_abort) != 0;
    };
    auto put_vx = [&](double x) {
      if (h == 0 && rowv) vx[wave + 1][row] = x;
    };
    auto put_vf = [&](float x) {
      if (h == 0 && rowv) vf[wave + 1][row] = x;
    };

    // ---- setup: the neighbours' right-hand-side rows (and warm-start rows)
    put_row(0, rhs);
    if (warm) put_row(1, lam);
    sync(0, warm ? 2 : 1);
    for (int t = tid; t < 2 * NX; t += NT) {
      const int s = t / NX, l = t % NX;
      hg[s][l] = hin[0][s][l];
      hr[s][l] = hin[0][s][l];
    }
    double rv = rhs;
    if (warm) {
      // r = gamma - S lambda_0 (lambda_0 of the neighbours' boundary knots from the setup)
      put_vx(lam);
      for (int t = tid; t < 2 * NX; t += NT) {
        const int s = t / NX, l = t % NX;
        vx[s ? KW + 1 : 0][l] = hin[1][s][l];
      }
      __syncthreads();
      rv = rhs - s_prod();
      put_row(0, rv);
      sync(0, 1);
      for (int t = tid; t < 2 * NX; t += NT) {
        const int s = t / NX, l = t % NX;
        hr[s][l] = hin[0][s][l];
      }
    }
    double eta = 0.0, eta_ref = 0.0, eta_new = 0.0;
    float rt;
    {
      __syncthreads();
      put_vf((float)rv);
      for (int t = tid; t < 2 * NX; t += NT) {
        const int s = t / NX, l = t % NX;
        vf[s ? KW + 1 : 0][l] = (float)hr[s][l];
      }
      __syncthreads();
      rt = p_prod();
      put_red(0, rv * (double)rt);
      if (warm) {  // eta_ref = gamma^T Phi^-1 gamma needs Phi^-1 gamma as well
        __syncthreads();
        put_vf((float)rhs);
        for (int t = tid; t < 2 * NX; t += NT) {
          const int s = t / NX, l = t % NX;
          vf[s ? KW + 1 : 0][l] = (float)hg[s][l];
        }
        __syncthreads();
        const float gt = p_prod();
        put_red(1, rhs * (double)gt);
      }
      put_row(0, (double)rt);
      sync(warm ? 2 : 1, 1);
      eta = uni(tot[0]);
      eta_ref = warm ? uni(tot[1]) : eta;
    }
    double p = (double)rt;
    for (int t = tid; t < 2 * NX; t += NT) {
      const int s = t / NX, l = t % NX;
      hp[s][l] = hin[0][s][l];
    }
    const double tau = a.stop_abs ? (double)a.eps : (double)a.eps * (double)a.eps * eta_ref;
    // two barriers per iteration: the cap keeps barrier indices within the tags' 24 bits
    const int max_iter = min(a.max_iter > 0 ? a.max_iter : N * NX, 1 << 22);
    int status = MPCPCG_NOT_CONVERGED, it = 0;
    double res = rv;  // r of Algorithm 1 (this lane's row)
    eta_new = eta;
    if (!(eta == eta) || !(eta_ref == eta_ref) || __builtin_isinf(eta) || __builtin_isinf(eta_ref)) {
      status = MPCPCG_BREAKDOWN;
    } else if (eta <= tau) {
      status = MPCPCG_OK;
    } else {
      for (it = 1; it <= max_iter && !aborted; ++it) {
        refresh();
        // Upsilon = S p, upsilon = p^T Upsilon
        __syncthreads();
        put_vx(p);
        for (int t = tid; t < 2 * NX; t += NT) {
          const int s = t / NX, l = t % NX;
          vx[s ? KW + 1 : 0][l] = hp[s][l];
        }
        __syncthreads();
        const double ups_row = s_prod();
        put_red(0, p * ups_row);
        put_row(0, ups_row);
        sync(1, 1);
        const double ups = uni(tot[0]);
        if (!(ups > 0.0) || __builtin_isinf(ups)) {
          status = MPCPCG_BREAKDOWN;
          break;
        }
        const double alpha = eta / ups;
        lam = __builtin_fma(alpha, p, lam);
        res = __builtin_fma(-alpha, ups_row, res);
        for (int t = tid; t < 2 * NX; t += NT) {
          const int s = t / NX, l = t % NX;
          hr[s][l] = __builtin_fma(-alpha, hin[0][s][l], hr[s][l]);
          vf[s ? KW + 1 : 0][l] = (float)hr[s][l];
        }
        // r~ = Phi^-1 r, eta' = r^T r~
        put_vf((float)res);
        __syncthreads();
        rt = p_prod();
        put_red(0, res * (double)rt);
        put_row(0, (double)rt);
        sync(1, 1);
        eta_new = uni(tot[0]);
        if (!(eta_new == eta_new) || __builtin_isinf(eta_new)) {
          status = MPCPCG_BREAKDOWN;
          break;
        }
        if (eta_new < tau) {
          status = MPCPCG_OK;
          break;
        }
        const double beta = eta_new / eta;
        p = __builtin_fma(beta, p, (double)rt);
        for (int t = tid; t < 2 * NX; t += NT) {
          const int s = t / NX, l = t % NX;
          hp[s][l] = __builtin_fma(beta, hp[s][l], hin[0][s][l]);
        }
        eta = eta_new;
      }
      if (it > max_iter) it = max_iter;
    }
    if (aborted) status = MPCPCG_TIMEOUT;
    if (h == 0 && mine) a.lamw[kb * NX + r] = lam;
    if (tid == 0 && part == 0)
      put_stats(a.stats + pd.id, it, status,
                eta_ref > 0.0 ? (float)__builtin_sqrt(eta_new > 0.0 ? eta_new / eta_ref : 0.0) : 0.0f);

    // ---- gang teardown: the last part out zeroes the gang's tagged words
    if (multi) {
      __syncthreads();
      if (tid == 0) {
        // a relaxed count after the barrier, which waited for every wave's stores (part 0's
        // stats, the abort flag): no L2 write-back at every task's end
        __builtin_amdgcn_s_waitcnt(0);
        const int d = __hip_atomic_fetch_add(&gang->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sh_task = d == G - 1;
      }
      __syncthreads();
      if (uni(sh_task)) {
        constexpr int kWords = sizeof(WTag) / sizeof(uint64_t);
        for (int i = tid; i < G * kWords; i += NT) {
          uint64_t *w = reinterpret_cast<uint64_t *>(&tws[pd.t0 + i / kWords]) + i % kWords;
          __hip_atomic_store(w, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid == 0) {
          const int ab = __hip_atomic_load(&gang->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (ab) __hip_atomic_store(reinterpret_cast<int *>(a.stats + pd.id) + 1, (int)MPCPCG_TIMEOUT,
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&gang->abort, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&gang->done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }

  // ---- launch teardown: the last workgroup out resets the queue
  __syncthreads();
  if (tid == 0) {
    __builtin_amdgcn_s_waitcnt(0);
    const int d = __hip_atomic_fetch_add(&g.queue[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (d == (int)gridDim.x - 1) {
      // a list whose XCD ran no workgroup of this launch (a placement the host did not
      // expect) leaves its problems unsolved: they report TIMEOUT instead of stale stats
      if (g.xoff) {
        for (int x = 0; x < 8; ++x) {
          const int popped = __hip_atomic_load(&g.queue[4 + x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          for (int t = g.xoff[x] + max(popped, 0); t < g.xoff[x + 1]; ++t) {
            const Task tk = g.tasks[t];
            if (tk.part == 0) put_stats(a.stats + g.probs[tk.prob].id, 0, MPCPCG_TIMEOUT, 0.0f);
          }
        }
      }
      __hip_atomic_store(&g.queue[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int x = 0; x < 8; ++x) __hip_atomic_store(&g.queue[4 + x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&g.queue[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&g.queue[1], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace wide
}  // namespace mpc
