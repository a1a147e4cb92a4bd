// Lane-level building blocks for 16-lane "knot groups" on CDNA4 (gfx950).
//
// A knot group is one 16-lane DPP row of a wave64.  Lane i of the group owns row i of
// every nx x nx block of its knot (rows >= nx hold zeros), so a matrix is NX registers
// per lane and a vector is one register per lane.  Products broadcast a row of the
// right-hand operand from its owner lane with DPP row_newbcast, which never leaves the
// 16-lane row, so four knots per wave run without interfering.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "dpp_asm.h"

namespace mpc {

constexpr int kGroup = 16;          // lanes per knot group (one DPP row)
constexpr int kRowNewBcast = 0x150; // DPP row_newbcast:n  (broadcast lane n of each row)
constexpr int kRowShr = 0x110;      // DPP row_shr:n       (lane i <- lane i-n, zero fill)

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// value of v in lane K of this lane's 16-lane group
template <int K>
__device__ __forceinline__ double bc(double v) { return dpp_f64<kRowNewBcast + K>(v); }
template <int K>
__device__ __forceinline__ float bcf(float v) { return dpp_f32<kRowNewBcast + K>(v); }

// Sum over the 16 lanes of the group; the full sum lands in lane 15 (other lanes hold
// partial prefix sums).
__device__ __forceinline__ double group_sum_to_last(double v) {
  v += dpp_f64<kRowShr + 1>(v);
  v += dpp_f64<kRowShr + 2>(v);
  v += dpp_f64<kRowShr + 4>(v);
  v += dpp_f64<kRowShr + 8>(v);
  return v;
}

// group_sum_to_last of two values, their steps interleaved (each rounds as on its own).
__device__ __forceinline__ void group_sums2(double &a, double &b) {
  a += dpp_f64<kRowShr + 1>(a);
  b += dpp_f64<kRowShr + 1>(b);
  a += dpp_f64<kRowShr + 2>(a);
  b += dpp_f64<kRowShr + 2>(b);
  a += dpp_f64<kRowShr + 4>(a);
  b += dpp_f64<kRowShr + 4>(b);
  a += dpp_f64<kRowShr + 8>(a);
  b += dpp_f64<kRowShr + 8>(b);
}

// 64-bit DPP move with a row mask: lanes of rows outside ROWS get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64_rows(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
constexpr int kRowBcast15 = 0x142;  // DPP row_bcast:15 (lane 15 of a row to the next row)

// Two 32-lane sums at once: lanes 0..31 carry the terms of the first sum, lanes 32..63
// those of the second.  Each is g0 + g1 of its two 16-lane row sums (fixed shape); both
// results are uniform (read from lanes 31 and 63).  One reduction chain serves both sums.
__device__ __forceinline__ void half_sums(double v, double &s0, double &s1) {
  double g = group_sum_to_last(v);
  g += dpp_f64_rows<kRowBcast15, 0xA>(g);  // rows 1, 3: + lane 15 of rows 0, 2
  const uint64_t u = __builtin_bit_cast(uint64_t, g);
  const uint32_t lo0 = __builtin_amdgcn_readlane((uint32_t)u, 31);
  const uint32_t hi0 = __builtin_amdgcn_readlane((uint32_t)(u >> 32), 31);
  const uint32_t lo1 = __builtin_amdgcn_readlane((uint32_t)u, 63);
  const uint32_t hi1 = __builtin_amdgcn_readlane((uint32_t)(u >> 32), 63);
  s0 = __builtin_bit_cast(double, ((uint64_t)hi0 << 32) | lo0);
  s1 = __builtin_bit_cast(double, ((uint64_t)hi1 << 32) | lo1);
}

// Sum over lanes 0..31 (the first two 16-lane rows), g0 + g1 of the row sums: what
// wave_sum gives when lanes 32..63 hold zeros, at half the cost.  Uniform result.
__device__ __forceinline__ double sum_rows01(double v) {
  const double g = group_sum_to_last(v);
  const uint64_t u = __builtin_bit_cast(uint64_t, g);
  const uint32_t lo0 = __builtin_amdgcn_readlane((uint32_t)u, 15), hi0 = __builtin_amdgcn_readlane((uint32_t)(u >> 32), 15);
  const uint32_t lo1 = __builtin_amdgcn_readlane((uint32_t)u, 31), hi1 = __builtin_amdgcn_readlane((uint32_t)(u >> 32), 31);
  return __builtin_bit_cast(double, ((uint64_t)hi0 << 32) | lo0) + __builtin_bit_cast(double, ((uint64_t)hi1 << 32) | lo1);
}

// Sum over the 64 lanes of the wave with a fixed reduction shape (identical rounding in
// every wave that calls it); the result is returned in every lane.
__device__ __forceinline__ double wave_sum(double v) {
  const double g = group_sum_to_last(v);
  const uint64_t u = __builtin_bit_cast(uint64_t, g);
  const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t l2 = __builtin_amdgcn_readlane(lo, 16 * q + 15);
    const uint32_t h2 = __builtin_amdgcn_readlane(hi, 16 * q + 15);
    s += __builtin_bit_cast(double, ((uint64_t)h2 << 32) | l2);
  }
  return s;
}

// ---- hot-loop matvec rows with the broadcast fused into the FMA -----------------------
// acc += sum_{j<NX} m[j] * x(lane j).  One asm block per 14-term row keeps the DPP
// broadcast folded into v_fmac (the compiler does not fuse row_newbcast by itself).  The
// leading s_nop covers the VALU-write -> DPP-read hazard on x, which the compiler cannot
// see through inline asm; x is not written inside the block.
// Operand %0 is the accumulator, %1 the broadcast source and %2..%15 the matrix
// entries; term K multiplies matrix operand K+2 by x broadcast from lane K.
#define MPC_F64_T(K, OP) "v_fmac_f64_dpp %0, %1, %" #OP " row_newbcast:" #K " row_mask:0xf bank_mask:0xf\n"
#define MPC_F32_T(K, OP) "v_fmac_f32_dpp %0, %1, %" #OP " row_newbcast:" #K " row_mask:0xf bank_mask:0xf\n"

__device__ __forceinline__ void row_fma14_f64(double &acc, double x, const double (&m)[14]) {
  asm volatile("s_nop 1\n" MPC_F64_T(0, 2) MPC_F64_T(1, 3) MPC_F64_T(2, 4) MPC_F64_T(3, 5)
                   MPC_F64_T(4, 6) MPC_F64_T(5, 7) MPC_F64_T(6, 8) MPC_F64_T(7, 9)
                       MPC_F64_T(8, 10) MPC_F64_T(9, 11) MPC_F64_T(10, 12) MPC_F64_T(11, 13)
                           MPC_F64_T(12, 14) MPC_F64_T(13, 15)
               : "+&v"(acc)
               : "v"(x), "v"(m[0]), "v"(m[1]), "v"(m[2]), "v"(m[3]), "v"(m[4]), "v"(m[5]),
                 "v"(m[6]), "v"(m[7]), "v"(m[8]), "v"(m[9]), "v"(m[10]), "v"(m[11]),
                 "v"(m[12]), "v"(m[13]));
}

__device__ __forceinline__ void row_fma14_f32(float &acc, float x, const float (&m)[14]) {
  asm volatile("s_nop 1\n" MPC_F32_T(0, 2) MPC_F32_T(1, 3) MPC_F32_T(2, 4) MPC_F32_T(3, 5)
                   MPC_F32_T(4, 6) MPC_F32_T(5, 7) MPC_F32_T(6, 8) MPC_F32_T(7, 9)
                       MPC_F32_T(8, 10) MPC_F32_T(9, 11) MPC_F32_T(10, 12) MPC_F32_T(11, 13)
                           MPC_F32_T(12, 14) MPC_F32_T(13, 15)
               : "+&v"(acc)
               : "v"(x), "v"(m[0]), "v"(m[1]), "v"(m[2]), "v"(m[3]), "v"(m[4]), "v"(m[5]),
                 "v"(m[6]), "v"(m[7]), "v"(m[8]), "v"(m[9]), "v"(m[10]), "v"(m[11]),
                 "v"(m[12]), "v"(m[13]));
}

// ---- small dense algebra on row-distributed matrices ---------------------------------
// All products go through the fused blocks of dpp_asm.h.  Sizes are 14 (state) or
// 7 (control) for the Kuka-shaped problems this library is built for.

template <int n> struct DAsm;
template <> struct DAsm<14> {
  template <int K, int LC, int LY> static __device__ __forceinline__ void axpy(double (&C)[LC], const double (&Y)[LY], double x) { dasm::axpy14<K>(C, Y, x); }
  template <int K, int LY, int LX> static __device__ __forceinline__ void dotk(double &acc, const double (&Y)[LY], const double (&X)[LX]) { dasm::dotk14<K>(acc, Y, X); }
  template <int LM> static __device__ __forceinline__ void rowdot(double &acc, double x, const double (&M)[LM]) { dasm::rowdot14(acc, x, M); }
  template <int LC> static __device__ __forceinline__ void outer(double (&C)[LC], double s, double x) { dasm::outer14(C, s, x); }
};
template <> struct DAsm<7> {
  template <int K, int LC, int LY> static __device__ __forceinline__ void axpy(double (&C)[LC], const double (&Y)[LY], double x) { dasm::axpy7<K>(C, Y, x); }
  template <int K, int LY, int LX> static __device__ __forceinline__ void dotk(double &acc, const double (&Y)[LY], const double (&X)[LX]) { dasm::dotk7<K>(acc, Y, X); }
  template <int LM> static __device__ __forceinline__ void rowdot(double &acc, double x, const double (&M)[LM]) { dasm::rowdot7(acc, x, M); }
  template <int LC> static __device__ __forceinline__ void outer(double (&C)[LC], double s, double x) { dasm::outer7(C, s, x); }
};

// sum_{k<K} m[k] * x(lane k)  (row of a matrix times a lane-distributed vector)
template <int K, int L>
__device__ __forceinline__ double row_dot(const double (&m)[L], double x) {
  double acc = 0.0;
  DAsm<K>::rowdot(acc, x, m);
  return acc;
}

// C = X Y : C[j] = sum_{m<M} X[m] Y(lane m)[j], j < J   (Y's rows owned by lanes m)
template <int M, int J, int LX, int LY, int LC>
__device__ __forceinline__ void mm_nn(const double (&X)[LX], const double (&Y)[LY],
                                      double (&C)[LC]) {
  static_assert(M <= LX && J <= LY && J <= LC, "shapes");
#pragma unroll
  for (int j = 0; j < J; ++j) C[j] = 0.0;
  static_for<0, M>([&](auto mm) {
    constexpr int K = decltype(mm)::value;
    DAsm<J>::template axpy<K>(C, Y, X[K]);
  });
}

// C = X Y^T : C[j] = sum_{m<M} X[m] Y(lane j)[m], j < J   (Y's rows owned by lanes j)
template <int M, int J, int LX, int LY, int LC>
__device__ __forceinline__ void mm_nt(const double (&X)[LX], const double (&Y)[LY],
                                      double (&C)[LC]) {
  static_assert(M <= LX && M <= LY && J <= LC, "shapes");
  static_for<0, J>([&](auto jj) {
    constexpr int K = decltype(jj)::value;
    double s = 0.0;
    DAsm<M>::template dotk<K>(s, Y, X);
    C[K] = s;
  });
}

// C[k] = s(lane k) * x for k < n  (a broadcast vector scaled by a lane value)
template <int n, int LC>
__device__ __forceinline__ void outer_row(double (&C)[LC], double s, double x) {
#pragma unroll
  for (int k = 0; k < n; ++k) C[k] = 0.0;
  DAsm<n>::outer(C, s, x);
}

// In-place Gauss-Jordan inverse of an n x n symmetric positive definite matrix whose row
// `lane` is a[0..n-1] (rows >= n must be zero and stay zero).  No pivoting is needed for
// SPD matrices: every pivot is a positive Schur complement.  Step k: the pivot row is
// scaled by d = 1/a_kk, every other row i loses (a_ik d) times the pivot row, and column
// k becomes (d for the pivot row, -a_ik d otherwise).  Written as t = s*a + c*bc_k(a)
// with (s, c) = (0, d) on the pivot lane and (1, -a_ik d) elsewhere.
// `positive` (optional) ends false when a pivot is not > 0, i.e. when the matrix is not
// positive definite (every pivot of an SPD matrix is positive).
template <int n, int L>
__device__ __forceinline__ void gj_inverse(double (&a)[L], int lane, bool *positive = nullptr) {
  static_for<0, n>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    const double piv = bc<k>(a[k]);
    if (positive) *positive = *positive && (piv > 0.0);
    // reciprocal of the pivot: hardware estimate + one Newton step (full FP64 accuracy
    // without the division's scaling and fix-up sequence)
    double d = __builtin_amdgcn_rcp(piv);
    d = __builtin_fma(d, __builtin_fma(-piv, d, 1.0), d);
    const bool me = (lane == k);
    const double f = a[k] * d;
    const double sc = me ? 0.0 : 1.0;
    const double c = me ? d : -f;
    double t[n];
#pragma unroll
    for (int j = 0; j < n; ++j) t[j] = a[j] * sc;
    DAsm<n>::template axpy<k>(t, a, c);
#pragma unroll
    for (int j = 0; j < n; ++j) a[j] = (j == k) ? (me ? d : -f) : t[j];
  });
}

}  // namespace mpc
