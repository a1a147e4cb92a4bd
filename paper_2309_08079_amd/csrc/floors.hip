// Measured floors of the device for the solver's rooflines (libmpcpcg_floors.so, used by
// bench.py; not part of the solve path):
//   floors_launch      latency of back-to-back empty kernel launches on one stream;
//   floors_barrier     one cross-workgroup barrier round with the solver's protocol (the
//                      sync points of PCG: every part publishes a tagged 16-byte word and
//                      polls its partners' words), isolated or with many gangs at once, gangs
//                      spread over the XCDs or each on one XCD, through device-scope words or
//                      (gangs on one XCD) through that XCD's L2;
//   floors_lds_read    aggregate LDS read bandwidth (ds_read_b128, conflict free);
//   floors_read        aggregate read bandwidth of a buffer of a given size, re-read by
//                      every workgroup (sizes that stay in L2, in the last-level cache, or
//                      that stream from HBM).
// Every wait is bounded; a probe whose wait gives up reports a negative time.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mpcpcg_floors.h"
#include "pcg_kernel.h"

namespace {

__global__ void empty_kernel() {}

struct BarrierArgs {
  void *words;     // [gangs][2][parts] 16-byte pairs, zero before the launch
  int parts;       // workgroups per gang (<= 64)
  int rounds;
  int sleep;       // s_sleep units (64 cycles) before the first poll of a round
  int pin;         // 1: the parts of gang g run on XCD g % 8
  int64_t spin;    // wall-clock ticks before a wait gives up
  int64_t *ticks;  // [gangs] wall-clock ticks of all rounds (part 0), -1 if a wait gave up
};

template <int L2X>
__global__ void __launch_bounds__(64) barrier_probe(BarrierArgs a) {
  const int b = blockIdx.x, lane = threadIdx.x;
  int gang, part;
  if (a.pin) {  // workgroup b runs on XCD b % 8
    gang = (b / (8 * a.parts)) * 8 + (b & 7);
    part = (b >> 3) % a.parts;
  } else {
    gang = b / a.parts;
    part = b % a.parts;
  }
  const __amdgpu_buffer_rsrc_t rs = mpc::ws_rsrc(a.words);
  auto off = [&](int par, int p) { return (uint32_t)((((int64_t)gang * 2 + par) * a.parts + p) * 16); };
  bool gave_up = false;
  const long long t0 = wall_clock64();
  for (int r = 0; r < a.rounds && !gave_up; ++r) {
    const int par = r & 1;
    const uint32_t tag = (uint32_t)r + 1u;
    if (lane == 0) {
      if (L2X)
        mpc::store_pair_l2(rs, off(par, part), tag, (double)r);
      else
        mpc::store_pair(rs, off(par, part), tag, (double)r);
    }
    if (a.sleep > 0) __builtin_amdgcn_s_sleep(24);
    const bool mine = lane < a.parts;
    const long long ts = wall_clock64();
    int polls = 0;
    while (true) {
      bool ok = true;
      if (mine) ok = mpc::pair_has(L2X ? mpc::load_pair_l2(rs, off(par, lane)) : mpc::load_pair(rs, off(par, lane)), tag);
      if (__ballot(ok) == ~0ull) break;
      __builtin_amdgcn_s_sleep(1);
      if ((++polls & 63) == 0 && wall_clock64() - ts > a.spin) {
        gave_up = true;
        break;
      }
    }
  }
  const long long t1 = wall_clock64();
  if (part == 0 && lane == 0) a.ticks[gang] = gave_up ? -1 : (int64_t)(t1 - t0);
}

constexpr int kLdsFloats = 8192;  // 32 KB per workgroup

// `step` is a kernel argument (256): the compiler cannot see that the read addresses repeat
// and reuse earlier loads, so every iteration issues its reads.
__global__ void __launch_bounds__(256) lds_probe(int iters, int step, float *sink) {
  __shared__ float4 buf[kLdsFloats / 4];
  for (int i = threadIdx.x; i < kLdsFloats / 4; i += 256)
    buf[i] = make_float4((float)i, 1.0f, 2.0f, 3.0f);
  __syncthreads();
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  const int mask = kLdsFloats / 4 - 1;
  int idx = threadIdx.x;
  for (int i = 0; i < iters; ++i) {
    // consecutive lanes read consecutive 16-byte slots: no bank conflicts
    const float4 v = buf[idx & mask];
    idx += step;
    acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
  }
  const float s = acc.x + acc.y + acc.z + acc.w;
  if (s == -1.0f) sink[blockIdx.x] = s;  // never true; keeps the loads
}

__global__ void __launch_bounds__(256) read_probe(const float4 *buf, int64_t n4, int passes, float *sink) {
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  // each workgroup sweeps the whole buffer (4 independent loads in flight per thread),
  // starting at a different offset; n4 is a multiple of 1024
  const int64_t start = ((int64_t)blockIdx.x * 4096) % n4;
  for (int p = 0; p < passes; ++p)
    for (int64_t i = threadIdx.x; i < n4; i += 1024) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        int64_t j = start + i + u * 256;
        if (j >= n4) j -= n4;
        v[u] = buf[j];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc.x += v[u].x; acc.y += v[u].y; acc.z += v[u].z; acc.w += v[u].w;
      }
    }
  const float s = acc.x + acc.y + acc.z + acc.w;
  if (s == -1.0f) sink[blockIdx.x] = s;
}

int64_t clock_khz() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      khz <= 0)
    khz = 100000;
  return khz;
}

#define FCHK(call)                            \
  do {                                        \
    if ((call) != hipSuccess) return -1;      \
  } while (0)

}  // namespace

extern "C" {

int floors_launch(int launches, double *us_per_launch) {
  if (launches < 1 || !us_per_launch) return -2;
  hipEvent_t e0, e1;
  FCHK(hipEventCreate(&e0));
  FCHK(hipEventCreate(&e1));
  hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, 0);
  FCHK(hipDeviceSynchronize());
  FCHK(hipEventRecord(e0, 0));
  for (int i = 0; i < launches; ++i) hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, 0);
  FCHK(hipEventRecord(e1, 0));
  FCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  FCHK(hipEventElapsedTime(&ms, e0, e1));
  *us_per_launch = ms * 1e3 / launches;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return 0;
}

int floors_barrier(int gangs, int parts, int rounds, int sleep, int pin, int l2, double *us_per_round) {
  if (gangs < 1 || parts < 2 || parts > 64 || rounds < 1 || !us_per_round) return -2;
  if (pin && gangs % 8) return -2;
  if (l2 && !pin) return -2;  // the XCD-local exchange needs every gang on one XCD
  int dev = 0, cus = 0;
  FCHK(hipGetDevice(&dev));
  FCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if ((int64_t)gangs * parts > (int64_t)cus * 8) return -2;  // every part co-resident
  const size_t wbytes = (size_t)gangs * 2 * parts * 16;
  void *words = nullptr;
  int64_t *ticks = nullptr;
  FCHK(hipMalloc(&words, wbytes));
  FCHK(hipMalloc(&ticks, sizeof(int64_t) * gangs));
  FCHK(hipMemset(words, 0, wbytes));
  BarrierArgs a;
  a.words = words; a.parts = parts; a.rounds = rounds; a.sleep = sleep; a.pin = pin;
  a.spin = 2000 * clock_khz();  // 2 s
  a.ticks = ticks;
  if (l2)
    hipLaunchKernelGGL(barrier_probe<1>, dim3(gangs * parts), dim3(64), 0, 0, a);
  else
    hipLaunchKernelGGL(barrier_probe<0>, dim3(gangs * parts), dim3(64), 0, 0, a);
  FCHK(hipGetLastError());
  FCHK(hipDeviceSynchronize());
  int64_t *h = new int64_t[gangs];
  FCHK(hipMemcpy(h, ticks, sizeof(int64_t) * gangs, hipMemcpyDeviceToHost));
  double sum = 0.0;
  bool bad = false;
  for (int g = 0; g < gangs; ++g) {
    if (h[g] < 0) bad = true;
    sum += (double)h[g];
  }
  delete[] h;
  (void)hipFree(words);
  (void)hipFree(ticks);
  *us_per_round = bad ? -1.0 : sum / gangs / rounds / (clock_khz() / 1000.0);
  return 0;
}

int floors_lds_read(int blocks, int iters, double *bytes_per_s) {
  if (blocks < 1 || iters < 1 || !bytes_per_s) return -2;
  float *sink = nullptr;
  FCHK(hipMalloc(&sink, sizeof(float) * blocks));
  hipEvent_t e0, e1;
  FCHK(hipEventCreate(&e0));
  FCHK(hipEventCreate(&e1));
  hipLaunchKernelGGL(lds_probe, dim3(blocks), dim3(256), 0, 0, 16, 256, sink);
  FCHK(hipDeviceSynchronize());
  FCHK(hipEventRecord(e0, 0));
  hipLaunchKernelGGL(lds_probe, dim3(blocks), dim3(256), 0, 0, iters, 256, sink);
  FCHK(hipEventRecord(e1, 0));
  FCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  FCHK(hipEventElapsedTime(&ms, e0, e1));
  *bytes_per_s = (double)blocks * 256 * 16 * (double)iters / (ms * 1e-3);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  return 0;
}

int floors_read(int64_t buffer_bytes, int blocks, int passes, double *bytes_per_s) {
  if (buffer_bytes < 16384 || buffer_bytes % 16384 || blocks < 1 || passes < 1 || !bytes_per_s) return -2;
  void *buf = nullptr;
  float *sink = nullptr;
  FCHK(hipMalloc(&buf, (size_t)buffer_bytes));
  FCHK(hipMalloc(&sink, sizeof(float) * blocks));
  FCHK(hipMemset(buf, 0, (size_t)buffer_bytes));
  hipEvent_t e0, e1;
  FCHK(hipEventCreate(&e0));
  FCHK(hipEventCreate(&e1));
  const int64_t n4 = buffer_bytes / 16;
  hipLaunchKernelGGL(read_probe, dim3(blocks), dim3(256), 0, 0, (const float4 *)buf, n4, 1, sink);
  FCHK(hipDeviceSynchronize());
  FCHK(hipEventRecord(e0, 0));
  hipLaunchKernelGGL(read_probe, dim3(blocks), dim3(256), 0, 0, (const float4 *)buf, n4, passes, sink);
  FCHK(hipEventRecord(e1, 0));
  FCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  FCHK(hipEventElapsedTime(&ms, e0, e1));
  *bytes_per_s = (double)blocks * (double)buffer_bytes * passes / (ms * 1e-3);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  (void)hipFree(sink);
  return 0;
}

}  // extern "C"
