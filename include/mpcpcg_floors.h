/*
 * libmpcpcg_floors -- measured floors of the device for the rooflines of libmpcpcg's
 * kernels (used by the benchmark; not part of the solve path).
 *
 * The solver's PCG meets at two inner products per iteration (Algorithm 1; the paper's
 * GPU version, Section IV-B and Algorithm 2, synchronises the whole grid at each), and its
 * batched form re-reads Phi^-1 from LDS every iteration.  These probes measure the costs
 * that bound it on this device:
 *   floors_launch    microseconds per launch of an empty kernel, `launches` back to back
 *                    on the null stream;
 *   floors_barrier   microseconds per barrier round of `gangs` independent gangs of `parts`
 *                    workgroups (2..64) using the solver's protocol (each part publishes a
 *                    tagged 16-byte word, then polls its partners'; sleep != 0 waits ~1,500
 *                    cycles before the first poll as the solver's device-scope barrier
 *                    does; pin = 1 runs each gang on one XCD and needs gangs % 8 == 0;
 *                    l2 = 0 exchanges device-scope words, l2 = 1 (needs pin = 1) exchanges
 *                    through the XCD's L2 as the solver does for gangs on one XCD);
 *                    gangs * parts must not exceed 8 per compute unit.  *us_per_round is
 *                    negative if a wait gave up (2 s);
 *   floors_lds_read  aggregate LDS read bandwidth in bytes/s over `blocks` workgroups of
 *                    256 threads, each reading `iters` conflict-free 16-byte words per thread;
 *   floors_read      aggregate read bandwidth in bytes/s of `blocks` workgroups each reading a
 *                    buffer of buffer_bytes (a multiple of 16384) `passes` times: a
 *                    buffer that fits in the L2 of each XCD measures L2, one beyond the L2s
 *                    but within the last-level cache measures that, a large one HBM.
 * Each call allocates what it needs, runs on the current device, synchronises it, and
 * returns 0, -1 (a HIP call failed) or -2 (bad argument).
 */
#ifndef MPCPCG_FLOORS_H
#define MPCPCG_FLOORS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int floors_launch(int launches, double *us_per_launch);
int floors_barrier(int gangs, int parts, int rounds, int sleep, int pin, int l2, double *us_per_round);
int floors_lds_read(int blocks, int iters, double *bytes_per_s);
int floors_read(int64_t buffer_bytes, int blocks, int passes, double *bytes_per_s);

#ifdef __cplusplus
}
#endif
#endif /* MPCPCG_FLOORS_H */
