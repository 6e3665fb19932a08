/*
 * sgweno_measure.h -- measurement hooks of libsgweno that are not part of the
 * sparse-grid WENO5 method: they time the stage launches of a batch and
 * calibrate the VALU issue rates that price kernel issue floors.  Benchmarks
 * and tuners use them; solving a problem never needs them.  Same conventions
 * as sgweno.h (status codes, sgw_last_error, caller-owned device memory).
 */
#ifndef SGWENO_MEASURE_H
#define SGWENO_MEASURE_H

#include "sgweno.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Measurement hook, outside any graph (callers time it with events on the batch
 * stream).  stage 0..2: reps launches of that RK stage, one stage at a time,
 * over all of the batch's boxes; stage 0 writes only the first stage buffer, so
 * repeating it leaves u^n unchanged.  stage 3: reps times the stage launches of
 * one step as the step graph runs them (all three stages of the grids that are
 * one box in one launch, the other grids stage by stage); this advances u^n
 * without advancing t.  Either way the solves' wave-speed slots are disturbed,
 * so re-restrict before trusting later results. */
sgw_status sgw_batch_launch_stage(sgw_batch_t* batch, int32_t stage, int32_t reps);
/* Measurement hook for one solver, outside any graph (callers time it with events
 * on the solver's stream): reps repetitions of one part of RK stage `stage` (0..2)
 * of the solver's current step, as sgw_advance enqueues it.  part 0: the whole
 * stage (moment pass, field launch, plane launch, sweeps or boxes); part 1: the
 * plane launch of a 4D plan (directions 1 and 2); part 2 + k: the line sweep of
 * direction k + 1 alone (line-mode plans).  Call it after sgw_advance has taken at
 * least one step; it reopens the solve (the final time goes to infinity) so the
 * kernels do their work, and it leaves the solve's state meaningless: re-restrict
 * before trusting later results.  SGW_ERR_INVALID_ARG for a part the plan does
 * not have. */
sgw_status sgw_solver_launch_stage(sgw_solver_t* solver, int32_t stage, int32_t part, int32_t reps);
/* Measurement hook for the VALU issue rates that price kernel issue floors (not
 * part of the method): enqueues on hip_stream one launch of `blocks` workgroups
 * of 256 threads running long chains of independent instructions of one class,
 * op 0 FP32 FMA, 1 FP32 multiply, 2 FP32 add, 3 INT32 add + xor, 4 FP64 FMA.
 * out_dev (device) receives one value per thread: blocks * 256 * 8 bytes.
 * *instructions_per_simd receives the wave64 instructions of the class each SIMD
 * issues (host, written before return); the caller times the launch with events,
 * so cycles per instruction = seconds * clock / *instructions_per_simd.  Returns
 * without waiting for the device. */
sgw_status sgw_calibrate_valu(int32_t op, int32_t blocks, void* out_dev, void* hip_stream,
                              double* instructions_per_simd);

#ifdef __cplusplus
}
#endif
#endif /* SGWENO_MEASURE_H */
