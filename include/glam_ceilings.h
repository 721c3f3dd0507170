/* Measured ceilings of the GPU the library runs on, for roofline fractions.  A
 * measuring tool next to the render library (it is built into its own shared library,
 * libglam_ceilings.so): each call allocates its own device buffers, launches a
 * microbenchmark kernel twice on the default stream (warm-up, then one timed launch
 * between HIP events), synchronises, frees, and returns the rate, or a negative value
 * when a HIP call failed.  Run it with no other work on the device.
 *
 * The work counted per kernel is what the kernel's loop does by construction:
 *   glamc_fma_tflops       FP32 fused multiply-adds (v_fma_f32, 2 FLOP each), eight
 *                          independent chains per lane: TFLOP/s
 *   glamc_exp_trate        v_exp_f32 (the transcendental behind exp and exp2), eight
 *                          independent chains per lane: results per second / 1e12
 *   glamc_lds_read_tbs     16-byte LDS reads without bank conflicts: TB/s
 *   glamc_hbm_copy_tbs     a device copy of `bytes` (bytes read + written): TB/s
 *   glamc_hbm_triad_tbs    a = b + s c over `bytes` per array (3 streams): TB/s
 *   glamc_mfma_fp32_tflops v_mfma_f32_16x16x4f32, four independent accumulators per
 *                          wave (2 x 16 x 16 x 4 FLOP each): TFLOP/s
 *   glamc_atomic_grate     device-scope FP32 atomic adds with unused results: on
 *                          distinct addresses (contended = 0) or all on one word
 *                          (contended = 1): G atomics per second
 */
#ifndef GLAM_CEILINGS_H
#define GLAM_CEILINGS_H

#ifdef __cplusplus
extern "C" {
#endif

double glamc_fma_tflops(void);
double glamc_exp_trate(void);
double glamc_lds_read_tbs(void);
double glamc_hbm_copy_tbs(long long bytes);
double glamc_hbm_triad_tbs(long long bytes);
double glamc_mfma_fp32_tflops(void);
double glamc_atomic_grate(int contended);

#ifdef __cplusplus
}
#endif
#endif
