/*
 * sq_probe.h -- measured hardware peaks for the rooflines of the SQ kernels
 * (part of libsq_mi355x.so).  Not an operation of the paper: the SQ
 * recurrence kernels (Sec. IV of arXiv 2006.03697) are bound by the LDS
 * reads of their stencil neighbours and by the vector ALU, and their
 * achieved LDS bandwidth is reported against the peak this probe measures.
 */
#ifndef SQ_PROBE_H
#define SQ_PROBE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Conflict-free LDS read bandwidth of the current device with ds_read of
 * bytes_per_lane = 4, 8 or 16 bytes: 8 workgroups of 256 threads per CU,
 * each lane reading 8 x 4096 times, timed with HIP events on hip_stream
 * (hipStream_t, NULL for the default stream) after one warm-up launch.
 * tb_per_s: whole-device TB/s (required); bytes_per_clk_per_cu: the same
 * per CU per clock at the device's peak shader clock (nullable).
 * Allocates and frees a 4-byte device word.  Returns 0 on success, 1 for a
 * bad argument, 2 if the allocation failed, 3 on a HIP runtime error. */
int sq_probe_lds(int bytes_per_lane, void* hip_stream, double* tb_per_s, double* bytes_per_clk_per_cu);

#ifdef __cplusplus
}
#endif

#endif /* SQ_PROBE_H */
