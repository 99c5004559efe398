/*
 * bls_probes.h -- micro-benchmarks of gfx950 rates behind the search
 * kernel's design (libbls_probes.so; measurement tooling, not part of the
 * search ABI).  Each call runs one warm-up and one timed launch of `grid`
 * workgroups of 256 threads on the current device's default stream and
 * writes the timed launch's duration (HIP events) to *ms.  Returns 0, -1 for
 * bad arguments, or a hipError_t.
 */
#ifndef BLS_PROBES_H
#define BLS_PROBES_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BLS_PROBE_ADD_U64 = 0,   /* ds_add_u64 (the fold's exact bin words)    */
    BLS_PROBE_ADD_U32 = 1,   /* ds_add_u32                                  */
    BLS_PROBE_ADD_F32 = 2    /* ds_add_f32 (rounded, order-dependent sums)  */
};
enum {
    BLS_PROBE_FMA_F32 = 0,   /* v_fma_f32 with inline constant and register,
                                8 independent chains per lane               */
    BLS_PROBE_MUL_F64 = 1,   /* v_mul_f64, 8 chains                         */
    BLS_PROBE_MAD_U32 = 2,   /* 32-bit integer shift-and-add, 8 chains      */
    BLS_PROBE_ADD_F32V = 3   /* v_add_f32 of two registers, 8 chains        */
};

/* Every thread performs `iters` LDS atomics of `kind` at pseudo-random
 * addresses among `span` words (a power of two, <= 4096) of its workgroup's
 * histogram.  Atomics per second = grid * 256 * iters / (ms / 1e3). */
int bls_probe_lds_atomic(int kind, int span, int iters, int grid, double *ms);

/* Every thread performs `iters` 64-bit LDS reads; lane l of each 16-lane
 * group reads word l * lane_stride + (its 16-lane group mod 8) + iteration
 * mod 64 (lane_stride 1: consecutive words; the bank pattern of one LDS
 * clock).  Reads per second = grid * 256 * iters / (ms / 1e3). */
int bls_probe_lds_read(int lane_stride, int iters, int grid, double *ms);

/* Every thread runs 8 independent chains of `iters` VALU operations of
 * `kind`.  Wave64 instructions per second = grid * 4 * 8 * iters / (ms /
 * 1e3). */
int bls_probe_valu(int kind, int iters, int grid, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* BLS_PROBES_H */
