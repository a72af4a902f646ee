/*
 * nx_micro.h -- C ABI of libnx_micro, the VALU issue-rate microbenchmarks behind the
 * roofline of libnx's sums on gfx950 (MI355X).  Measurement support, not part of the
 * scattering library.
 *
 * The sums of the direct scattering amplitude (Favre-Nicolin et al., J. Appl. Cryst.
 * 2010, Section 2.1 Eq. 2) are bound by vector-ALU issue; the paper counts their work as
 * 8 flop per atom-point pair (Section 2.2, Eq. 3).  Each kernel here repeats the
 * per-pair instruction sequence of one sum on register operands only (no memory
 * traffic), in up to three shapes: `wide` = 0 runs 4 (FP64-phase mixes) or 8 (FP32
 * mixes) independent pairs per lane at 8 waves per SIMD, `wide` = 1 twice as many at 4
 * waves per SIMD, and `wide` = 2 (FP64-phase mixes only) the sums' own shape, 1 point
 * (forward) or 2 atoms (adjoint) per lane against 16 wave-uniform stream items per
 * iteration; the mixes of the sums over grid rows (Eq. 2 over a regular grid, the phase
 * formed from the point's index along the row) exist in that shape only.  The best rate, in pairs per second, is the issue ceiling of that instruction
 * mix on the chip under load.
 *
 * nxm_run queues one launch of n_blocks work-groups of nxm_threads_per_block() lanes,
 * each lane computing iters * nxm_pairs_per_lane_iter(mix, wide) pairs, on `stream` (a
 * hipStream_t, NULL = null stream).  `out` is a DEVICE array of n_blocks *
 * nxm_threads_per_block() floats (overwritten with meaningless values).  Returns 0, -1 for
 * invalid sizes, a NULL out, `wide` outside 0..2 or a shape the mix does not have (then
 * nxm_pairs_per_lane_iter returns 0), -2 for an unknown mix, -4 if the launch failed.  The call
 * does not synchronise; time it with events on the same stream.
 */
#ifndef NX_MICRO_H
#define NX_MICRO_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NXM_FWD_PH64_CF = 0,   /* forward, FP64 phase, complex f: 3 fma64, cvt_i32, mul, cos, sin, 2 fma */
  NXM_FWD_PH64_F1 = 1,   /* forward, FP64 phase, f = 1: the same with 2 adds */
  NXM_BWD_PH64_CF = 2,   /* adjoint, FP64 phase, complex f: 3 fma64, add64, cvt_i32, mul, sin, 3 fma */
  NXM_BWD_PH64_F1 = 3,   /* adjoint, FP64 phase, f = 1: without the add64 */
  NXM_FWD_F32_CF = 4,    /* forward, FP32: 3 fma, fract, cos, sin, 4 fma */
  NXM_FWD_F32_F1 = 5,    /* forward, FP32, f = 1: 3 fma, fract, cos, sin, 2 add */
  NXM_BWD_F32_CF = 6,    /* adjoint, FP32, complex f: 3 fma, fract, cos, sin, 6 (w, v), 3 fma */
  NXM_BWD_F32_F1 = 7,    /* adjoint, FP32, f = 1: 3 fma, fract, cos, sin, 2 (Im w), 3 fma */
  NXM_OP_FMA_F32 = 8,    /* one instruction kind alone: FP32 fma, a scalar operand (v_fma_f32) */
  NXM_OP_FMA_F64 = 9,    /*   FP64 fma, a scalar operand (v_fma_f64) */
  NXM_OP_SIN_F32 = 10,   /*   v_sin_f32 */
  NXM_OP_FMAC_F32 = 11,  /*   FP32 fma into its destination, vector operands (v_fmac_f32_e32) */
  NXM_OP_FMAC_F64 = 12,  /*   FP64 fma into its destination, vector operands (v_fmac_f64_e32) */
  NXM_OP_ADD_F64 = 13,   /*   v_add_f64 */
  NXM_OP_RNDNE_F64 = 14, /*   v_rndne_f64 (round to nearest even integer) */
  NXM_OP_FRACT_F64 = 15, /*   v_fract_f64 */
  NXM_OP_CVT_F32_I32 = 16, /* v_cvt_f32_i32 */
  NXM_OP_COS_F32 = 17,   /*   v_cos_f32 */
  NXM_OP_MUL_F32 = 18,   /*   v_mul_f32_e32 */
  NXM_OP_FMA_F32_V = 19, /*   FP32 fma, vector operands, three-operand encoding (v_fma_f32) */
  NXM_OP_ADD_F32 = 20,   /*   v_add_f32_e32 */
  NXM_FWD_GRID_CF = 21,  /* forward over grid rows, 2 x 2 x 2 points: per atom 1 fma64, cvt_i32, mul, cos,
                            sin, 7 steps (4 fma each), 8 x 2 fma */
  NXM_FWD_GRID_F1 = 22,  /* the same for f = 1, 8 x 2 adds */
  NXM_BWD_GRID_CF = 23,  /* adjoint over grid rows: 1 fma64, add64, cvt_i32, mul, sin, 3 fma */
  NXM_BWD_GRID_F1 = 24   /* adjoint over grid rows, f = 1: the same sequence */
} nxm_mix;

/* Work items per lane and iteration: atom-point pairs for the mixes, instructions for the
 * single-instruction kinds. */
int nxm_pairs_per_lane_iter(int mix, int wide);
int nxm_threads_per_block(void);
/* Rate of the real-time counter the kernels read (kHz), or -4. */
int nxm_wallclock_khz(void);
/* `clk`: DEVICE array of 2 * n_blocks counters or NULL; thread 0 of work-group b stores the
 * shader-clock cycles (s_memtime) and real-time ticks (s_memrealtime) between its start and
 * its end in clk[2 b] and clk[2 b + 1], so that cycles / ticks * nxm_wallclock_khz() is the
 * clock under this load. */
int nxm_run(int mix, int wide, int n_blocks, int iters, float* out, unsigned long long* clk,
            void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NX_MICRO_H */
