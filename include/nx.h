/*
 * nx.h -- C ABI of libnx, the gfx950 (MI355X) direct scattering-sum library.
 *
 * The library evaluates the kinematic scattering amplitude of an atomistic model
 * (Favre-Nicolin, Coraux, Richard & Renevier, "Fast computing of scattering maps of
 * nanostructures using graphical processing units", J. Appl. Cryst. 2010, Section
 * 2.1, Eq. 2):
 *
 *     A(S_k) = sum_j f_j exp(2 i pi S_k . r_j)
 *
 * over every atom j and every reciprocal-space point k, the adjoint of that sum with
 * respect to the atom positions and the factors (for fitting displacement fields,
 * occupancies or compositions to measured intensities), and the species-factorised
 * form of Section 4.2.
 *
 * Units and layout (all arrays flat and row-major; the order of atoms and of points
 * is irrelevant, as Section 3 of the paper notes for its own inputs):
 *   - r_j in lattice (fractional) units, S_k in reciprocal-lattice units, so S.r is in
 *     cycles (Section 4.2 converts orthonormal coordinates to fractional ones);
 *   - xyz:      n_atoms  x 3 values (x, y, z);
 *   - f:        n_atoms complex values stored as (re, im) pairs, or NULL for f_j = 1
 *               (the unit-occupancy sum of Section 3); occupancy and species
 *               factors are folded into f_j by the caller (Section 4.2 factors the
 *               S-dependent atomic factor out of the sum);
 *   - S:        n_points x 3 values (h, k, l);
 *   - A, G:     n_points complex values stored as (re, im) pairs;
 *   - grad_xyz: n_atoms  x 3 values.
 *
 * Ownership and execution: every pointer except those of nx_workspace_bytes and
 * nx_last_error is a DEVICE pointer owned by the caller.  The library never
 * allocates, frees, copies to or from the host, or synchronises: all work is queued
 * on `stream` (a hipStream_t; NULL = the null stream) and the call returns once it
 * is queued.  Outputs must not alias inputs.  The workspace `ws` is caller-owned
 * device memory of at least nx_workspace_bytes(...) bytes, used for the packed atom
 * or point records and the split/chunk partial sums; its contents on entry are
 * ignored and it must not be used by other work until the queued calls finish.
 * Calls that share a workspace must be ordered on one stream.
 *
 * Errors: every entry point validates its arguments on the host before any HIP call
 * and returns a negative nx_status on failure (nothing is queued then); the text of
 * the last error of the calling thread is available from nx_last_error().  Faults
 * during kernel execution surface at the caller's next synchronisation.  Non-finite
 * inputs propagate to the outputs.
 *
 * Results are bitwise reproducible for a fixed mode, input and size: partial sums
 * are combined in a fixed order and no atomics are used.
 */
#ifndef NX_H
#define NX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NX_OK = 0,
  NX_ERR_ARG = -1,        /* negative count, count too large, NULL pointer with count > 0,
                             misaligned complex array, or an invalid species partition */
  NX_ERR_MODE = -2,       /* unknown mode or op */
  NX_ERR_WORKSPACE = -3,  /* workspace missing or smaller than nx_workspace_bytes() */
  NX_ERR_DEVICE = -4      /* a HIP call failed (message in nx_last_error) */
} nx_status;

/* Precision modes of the single-precision entry points.
 *   NX_F32      the paper's own arithmetic (Section 2.2-2.3): phase S.r formed and
 *               reduced modulo one cycle in FP32, FP32 sin/cos, plain FP32 sums.
 *               Its error grows with |S.r| and with the number of atoms
 *               (the single-precision discussion of Section 2.3).
 *   NX_F32_PH64 the phase S.r is formed and reduced modulo one cycle in FP64 (exact for
 *               FP32 inputs up to the final rounding), sin/cos and the multiply-adds
 *               run in FP32, and the sums are compensated (FP32 group partial sums
 *               folded into a two-word FP32 accumulator by Kahan's compensated
 *               addition).  FP64 is used in the phase reduction only.  A complex f_j
 *               enters in polar form, its angle added to the FP64 phase.  In the
 *               forward every compensated group also carries a pseudo-random eighth
 *               turn, added to its phases and undone when the group is folded in, so
 *               that the periodic error of the hardware sin/cos does not add up
 *               coherently over lattice sites.  */
typedef enum { NX_F32 = 0, NX_F32_PH64 = 1 } nx_mode;

/* Operation selector for nx_workspace_bytes. */
typedef enum {
  NX_OP_FWD = 0,          /* nx_scatter_fwd                                  */
  NX_OP_BWD = 1,          /* nx_scatter_bwd, nx_scatter_bwd_ex without grad_f */
  NX_OP_FWD_F64 = 2,      /* nx_scatter_fwd_f64                              */
  NX_OP_BWD_F64 = 3,      /* nx_scatter_bwd_f64                              */
  NX_OP_LOSS = 4,         /* nx_loss_grad                                    */
  NX_OP_BWD_GF = 5,       /* nx_scatter_bwd_ex with grad_f                   */
  NX_OP_BWD_GF_F64 = 6,   /* nx_scatter_bwd_ex_f64 with grad_f               */
  NX_OP_FIT = 7           /* nx_fit_step                                     */
} nx_op;

/* Most species accepted by the species-factorised entry points. */
#define NX_MAX_SPECIES 16

/* Largest n_atoms / n_points accepted by any entry point. */
#define NX_MAX_COUNT ((int64_t)1 << 30)

/* Library ABI version (major * 100 + minor). */
int nx_version(void);

/* Bytes of device workspace the call (op, mode, n_atoms, n_points) needs; 0 when it
 * needs none.  `f_is_null` must match the f argument of the later call (1 when f
 * will be NULL).  `mode` is ignored for the FP64 and loss ops.  Returns 0 and sets
 * the last error on invalid arguments. */
size_t nx_workspace_bytes(int64_t n_atoms, int64_t n_points, int mode, int op, int f_is_null);

/* Forward sum, Section 2.1 Eq. 2:  A_k = sum_j f_j exp(2 i pi S_k . r_j).
 *   xyz  float[n_atoms*3], f float[n_atoms*2] or NULL, S float[n_points*3],
 *   A    float[n_points*2] (complex64), overwritten.
 * n_atoms == 0 writes A = 0; n_points == 0 queues nothing. */
int nx_scatter_fwd(const float* xyz, const float* f, int64_t n_atoms,
                   const float* S, int64_t n_points, float* A,
                   int mode, void* ws, size_t ws_bytes, void* stream);

/* Bytes of the static device scratch of nx_scatter_fwd_noalloc (per GPU). */
#define NX_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* Forward sum without allocation, for callers that cannot allocate device memory or
 * pass a workspace (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): nx_scatter_fwd with the same arguments but no workspace.  Its
 * workspace is a static device array of NX_NOALLOC_SCRATCH_BYTES (128 MiB) that every
 * GPU the library runs on holds from the library's load until the process ends; the call
 * itself allocates nothing.  The work is queued on `stream`, which must belong to the
 * current device (the scratch used is the current device's).
 * The launch plan is nx_scatter_fwd's, with fewer stream slices when its workspace would
 * not fit the scratch: the result then differs from nx_scatter_fwd's only by rounding
 * (the same tolerance), and is bitwise equal when the plan is the same.  Sizes that do not
 * fit even with one slice (about n_atoms * 48 bytes of atom records, plus n_points * 16
 * bytes when the atoms are cut into several launches) return NX_ERR_WORKSPACE before any
 * HIP call.  Nothing in the scratch has to start at zero (each call writes what it reads
 * back).  Every call on one GPU shares that GPU's scratch and leaves its contents behind:
 * calls that overlap on one GPU (on different streams or threads) race and give wrong
 * results; order them on one stream. */
int nx_scatter_fwd_noalloc(const float* xyz, const float* f, int64_t n_atoms,
                           const float* S, int64_t n_points, float* A, int mode, void* stream);

/* Adjoint of the forward sum with respect to the positions (chain rule through Eq. 2).
 * For a real loss L(A) with seed G_k = dL/dRe A_k + i dL/dIm A_k (the complex gradient
 * convention of PyTorch):
 *     grad_xyz_j = dL/dr_j = Re sum_k conj(G_k) f_j (2 i pi S_k) exp(2 i pi S_k . r_j)
 *   G float[n_points*2], grad_xyz float[n_atoms*3], overwritten.
 * n_points == 0 writes grad_xyz = 0; n_atoms == 0 queues nothing. */
int nx_scatter_bwd(const float* xyz, const float* f, int64_t n_atoms,
                   const float* S, int64_t n_points, const float* G, float* grad_xyz,
                   int mode, void* ws, size_t ws_bytes, void* stream);

/* All-FP64 forward (Eq. 2 with FP64 phase, FP64 sin/cos and FP64 sums): the
 * double-precision comparator mentioned at the end of Section 2.3.  Same layout as
 * nx_scatter_fwd with double arrays; A is complex128. */
int nx_scatter_fwd_f64(const double* xyz, const double* f, int64_t n_atoms,
                       const double* S, int64_t n_points, double* A,
                       void* ws, size_t ws_bytes, void* stream);

/* All-FP64 adjoint: the chain rule through Eq. 2 (Section 2.1) for the positions,
 *     grad_xyz_j = Re sum_k conj(G_k) f_j (2 i pi S_k) exp(2 i pi S_k . r_j),
 * with FP64 phase, sin/cos and sums: the double-precision comparator of the end of
 * Section 2.3, applied to the adjoint.  Same layout, ownership and errors as
 * nx_scatter_bwd with double arrays (G and f complex128 as (re, im) pairs). */
int nx_scatter_bwd_f64(const double* xyz, const double* f, int64_t n_atoms,
                       const double* S, int64_t n_points, const double* G, double* grad_xyz,
                       void* ws, size_t ws_bytes, void* stream);

/* Intensity misfit and its seed for fitting a model to measured intensities I (the
 * paper computes intensity maps |A|^2 of strained nanostructures, Sections 4.1-4.3, and
 * its conclusion, Section 6, points to fitting such models to measured maps; the
 * paper prints no loss, so this least-squares misfit in intensity is this library's
 * choice of objective):
 *     e_k = |A_k|^2 - I_k,   L = sum_k e_k^2,   G_k = 4 e_k A_k
 * (G is dL/dRe A + i dL/dIm A, the input nx_scatter_bwd expects).  e and L are
 * evaluated in FP64 from the FP32 inputs; G is rounded once to FP32.  L is reduced in
 * a fixed order (deterministic).
 *   A float[n_points*2], I float[n_points], L double[1] (device), G float[n_points*2]
 *   (may be NULL when only L is wanted).  n_points == 0 writes L = 0. */
int nx_loss_grad(const float* A, const float* I, int64_t n_points, double* L, float* G,
                 void* ws, size_t ws_bytes, void* stream);

/* One fitting step, queued by one call: the forward sum (Eq. 2), the intensity misfit
 * and its seed (as nx_loss_grad), then the adjoint with respect to the positions (the
 * chain rule through Eq. 2, as nx_scatter_bwd), on `stream`, in that order:
 *     A = nx_scatter_fwd(xyz, f, S);  (L, G) = misfit(A, I);  grad_xyz = adjoint(G).
 * The results are those of the three calls made one after the other (bitwise).  The one
 * workspace serves the three stages in turn: nx_workspace_bytes(..., NX_OP_FIT, ...) is the
 * largest of the three needs.  It exists for callers whose steps are short enough that
 * three calls cost more host time than the GPU work (a few thousand atoms and points).
 *   I float[n_points]; A float[n_points*2], L double[1], G float[n_points*2],
 *   grad_xyz float[n_atoms*3]: outputs (device), overwritten.  Errors as for the three
 *   calls; nothing is queued when the arguments are invalid. */
int nx_fit_step(const float* xyz, const float* f, int64_t n_atoms, const float* S,
                int64_t n_points, const float* I, float* A, double* L, float* G,
                float* grad_xyz, int mode, void* ws, size_t ws_bytes, void* stream);

/* A regular grid of reciprocal-space points, given exactly (FP64, r.l.u.): point
 * (i1, i2, i3), 0 <= i_a < n_a, is S = origin + i1 step1 + i2 step2 + i3 step3, and the points
 * are listed with i1 fastest, k = i1 + n1 (i2 + n2 i3) (the order of A, G and I).  The maps
 * of reciprocal space around a reflection (Section 4's examples) are such grids.  The
 * grid entry points compute the same sums as their point-list counterparts over these
 * points, in the FP64-phase mode only (mode NX_F32_PH64; other modes: NX_ERR_MODE).  Where
 * n1 is a multiple of 64 they walk the grid by rows: the phase S.r_j is i1 (step1.r_j)
 * plus a row term formed once per atom and row, one FP64 fma per atom-point pair instead of
 * three; otherwise they form every grid point in FP64 and run the point-list kernels.
 * Counts: n_a >= 0, n1 n2 n3 <= NX_MAX_COUNT; origin and steps finite (else NX_ERR_ARG). */
typedef struct nx_grid {
  double origin[3], step1[3], step2[3], step3[3];
  int64_t n1, n2, n3;
} nx_grid;

/* Workspace (bytes) of the grid entry points for op NX_OP_FWD (nx_scatter_fwd_grid),
 * NX_OP_BWD (nx_scatter_bwd_grid) or NX_OP_FIT (nx_fit_step_grid); 0 with the error set
 * for invalid arguments. */
size_t nx_workspace_bytes_grid(int64_t n_atoms, const nx_grid* grid, int op, int f_is_null);

/* Forward sum (Eq. 2) over the points of `grid` (host pointer):
 *   A_k = sum_j f_j exp(2 i pi S_k . r_j),  S_k the grid's k-th point in FP64.
 * xyz, f, A as for nx_scatter_fwd (A float[n1 n2 n3 * 2], device, overwritten). */
int nx_scatter_fwd_grid(const float* xyz, const float* f, int64_t n_atoms, const nx_grid* grid,
                        float* A, int mode, void* ws, size_t ws_bytes, void* stream);

/* Adjoint with respect to the positions over the points of `grid` (the chain rule through
 * Eq. 2, as nx_scatter_bwd): G float[n1 n2 n3 * 2] (device), grad_xyz float[n_atoms * 3]
 * (device, overwritten; zero for an empty grid). */
int nx_scatter_bwd_grid(const float* xyz, const float* f, int64_t n_atoms, const nx_grid* grid,
                        const float* G, float* grad_xyz, int mode, void* ws, size_t ws_bytes,
                        void* stream);

/* One fitting step over the points of `grid`, queued by one call: nx_scatter_fwd_grid, the
 * misfit of nx_loss_grad, nx_scatter_bwd_grid, on one workspace (op NX_OP_FIT of
 * nx_workspace_bytes_grid); bitwise the three calls.  Arguments as nx_fit_step's. */
int nx_fit_step_grid(const float* xyz, const float* f, int64_t n_atoms, const nx_grid* grid,
                     const float* I, float* A, double* L, float* G, float* grad_xyz, int mode,
                     void* ws, size_t ws_bytes, void* stream);

/* Adjoint with the gradient with respect to the factors as well (for fitting
 * occupancies or compositions):
 *     grad_f_j = dL/dRe f_j + i dL/dIm f_j = conj( sum_k conj(G_k) exp(2 i pi S_k . r_j) )
 * grad_f float[n_atoms*2] (complex64) or NULL (then this is nx_scatter_bwd);
 * grad_xyz may be NULL when only grad_f is wanted.  Workspace: op NX_OP_BWD_GF. */
int nx_scatter_bwd_ex(const float* xyz, const float* f, int64_t n_atoms,
                      const float* S, int64_t n_points, const float* G, float* grad_xyz,
                      float* grad_f, int mode, void* ws, size_t ws_bytes, void* stream);

/* All-FP64 counterpart of nx_scatter_bwd_ex (workspace op NX_OP_BWD_GF_F64). */
int nx_scatter_bwd_ex_f64(const double* xyz, const double* f, int64_t n_atoms,
                          const double* S, int64_t n_points, const double* G, double* grad_xyz,
                          double* grad_f, void* ws, size_t ws_bytes, void* stream);

/* Species-factorised sum (Section 4.2 of the paper: the atoms of one type are summed
 * with unit factor, and each type's sum is multiplied by that type's scattering factor at
 * S, which may depend on |S| and on the energy):
 *     A_k = sum_s fs[s][k] * sum_{j in species s} exp(2 i pi S_k . r_j)
 * The atoms are listed species by species: species s holds atoms
 * [species_start[s], species_start[s+1]); species_start is a HOST array of n_species + 1
 * non-decreasing entries from 0 to n_atoms, 1 <= n_species <= NX_MAX_SPECIES.
 *   fs        float[n_species * n_points * 2] (complex64, species-major), or NULL for 1;
 *   A         float[n_points * 2], overwritten;
 *   A_species float[n_species * n_points * 2] or NULL: the per-species sums (needed by
 *             nx_scatter_bwd_species for the gradient with respect to fs).
 * The per-species (sum, comp) states are combined in FP64 and rounded once.
 * Workspace: nx_workspace_bytes_species(..., op = 0).  Errors as for nx_scatter_fwd,
 * plus NX_ERR_ARG for an invalid species partition. */
int nx_scatter_fwd_species(const float* xyz, int64_t n_atoms, const int64_t* species_start,
                           int n_species, const float* fs, const float* S, int64_t n_points,
                           float* A, float* A_species, int mode, void* ws, size_t ws_bytes,
                           void* stream);

/* Adjoint of nx_scatter_fwd_species for the seed G:
 *   grad_xyz (may be NULL): dL/dr_j for every atom (the per-species seeds G conj(fs[s])
 *            drive the unit-factor adjoint over that species' atoms);
 *   grad_fs  (may be NULL): dL/dRe fs[s][k] + i dL/dIm fs[s][k] = G_k conj(A_species[s][k]),
 *            complex64 [n_species][n_points]; needs A_species.
 * Workspace: nx_workspace_bytes_species(..., op = 1) (only when grad_xyz is wanted). */
int nx_scatter_bwd_species(const float* xyz, int64_t n_atoms, const int64_t* species_start,
                           int n_species, const float* fs, const float* S, int64_t n_points,
                           const float* G, const float* A_species, float* grad_xyz,
                           float* grad_fs, int mode, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes of the species-factorised calls: op 0 forward, op 1 adjoint.  Returns 0
 * and sets the last error on invalid arguments. */
size_t nx_workspace_bytes_species(const int64_t* species_start, int n_species, int64_t n_points,
                                  int mode, int op);

/* The species-factorised sum of Section 4.2 over the points of `grid` (host pointer; the
 * maps of Section 4 are such grids, their atoms of a few types): nx_scatter_fwd_species
 * with S_k the grid's k-th point, each species' unit-factor sum walked over the grid as
 * nx_scatter_fwd_grid walks it.  fs, A, A_species as for nx_scatter_fwd_species with
 * n_points = n1 n2 n3 (points in the grid's order); mode NX_F32_PH64 only (else
 * NX_ERR_MODE).  Workspace: nx_workspace_bytes_species_grid(..., op = 0).  Errors as for
 * nx_scatter_fwd_species and nx_scatter_fwd_grid. */
int nx_scatter_fwd_species_grid(const float* xyz, int64_t n_atoms, const int64_t* species_start,
                                int n_species, const float* fs, const nx_grid* grid, float* A,
                                float* A_species, int mode, void* ws, size_t ws_bytes,
                                void* stream);

/* Adjoint of nx_scatter_fwd_species_grid for the seed G (float[n1 n2 n3 * 2], device):
 * grad_xyz and grad_fs as for nx_scatter_bwd_species (each species' seed G conj(fs[s])
 * drives the grid adjoint over that species' atoms; grad_xyz is zero for an empty grid).
 * Workspace: nx_workspace_bytes_species_grid(..., op = 1) (only when grad_xyz is wanted). */
int nx_scatter_bwd_species_grid(const float* xyz, int64_t n_atoms, const int64_t* species_start,
                                int n_species, const float* fs, const nx_grid* grid, const float* G,
                                const float* A_species, float* grad_xyz, float* grad_fs, int mode,
                                void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes of the species-factorised calls over a grid: op 0 forward, op 1 adjoint.
 * Returns 0 and sets the last error on invalid arguments. */
size_t nx_workspace_bytes_species_grid(const int64_t* species_start, int n_species,
                                       const nx_grid* grid, int op);

/* Message of the calling thread's last error ("" if none).  The pointer stays valid
 * until the thread's next call into the library. */
const char* nx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NX_H */
