/*
 * libtersoff: Tersoff multi-body potential on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  Unless stated otherwise:
 *   - "device" pointers are HIP device memory (hipMalloc, or torch CUDA tensors
 *     on ROCm) owned by the caller; the library never frees them;
 *   - "host" pointers are ordinary host memory, read during the call only;
 *   - every call is asynchronous on the context's HIP stream unless it says
 *     it synchronises;
 *   - positions are FP64 [n][3] row-major (x, y, z of atom 0, then atom 1 ...),
 *     species are int32 [n] in [0, ntypes), and every output is FP64;
 *   - units are Angstrom, eV, eV/Angstrom, amu, ps ("metal" units);
 *   - boxes are orthorhombic, periodic in x, y and z, given as three side
 *     lengths (host memory).  Positions may lie outside [0, L): they are
 *     folded internally.
 * Errors are returned as ters_status; ters_last_error() gives a message.  No
 * C++ exception crosses this interface.
 *
 * The potential (the paper, Section III, Eqs. ters-1..ters-3):
 *   E = 1/2 sum_i sum_{j in N_i} f_C(r_ij) [f_R(r_ij) + b_ij f_A(r_ij)],
 *   b_ij = (1 + (beta zeta_ij)^n)^(-1/(2n)),
 *   zeta_ij = sum_{k in N_i \ {j}} f_C(r_ik) g(theta_ijk) exp(lambda3^m (r_ij - r_ik)^m),
 * with Tersoff's forms f_R = A exp(-lambda1 r), f_A = -B exp(-lambda2 r),
 * g = gamma (1 + c^2/d^2 - c^2/(d^2 + (cos theta - h)^2)), and f_C the sine
 * switch from 1 at R-D to 0 at R+D.  Forces are F = -dE/dx (Eq. pot-force);
 * the virial is W = sum over terms of (x_a - x_i) (x) f_a, six values
 * xx, yy, zz, xy, xz, yz, in eV.
 */
#ifndef TERSOFF_H
#define TERSOFF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ters_ctx ters_ctx;
typedef struct ters_plan ters_plan;

typedef enum {
  TERS_OK = 0,
  TERS_ERR_INVALID_ARG = 1,    /* null pointer, negative size, bad enum */
  TERS_ERR_BOX_TOO_SMALL = 2,  /* a box side is below twice the list cutoff */
  TERS_ERR_NLIST_OVERFLOW = 3, /* an atom has more neighbours than supported */
  TERS_ERR_PARAMS = 4,         /* parameter table fails validation */
  TERS_ERR_NOT_FINITE = 5,     /* non-finite position or result */
  TERS_ERR_HIP = 6,            /* a HIP runtime call failed */
  TERS_ERR_UNSUPPORTED = 7,    /* valid request the library does not handle */
  TERS_ERR_NO_LIST = 8         /* compute before ters_build_nlist, or n changed */
} ters_status;

/* precision modes */
enum {
  TERS_FP64 = 0, /* all arithmetic in FP64 */
  TERS_MIXED = 1, /* FP32 arithmetic; FP64 displacements x_j - x_i (rounded
                    to FP32 afterwards), FP64 rebuild check, FP64 force,
                    energy, virial and gradient accumulators (the paper,
                    Section V-F, mode Opt-M) */
  TERS_SINGLE = 2 /* everything in FP32: positions rounded to FP32 before the
                    displacement, FP32 accumulators for the forces, energy and
                    virial of each wavefront (the paper, Section V-F, mode
                    Opt-S); the per-wavefront sums, the per-atom force gather
                    and the integration stay FP64.  Forward only: ters_compute
                    (without TERS_PARAM_GRAD), ters_md_run, ters_autotune and
                    ters_profile_forward; TERS_ERR_UNSUPPORTED elsewhere. */
};

/* output selection for ters_compute */
enum {
  TERS_ENERGY = 1u,
  TERS_FORCES = 2u,
  TERS_VIRIAL = 4u,
  TERS_PER_ATOM_E = 8u,  /* e_i = 1/2 sum_j V_ij */
  TERS_ACCUMULATE = 16u, /* add to the outputs instead of overwriting them */
  TERS_PARAM_GRAD = 32u  /* also dE/dtable into param_grad (ters_compute_ex) */
};

/* Parameter-table layout: table[ti][tj][tk][14] (FP64, host) with fields
 *   0 m  1 gamma  2 lambda3  3 c  4 d  5 h(=cos theta0)  6 n  7 beta
 *   8 lambda2  9 B  10 R  11 D  12 lambda1  13 A
 * Pair quantities of (i,j) (A, B, lambda1, lambda2, beta, n and the cutoff of
 * r_ij) are read from entry [ti][tj][tj]; three-body quantities of (i,j,k)
 * (m, gamma, lambda3, c, d, h and the cutoff of r_ik) from [ti][tj][tk]. */
#define TERS_NFIELD 14

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, issuing work on `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  The context owns all
 * internal scratch (cell bins, neighbour list, partial sums).  One context
 * per stream; not safe to use from two host threads at once. */
ters_status ters_create(ters_ctx **out, int device, void *hip_stream);
ters_status ters_destroy(ters_ctx *ctx);
ters_status ters_set_stream(ters_ctx *ctx, void *hip_stream);
/* Wait for the context's stream; report any error latched by a kernel. */
ters_status ters_sync(ters_ctx *ctx);
/* Message for the last error on this context (never NULL). */
const char *ters_last_error(const ters_ctx *ctx);

/* ---- parameters (the paper, Section III: per-species parameters) ---------
 * Copy a parameter table (host, [ntypes]^3 x 14 FP64, layout above) and the
 * per-species masses (host, [ntypes] amu, may be NULL if no MD is run) to
 * the device.  Validation: 1 <= ntypes <= 8; n > 0, beta > 0, d != 0, D > 0,
 * R > D, A, B, lambda1, lambda2 finite; m in {1, 3}.  Fails with
 * TERS_ERR_PARAMS otherwise.  Synchronises. */
ters_status ters_set_params(ters_ctx *ctx, int32_t ntypes, const double *table_host,
                            const double *mass_host);

/* ---- neighbour list (the paper, Section II Eq. neigh and Section III skin)
 * Build the full list N_i = { j != i : |x_j - x_i| <= r_list } with
 * r_list = (largest R + D in the table) + skin, by binning atoms into cells of
 * side >= r_list (minimum image).  x: device [n][3]; type: device [n];
 * box: host [3].  Stores the list and a copy of x (the reference for the
 * rebuild check) in the context.  Fails with TERS_ERR_BOX_TOO_SMALL if a side
 * is below 2 r_list.  Grows the list capacity and retries when an atom has
 * more entries than fit (synchronises to read the largest row length). */
ters_status ters_build_nlist(ters_ctx *ctx, int32_t n, const double *x, const int32_t *type,
                             const double *box, double skin);

/* Largest displacement since the last build above skin/2 (FP64, minimum
 * image)?  Writes 1 or 0 to flag_dev (device int32[1]).  No synchronisation. */
ters_status ters_needs_rebuild(ters_ctx *ctx, const double *x, int32_t *flag_dev);

/* Neighbour-list statistics from the last build (synchronises):
 * out[0] = n, out[1] = total entries, out[2] = longest row, out[3] = capacity. */
ters_status ters_nlist_stats(ters_ctx *ctx, int64_t *out4);

/* ---- energy, forces, virial (the paper, Algorithm 3 over the list) --------
 * Evaluate the potential for the n atoms (device x, type; host box) with the
 * context's current list, which must have been built for n atoms with
 * positions within skin/2 of x.  precision: TERS_FP64 or TERS_MIXED.
 * flags: any of TERS_ENERGY, TERS_FORCES, TERS_VIRIAL, TERS_PER_ATOM_E,
 * TERS_ACCUMULATE.  Outputs (device, FP64, caller-owned; NULL allowed when the
 * matching flag is off): energy[1], forces[n][3], virial[6], e_atom[n]. */
ters_status ters_compute(ters_ctx *ctx, int32_t n, const double *x, const int32_t *type,
                         const double *box, int precision, uint32_t flags, double *energy,
                         double *forces, double *virial, double *e_atom);

/* ---- the same without allocation ------------------------------------------
 * For callers that cannot allocate device memory at call time: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * One call builds the neighbour list (skin 0) of the n atoms and evaluates
 * them like ters_build_nlist followed by ters_compute (same kernels, the
 * context's schedule and force mode), with every work buffer (cell bins,
 * list of at most TERS_STATIC_CAP entries per atom, reverse map, force slots,
 * partial sums) in one static device array of the library, of fixed size
 * (about 23 MB), that each GPU holds from the first ters_create on it until
 * the process ends.  It calls no hipMalloc, hipFree or other allocating
 * routine and does not synchronise.  Limits: n <= TERS_STATIC_MAX_ATOMS
 * (TERS_ERR_UNSUPPORTED beyond); at most TERS_STATIC_CAP list entries per
 * atom, else TERS_ERR_NLIST_OVERFLOW is latched and reported by ters_sync
 * (the outputs are then not valid); along an axis with many cells, larger
 * cells are used (results unchanged).  Every call on one GPU shares that
 * GPU's array, so calls that overlap in time on one GPU (two streams, two
 * contexts, two host threads) race and must be serialised by the caller.
 * Arguments, outputs and flags as ters_compute (TERS_PARAM_GRAD refused);
 * it does not touch the context's own list. */
#define TERS_STATIC_MAX_ATOMS 16384
#define TERS_STATIC_CAP 32
ters_status ters_compute_static(ters_ctx *ctx, int32_t n, const double *x, const int32_t *type,
                                const double *box, int precision, uint32_t flags, double *energy,
                                double *forces, double *virial, double *e_atom);

/* As ters_compute, plus with TERS_PARAM_GRAD the derivative of E with
 * respect to every table entry: param_grad device [ntypes^3][14], accumulated
 * into (the caller zeroes it unless accumulating on purpose). */
ters_status ters_compute_ex(ters_ctx *ctx, int32_t n, const double *x, const int32_t *type,
                            const double *box, int precision, uint32_t flags, double *energy,
                            double *forces, double *virial, double *e_atom, double *param_grad);

/* ---- a pair potential on the same list (the paper, Section II, Algorithm 1)
 * Truncated Lennard-Jones V(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6) for
 * r < rc (eV, Angstrom), E = 1/2 sum_i sum_{j in N_i} V(r_ij), over the
 * context's current list, which must have been built for these n atoms and
 * this box (ters_build_nlist) with a list radius minus skin of at least rc
 * (the Tersoff parameters fix that radius).  precision: TERS_FP64 or
 * TERS_MIXED (FP32 arithmetic, FP64 displacements and accumulators).  flags:
 * TERS_ENERGY, TERS_FORCES, TERS_VIRIAL, TERS_ACCUMULATE.  Outputs (device,
 * FP64, caller-owned; NULL allowed when the flag is off): energy[1],
 * forces[n][3], virial[6] (the convention of ters_compute).  Errors:
 * TERS_ERR_NO_LIST without a matching list, TERS_ERR_INVALID_ARG for rc
 * beyond the list, a different box, non-positive sigma or rc. */
ters_status ters_pair_compute(ters_ctx *ctx, int32_t n, const double *x, const double *box,
                              double eps, double sigma, double rc, int precision, uint32_t flags,
                              double *energy, double *forces, double *virial);

/* ---- adjoint (vector-Jacobian product of (E, F) wrt (x, table)) ----------
 * Given cotangents e_bar (host scalar) and f_bar (device [n][3]) of the
 * outputs E and F, writes
 *   x_grad     = e_bar dE/dx + sum_a f_bar_a dF_a/dx      (device [n][3])
 *   param_grad = e_bar dE/dtheta + sum_a f_bar_a dF_a/dtheta (device [ntypes^3][14])
 * Both are overwritten.  Computed by one pass of the force kernel in
 * forward-mode dual arithmetic along f_bar; zeta is recomputed, no triplet
 * is stored.  The derivative with respect to the integer m uses the
 * continuation sgn(u)|u|^m, u = lambda3 (r_ij - r_ik).  Needs a current list. */
ters_status ters_backward(ters_ctx *ctx, int32_t n, const double *x, const int32_t *type,
                          const double *box, int precision, double e_bar, const double *f_bar,
                          double *x_grad, double *param_grad);

/* ---- molecular dynamics ---------------------------------------------------
 * nsteps velocity-Verlet steps (dt_ps in ps) on device x, v, f ([n][3] FP64,
 * updated in place; f must hold the forces at x on entry, e.g. from
 * ters_compute).  The list is rebuilt on the device whenever the largest
 * displacement since the last build exceeds skin/2; no host synchronisation
 * inside the loop.  energy_trace: device [nsteps] potential energy after
 * each step, or NULL.  Needs masses (ters_set_params) and a list built with
 * the same skin.  When use_graph is non-zero one step is captured into a
 * hipGraph once and replayed. */
ters_status ters_md_run(ters_ctx *ctx, int32_t n, double *x, double *v, double *f,
                        const int32_t *type, const double *box, double dt_ps, int32_t nsteps,
                        double skin, int precision, double *energy_trace, int use_graph);
/* The same steps as ters_md_run, launched one by one (no graph), with a pair
 * of HIP events recorded on the context's stream around every force-kernel
 * launch.  force_us (host, required) gets the average force-kernel duration
 * in microseconds over the nsteps steps (synchronises).  For measurement. */
ters_status ters_md_run_timed(ters_ctx *ctx, int32_t n, double *x, double *v, double *f,
                              const int32_t *type, const double *box, double dt_ps,
                              int32_t nsteps, double skin, int precision, double *energy_trace,
                              double *force_us);
/* Number of list rebuilds done by ters_md_run calls so far (synchronises). */
ters_status ters_md_rebuilds(ters_ctx *ctx, int64_t *out);

/* ---- batches of independent configurations -------------------------------
 * A plan covers nconf configurations concatenated along the atom axis:
 * natoms_host[c] atoms each (config c occupies rows off_c .. off_c+n_c-1 with
 * off_c = sum of earlier n), boxes_host [nconf][3].  Lists are built with
 * skin 0, inside each run's graph, and only when an atom is not where the
 * last build found it (bitwise, up to whole box vectors), a species lies
 * outside the table or the last build overflowed a row: a fitting loop over
 * fixed frames builds them once.  The plan owns device scratch, the
 * autotuned schedule and the
 * hipGraphs of the evaluation.  ters_batch_run evaluates all configurations
 * with one graph launch: energies e[nconf], forces f_cat[N][3], virials
 * w[nconf][6] (device, FP64; any may be NULL).  If f_bar is non-NULL the
 * graph also runs the adjoint with per-configuration e_bar[nconf] (device)
 * and f_bar_cat [N][3] (device), writing x_grad_cat [N][3] and param_grad
 * (summed over configurations) [ntypes^3][14]; with f_bar set and e, f_cat
 * and w all NULL the forward pass is left out (the adjoint does not need its
 * results: a fitting loop that has the energies and forces of these
 * positions from a forward-only run asks for the gradients alone).  x_cat,
 * type_cat device.
 * Inside the graph: the lists of all configurations (one set of launches),
 * then one persistent launch of the wavefront force kernel whose workgroups
 * (as many as stay resident on the device, or as the chunks keep busy when
 * they are fewer) take chunks of atoms, never spanning two configurations,
 * from eight work queues (one per XCD, atomic counters reset at the start of
 * the graph) until all are done, and, with f_bar, one such launch of the
 * adjoint kernel.  The atoms per chunk of each pass are timed on the data of
 * the first run that needs the pass (synchronising).
 * The pointers of a run are baked into its graph: the plan keeps the graphs
 * of the four most recently used argument sets (a forward-only run and a run
 * with the adjoint, alternating, replay two graphs), and a run with another
 * set captures a new one in place of the least recently launched.  Errors
 * latched by the graph (list overflow, non-finite positions, species outside
 * the table) are reported by ters_sync.  A plan refuses runs once
 * ters_set_params changed the number of species or raised a cutoff beyond
 * the plan's list radius. */
ters_status ters_batch_plan(ters_ctx *ctx, int32_t nconf, const int32_t *natoms_host,
                            const double *boxes_host, int precision, uint32_t flags,
                            ters_plan **out);
ters_status ters_batch_run(ters_plan *plan, const double *x_cat, const int32_t *type_cat,
                           double *e, double *f_cat, double *w, const double *e_bar,
                           const double *f_bar_cat, double *x_grad_cat, double *param_grad);
/* Destroying a context releases the device resources of its plans; such a
 * plan then fails ters_batch_run with TERS_ERR_INVALID_ARG, and
 * ters_plan_destroy still frees it. */
ters_status ters_plan_destroy(ters_plan *plan);
/* Schedule chosen by the plan's autotuner (host double[6]): out[0] = atoms
 * per chunk of the forward pass, out[1] = kernel (2: the wavefront schedule,
 * persistent form), out[2] = measured microseconds of the forward pass,
 * out[3] = atoms per chunk of the adjoint pass (0 until a run with f_bar),
 * out[4] = its microseconds, out[5] = workgroups of the forward launch (those
 * that fill the device, or fewer when the chunks are fewer). */
ters_status ters_plan_schedule(const ters_plan *plan, double *out6);

/* ---- schedule control ------------------------------------------------------
 * kernel: 1 = workgroup schedule (a workgroup of 256 lanes stages a run of
 * atoms' pairs in LDS and keeps dzeta/dx_k of up to k_max neighbours per pair,
 * the paper's Algorithm 3), 2 = wavefront schedule (each wavefront works alone,
 * pair data in registers exchanged by cross-lane permutes, the two K loops of
 * Algorithm 2 with dzeta/dx_k of the first four k kept), 3 = thread per atom
 * (the paper's mapping scheme (c), Section IV-B: one thread walks its atom's
 * j and k; forward only, forces scattered with FP64 atomics whatever the
 * force mode; kept as a baseline), 0 = default (2).  atoms: atoms per
 * workgroup (kernel 1, <= 64) or per wavefront (kernel 2, <= 32), ignored by
 * kernel 3; 0 = default (kernel 1: 64; kernel 2: 32 with one species, 24
 * with several).  kmax (kernel 1): stored dzeta/dx_k per pair before
 * falling back to recomputing them (the paper's k_max, Section IV-A); 0 =
 * store all that fit; -1 = store none, so that the second K loop recomputes
 * every term (the paper's Algorithm 2).  Applies to the FP64 and mixed precisions (the single
 * mode always runs kernel 2).  ters_backward refuses kernel 3 with
 * TERS_ERR_UNSUPPORTED. */
ters_status ters_set_schedule(ters_ctx *ctx, int32_t kernel, int32_t atoms, int32_t kmax);
/* Current schedule for a precision (TERS_FP64, TERS_MIXED or TERS_SINGLE):
 * out3[0] = kernel (1, 2 or 3), out3[1] = atoms per workgroup/wavefront
 * (the default resolved), out3[2] = force mode. */
ters_status ters_get_schedule(const ters_ctx *ctx, int32_t precision, int32_t *out3);
/* How forces reach their atoms: 1 (default) = owner gather: the force kernel
 * stores, for every list slot (i, j), the force that atom i's terms exert on
 * j, and a second pass sums each atom's incoming slots in a fixed order
 * through a reverse-slot map built with the list (no atomics; results are
 * bitwise reproducible); 0 = scatter with FP64 atomic adds. */
ters_status ters_set_force_mode(ters_ctx *ctx, int32_t mode);
/* The filter of the paper's Section IV-B/IV-D (only list entries inside the
 * largest cutoff reach the compute lanes): 1 (default) = on; 0 = off, every
 * list entry, skin included, takes a lane and the cutoff is applied inside
 * the K loops.  Results are the same either way; the switch exists to
 * measure the filter.  The wavefront schedule honours it; the workgroup
 * schedule always filters.  TERS_ERR_INVALID_ARG for other values. */
ters_status ters_set_filter(ters_ctx *ctx, int32_t enabled);
/* Time the candidate schedules (both kernels, several atom counts) on the
 * current list and keep the fastest for this precision (synchronises).
 * out_us (host, may be NULL) gets the best time. */
ters_status ters_autotune(ters_ctx *ctx, int32_t n, const double *x, const int32_t *type,
                          const double *box, int precision, double *out_us);

/* Average duration in microseconds of the force kernel alone (energy, forces
 * and virial, no output zeroing or final reduction), from HIP events around
 * `reps` back-to-back launches on the context's stream, with the current list
 * (synchronises).  with_gather != 0 adds, in owner-gather mode, the pass that
 * sums each atom's slots into its force, so that the time covers all work up
 * to the forces (it has no effect in scatter mode).  Forces go to internal
 * scratch. */
ters_status ters_profile_forward(ters_ctx *ctx, int32_t n, const double *x, const int32_t *type,
                                 const double *box, int precision, int32_t reps,
                                 int32_t with_gather, double *avg_us);

/* ---- parameter tables (Si/C mixing rules, Tersoff 1989) -------------------
 * Fill a host table [2][2][2][14] for species 0 = Si (Tersoff's Si(C) set),
 * 1 = C, with Si-C cross terms by the geometric/arithmetic mixing rules and
 * chi = 0.9776.  Fill a [1][1][1][14] table for one of the element sets
 * 0 = Si(B), 1 = Si(C), 2 = C. */
ters_status ters_table_sic(double *table_host);
ters_status ters_table_element(int32_t which, double *table_host);

/* Library version string. */
const char *ters_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TERSOFF_H */
