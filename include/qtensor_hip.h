/*
 * qtensor_hip.h -- C-ABI of the MI355X bucket-elimination contractor for
 * QAOA MaxCut tensor networks with step-dependent slicing.
 *
 * The method (Lykov et al., "Tensor Network Quantum Simulator With
 * Step-Dependent Parallelization"):
 *   circuit -> tensor expression over binary variables (Section IV-A, IV-B)
 *   -> elimination order and slice set (Section V-A, Section VI-C, VI-D)
 *   -> bucket elimination, sliced part batched over slices, then a sum over
 *      slices (Algorithm 1; Eq. (2)).
 *
 * General conventions
 *   - Every call returns a qt_status; no exception or abort crosses the ABI.
 *     On failure qt_last_error() (thread-local) holds a message; HIP errors
 *     come back as QT_EHIP with the HIP error string in the message.
 *   - The caller owns every buffer it passes; the library copies what it
 *     keeps.  Objects returned through qt_network** / qt_plan** are owned by
 *     the caller and released with qt_free_network / qt_free_plan (a plan
 *     keeps its own copy of the network; the network may be freed first).
 *   - Parameter arrays (gammas, betas) and outputs may be host or device
 *     pointers.  Results written to host memory are complete when the call
 *     returns (the call synchronises `hip_stream`); results written to
 *     device memory are ordered on `hip_stream` and the call does not wait.
 *     Device parameter (and weight) arrays are read by the call's launches
 *     where they are, in stream order, and device results are written by
 *     them in place: change or free such arrays only after the work on
 *     `hip_stream` has run.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  The
 *     library allocates its device workspace on first use of a plan and
 *     keeps it with the plan; calls on one plan must not overlap.
 *   - A value is reported as qt_amp: (re + i im) * 2^log2_scale, with re/im
 *     and the scale in FP64.  Gate tensors |+> are stored as (1, 1) and
 *     their 2^{-1/2} factors are carried exactly in log2_scale.
 */
#ifndef QTENSOR_HIP_H
#define QTENSOR_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qt_network qt_network; /* opaque, library-owned storage */
typedef struct qt_plan qt_plan;       /* opaque, library-owned storage */

typedef enum {
  QT_OK = 0,
  QT_EINVAL = -1,          /* bad argument (null pointer, size out of range) */
  QT_ENOMEM = -2,          /* host or device allocation failed */
  QT_EPLAN = -3,           /* order / slice schedule inconsistent with the network */
  QT_EHIP = -4,            /* a HIP runtime call failed */
  QT_EUNSUPPORTED = -5,    /* valid request outside what this build handles */
  QT_EFAULT_INJECTED = -6  /* test hook QT_FAULT_AFTER_SLICE fired */
} qt_status;

/* Arithmetic of the bucket steps.
 *   QT_C128         complex128 throughout, no scaling: the plain path.
 *   QT_C64_SCALED   complex64 mantissas with a per-tensor power-of-two
 *                   exponent (renormalised after every step from the
 *                   measured max|x|), FP64 slice sum.
 *   QT_C64_SCALED_MFMA_FP32
 *                   as QT_C64_SCALED, and a bucket whose two largest
 *                   tensors share variables held by no other tensor (but
 *                   vectors) sums the bucket variable and those variables
 *                   in one step, a batched complex GEMM
 *                   C[b,m,n] = sum_k A[b,m,k] B[b,n,k] on the matrix cores
 *                   (FP32 inputs and accumulation), when the unfused output
 *                   would have rank >= 12 (QT_GEMM_MIN_RANK), K >= 8,
 *                   M, N >= 16 and A, B and C have rank <= 28 per batch
 *                   item.  Same values as eliminating the variables one by
 *                   one, with a smaller intermediate.
 *   QT_C64_SCALED_MFMA_BF16X3
 *                   as QT_C64_SCALED_MFMA_FP32, and fused buckets with
 *                   K >= 32 take their products on the BF16 matrix cores:
 *                   each FP32 operand value is split into three BF16 parts
 *                   (about 24 significant bits), a real product is the sum
 *                   of the six part products above 2^-16 of it, and a complex
 *                   product takes three real ones (3M: Ar Br, Ai Bi and
 *                   (Ar + Ai)(Br + Bi)), all accumulated in FP32.  Shorter
 *                   fused sums use the FP32 products. */
typedef enum {
  QT_C128 = 0,
  QT_C64_SCALED = 1,
  QT_C64_SCALED_MFMA_FP32 = 2,
  QT_C64_SCALED_MFMA_BF16X3 = 3
} qt_precision;

/* Tensor kinds (Section III-A gates; Section IV-B graph model: diagonal
 * gates are written on the variables they share with their wires).
 *   VEC_PLUS   |+> (also <+| of the energy network) on (x)          values (1, 1) * 2^{-1/2}
 *   ZZ         exp(-i gamma_k (1 - Z_a Z_b)/2) on (x_a, x_b)       [[1, e^{-i g}], [e^{-i g}, 1]]
 *   RX         exp(-i beta_k X) from x_in to x_out                  [[cos b, -i sin b], [-i sin b, cos b]]
 *   BRA_BIT    <z| on an output variable (layer field = z)          e_z
 *   ZZ_DAG     adjoint of ZZ, analytic in gamma                     [[1, e^{+i g}], [e^{+i g}, 1]]
 *   RX_DAG     adjoint of RX, analytic in beta                      [[cos b, i sin b], [i sin b, cos b]]
 *   OBS_CUT    (1 - Z_u Z_v)/2 on (x_u, x_v)                        [[0, 1], [1, 0]]
 *   DENSE      caller-supplied values
 * Parametrised kinds take gamma_k / beta_k with k = `layer` (1-based). */
typedef enum {
  QT_T_VEC_PLUS = 0,
  QT_T_ZZ = 1,
  QT_T_RX = 2,
  QT_T_BRA_BIT = 3,
  QT_T_ZZ_DAG = 4,
  QT_T_RX_DAG = 5,
  QT_T_OBS_CUT = 6,
  QT_T_DENSE = 7
} qt_tkind;

typedef struct {
  int32_t kind;         /* qt_tkind */
  int32_t rank;         /* number of variables: 1 (VEC_PLUS, BRA_BIT), 2 (ZZ, RX, *_DAG, OBS_CUT), 1..24 (DENSE) */
  int32_t layer;        /* 1..p for ZZ/RX/ZZ_DAG/RX_DAG; the bit z (0/1) for BRA_BIT; ignored otherwise */
  const int32_t* vars;  /* `rank` distinct variable ids in [0, n_vars) */
  const double* dense;  /* DENSE only: 2^rank interleaved (re, im); vars[0] is the most significant axis */
} qt_tensor_desc;

typedef struct {
  int32_t n_vars;       /* size of the variable id space (ids need not all be used) */
  int32_t n_tensors;
  int32_t p;            /* number of QAOA layers (length of gammas / betas) */
  const qt_tensor_desc* tensors;
} qt_network_desc;

/* Elimination order and step-dependent slicing schedule (Section VI-C, VI-D;
 * Algorithm 1).  `order` lists every variable of the network that is not
 * sliced, in elimination order.  Group g fixes its `group_len[g]` variables
 * (concatenated in `slice_vars`) after `group_step[g]` variables of `order`
 * have been eliminated; the first group_step[0] buckets form the serial
 * prefix, run once and shared by every slice.  The slice id's bits are the
 * slice variables' values, first listed variable most significant (the
 * binary representation of the rank in Algorithm 1), group by group.
 * Several groups (r < n in Section VI-D) must have non-decreasing steps;
 * they are executed with every group's variables fixed at the last group's
 * step: the steps between two group steps then run once on tensors that
 * hold the earlier groups' variables as their top bits, the same
 * arithmetic as running them once per earlier-group slice on the blocks,
 * so the per-slice values are those of the branched schedule. */
typedef struct {
  const int32_t* order;
  int32_t n_order;
  int32_t n_groups;
  const int32_t* group_step;
  const int32_t* group_len;
  const int32_t* slice_vars;
  int32_t precision;    /* qt_precision */
  int64_t slice_batch;  /* slices processed per launch; 0 = as many as fit the workspace budget */
  int32_t flags;        /* QT_PLAN_* bits */
  /* Open output variables (a batch of amplitudes, Section VII): `n_open`
   * variables (0..20) that are neither eliminated nor sliced; the value of
   * the contraction is then a tensor over them, 2^n_open values, computed
   * in one contraction.  Output index bit a-1-q is the value of open_vars[q]
   * (open_vars[0] most significant).  NULL / 0: a scalar amplitude. */
  int32_t n_open;
  const int32_t* open_vars;
  /* MFMA precisions: a bucket is fused into one complex GEMM only when its
   * output has at least this rank (4..28); smaller buckets stay bucket
   * steps.  0: the default (12, or QT_GEMM_MIN_RANK). */
  int32_t gemm_min_rank;
} qt_plan_desc;

/* Plan flags.
 *   QT_PLAN_PLAIN: one launch per bucket step (no fusion of small steps into
 *     LDS-resident segments); with slice_batch = 1 this is the plain path,
 *     one launch per step per slice.
 *   QT_PLAN_FOLD_PREFIX: run the serial prefix inside every slice with the
 *     slice variables already fixed (same order, same per-slice values),
 *     instead of once before the slices.
 *   QT_PLAN_GRAPH: when parameters and results are device memory,
 *     qt_contract_batch captures the launch sequence as a HIP graph on first
 *     use (per addresses and batch shape) and replays it afterwards; set on
 *     lightcones[0], qt_energy_grad does the same for its sequence. */
enum { QT_PLAN_PLAIN = 1, QT_PLAN_FOLD_PREFIX = 2, QT_PLAN_GRAPH = 4 };

typedef struct {
  double re, im;        /* mantissa */
  double log2_scale;    /* value = (re + i im) * 2^log2_scale */
} qt_amp;

/* Summary of a compiled plan (for reporting; algorithmic counts per point). */
typedef struct {
  int32_t n_steps;          /* bucket steps (prefix + per-slice) */
  int32_t n_prefix_steps;
  int32_t width;            /* max over steps of the eliminated variable's neighbour count (contraction width c) */
  int32_t prefix_width;
  int32_t slice_width;      /* width of the per-slice part */
  int32_t n_slice_vars;
  int64_t n_slices;
  int64_t slice_batch;      /* slices per launch actually used */
  double prefix_bytes;      /* algorithmic bytes of the prefix (inputs read + output written) */
  double slice_bytes;       /* algorithmic bytes of one slice's steps */
  double prefix_flops;      /* real flops of the prefix */
  double slice_flops;       /* real flops of one slice */
  int64_t workspace_bytes;  /* device workspace of the last run */
  int32_t element_bytes;    /* 8 (complex64) or 16 (complex128) */
  int32_t n_launches;       /* kernel launches of one amplitude at the last run's batch */
  int32_t n_open;           /* open output variables: each contraction gives 2^n_open values */
  int32_t n_groups;         /* slice groups of the schedule */
} qt_plan_info;

/* Copy a tensor network (Section IV-A: tensors over binary variables, each a
 * clique of the line graph, Section IV-B).  Checks kinds, ranks and variable
 * ids.  All inputs are copied. */
qt_status qt_load_network(const qt_network_desc* desc, qt_network** out);

/* Compile a plan: validate the order and slice schedule (QT_EPLAN if `order`
 * is not a permutation of the unsliced variables, if slice variables repeat
 * or overlap the order, or if group steps are out of [0, n_order]), run the
 * bucket assignment of Algorithm 1 symbolically (each tensor goes to the
 * bucket of its earliest variable; each result to the bucket of its earliest
 * remaining variable), lay out every intermediate, and upload the step
 * tables.  No kernel runs. */
qt_status qt_load_plan(const qt_network* net, const qt_plan_desc* desc, qt_plan** out);

/* One amplitude at one parameter point: gate tensors materialised on the
 * device from (gamma, beta) (p values each), the serial prefix, all slices
 * (batched), the FP64 slice sum.  `out` receives the sum (2^n_open values
 * for a plan with open output variables). */
qt_status qt_contract_amplitude(qt_plan* plan, const double* gammas, const double* betas,
                                qt_amp* out, void* hip_stream);

/* Batched contraction: every plan at every point (gammas/betas are
 * [n_points][p], row-major), restricted to slice ids in
 * [slice_begin, slice_end) (the resumable unit of work; slices are
 * independent, Eq. (2)).  out: [n_plans][n_points][2^a] partial sums over
 * the range, a = the plans' n_open (all plans of a call have the same).
 * per_slice_out (optional, NULL to skip): [n_plans][n_points][2^a]
 * [slice_end - slice_begin][3] doubles (re, im, log2_scale) per slice, the
 * journal a caller keeps to resume.  Slices are summed in FP64 in slice-id
 * order, so results are bitwise reproducible.  The test hook environment
 * variable QT_FAULT_AFTER_SLICE=j makes the call return QT_EFAULT_INJECTED
 * after the slices below j have been written to per_slice_out. */
qt_status qt_contract_batch(qt_plan* const* plans, int32_t n_plans, int32_t n_points,
                            const double* gammas, const double* betas,
                            int64_t slice_begin, int64_t slice_end,
                            qt_amp* out, double* per_slice_out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * qt_contract_batch for a single plan, with the same arguments, results
 * and journal layout (n_plans = 1), whose whole device workspace -- gate
 * tensors, intermediates, exponent and max slots, step tables, per-slice
 * results -- lives in a static device array of QT_NOALLOC_SCRATCH_BYTES
 * that each GPU the library runs on holds until the process ends.  No
 * device memory is allocated or freed by the call.  The slice batch is the
 * largest power of two whose workspace fits; a contraction that does not
 * fit at one slice per launch is rejected with QT_EINVAL and the size it
 * needs in qt_last_error().  All calls on one GPU share the array: when it
 * holds another plan's (or another shape's) workspace, the call waits for
 * the device to drain and uploads its tables again; calls that overlap on
 * one GPU (other threads, or streams still running an earlier call) race
 * and must be serialised by the caller.  QT_PLAN_GRAPH is ignored. */
#define QT_NOALLOC_SCRATCH_BYTES (64ll << 20)
qt_status qt_contract_batch_noalloc(qt_plan* plan, int32_t n_points,
                                    const double* gammas, const double* betas,
                                    int64_t slice_begin, int64_t slice_end,
                                    qt_amp* out, double* per_slice_out, void* hip_stream);

/* QAOA MaxCut energy E = sum_e <C_e> from per-edge lightcone networks
 * (Section III-B: the energy is one amplitude of a duplicated expression;
 * lightcone optimisation, Section III-A), all edges and points in one batched
 * launch, and optionally its gradient by reverse-mode bucket elimination.
 * `lightcones[e]` is the compiled plan of edge e's network (built with
 * OBS_CUT, ZZ_DAG and RX_DAG tensors, no slicing).  gammas/betas are
 * [n_points][p].  energy: [n_points] (required); dE_dgamma, dE_dbeta:
 * [n_points][p] or NULL (no gradient pass); per_edge: [n_points][n_edges]
 * or NULL.  Sums over edges run in FP64 in edge order.
 * Execution: one launch of one workgroup per (edge, point), in order of
 * decreasing cost.  Lightcones whose tensors fit the launch's LDS keep them
 * there; larger ones run the same schedule from a global scratch area of
 * their own (forward lightcones above 2^22 tensor elements instead take the
 * plan's per-step schedule, outside the launch).  The device buffers of a
 * list of lightcones (parameters, per-edge results, scratch) are built on
 * first use and cached with it until one of its plans is freed; calls on
 * the same list that overlap on different streams race on them and must be
 * serialised by the caller (calls on one stream are ordered).
 * Precision: without gradient outputs the lightcones run in the plans'
 * precision.  With them, the forward and reverse pass run in complex128
 * whatever the plans' precision, and the energies returned are that pass's:
 * a derivative is a sum of per-gate terms about as large as the edge energy
 * that cancel to a far smaller value near stationary points, so complex64
 * arithmetic loses the 1e-5 relative bound there (measured 1.2e-5 normwise
 * on a 200-node, p = 2 point), at a cost in time of under 10 percent. */
qt_status qt_energy_grad(qt_plan* const* lightcones, int32_t n_edges, int32_t n_points,
                         const double* gammas, const double* betas,
                         double* energy, double* dE_dgamma, double* dE_dbeta,
                         double* per_edge, void* hip_stream);

/* qt_energy_grad with per-edge weights in the FP64 sums over edges:
 * energy = sum_e w_e <C_e>, the gradient likewise; per_edge stays the
 * unweighted <C_e>.  edge_weights: [n_edges] non-negative doubles, host or
 * device (QT_EINVAL on a negative or NaN host weight).  With lightcones
 * deduplicated up to isomorphism (Section III-A's symmetry argument: edges
 * whose lightcones are isomorphic, with the edge's endpoints mapped to each
 * other, have equal <C_e>), one plan per class weighted by the class size
 * gives the full-graph energy and gradient. */
qt_status qt_energy_grad_weighted(qt_plan* const* lightcones, const double* edge_weights, int32_t n_edges,
                                  int32_t n_points, const double* gammas, const double* betas,
                                  double* energy, double* dE_dgamma, double* dE_dbeta,
                                  double* per_edge, void* hip_stream);

/* Introspection of a compiled plan. */
qt_status qt_plan_get_info(const qt_plan* plan, qt_plan_info* out);

/* Kernel classes reported by the profiler. */
typedef enum {
  QT_KCLASS_STEP_STREAM = 0, /* streaming bucket step, output >= 1024 elements per item */
  QT_KCLASS_STEP_SMALL = 1,  /* bucket step with smaller outputs, one element per thread */
  QT_KCLASS_LDS = 2,         /* LDS-resident multi-step contraction */
  QT_KCLASS_GEMM = 3,        /* fused bucket as complex GEMM on MFMA */
  QT_KCLASS_OTHER = 4,       /* gate materialisation, fills, per-slice products, slice sum */
  QT_KCLASS_COUNT = 8
} qt_kclass;

typedef struct {
  int64_t launches;
  double ms;     /* summed kernel durations from HIP events recorded around each launch */
  double bytes;  /* algorithmic bytes: elements of every input read plus the output written */
  double flops;  /* algorithmic real flops */
} qt_kernel_stats;

/* Tracing: with `enable` != 0, later calls on `plan` record a HIP event pair
 * around every kernel launch on the caller's stream (adds a few
 * microseconds per launch); 0 turns recording off. */
qt_status qt_profile_enable(qt_plan* plan, int32_t enable);

/* Waits for the recorded events and adds their durations into
 * out[QT_KCLASS_COUNT]; with `reset` != 0 the accumulated statistics are
 * cleared afterwards (those of qt_profile_read_ops too). */
qt_status qt_profile_read(qt_plan* plan, qt_kernel_stats* out, int32_t reset);

/* Launch statistics of one operation of the schedule: a bucket step
 * (streaming or fused GEMM; `op` = its index in the plan's step list), an
 * LDS-executor segment (`op` = segment index), or all other kernels
 * together (`op` = -1). */
typedef struct {
  int32_t kclass;  /* qt_kclass */
  int32_t op;
  int64_t launches;
  double ms;       /* summed HIP-event durations */
  double bytes;    /* algorithmic bytes */
  double flops;    /* algorithmic real flops */
} qt_op_stats;

/* The recorded statistics per operation, in order of first launch: writes
 * min(cap, count) records to `out` and the count to *n_ops; `reset` as for
 * qt_profile_read. */
qt_status qt_profile_read_ops(qt_plan* plan, qt_op_stats* out, int32_t cap, int32_t* n_ops, int32_t reset);

/* Execution tunables of a plan; 0 selects the library default (or the
 * QT_LDS_WAVES, QT_LDS_MAX_RANK, QT_LDS_WAVES_MULTI, QT_LDS_WAVES_GRAD,
 * QT_STEP_LG_TILES (log2 of step_tiles), QT_GEMM_TILES, QT_MULTI_LDS_CAP,
 * QT_GRAD_LDS_CAP environment variables when set).  They choose launch shapes and which
 * steps run from LDS rather than streaming, the role Eq. (1) of the paper
 * gives to its thread count per pairwise product; results stay within the
 * stated tolerances and are bitwise reproducible for fixed tunables.
 *   lds_waves     wavefronts per workgroup of the LDS executor (1..16)
 *   lds_max_rank  largest step output rank the LDS executor takes (6..16);
 *                 larger steps stream from HBM
 *   multi_waves   wavefronts per workgroup of the batched lightcone launch
 *                 of qt_energy_grad (read from lightcones[0])
 *   grad_waves    the same for its gradient launch
 *   step_tiles    output tiles of 1024 elements per workgroup of the
 *                 streaming bucket-step kernel (1, 2, 4, 8, 16)
 *   gemm_tiles    output tiles per workgroup of the fused GEMM kernel
 *                 (power of two, 1..64)
 *   multi_lds_cap LDS bytes per workgroup of the batched lightcone launch
 *                 (4096..163840): as many points of a lightcone as fit
 *                 share a workgroup; lightcones needing more than one
 *                 point's worth run from global scratch in the same launch
 *                 (read from lightcones[0])
 *   grad_lds_cap  the same for the gradient launch */
typedef struct {
  int32_t lds_waves;
  int32_t lds_max_rank;
  int32_t multi_waves;
  int32_t grad_waves;
  int32_t step_tiles;
  int32_t gemm_tiles;
  int32_t multi_lds_cap;
  int32_t grad_lds_cap;
} qt_tuning;

/* Sets a plan's tunables (QT_EINVAL outside the ranges above).  A change of
 * lds_waves or lds_max_rank drops the plan's compiled schedule and device
 * workspace, rebuilt by the next contraction; call it between contractions
 * of the plan, never while one is in flight. */
qt_status qt_plan_set_tuning(qt_plan* plan, const qt_tuning* tuning);
/* The tunables as set (0: default). */
qt_status qt_plan_get_tuning(const qt_plan* plan, qt_tuning* out);

/* Host-only description of the launch schedule the plan would run with the
 * current environment: LDS-executor segments (steps, dependency levels,
 * LDS bytes, staged inputs) and streaming steps, as JSON.  Writes at most
 * `cap` bytes (NUL-terminated) to `buf` and the full length to *needed;
 * QT_EINVAL if `buf` is too small.  Touches no GPU. */
qt_status qt_plan_describe(const qt_plan* plan, char* buf, int64_t cap, int64_t* needed);

void qt_free_plan(qt_plan* plan);
void qt_free_network(qt_network* net);
const char* qt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QTENSOR_HIP_H */
