/*
 * tsne.h - C ABI of the MI355X (gfx950) t-SNE gradient library.
 *
 * One t-SNE gradient iteration as in Linderman et al., "Efficient Algorithms
 * for t-distributed Stochastic Neighborhood Embedding" (FIt-SNE):
 *   - repulsion by piecewise Lagrange interpolation of the Cauchy kernels on an
 *     equispaced grid and a circulant-embedded FFT convolution (Section 2,
 *     Algorithm 1, Section 2.4 for s = 2, the Appendix for the s+2 sums),
 *   - attraction over a sparse symmetric P (Section 3),
 *   - the gradient with early/late exaggeration (Section 1.1, Section 1.2,
 *     Section 4) and a momentum/gain descent step.
 *
 * Conventions shared by every entry point
 *   - Every call returns tsne_status and never throws.  Argument errors are
 *     detected on the host before anything is enqueued (TSNE_E_ARG,
 *     TSNE_E_UNSUPPORTED, TSNE_E_WORKSPACE).  Conditions found on the device
 *     (grid capacity exceeded, non-finite coordinates) are latched in a status
 *     word of the plan; the iteration that meets them is not committed (Y, uY,
 *     gains and outputs are left as they were) and every later call on the
 *     plan is a no-op until tsne_query reports and clears them.
 *   - Pointers are DEVICE pointers unless marked "host".  They are owned by
 *     the caller, borrowed for the duration of the call (P: until rebound or
 *     the plan is destroyed) and must stay valid until the enqueued work has
 *     completed on the plan's stream.
 *   - Y is [n, s] row-major: y_i(d) = Y[i*s + d].  Arrays of per-point
 *     vectors (F_rep, F_attr, uY, gains) share that layout.  The element type
 *     is float (TSNE_F32) or double (TSNE_F64) as set in the descriptor.
 *     Each such array is aligned to a whole point (s times the element size;
 *     for s = 3 one element), since kernels move a point's coordinates as one
 *     vector; every entry
 *     point that takes Y (and tsne_step, tsne_run, tsne_batch_admit for uY
 *     and gains) returns TSNE_E_ARG for one that is not.
 *   - F_rep follows the sign of the attractive/repulsive split of Section 1.1:
 *     F_rep,i = sum_{j != i} (y_i - y_j) / (1 + |y_i - y_j|^2)^2 / Z, pointing
 *     away from the other points; Z = sum_{k != l} 1/(1 + |y_k - y_l|^2).
 *     F_attr,i = sum_j p_ij (y_i - y_j) / (1 + |y_i - y_j|^2) (Section 3).
 *     The gradient is 4 (alpha F_attr - F_rep).
 *   - The library allocates no device memory and creates no streams: the
 *     caller provides a workspace and a stream (hipStream_t, or NULL for the
 *     default stream).  All work is enqueued asynchronously on that stream;
 *     only tsne_query and tsne_batch_poll synchronise.
 *   - A plan is used by one host thread at a time; distinct plans are
 *     independent.
 */
#ifndef TSNE_MI355X_H
#define TSNE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TSNE_OK = 0,
    TSNE_E_ARG = 1,          /* invalid argument (host check) */
    TSNE_E_UNSUPPORTED = 2,  /* valid but not built (e.g. p outside 2..6) */
    TSNE_E_WORKSPACE = 3,    /* workspace missing, misaligned or too small */
    TSNE_E_CAPACITY = 4,     /* the box needs more intervals than max_intervals */
    TSNE_E_NONFINITE = 5,    /* a coordinate of Y is NaN or infinite */
    TSNE_E_HIP = 6,          /* a HIP runtime call failed */
    TSNE_E_STATE = 7,        /* call not valid in the plan's state (e.g. no P bound) */
    TSNE_E_INTERNAL = 8      /* the binning's look-back did not complete (latched on the
                                device; the iteration's results are invalid) */
} tsne_status;

typedef enum { TSNE_F32 = 0, TSNE_F64 = 1 } tsne_dtype;

/* Box / interval policy.  With L = max_d (max_i y_i(d) - min_i y_i(d)) the
 * box is the square (Section 2.4) of side N_int w centred on the mid-range
 * (max + min)/2 of each dimension, and the nodes of interval l sit at
 * origin + (l p + m + 1/2) w/p, m = 0..p-1 (eq. (equinodes) mapped onto the
 * box).  A point y falls in interval clamp(floor((y - origin)/w), 0, N_int-1).
 *   TSNE_GRID_PAPER: N_int = max(min_intervals, ceil(L)), w = L / N_int
 *                    (the interval count of the experiments of Section 2.5);
 *   TSNE_GRID_FIXED: w = interval_width, N_int = ceil(L/w); a box narrower than
 *                    min_intervals * interval_width gets N_int = min_intervals
 *                    and w = L / N_int (no interval wider than L / min_intervals,
 *                    as under the interval count of Section 2.5).
 * L is floored at 1e-6.  The FFT length M (a 4^a 3^b 5^c number >= 2 N_int p)
 * is chosen on the device every call, with hysteresis; the FP64 kernel spectra
 * are rebuilt whenever M or the node spacing w/p changes: under FIXED only
 * when M changes, under PAPER at nearly every call. */
typedef enum { TSNE_GRID_PAPER = 0, TSNE_GRID_FIXED = 1 } tsne_grid_policy;

/* Which kernel sums are formed (Section 2 and the Appendix).
 *   TSNE_FORM_A: K1 with charge 1; K2 with charges 1 and y(d) (the Appendix);
 *   TSNE_FORM_B: K2 with charges 1, y(d) and |y|^2; the K1 sum follows from
 *                K1 = (1 + r^2) K2.
 *   TSNE_FORM_V: not in the paper; the same interpolation with the single
 *                charge 1 against K1 and the s odd kernels z_d K2(|z|^2),
 *                whose sums are the numerators of eq. (frep) themselves:
 *                one spread grid, s + 1 potentials and no cancellation.
 * Charges are centred at the box centre. */
typedef enum { TSNE_FORM_A = 0, TSNE_FORM_B = 1, TSNE_FORM_V = 2 } tsne_form;

typedef struct {
    int64_t n;               /* number of points, >= 2 (< 2^31) */
    int32_t s;               /* embedding dimension: 1, 2 or 3.  s = 3 (Section 2's
                                sums for any s, tensor-product nodes on a cube): forms
                                A and B, the square box, the CSR attraction in one
                                slab, circulant lengths up to 400 per axis
                                (2 max_intervals p <= 400); TSNE_E_UNSUPPORTED
                                otherwise */
    int32_t dtype;           /* tsne_dtype of Y, forces, uY, gains, P values */
    int32_t p;               /* Lagrange nodes per interval, 2..6 (Section 2.3) */
    int32_t policy;          /* tsne_grid_policy */
    int32_t form;            /* tsne_form */
    int32_t min_intervals;   /* lower bound on N_int, >= 1 */
    int32_t max_intervals;   /* capacity: the largest N_int the plan holds */
    double interval_width;   /* w for TSNE_GRID_FIXED (> 0); ignored otherwise */
    int64_t nnz;             /* non-zeros of P; 0 if attraction is not used */
    int32_t lanes_per_row;   /* CSR lanes per row: 0 (auto), 4, 8, 16, 32 or 64 */
    int32_t points_per_lane; /* spreading points per lane: 0 (auto), 1..64 */
    int32_t attr_slabs;      /* CSR layout: column slabs of P, 0 (auto), 1, 2, 4 or 8;
                                each slab is handled by 8/slabs of the 8 XCDs */
    int32_t attr_layout;     /* attraction: 1 CSR rows (lanes per row over the bound
                                CSR), 2 row blocks (P re-bucketed at bind time by
                                blocks of about n/256 rows, at most 3968 (FP32) or
                                1984 (FP64), and 32 KB column windows; each
                                workgroup keeps its rows in LDS and sweeps the
                                windows its non-zeros touch, staged in LDS; row
                                sums in 64-bit fixed point, so the result does not
                                depend on timing).  0 auto: row blocks when s <= 2,
                                n >= 300,000 and lanes_per_row and attr_slabs are
                                0, else CSR rows.  Layout 2 needs s <= 2; binding P
                                then also rejects non-finite values (TSNE_E_ARG) */
    int32_t rect;            /* box shape (s = 2): 0 the square box of Section 2.4;
                                1 a rectangle of equal spacing: the widest axis
                                keeps the policy's N_int and w, a narrower axis d
                                gets min(N_int, max(min_intervals, ceil(L_d / w)))
                                intervals, and each axis its own FFT length.
                                Ignored for s = 1. */
    int32_t keep_h1;         /* 1: keep each point's K1 sum h1_i = sum_j K1(y_i, y_j)
                                (self pair included, so Z = sum_i h1_i - n) of the
                                last repulsion, FP64 in point order, for
                                tsne_debug_export(what = 5); the workspace grows by
                                8 n bytes.  0: not kept. */
} tsne_desc;

/* Descent schedule, indexed by the absolute iteration it:
 *   alpha(it) = le_alpha if it >= le_start, else ee_alpha if it < ee_stop, else 1
 *               (early exaggeration, Section 1.2; late exaggeration, Section 4);
 *   mom(it)   = mom0 if it < mom_switch else mom1.
 * Per component: grad = 4 (alpha F_attr - F_rep);
 *   gain = ((grad > 0) != (uY > 0)) ? gain + gain_inc : gain * gain_dec,
 *   gain = max(gain, gain_min); uY = mom uY - eta gain grad;
 *   Y = (Y - mean(Y)) + uY if recentre, else Y + uY.
 * The momentum/gain rule is not stated in the paper; it is the rule of the
 * t-SNE implementations the paper builds on. */
typedef struct {
    double eta;
    double mom0, mom1;
    int32_t mom_switch;
    double ee_alpha;
    int32_t ee_stop;
    double le_alpha;
    int32_t le_start;
    double gain_inc, gain_dec, gain_min;
    int32_t recentre;
} tsne_sched;

/* Snapshot returned by tsne_query (host struct). */
typedef struct {
    int32_t status;          /* latched tsne_status of the device, then cleared */
    int32_t n_int;           /* N_int of the last iteration */
    int32_t n_nodes;         /* N_int * p */
    int32_t fft_len;         /* circulant length M per dimension */
    int32_t iter;            /* device iteration counter (next iteration to run) */
    int32_t max_intervals;   /* capacity of the plan */
    double origin[2];        /* box origin of the last iteration */
    double w_int;            /* interval width of the last iteration */
    double box_side;         /* L of the last iteration */
    double Z;                /* normalisation of the last repulsion */
    int32_t n_int_y;         /* second axis (s = 2): N_int, nodes and FFT length; */
    int32_t n_nodes_y;       /* equal to the first axis' for the square box */
    int32_t fft_len_y;
    double origin_z;         /* s = 3: box origin along the third axis */
} tsne_stats;

typedef struct tsne_plan tsne_plan;

/* Device workspace needed by a plan for this descriptor (bytes; 0 if the
 * descriptor is invalid). */
size_t tsne_workspace_bytes(const tsne_desc* desc);

/* Create a plan over a caller-owned device workspace (256-byte aligned, at
 * least tsne_workspace_bytes(desc) bytes) for the given stream.  Initialises
 * the workspace (twiddle tables, counters, kernel spectra under FIXED) with
 * work enqueued on the stream.  *out receives the plan (host object). */
tsne_status tsne_plan_create(const tsne_desc* desc, void* workspace, size_t bytes,
                             void* stream, tsne_plan** out);

/* Release the host object.  The workspace belongs to the caller. */
tsne_status tsne_plan_destroy(tsne_plan* plan);

/* Bind the sparse symmetric P in CSR form (Section 3): row_ptr int64 [n+1]
 * (row_ptr[0] = 0, row_ptr[n] = desc.nnz), col int32 [nnz], val [nnz] of the
 * plan's dtype.  Checked on the host (synchronous; TSNE_E_ARG on failure):
 * row_ptr monotone from 0 to nnz, columns in [0, n) and increasing within each
 * row.  Not checked: symmetry, zero diagonal, sum of values 1.  Also builds the
 * per-row slab split table in the workspace, and for FP32 plans with the CSR
 * layout copies (column, value) pairs into the workspace (enqueued on the
 * plan's stream): the attraction and the divergence then read the copy, so
 * a change to P's values takes effect at the next bind.  With attr_layout 2
 * the values must be finite (TSNE_E_ARG otherwise) and are copied, re-bucketed
 * by row block and column window, with the sweep steps and the fixed-point
 * scale of the row sums (2^61 over the largest row sum of |p|, rounded down
 * to a power of two).  The arrays stay borrowed: the CSR layout reads
 * row_ptr (and, in FP64, col and val) at every call; the row-block layout
 * reads only its copy. */
tsne_status tsne_bind_P(tsne_plan* plan, const int64_t* row_ptr,
                        const int32_t* col, const void* val);

/* Repulsion (steps of Algorithm 1 / Section 2.4 with FFT convolution):
 * writes F_rep [n, s] and *Z (device double). */
tsne_status tsne_repulsive(tsne_plan* plan, const void* Y, void* F_rep, double* Z);

/* Attraction over the bound P (Section 3: the attractive term of the
 * gradient is a sum over the non-zeros of P only, computed directly):
 * F_attr,i = sum_j p_ij (y_i - y_j) / (1 + |y_i - y_j|^2).  Y [n, s] and
 * F_attr [n, s] device, in the plan's dtype; TSNE_E_STATE without a bound P. */
tsne_status tsne_attractive(tsne_plan* plan, const void* Y, void* F_attr);

/* One full iteration at absolute iteration index iter (>= 0): the gradient
 * of Section 1.1 split as in Sections 2 and 3, 4 (alpha F_attr - F_rep / Z)
 * with the exaggeration alpha of tsne_sched, then the descent step of
 * tsne_sched (gains, momentum), updating Y, uY and gains in place.  Sets the
 * device iteration counter to iter + 1. */
tsne_status tsne_step(tsne_plan* plan, void* Y, void* uY, void* gains,
                      const tsne_sched* sched, int32_t iter);

/* n_iter iterations (each as tsne_step: Section 1.1's gradient, its
 * repulsion by Sections 2 and 2.4, its attraction by Section 3) starting at
 * absolute iteration iter0 (the schedule is indexed by absolute iteration,
 * so a run can be split and resumed).  The
 * iteration is captured once in a HIP graph (device-side iteration counter and
 * schedule) and replayed n_iter times. */
tsne_status tsne_run(tsne_plan* plan, void* Y, void* uY, void* gains,
                     const tsne_sched* sched, int32_t iter0, int32_t n_iter);

/* Kullback-Leibler divergence C = KL(P || Q) of Section 1.1 at Y, with
 * q_ij = K1(y_i, y_j) / Z: the repulsion's interpolated Z (Section 2) and one
 * pass over the bound P, C = sum p log(p (1 + |y_i - y_j|^2)) + (sum p) log Z.
 * Y [n, s] device; *kl one device double, written when the enqueued work
 * completes.  Needs a bound P (TSNE_E_STATE otherwise); Y, uY, gains and the
 * iteration counter are not touched.  The logarithms run in the element type,
 * the sums in FP64. */
tsne_status tsne_kl_divergence(tsne_plan* plan, const void* Y, double* kl);

/* Synchronise the plan's stream, fill *out (host) and clear the latched
 * device status. */
tsne_status tsne_query(tsne_plan* plan, tsne_stats* out);

/* Copy an internal array of the last iteration to host memory (testing and
 * inspection; synchronises).  what: 0 = charge grids W [C][n_cap][n_cap] (s=2)
 * or [C][n_cap] (s=1), 1 = potential grids V [s+2][...] same layout,
 * 2 = unnormalised repulsion numerators [n, s], 3 = cell start offsets
 * [N_int^s + 1] (int32), 4 = the sorted order [n] (int32: point at each
 * sorted position; points by cell, x interval + N_int * y interval, and by
 * index within a cell), 5 = h1 [n] (double, point order; TSNE_E_STATE unless
 * the plan was created with keep_h1).  *bytes is the size copied (or needed
 * if dst_host is NULL). */
tsne_status tsne_debug_export(tsne_plan* plan, int32_t what, void* dst_host,
                              size_t* bytes);

const char* tsne_status_str(tsne_status status);

/* Size of the device scratch array behind tsne_repulsive_static (bytes). */
#define TSNE_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

/* Repulsion without any device allocation, for callers that cannot allocate
 * device memory or hand over a workspace: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Computes exactly what
 * tsne_plan_create + tsne_repulsive + tsne_plan_destroy compute for desc (same
 * kernels; desc->nnz and the attraction fields are ignored), with the plan's
 * workspace in a fixed device array of TSNE_STATIC_SCRATCH_BYTES (128 MiB)
 * that the library holds on each GPU it runs on until the process ends, and
 * its host record in static storage.  That covers, for example, FP32 n <= 1e6
 * with max_intervals <= 128, or FP64 n <= 2e5 with max_intervals <= 128.
 *   desc   host; validated as for tsne_plan_create (TSNE_E_ARG,
 *          TSNE_E_UNSUPPORTED); TSNE_E_WORKSPACE when
 *          tsne_workspace_bytes(desc with nnz = 0) exceeds the scratch size.
 *   Y      device [n, s], F_rep device [n, s] (written), both point-aligned
 *          (TSNE_E_ARG otherwise); Z device double (written) or NULL.
 *   stream hipStream_t or NULL.
 * Every call re-initialises the scratch of the current device (geometry,
 * counters, kernel spectra; the initialisation synchronises the stream), so
 * no state carries over from an earlier call.  Calls on one GPU share that
 * GPU's scratch: calls that overlap on one device (two host threads, or two
 * streams whose work is still in flight) race and give undefined results.
 * Device conditions (TSNE_E_CAPACITY, TSNE_E_NONFINITE) latched by a call
 * leave F_rep and Z unwritten; they are not reported (there is no plan to
 * query), so a caller that needs them uses tsne_repulsive. */
tsne_status tsne_repulsive_static(const tsne_desc* desc, const void* Y, void* F_rep, double* Z,
                                  void* stream);

/* ---------------------------------------------------------------------- */
/* Input affinities (Section 1.1) over the k nearest neighbours (Section 3) */
/* ---------------------------------------------------------------------- */

/* Exact k nearest neighbours of every row of X [n, dim] (row-major FP32,
 * device): squared Euclidean distances accumulated in FP32 over the
 * coordinate differences, the point itself excluded, equal distances ordered
 * by index.  idx [n, k] int32 and dist2 [n, k] FP32 (device, caller-owned)
 * receive each row's neighbours in ascending distance.  1 <= k < n,
 * k <= 256 (TSNE_E_UNSUPPORTED above); n < 2^31.  Enqueued on stream; no
 * workspace. */
tsne_status tsne_knn(const float* X, int64_t n, int32_t dim, int32_t k, int32_t* idx, float* dist2,
                     void* stream);

/* Conditional affinities p_{j|i} = exp(-beta_i d_ij) / sum_l exp(-beta_i d_il)
 * over the k neighbour distances of each row (dist2 [n, k] FP32, device), with
 * beta_i = 1 / (2 sigma_i^2) found by bisection in FP64 so that the
 * perplexity exp(-sum p ln p) equals the target: distances shifted by the row
 * minimum, doubling or halving beta until the target is bracketed, then
 * halving the bracket, until the entropy is within 1e-10 of ln(perplexity)
 * or after 200 steps.  p [n, k] FP32 (device); beta [n] FP64 (device, may be
 * NULL).  k <= 128. */
tsne_status tsne_perplexity(const float* dist2, int64_t n, int32_t k, double perplexity, float* p,
                            double* beta, void* stream);

/* Workspace bytes of tsne_symmetrize (0 for invalid sizes). */
size_t tsne_symmetrize_workspace_bytes(int64_t n, int32_t k);

/* Joint affinities p_ij = (p_{j|i} + p_{i|j}) / (2N) (Section 1.1) from the
 * conditional rows idx [n, k], p [n, k] (device) as CSR for tsne_bind_P:
 * row_ptr [n+1] int64, col [<= 2nk] int32 ascending within each row, val
 * [<= 2nk] FP32 (device, caller-owned; nnz = row_ptr[n]).  Equal (row,
 * column) pairs are summed.  A row longer than 16384 entries (a point in
 * more than 16384 - k neighbour lists) is left empty and sets *status
 * (device int, may be NULL) to 1; otherwise *status is 0.  workspace: 256-byte
 * aligned, tsne_symmetrize_workspace_bytes(n, k) bytes. */
tsne_status tsne_symmetrize(const int32_t* idx, const float* p, int64_t n, int32_t k, void* workspace,
                            size_t bytes, void* stream, int64_t* row_ptr, int32_t* col, float* val,
                            int* status);

/* ---------------------------------------------------------------------- */
/* Batching: independent embeddings of uneven n sharing every launch.      */
/* ---------------------------------------------------------------------- */

/* A batch holds up to max_slots instances that have the same s, dtype, p and
 * form.  Each admitted job has its own plan workspace (tsne_workspace_bytes of
 * its descriptor) and its own n, nnz, capacity and grid; one tick runs one
 * iteration of every live slot with a single launch per kernel, each launch
 * covering every slot's work (per-slot grid sizes come from a device table). */
typedef struct tsne_batch tsne_batch;

/* Workspace for the batch's own tables (bytes). */
size_t tsne_batch_workspace_bytes(int32_t max_slots);

/* lanes_per_row: CSR lanes per row of the shared attraction launch (0 = 32,
 * else 4, 8, 16, 32 or 64); admitted descriptors must leave it 0 or match.  The
 * attraction of a batch always uses the CSR layout with one column slab. */
tsne_status tsne_batch_create(int32_t max_slots, int32_t s, int32_t dtype, int32_t p,
                              int32_t form, int32_t lanes_per_row, void* workspace,
                              size_t bytes, void* stream, tsne_batch** out);
tsne_status tsne_batch_destroy(tsne_batch* batch);

/* Admit a job into a free slot.  The job runs iterations [iter0, iter0+n_iter)
 * of sched on Y, uY, gains with the bound CSR P.  plan_ws is the job's plan
 * workspace.  *slot receives the slot index. */
tsne_status tsne_batch_admit(tsne_batch* batch, const tsne_desc* desc, void* plan_ws,
                             size_t plan_ws_bytes, void* Y, void* uY, void* gains,
                             const int64_t* row_ptr, const int32_t* col, const void* val,
                             const tsne_sched* sched, int32_t iter0, int32_t n_iter,
                             int32_t* slot);

/* Run n_ticks iterations of every live slot (a slot that has finished its
 * n_iter iterations is skipped on the device).  Replays a captured graph of
 * one tick when the set of slots is unchanged. */
tsne_status tsne_batch_tick(tsne_batch* batch, int32_t n_ticks);

/* Synchronise and report a slot: iterations done and latched status. */
tsne_status tsne_batch_poll(tsne_batch* batch, int32_t slot, int32_t* iters_done,
                            int32_t* status);

/* Free a slot (its buffers belong to the caller). */
tsne_status tsne_batch_retire(tsne_batch* batch, int32_t slot);

#ifdef __cplusplus
}
#endif

#endif /* TSNE_MI355X_H */
