/*
 * dp.h -- C ABI of libdpse: Deep Potential smooth-edition (se_a) energy,
 * forces and virial on one AMD Instinct MI355X (gfx950).
 *
 * The operation (Background section, DeePMD-kit subsection, Fig. 1): for each
 * atom i, a neighbour list within the cut-off r_c; the environment matrix R_i
 * whose smoothed first column s(r) feeds the per-type-pair embedding net G;
 * the descriptor D_i = (G^T R)(R^T G<); the per-type fitting net giving E_i;
 * E = sum_i E_i; forces F_i = -dE/dx_i by back-propagation; the virial.
 * Precision modes follow the Computation Optimization section (mixed
 * precision subsection): FP64 everywhere, or the embedding and fitting GEMMs
 * on low-precision matrix cores with FP32 accumulation while the environment
 * matrix, force/virial accumulation and integrator stay FP64.
 *
 * Conventions
 *   units      metal: Angstrom, eV, eV/Angstrom, amu, fs; virial in eV.
 *   coords     [n, 3] float64, device, atom-major, wrapped into [0, L_d) when
 *              a neighbour list is built.
 *   types      [n] int32, device, values in [0, ntypes).
 *   box        [9] float64, HOST, row vectors; must be diagonal
 *              (orthorhombic) with r_c < every edge.
 *   nlist      [n, nm] int32, device, nm = sum(sel).  Slots are split into
 *              ntypes sections of sel[t] slots (neighbours of type t), each
 *              sorted by (r^2, packed) ascending and padded with -1.  An entry
 *              is packed = 27*j + (sx+1) + 3*(sy+1) + 9*(sz+1): neighbour atom j
 *              (global index in a batch) seen through image shift (sx,sy,sz)
 *              in {-1,0,1}^3, i.e. d_ij = x_j + s*L - x_i.
 *   streams    every call is asynchronous on the given hipStream_t (0 = the
 *              null stream).  Output buffers are owned by the caller and must
 *              stay valid until the stream reaches the call.  One context may
 *              be used by one stream at a time; calls are not thread-safe per
 *              context.
 *   errors     functions return DP_OK (0) or a negative DP_ERR_* code and set
 *              a thread-local message readable with dp_last_error().  Host
 *              argument checks run before any GPU work is queued.  Conditions
 *              only the device can see (capacity, r = 0, non-finite energy,
 *              unwrapped coordinates) set bits in a device status word read
 *              by dp_ctx_status().
 *   memory     all device memory is allocated by dp_model_create,
 *              dp_model_compress and dp_ctx_create (set-up calls); no other
 *              call allocates (Computation Optimization section: memory is
 *              allocated at start-up).
 */
#ifndef DPSE_DP_H
#define DPSE_DP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DP_MAX_TYPES 4
#define DP_MAX_LAYERS 4

/* Return codes */
#define DP_OK 0
#define DP_ERR_BAD_ARG -1      /* null pointer, size out of range, bad descriptor */
#define DP_ERR_UNSUPPORTED -2  /* model shape or box the kernels do not implement */
#define DP_ERR_CAPACITY -3     /* n above the context's max_atoms / frames, etc. */
#define DP_ERR_NOT_WRAPPED -4  /* coordinates outside [0, L) (device flag) */
#define DP_ERR_OVERLAP -5      /* two atoms at distance 0 (device flag) */
#define DP_ERR_NONFINITE -6    /* non-finite energy (device flag) */
#define DP_ERR_HIP -7          /* a HIP runtime call failed */
#define DP_ERR_STATE -8        /* call order (e.g. backward without compute) */

/* Device status bits (dp_ctx_status) */
#define DP_FLAG_NOT_WRAPPED 1
#define DP_FLAG_OVERLAP 2
#define DP_FLAG_NONFINITE 4
/* DP_FLAG_CAND_CAPACITY: more pairs than the per-atom capacity (512 within
 * r_c + skin for a Verlet build; within r_c, 256 when sum(sel) <= 256, else
 * 512). */
#define DP_FLAG_CAND_CAPACITY 8
#define DP_FLAG_SEL_OVERFLOW 16 /* some section had more neighbours than sel (truncated) */
#define DP_FLAG_BAD_INPUT 32    /* a type outside [0, ntypes) or a neighbour index >= n (ignored) */
#define DP_FLAG_SKIN_EXCEEDED 64 /* an atom moved more than skin/2 since the Verlet build (list may miss pairs) */
#define DP_FLAG_TABLE_RANGE 128  /* DP_FP64_TAB: an embedding input at or beyond the table's end (value held) */

/* Precision modes (Computation Optimization section, mixed precision) */
#define DP_FP64 0     /* everything in FP64 */
#define DP_MIX_BF16 1 /* embedding layers 2.. and fitting GEMMs: BF16 inputs, FP32 accumulate */
#define DP_MIX_FP16 2 /* same with FP16 inputs */
/* The paper's own recipes (Evaluation section, accuracy: "MIX-fp32" and
 * "MIX-fp16"; Computation Optimization section, mixed precision): */
#define DP_MIX_FP32 3      /* embedding and fitting nets in FP32 (FP32 matrix-core products, FP32 tanh) */
#define DP_MIX_FP16_FIT1 4 /* as DP_MIX_FP32, with the first fitting layer's products in FP16 */
/* FP64 with the embedding nets evaluated from the DP-compress table of
 * dp_model_compress (Background section: the compression of the embedding
 * net); energies, forces and virial only (no dp_backward_params). */
#define DP_FP64_TAB 5

/* Model hyper-parameters (Evaluation section: cut-offs, sel, fitting widths).
 *   emb[0..n_emb)  embedding widths, input width 1; layer l adds an identity
 *                  skip when its width equals (or doubles, by concatenation)
 *                  the previous width.
 *   fit[0..n_fit)  fitting widths; same skip rule; a linear output follows.
 *   m2             axis neurons: D_i has emb[n_emb-1] * m2 entries.
 *   std_s, std_v   the environment matrix is divided column-wise by std_s
 *                  (radial column) and std_v (three vector columns); its
 *                  mean is fixed at 0.
 *   masses         per type, amu (used by the integrator entry points).
 * Implemented shapes: n_emb = 3 with widths (w, 2w, 4w), w <= 32, m2 = 16;
 * n_fit = 3 equal widths, a multiple of 16 and <= 256; ntypes <= 4;
 * sum(sel) <= 1024.  Others return DP_ERR_UNSUPPORTED. */
typedef struct dp_model_desc {
  int32_t ntypes;
  int32_t sel[DP_MAX_TYPES];
  int32_t n_emb;
  int32_t emb[DP_MAX_LAYERS];
  int32_t m2;
  int32_t n_fit;
  int32_t fit[DP_MAX_LAYERS];
  double rcut;
  double rcut_smth;
  double std_s;
  double std_v;
  double masses[DP_MAX_TYPES];
} dp_model_desc;

typedef struct dp_model dp_model;
typedef struct dp_ctx dp_ctx;

/* Number of FP64 parameters of the flat layout for this descriptor, or a
 * negative error.  Layout: embedding nets for (t_i, t_j) in row-major order,
 * each W_1 [1 x w_1], b_1, W_2 [w_1 x w_2], b_2, ... (row-major); then per
 * centre type the fitting net W_1 [nd x f_1], b_1, ..., w_out [f_L], b_out;
 * then e_bias [ntypes]. */
int64_t dp_model_n_params(const dp_model_desc* desc);

/* Copies the parameters (host, FP64) to the device and derives the
 * pre-arranged matrix-core operand copies of every weight matrix: the
 * forward and the transposed (backward) forms, in FP64, BF16 and FP16
 * (Computation Optimization section: the transpose is prepared once at
 * start-up so that no transposed product runs in the step). */
int dp_model_create(const dp_model_desc* desc, const double* params_host, int64_t n_params, dp_model** out);
/* Replaces the parameters of an existing model (same descriptor), host
 * FP64 values checked finite (DP_ERR_BAD_ARG otherwise).  The operand copies
 * are re-derived on the device by gathers through index maps built at
 * creation; nothing is allocated.  Runs on the null stream and returns when
 * the model is updated; computes using the model on other streams must not
 * be in flight. */
int dp_model_set_params(dp_model* model, const double* params_host, int64_t n_params);
/* The same from device FP64 parameters [n_params], asynchronously on
 * `stream` (a copy into the model, then the gathers): no allocation, no host
 * wait, so a training loop can update the model every step.  Values are not
 * checked on the host; non-finite parameters give non-finite energies, which
 * the computes flag with DP_FLAG_NONFINITE. */
int dp_model_set_params_device(dp_model* model, const double* params_dev, int64_t n_params, hipStream_t stream);
int dp_model_destroy(dp_model* model);

/* DP-compress (Background section: the compression of the embedding net):
 * tabulates every embedding net G(x) of its input x = R~[0] as piecewise
 * fifth-order polynomials that match G, dG/dx and d2G/dx2 at the ends of
 * each interval, on a fine stride h over [0, X1) and a coarse stride 10 h
 * over [X1, X2), where X1 = ceil(x_fine / h) h and X2 = X1 + ceil((x_max -
 * X1) / (10 h)) 10 h.  Inputs at or beyond X2 take the value at X2 (zero
 * slope) and raise DP_FLAG_TABLE_RANGE.  Computes with mode DP_FP64_TAB
 * use it; the table is rebuilt on the device from the parameters at every
 * dp_model_set_params[_device].  A set-up call: it allocates the table
 * (n_types^2 * n_intervals * 6 * m1 doubles) and waits for the build.
 * DP_ERR_BAD_ARG for h <= 0, x_fine <= 0, x_max < x_fine or more than
 * 10^6 intervals. */
int dp_model_compress(dp_model* model, double x_fine, double x_max, double h);
/* Copies the table (layout [t_i * ntypes + t_j][interval][power 0..5][m1
 * features], FP64) into dst (device, caller-owned) and writes its value
 * count to *n_values; with dst NULL only the count.  Waits for the copy.
 * DP_ERR_STATE when the model is not compressed. */
int dp_model_copy_table(const dp_model* model, double* dst, int64_t* n_values);

/* Allocates every work buffer for up to max_atoms atoms in up to max_frames
 * frames (Computation Optimization section: all memory is allocated in the
 * initial phase).  workspace_budget_bytes caps the embedding-activation store
 * (at most max_atoms * T * 16 * m1 * 8 bytes are taken, with T = sum over
 * neighbour types of ceil(sel_t / 16) row tiles per atom): a DP_FP64 compute
 * on n atoms keeps the last embedding layer's tanh output there when
 * n * T * 16 * m1 * 8 bytes fit, and otherwise (or with a budget of 0) the
 * backward pass recomputes it.  The mixed modes always recompute (their
 * half-precision layer costs less than the store's memory traffic). */
int dp_ctx_create(const dp_model* model, int64_t max_atoms, int32_t max_frames, int64_t workspace_budget_bytes,
                  dp_ctx** out);
int dp_ctx_destroy(dp_ctx* ctx);

/* Neighbour list of one frame (Background section, Fig. 1(a)): cell binning
 * with cells of edge >= r_c, a 27-cell stencil search with the strict test
 * r^2 < r_c^2 on r^2 = (dx*dx + dy*dy) + dz*dz evaluated without fused
 * multiply-add, per-type sections sorted by (r^2, packed), truncated to sel
 * and padded with -1.  Neighbours beyond sel are dropped and counted into
 * *n_overflow_out (device int32, written, not accumulated).
 * nlist_out: [n, nm] int32 device.  n may be 0. */
int dp_build_nlist(dp_ctx* ctx, const double* coords, const int32_t* types, const double* box, int64_t n,
                   int32_t* nlist_out, int32_t* n_overflow_out, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the neighbour
 * list of dp_build_nlist -- the same list, bit for bit -- with no context.
 * Its scratch (cell grid and counts, frame table, status word) is a static
 * device array of about 2 MB per GPU, held until the process ends; the call
 * allocates nothing, and the model only supplies r_c and sel.  Limits:
 * n <= 65536 atoms and at most 131072 cells (floor(L_d / r_c) per axis),
 * else DP_ERR_CAPACITY before any launch.  flags_out (device int32,
 * nullable) receives the call's DP_FLAG_* bits (written, not accumulated).
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (two streams, two threads) race and must be serialised by the
 * caller. */
int dp_build_nlist_noalloc(const dp_model* model, const double* coords, const int32_t* types, const double* box,
                           int64_t n, int32_t* nlist_out, int32_t* n_overflow_out, int32_t* flags_out,
                           hipStream_t stream);

/* Verlet (skin) list for MD (Evaluation section: the neighbour list is
 * rebuilt every 50 steps with a 2 A skin).
 * dp_nlist_skin_build first wraps coords [n, 3] (device f64, in place) into
 * [0, L) by whole box lengths, adding the lengths moved to images [n, 3]
 * (device int32, may be NULL), then keeps in the context every pair image
 * (j, s) with r^2 < (r_c + skin)^2 and the positions of the build.  Needs
 * r_c + skin below every box edge (DP_ERR_UNSUPPORTED).
 * dp_nlist_skin_format writes, from the current coords (not wrapped since
 * the build: r_ij keeps the image of the build), the list dp_build_nlist
 * defines: same cut-off test, order, truncation, padding and n_overflow_out
 * (device int32, written) -- exactly the list of all pairs within r_c while
 * no atom has moved more than skin/2 since the build; beyond that
 * DP_FLAG_SKIN_EXCEEDED is raised and pairs may be missing.  It also
 * prepares the reverse-entry index that dp_compute uses with this list.
 * DP_ERR_STATE when no build with the same n preceded on this context. */
int dp_nlist_skin_build(dp_ctx* ctx, double* coords, const int32_t* types, const double* box, int64_t n, double skin,
                        int32_t* images, hipStream_t stream);
int dp_nlist_skin_format(dp_ctx* ctx, const double* coords, const int32_t* types, int64_t n, int32_t* nlist_out,
                         int32_t* n_overflow_out, hipStream_t stream);

/* One MD step's list with the rebuild decided on the device (no host wait):
 * when some atom has moved more than skin/2 since the last Verlet build
 * (the condition under which the formatted list is exact), or when `every`
 * > 0 updates have passed since that build, the candidates are rebuilt in
 * place exactly as dp_nlist_skin_build does (coords wrapped in place, image
 * counters [n, 3] updated when images is non-NULL), with the skin and box of
 * the last dp_nlist_skin_build; then the list is formatted as
 * dp_nlist_skin_format does.  rebuild_count (device int32, nullable) is
 * incremented once per rebuild (accumulated, never cleared).  Types must be
 * those of that build.  DP_ERR_STATE when no build with the same n preceded
 * on this context. */
int dp_nlist_skin_update(dp_ctx* ctx, double* coords, const int32_t* types, int64_t n, int32_t every, int32_t* images,
                         int32_t* nlist_out, int32_t* n_overflow_out, int32_t* rebuild_count, hipStream_t stream);

/* Batched form: frames f = 0..B-1 hold atoms [frame_off[f], frame_off[f+1])
 * of coords/types; boxes [B, 9] and frame_off [B+1] are HOST arrays.  Entries
 * use global atom indices; atoms of different frames never neighbour. */
int dp_build_nlist_batch(dp_ctx* ctx, const double* coords, const int32_t* types, const double* boxes,
                         const int64_t* frame_off, int32_t nframes, int32_t* nlist_out, int32_t* n_overflow_out,
                         hipStream_t stream);

/* Energy, forces and virial of one frame from a neighbour list built for the
 * same atoms (Background section, Fig. 1(b)).
 *   energy      [1] device f64: E = sum_i E_i
 *   atom_energy [n] device f64 or NULL: E_i
 *   forces      [n, 3] device f64: F_i = -dE/dx_i (overwritten)
 *   virial      [9] device f64: W_ab = -sum_ij d_a (dE/dd)_b, row-major
 *   mode        DP_FP64, DP_MIX_BF16, DP_MIX_FP16, DP_MIX_FP32,
 *               DP_MIX_FP16_FIT1 or DP_FP64_TAB.
 * The list has the layout dp_build_nlist writes: per neighbour-type section
 * the real entries first, then -1 padding (entries after a section's padding
 * starts are not used).
 * Positions may drift from where the list was built; r_ij uses the stored
 * image shift.  The types must be the ones the list was built with (its
 * sections are by neighbour type): for a list built or formatted by this
 * context, the column order by type from the last sort is reused while the
 * types pointer, n and the frames are unchanged, so types changed in place
 * need a new list.  State for dp_backward_params is kept in the context. */
int dp_compute(dp_ctx* ctx, const double* coords, const int32_t* types, const double* box, int64_t n,
               const int32_t* nlist, int32_t mode, double* energy, double* atom_energy, double* forces,
               double* virial, hipStream_t stream);

/* Batched form (frames as in dp_build_nlist_batch): energies [B], forces
 * [N, 3], virials [B, 9], all device f64. */
int dp_compute_batch(dp_ctx* ctx, const double* coords, const int32_t* types, const double* boxes,
                     const int64_t* frame_off, int32_t nframes, const int32_t* nlist, int32_t mode,
                     double* energies, double* forces, double* virials, hipStream_t stream);

/* Parameter gradient of a loss L through the energies of the last
 * dp_compute / dp_compute_batch on this context: grad_params [n_params]
 * device f64 receives sum_f dL/dE_f * dE_f/dtheta (overwritten, flat layout
 * of dp_model_n_params), for dL_dE [B] device f64 (B = frames of that
 * compute), with the compute's inputs unchanged; DP_ERR_STATE if no compute
 * preceded.  After a mixed-precision compute the layer inputs, deltas and
 * g_T of its half-precision passes are used (widened to FP64 for the
 * weight-gradient reductions; the embedding nets are re-evaluated in FP64),
 * so the result is the mixed model's gradient to mixed-precision accuracy.
 * Gradients are accumulated with atomics (summation order not fixed). */
int dp_backward_params(dp_ctx* ctx, const double* dL_dE, double* grad_params, hipStream_t stream);

/* Velocity-Verlet halves (FP64; Evaluation section time steps).
 *   dp_md_kick_drift: v += dt/2 * F/m; x += dt * v; with wrap != 0, x is
 *                     wrapped into [0, L) (image counters [n,3] int32
 *                     updated when non-NULL); with wrap = 0 (between Verlet
 *                     builds) positions are left unwrapped and box may be NULL.
 *   dp_md_kick:       v += dt/2 * F/m; ke [1] device f64 = sum 1/2 m v^2 (eV).
 * dt in fs, v in Angstrom/fs, masses from the model descriptor. */
int dp_md_kick_drift(dp_ctx* ctx, double* coords, double* vel, const double* forces, const int32_t* types,
                     const double* box, int64_t n, double dt, int32_t wrap, int32_t* images, hipStream_t stream);
int dp_md_kick(dp_ctx* ctx, double* vel, const double* forces, const int32_t* types, int64_t n, double dt,
               double* ke, hipStream_t stream);

/* Device status word accumulated since the last call (DP_FLAG_*); waits for
 * the context's last stream, then clears the word. */
int dp_ctx_status(dp_ctx* ctx, int32_t* flags);

/* Embedding-activation store of the context (the budget given to
 * dp_ctx_create): *capacity_bytes receives its size (0 when the budget was 0),
 * *last_used 1 when the last dp_compute / dp_compute_batch kept the last
 * embedding layer's activations there instead of recomputing them in the
 * backward pass; 2 when that compute was a mixed-precision one and a
 * dp_backward_params after it filled the store (FP64 embedding forward of the
 * same frame) for its embedding-gradient pass to read; else 0.  Either
 * pointer may be NULL.  Host-only; no wait. */
int dp_ctx_store_info(dp_ctx* ctx, int64_t* capacity_bytes, int32_t* last_used);

/* Inspection of intermediate buffers of the last compute (tests, debugging).
 * which: 0 = environment matrix [n, nm, 4] f64 (atom order);
 *        1 = T [n, m1, 4] f64 (atom order; FP32 in mixed modes, widened);
 *        2 = descriptor D [n, m1*m2] f64 (atom order);
 *        3 = dE/dD [n, m1*m2] f64 (atom order);
 *        4 = net_deriv = dE/dR~ [n, nm, 4] f64 (atom order);
 *        5 = g_T = dE/dT [n, m1, 4] f64 (atom order; FP32 in mixed modes).
 * Where the compute folded D and dE/dD into the first fitting layer (the
 * BF16 / FP16 first layer on frames of many atoms) they are formed on
 * request from the compute's T and dz1 by the plain descriptor and GEMM
 * passes.  Copies into dst (device, caller-owned, at least the stated size)
 * on stream; *nbytes receives the size. */
int dp_ctx_copy_buffer(dp_ctx* ctx, int32_t which, void* dst, int64_t* nbytes, hipStream_t stream);

/* Opt-in per-stage timing with HIP events recorded on the call's stream
 * around the stages of dp_build_nlist / dp_nlist_skin_* / dp_compute / the
 * integrator.  stage_mask selects the stages timed (bit s for stage s, -1
 * for all); a non-zero mask allocates an event pool (setup call, not for
 * loops that forbid allocation), 0 releases it.  dp_ctx_stage_times waits
 * for the recorded events, adds their durations into total_ms[s] and
 * counts[s] (arrays of DP_NSTAGES, caller-owned, host) and clears the
 * record. */
#define DP_NSTAGES 12
#define DP_STAGE_NLIST 0
#define DP_STAGE_TYPESORT 1
#define DP_STAGE_ENV 2
#define DP_STAGE_EMBED_FWD 3
#define DP_STAGE_DESCRIPTOR 4
#define DP_STAGE_FIT_FWD 5
#define DP_STAGE_FIT_BWD 6
#define DP_STAGE_DESC_BWD 7
#define DP_STAGE_EMBED_BWD 8
#define DP_STAGE_FORCE 9
#define DP_STAGE_REDUCE 10
#define DP_STAGE_MD 11
int dp_ctx_profile(dp_ctx* ctx, int32_t stage_mask);
int dp_ctx_stage_times(dp_ctx* ctx, double* total_ms, int64_t* counts);

/* Message of the last error on this thread ("" if none). */
const char* dp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DPSE_DP_H */
