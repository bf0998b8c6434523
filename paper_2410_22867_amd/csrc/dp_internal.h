// Internal structures of libdpse shared by the host driver and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dp.h"

namespace dpse {

constexpr int kMaxT = DP_MAX_TYPES;
constexpr int kColPad = 128;     // fitting-GEMM column tile; type segments are padded to it
// Split-K form of the first fitting layer for frames with few atoms: at most
// kSplitMax partial sums over K ranges, for up to kSplitCols columns (plus
// the type segments' padding)
constexpr int kSplitMax = 16, kSplitCols = 2048;
constexpr int kCandCap = 512;    // neighbour candidates inside r_c per atom (LDS capacity)
constexpr int kMaxNm = 1024;     // sum(sel)
constexpr int kRedChunk = 256;  // atoms per partial sum of the per-frame reductions

// Slot layout of the embedding activations (see k_embed.hip): widths
// (w, 2w, 4w) with w <= 32 occupy 32, 64 and 128 slots.
constexpr int kP1 = 32, kP2 = 64, kP3 = 128;

// Per-frame table (device).
struct FrameInfo {
  int32_t atom_off;   // first atom
  int32_t natoms;
  int32_t cell_off;   // first cell of the frame's grid
  int32_t chunk_off;  // first reduction chunk of the frame (chunks of kRedChunk atoms)
  int32_t ncell[3];
  double L[3];        // orthorhombic edges
};

// Fragment-arranged weights of one embedding net in one precision.
// Element counts (per net) for every precision:
//   F2   : fwd layer 2 (T layout)        4 ot x 32 in-slots  x 16 = 2048
//   F3n  : fwd layer 3, rows as M        n3 ot x 64 in-slots x 16 (n3 = m1/16 rounded up)
//   F3t  : fwd layer 3 (T layout)        8 ot x 64 x 16 = 8192
//   B3   : bwd dh2 = W3 dz3              4 it x 128 x 16 = 8192
//   B2   : bwd dh1 = W2 dz2              2 it x 64 x 16 = 2048
struct EmbFragOffsets {
  int64_t F2, F3n, F3t, B3, B2, per_net;
};

// Fitting-net fragments per centre type: forward layer l uses W_l^T
// (out x in), backward uses W_l (in x out).  Offsets in elements.
struct FitFragOffsets {
  int64_t fwd[3], bwd[3], per_type;
};

// One device copy of the parameters: dst[k] = P[idx[k]] (0 where
// idx[k] < 0) in precision kind (0 f64, 1 f32, 2 bf16, 3 f16).
struct ParamMap {
  int32_t* idx;          // owned map (NULL when shared with an earlier entry)
  const int32_t* idx_use;
  int64_t n;
  int kind;
  void* dst;
};

// DP-compress grid (see k_tab.hip): fine stride h on [0, X1) with n1
// intervals, coarse stride H = 10 h on [X1, X2) with n2 intervals.
struct TabGrid {
  double h, H, X1, X2;
  int n1, n2, nint;
};
// Flat-parameter offsets of each embedding net's W_l and b_l.
struct TabNetOffsets {
  int64_t W[kMaxT * kMaxT][3], b[kMaxT * kMaxT][3];
};

// Element kinds of the matrix stages of a mixed mode (1 BF16, 2 FP16,
// 3 FP32): the embedding nets, the first fitting layer (forward GEMM and
// its backward GEMM, hence D and dz1), the fitting layer pairs 2-3.
struct MixKinds {
  int emb, fit1, fit23;
};
inline MixKinds mix_kinds(int mode) {
  switch (mode) {
    case DP_MIX_BF16: return {1, 1, 1};
    case DP_MIX_FP16: return {2, 2, 2};
    case DP_MIX_FP32: return {3, 3, 3};
    default: return {3, 2, 3};  // DP_MIX_FP16_FIT1
  }
}
template <class T16, class T32>
inline const void* frag_of(const T16* bf, const T16* hf, const T32* f32, int kind) {
  return kind == 1 ? (const void*)bf : (kind == 2 ? (const void*)hf : (const void*)f32);
}

}  // namespace dpse

struct dp_model {
  dp_model_desc desc;
  int nm;
  int sec[DP_MAX_TYPES + 1];
  int w1;          // first embedding width (25 or 32 ...)
  int m1;          // last embedding width
  int n3;          // m-tiles of m1
  int tpa;         // 16-row neighbour tiles per atom: sum_t ceil(sel_t / 16)
  int toff[DP_MAX_TYPES + 1];  // first tile of each neighbour section
  int nd;          // m1 * m2
  int fw;          // fitting width
  int64_t n_params;
  // device buffers
  double* params;            // flat FP64 copy
  // embedding small vectors per net (FP64 and FP32 copies), slot/feature mapped:
  //   W1s[32], b1s[32], b2s[64], b3s[128] (slot order), b3f[128] (feature order)
  double* emb_vec64;
  float* emb_vec32;
  int64_t emb_vec_per_net;   // = 32+32+64+128+128
  double* emb_frag64;
  // the FP64 force kernels' copies in the denser width-2w layout (w = 25;
  // the same as the plain ones otherwise); the gradient kernels and the
  // mixed kernels use the plain layout
  double* emb_vec64d;
  double* emb_frag64d;
  uint16_t* emb_frag_bf16;
  uint16_t* emb_frag_f16;
  float* emb_frag_f32;
  dpse::EmbFragOffsets efo;
  // fitting
  double* fit_frag64;
  uint16_t* fit_frag_bf16;
  uint16_t* fit_frag_f16;
  float* fit_frag_f32;
  dpse::FitFragOffsets ffo;     // FP64 fragment offsets
  dpse::FitFragOffsets ffo_lp;  // BF16/FP16 fragment offsets (K padded to 32)
  // flat-parameter offsets used by the gradient kernels
  int64_t emb_param_off[DP_MAX_TYPES * DP_MAX_TYPES][6];  // W1 b1 W2 b2 W3 b3 per net
  int64_t fit_param_off[8];   // type 0: W1 W2 W3 b1 b2 b3 w_out b_out
  int64_t fit_param_stride;   // parameters per fitting net
  int64_t ebias_off;
  double* fit_vec64;   // per type: b1, b2, b3, wo [fw each], bo, ebias  (4*fw + 2)
  float* fit_vec32;
  int64_t fit_vec_per_type;
  // index maps of every copy above (built once at creation)
  dpse::ParamMap maps[16];
  int n_maps;
  // DP-compress table (dp_model_compress; NULL without): [nets][nint][6][m1]
  // quintic coefficients, rebuilt from params whenever they change
  double* table;
  double* tab_nodes;         // [nets][nint + 1][3][m1] node values, slopes, curvatures
  dpse::TabGrid tab_grid;
  dpse::TabNetOffsets tab_off;
  int device;
};

struct dp_ctx {
  const dp_model* model;
  int64_t max_atoms;
  int32_t max_frames;
  int64_t max_cols;
  int64_t max_cells;
  int device;
  // frame table
  dpse::FrameInfo* frames_dev;
  dpse::FrameInfo* frames_host;  // pinned staging
  dpse::FrameInfo* frames_prev;  // host copy of the table on the device
  int32_t nframes_dev;           // entries of that table (-1: none)
  int64_t frames_gen;            // bumped whenever the device table changes
  hipEvent_t frames_ev;
  bool frames_ev_pending;
  // inputs of the last type sort (column order), see type_sort()
  bool ts_valid;
  const int32_t* ts_types;
  int64_t ts_n;
  int32_t ts_nframes;
  int64_t ts_frames_gen;
  int32_t nframes_last;
  int64_t natoms_last;
  int32_t mode_last;
  bool have_state;
  bool train_h;   // a parameter-gradient pass has run on this context: computes keep h2, h3, dz2
  bool h_stored;  // the last compute stored h2, h3, dz2
  const int32_t* types_last;
  // status
  int32_t* flags_dev;
  int32_t* flags_host;  // pinned
  hipStream_t last_stream;
  // nlist scratch
  int32_t* cell_of;
  int32_t* cell_count;
  int32_t* cell_start;
  int32_t* cell_fill;
  int32_t* cell_atoms;
  // type sort
  int32_t* chunk_counts;   // [nchunks * kMaxT]
  int32_t* type_meta;      // [2*kMaxT]: n_t, cbase_t
  int32_t* col_of;         // [max_atoms]
  int32_t* atom_at;        // [max_cols]
  int32_t* frame_of;       // [max_atoms]
  int32_t ncu;             // compute units of the device
  int32_t* emb_ctr;        // [nets][3 ncu][32] next-column counter of each embedding work-group (one per 128-byte line)
  // compute buffers
  double* R;               // [N, nm, 4] f64
  int32_t* nnei;           // [N, kMaxT]
  void* Tpart;             // [ntypes, cols, m1, 4] f64 / f32 (per neighbour section)
  void* T;                 // [cols, m1, 4]   f64 / f32
  void* D;                 // [cols, nd]      f64 / lp
  void* dD;                // [cols, nd]      f64 / f32
  void* gT;                // [cols, m1, 4]   f64 / f32
  // fitting activations [cols, fw]
  void* fa[12];
  double* split_part;   // [kSplitMax][split_cols][fw] partial sums (FP64, or FP32 in the same bytes)
  int64_t split_cols;
  double* Ei_col;          // [cols]
  double* Ei_atom;         // [N]
  double* netd;            // [N, nm, 4] f64
  int32_t* rev;            // [N, nm] reverse-entry index of the list in use
  // Verlet (skin) list of the last dp_nlist_skin_build
  int32_t* skin_cand;      // [N, kCandCap] packed candidates, sorted by packed value
  int32_t* skin_ncand;     // [N]
  int32_t* skin_crev;      // [N, kCandCap] position of the reverse pair in j's candidates (-1: absent)
  int32_t* skin_slot;      // [N, kCandCap] list entry i*nm + q of the candidate after the last format (-1)
  int32_t* skin_cof;       // [N, nm] candidate behind each list slot
  double* skin_xref;       // [N, 3] positions at the build
  double skin_L[3];
  double skin;
  int64_t skin_n;          // atoms of the build (-1: no build)
  int32_t skin_ncells;     // cells of the build's grid (edge >= r_c + skin)
  dpse::FrameInfo* skin_frame;  // [1] frame table of the build (device)
  int32_t* skin_gate;      // [2] rebuild decided by the device, formats since the build (inside ovf_ctr)
  // last embedding layer's tanh output per 16-row neighbour tile, [N, tpa,
  // m1, 16] f64 (FP64) or f32 (mixed), when it fits the workspace budget
  void* act;
  int64_t act_bytes;
  bool act_used_last;
  bool grad_act;       // act holds the FP64 records of the last compute's frame, written by the gradient pass
  const int32_t* rev_list; // neighbour list rev was built for (by dp_build_nlist on this ctx)
  int64_t natoms_rev;      // atom count of that build
  double* vatom;           // [N, 9]
  double* ke_part;         // [N/256 + 1] per-block kinetic energies
  int32_t* ovf_ctr;        // truncated neighbours counted by the Verlet format (moved out and reset by its second pass)
  int32_t* frame_ctr;      // [max_frames] chunk blocks of the frame reduction done (reset by the last)
  int32_t* ke_ctr;         // blocks of the kick that have written their partial (reset by the last)
  double* red_part;        // [chunks, 10] per-chunk energy + virial partial sums
  int32_t nchunks_last;
  // parameter-gradient scratch
  double* gE_col;          // [cols]
  double* grad_tmp;        // [n_params]
  double* gpart;           // partial sums of the parameter-gradient reductions
  int32_t grad_chunks;     // column chunks per type of the fitting reductions
  int32_t grad_slots;      // work-group records per net of the embedding reductions
  // opt-in stage timing
  hipEvent_t* prof_ev;     // [2 * prof_cap]
  int32_t* prof_stage;     // [prof_cap]
  int32_t prof_cap, prof_n;
  int32_t prof_mask;       // stages timed (bit s = stage s)
  double prof_ms[DP_NSTAGES];
  int64_t prof_cnt[DP_NSTAGES];
};

namespace dpse {

// Error plumbing
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// ---------------------------------------------------------------- launchers
// nlist
void launch_nl_bin(dp_ctx* c, const double* x, int32_t ntot, int32_t nframes, hipStream_t s);
void launch_nl_scan(dp_ctx* c, int32_t ncells, hipStream_t s);
void launch_nl_scatter(dp_ctx* c, int32_t ntot, hipStream_t s);
void launch_nl_search(dp_ctx* c, const double* x, const int32_t* types, int32_t ntot, int32_t nframes,
                      int32_t* nlist, int32_t* overflow, hipStream_t s);
void launch_nl_reverse(dp_ctx* c, const double* x, const int32_t* types, const int32_t* nlist, int32_t ntot,
                       hipStream_t s);
// Verlet build: wraps x in place (image counters when non-NULL), bins on the
// build's grid and keeps the candidates within r_c + skin.
void launch_nl_skin_build(dp_ctx* c, double* x, const int32_t* types, int32_t ntot, int32_t ncells, int32_t* images,
                          hipStream_t s);
// Verlet update: the same build, run only when the device finds an atom
// moved more than skin/2 since the last build or `every` updates passed.
void launch_nl_skin_update(dp_ctx* c, double* x, const int32_t* types, int32_t ntot, int32_t every, int32_t* images,
                           int32_t* rebuilds, hipStream_t s);
void launch_nl_skin_format(dp_ctx* c, const double* x, const int32_t* types, int32_t ntot, int32_t* nlist,
                           int32_t* overflow, hipStream_t s);
// small utilities
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
void launch_copy_i32(const int32_t* a, int32_t* b, int64_t n, hipStream_t s);
// dst[k] = P[idx[k]] (0 where idx[k] < 0) converted to kind (0 f64, 1 f32,
// 2 bf16, 3 f16; the half forms round through FP32, to nearest even)
void launch_param_gather(const double* P, const int32_t* idx, int64_t n, int kind, void* dst, hipStream_t s);
// writes one frame-table entry and clears a status word (kernel arguments
// only: no host staging buffer)
void launch_set_frame(FrameInfo* dst, const FrameInfo& F, int32_t* flags, hipStream_t s);
void launch_type_sort(dp_ctx* c, const int32_t* types, int32_t ntot, int32_t nframes, hipStream_t s);
// compute
void launch_env(dp_ctx* c, const double* x, const int32_t* types, const int32_t* nlist, int32_t ntot, double* forces,
                hipStream_t s);
void launch_embed_fwd(dp_ctx* c, const int32_t* types, int32_t mode, hipStream_t s);
void launch_descriptor(dp_ctx* c, int32_t mode, hipStream_t s);
void launch_descriptor_ex(dp_ctx* c, int32_t mode, bool write_d, hipStream_t s);
void launch_fit_forward(dp_ctx* c, int32_t mode, bool keep_h, hipStream_t s);
void launch_fit_backward(dp_ctx* c, int32_t mode, bool keep_dz2, hipStream_t s);
void launch_desc_bwd(dp_ctx* c, int32_t mode, hipStream_t s);
bool fit1_fused(const dp_ctx* c, int32_t mode);
void launch_fit1_bwd_gemm(dp_ctx* c, int32_t mode, hipStream_t s);
void launch_embed_bwd(dp_ctx* c, const int32_t* types, int32_t mode, hipStream_t s);
// DP-compress: table from the model's parameters; tabulated embedding
// forward (T sections) or backward (net_deriv) of the FP64 path
void launch_tab_build(const dp_model* m, hipStream_t s);
void launch_embed_tab(dp_ctx* c, bool bwd, hipStream_t s);
void launch_force(dp_ctx* c, const double* x, const int32_t* nlist, int32_t ntot, double* forces, hipStream_t s);
void launch_frame_reduce(dp_ctx* c, int32_t nframes, double* energies, double* atom_energy, double* virials,
                         hipStream_t s);
// md
void launch_kick_drift(dp_ctx* c, double* x, double* v, const double* f, const int32_t* types, int32_t n,
                       double dt, const double* L, int32_t* images, hipStream_t s);
void launch_wrap(dp_ctx* c, double* x, int32_t n, const double L[3], int32_t* images, hipStream_t s);
void launch_kick(dp_ctx* c, double* v, const double* f, const int32_t* types, int32_t n, double dt, double* ke,
                 hipStream_t s);
// parameter gradients from the state of the last compute, in FP64: the layer
// inputs X_l and deltas dz_l of the fitting net (columns, leading dims ldx/ldz)
// and g_T; FP64 computes pass their own buffers, mixed ones widened copies
struct ParamGradInputs {
  const double* X[3];
  int ldx[3];
  const double* dz[3];
  const double* h3;
  int ldz;
  const double* gT;
};
void launch_param_grads(dp_ctx* c, const ParamGradInputs& in, const double* dLdE, double* grad, hipStream_t s);
// widens a [rows][width] block of FP32 (kind 0), BF16 (1) or FP16 (2) values
void launch_widen(const void* src, int kind, int ld_src, double* dst, int ld_dst, int width, int64_t rows,
                  hipStream_t s);
// inspection
void launch_gather_cols(dp_ctx* c, int32_t which, int32_t mode, int32_t ntot, double* dst, hipStream_t s);

}  // namespace dpse
