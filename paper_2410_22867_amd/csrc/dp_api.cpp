// Host side of libdpse: argument validation, model preparation (weight
// fragments), context allocation and the launch sequences behind the C ABI
// declared in include/dp.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "dp_internal.h"

using namespace dpse;

namespace dpse {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return DP_ERR_HIP;
}

}  // namespace dpse

#define HIPCHECK(x)                            \
  do {                                         \
    hipError_t e_ = (x);                       \
    if (e_ != hipSuccess) return hip_fail(e_, #x); \
  } while (0)

namespace {

// ------------------------------------------------------------ descriptor
int validate_desc(const dp_model_desc* d) {
  if (!d) { set_error("desc is NULL"); return DP_ERR_BAD_ARG; }
  if (d->ntypes < 1 || d->ntypes > DP_MAX_TYPES) { set_error("ntypes %d out of [1,%d]", d->ntypes, DP_MAX_TYPES); return DP_ERR_BAD_ARG; }
  int nm = 0;
  for (int t = 0; t < d->ntypes; ++t) {
    if (d->sel[t] < 1) { set_error("sel[%d] = %d must be >= 1", t, d->sel[t]); return DP_ERR_BAD_ARG; }
    nm += d->sel[t];
  }
  if (d->n_emb < 1 || d->n_emb > DP_MAX_LAYERS || d->n_fit < 1 || d->n_fit > DP_MAX_LAYERS) {
    set_error("layer counts out of range"); return DP_ERR_BAD_ARG;
  }
  for (int l = 0; l < d->n_emb; ++l) if (d->emb[l] < 1) { set_error("emb width < 1"); return DP_ERR_BAD_ARG; }
  for (int l = 0; l < d->n_fit; ++l) if (d->fit[l] < 1) { set_error("fit width < 1"); return DP_ERR_BAD_ARG; }
  if (d->m2 < 1 || d->m2 > d->emb[d->n_emb - 1]) { set_error("m2 out of range"); return DP_ERR_BAD_ARG; }
  if (!(d->rcut > 0) || !(d->rcut_smth >= 0) || !(d->rcut_smth < d->rcut)) { set_error("need 0 <= rcut_smth < rcut"); return DP_ERR_BAD_ARG; }
  if (!(d->std_s > 0) || !(d->std_v > 0)) { set_error("std_s, std_v must be > 0"); return DP_ERR_BAD_ARG; }
  // shapes the kernels implement
  const int w = d->emb[0];
  if (d->n_emb != 3 || !(w == 25 || w == 32) || d->emb[1] != 2 * w || d->emb[2] != 4 * w) {
    set_error("embedding widths must be (w, 2w, 4w) with w in {25, 32}"); return DP_ERR_UNSUPPORTED;
  }
  if (d->m2 != 16) { set_error("m2 must be 16"); return DP_ERR_UNSUPPORTED; }
  if (d->n_fit != 3 || d->fit[1] != d->fit[0] || d->fit[2] != d->fit[0] || d->fit[0] % 16 || d->fit[0] > 256) {
    set_error("fitting widths must be three equal multiples of 16 <= 256"); return DP_ERR_UNSUPPORTED;
  }
  if (nm > kMaxNm) { set_error("sum(sel) = %d exceeds %d", nm, kMaxNm); return DP_ERR_UNSUPPORTED; }
  for (int t = 0; t < d->ntypes; ++t)
    if (!(d->masses[t] > 0)) { set_error("masses must be > 0"); return DP_ERR_BAD_ARG; }
  return DP_OK;
}

struct ParamLayout {
  int64_t embW[kMaxT][kMaxT][DP_MAX_LAYERS], embB[kMaxT][kMaxT][DP_MAX_LAYERS];
  int64_t fitW[kMaxT][DP_MAX_LAYERS], fitB[kMaxT][DP_MAX_LAYERS], wo[kMaxT], bo[kMaxT], ebias;
  int64_t total;
};

ParamLayout layout_of(const dp_model_desc* d) {
  ParamLayout L;
  memset(&L, 0, sizeof(L));
  int64_t off = 0;
  for (int a = 0; a < d->ntypes; ++a)
    for (int b = 0; b < d->ntypes; ++b) {
      int prev = 1;
      for (int l = 0; l < d->n_emb; ++l) {
        L.embW[a][b][l] = off; off += (int64_t)prev * d->emb[l];
        L.embB[a][b][l] = off; off += d->emb[l];
        prev = d->emb[l];
      }
    }
  const int nd = d->emb[d->n_emb - 1] * d->m2;
  for (int t = 0; t < d->ntypes; ++t) {
    int prev = nd;
    for (int l = 0; l < d->n_fit; ++l) {
      L.fitW[t][l] = off; off += (int64_t)prev * d->fit[l];
      L.fitB[t][l] = off; off += d->fit[l];
      prev = d->fit[l];
    }
    L.wo[t] = off; off += prev;
    L.bo[t] = off; off += 1;
  }
  L.ebias = off; off += d->ntypes;
  L.total = off;
  return L;
}

template <typename T>
int dev_alloc(T** p, size_t count, const char* what) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return hip_fail(e, what);
  return DP_OK;
}

// Slot maps of the embedding activations (widths w, 2w, 4w).
int feat1(int w, int p) { return p < w ? p : -1; }
int feat2(int w, int p) { return (p & 31) < w ? (p >> 5) * w + (p & 31) : -1; }
int feat3(int w, int p) {
  const int f = feat2(w, p & 63);
  return f < 0 ? -1 : (p >> 6) * 2 * w + f;
}

// Slot order of the half-precision kernels, whose lane group g holds slots
// 16t + 4g + v of tile t in element v: for w <= 28 the layer-1 slots
// 16 + 4g + 3 (g = 0..3) and their copies in the wider layers hold no
// feature, so that element 3 of every odd tile is padding in all four lane
// groups and the kernels skip its activation; the features fill the other
// slots in order.
int feat1h(int w, int p) {
  if (w > 28) return feat1(w, p);
  if (p >= 16 && (p & 3) == 3) return -1;
  const int f = p < 16 ? p : 16 + 3 * ((p - 16) >> 2) + ((p - 16) & 3);
  return f < w ? f : -1;
}
int feat2h(int w, int p) {
  const int f = feat1h(w, p & 31);
  return f < 0 ? -1 : (p >> 5) * w + f;
}
int feat3h(int w, int p) {
  const int f = feat2h(w, p & 63);
  return f < 0 ? -1 : (p >> 6) * 2 * w + f;
}

// Denser layout of the FP64 force kernels for w = 25 (the last feature of
// each half of the width-2w layer shares one k-step; slots 26, 27 are
// copies of features 24, 49 that feed nothing but the identity skip, and
// layer-1 slots 25..27 copies of layer-1 feature 24 that feed only those).
// val*: the feature whose value a slot carries; wt*: the feature whose
// outgoing weights it carries (-1 for padding and copies).
bool dense2(int w) { return w == 25; }
int val1(int w, int p) { return dense2(w) && p >= w && p < w + 3 ? w - 1 : feat1(w, p); }
int wt1(int w, int p) { return feat1(w, p); }
int val2(int w, int q) {
  if (!dense2(w)) return feat2(w, q);
  if (q >= w - 1 && q < w + 3) return ((q - (w - 1)) & 1) ? 2 * w - 1 : w - 1;
  if (q >= 32 + w - 1) return -1;
  return feat2(w, q);
}
int wt2(int w, int q) { return dense2(w) && (q == w + 1 || q == w + 2) ? -1 : val2(w, q); }
int val3(int w, int p) {
  if (!dense2(w)) return feat3(w, p);
  const int q = p & 63;
  if (q >= w - 1 && q < w + 3) return p < 64 ? (w - 1) + w * (q - (w - 1)) : -1;
  const int f = val2(w, q);
  return f < 0 ? -1 : (p >> 6) * 2 * w + f;
}

// Packed-index helpers of the two fragment kinds.
//   f64 16x16x4 : element (t, v, lane) with k-feature 16t + 4(lane/16) + v when
//                 the other operand is read from memory, 16t + 4v + lane/16
//                 when it is a register tile produced by the previous MFMA.
//   16x16x32    : element (t, lane, j) with k-feature 32t + 16(j/4) + 4(lane/16) + (j%4).
inline int kfeat64(int t, int v, int lane) { return 16 * t + 4 * (lane >> 4) + v; }       // memory-fed
inline int kfeat64c(int t, int v, int lane) { return 16 * t + 4 * v + (lane >> 4); }      // register-chained
inline int kfeat32(int t, int lane, int j) { return 32 * t + 16 * (j >> 2) + 4 * (lane >> 4) + (j & 3); }

// Builds one fragment block: out[mtile][ktile...] for a weight accessor
// wfun(m_index, k_index) -> value (0 when padded).  For f64 the k tiles are
// (t, v) pairs with ktiles16 = K/16; for lp they are t with ktiles32 = K/32.
// Register-chained f64 blocks (embedding nets, read from LDS one v at a time)
// are ordered [mt][t][v][lane]; memory-fed ones (fitting GEMMs, whose lanes
// read all four v of a step with one 32-byte load) [mt][t][lane][v].
template <class T, class F>
void frag_block64(std::vector<T>& out, int64_t base, int mtiles, int ktiles16, F wfun, bool chained) {
  for (int mt = 0; mt < mtiles; ++mt)
    for (int t = 0; t < ktiles16; ++t)
      for (int v = 0; v < 4; ++v)
        for (int l = 0; l < 64; ++l) {
          const int64_t tile = (int64_t)mt * ktiles16 + t;
          out[base + (chained ? (tile * 4 + v) * 64 + l : (tile * 64 + l) * 4 + v)] =
              wfun(16 * mt + (l & 15), chained ? kfeat64c(t, v, l) : kfeat64(t, v, l));
        }
}
template <class T, class F>
void frag_block32(std::vector<T>& out, int64_t base, int mtiles, int ktiles32, F wfun) {
  for (int mt = 0; mt < mtiles; ++mt)
    for (int t = 0; t < ktiles32; ++t)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 8; ++j)
          out[base + (((int64_t)mt * ktiles32 + t) * 64 + l) * 8 + j] = wfun(16 * mt + (l & 15), kfeat32(t, l, j));
}

template <class T>
int upload_vec(T** dst, const std::vector<T>& v, const char* what) {
  int rc;
  if ((rc = dev_alloc(dst, v.size(), what))) return rc;
  hipError_t e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, what);
  return DP_OK;
}

void free_model(dp_model* m) {
  if (!m) return;
  void* ptrs[] = {m->params, m->emb_vec64, m->emb_vec32, m->emb_frag64, m->emb_vec64d, m->emb_frag64d,
                  m->emb_frag_bf16, m->emb_frag_f16, m->emb_frag_f32,
                  m->fit_frag64, m->fit_frag_bf16, m->fit_frag_f16, m->fit_frag_f32, m->fit_vec64, m->fit_vec32,
                  m->table, m->tab_nodes};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int k = 0; k < m->n_maps; ++k)
    if (m->maps[k].idx) (void)hipFree(m->maps[k].idx);
  delete m;
}

// Every device copy of the parameters is a gather from the flat vector:
// element k of a copy holds P[idx[k]] (0 where idx[k] < 0) converted to the
// copy's precision.  The index maps depend only on the descriptor, so they
// are derived once here; dp_model_create and both parameter updates then run
// the same gathers on the device, with no allocation after creation.
int build_maps(dp_model* m) {
  const dp_model_desc& d = m->desc;
  const ParamLayout L = layout_of(&d);
  const int w = m->w1, nt = d.ntypes, fw = m->fw, nd = m->nd;
  const int nnets = nt * nt;
  int rc;
  // ---- flat-parameter offsets for the gradient kernels
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nt; ++b)
      for (int l = 0; l < 3; ++l) {
        m->emb_param_off[a * nt + b][2 * l] = L.embW[a][b][l];
        m->emb_param_off[a * nt + b][2 * l + 1] = L.embB[a][b][l];
      }
  for (int l = 0; l < 3; ++l) {
    m->fit_param_off[l] = L.fitW[0][l];
    m->fit_param_off[3 + l] = L.fitB[0][l];
  }
  m->fit_param_off[6] = L.wo[0];
  m->fit_param_off[7] = L.bo[0];
  m->fit_param_stride = nt > 1 ? L.fitW[1][0] - L.fitW[0][0] : 0;
  m->ebias_off = L.ebias;
  typedef std::vector<int32_t> Map;
  auto I = [](int64_t k) -> int32_t { return (int32_t)k; };
  // ---- embedding vectors, slot order (plain and denser layouts)
  m->emb_vec_per_net = 384;
  Map ev((size_t)nnets * 384, -1), evd((size_t)nnets * 384, -1), evh((size_t)nnets * 384, -1);
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nt; ++b) {
      int32_t* v = &ev[(size_t)(a * nt + b) * 384];
      int32_t* vd = &evd[(size_t)(a * nt + b) * 384];
      int32_t* vh = &evh[(size_t)(a * nt + b) * 384];
      for (int p = 0; p < 32; ++p) {
        int f = feat1(w, p);
        if (f >= 0) { v[p] = I(L.embW[a][b][0] + f); v[32 + p] = I(L.embB[a][b][0] + f); }
        f = val1(w, p);
        if (f >= 0) { vd[p] = I(L.embW[a][b][0] + f); vd[32 + p] = I(L.embB[a][b][0] + f); }
        f = feat1h(w, p);
        if (f >= 0) { vh[p] = I(L.embW[a][b][0] + f); vh[32 + p] = I(L.embB[a][b][0] + f); }
      }
      for (int p = 0; p < 64; ++p) {
        int f = feat2(w, p);
        if (f >= 0) v[64 + p] = I(L.embB[a][b][1] + f);
        f = val2(w, p);
        if (f >= 0) vd[64 + p] = I(L.embB[a][b][1] + f);
        f = feat2h(w, p);
        if (f >= 0) vh[64 + p] = I(L.embB[a][b][1] + f);
      }
      for (int p = 0; p < 128; ++p) {
        int f = feat3(w, p);
        if (f >= 0) v[128 + p] = I(L.embB[a][b][2] + f);
        f = val3(w, p);
        if (f >= 0) vd[128 + p] = I(L.embB[a][b][2] + f);
        f = feat3h(w, p);
        if (f >= 0) vh[128 + p] = I(L.embB[a][b][2] + f);
      }
      for (int f = 0; f < 4 * w; ++f) v[256 + f] = vd[256 + f] = vh[256 + f] = I(L.embB[a][b][2] + f);
    }
  // ---- embedding fragments (same element counts for both kinds)
  EmbFragOffsets& fo = m->efo;
  fo.F2 = 0;
  fo.F3n = fo.F2 + 2048;
  fo.F3t = fo.F3n + (int64_t)m->n3 * 1024;
  fo.B3 = fo.F3t + 8192;
  fo.B2 = fo.B3 + 8192;
  fo.per_net = fo.B2 + 2048;
  Map e64((size_t)nnets * fo.per_net, -1), e64d((size_t)nnets * fo.per_net, -1), e32((size_t)nnets * fo.per_net, -1);
  const int m1 = 4 * w;
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nt; ++b) {
      const int64_t W2 = L.embW[a][b][1];  // [w][2w]
      const int64_t W3 = L.embW[a][b][2];  // [2w][4w]
      const int64_t base = (int64_t)(a * nt + b) * fo.per_net;
      auto w2 = [&](int in_slot, int out_slot) -> int32_t {  // slots of layer 1 -> layer 2
        const int fi = feat1(w, in_slot), fo2 = feat2(w, out_slot);
        return (fi < 0 || fo2 < 0) ? -1 : I(W2 + (int64_t)fi * 2 * w + fo2);
      };
      auto w3s = [&](int in_slot, int out_slot) -> int32_t {  // layer-2 slot -> layer-3 slot
        if (in_slot >= 64 || out_slot >= 128) return -1;
        const int fi = feat2(w, in_slot), fo3 = feat3(w, out_slot);
        return (fi < 0 || fo3 < 0) ? -1 : I(W3 + (int64_t)fi * 4 * w + fo3);
      };
      auto w3f = [&](int in_slot, int out_feat) -> int32_t {  // layer-2 slot -> layer-3 feature
        const int fi = feat2(w, in_slot);
        return (fi < 0 || out_feat >= m1) ? -1 : I(W3 + (int64_t)fi * 4 * w + out_feat);
      };
      // the half-precision kernels' slot order
      auto w2h = [&](int in_slot, int out_slot) -> int32_t {
        const int fi = feat1h(w, in_slot), fo2 = feat2h(w, out_slot);
        return (fi < 0 || fo2 < 0) ? -1 : I(W2 + (int64_t)fi * 2 * w + fo2);
      };
      auto w3sh = [&](int in_slot, int out_slot) -> int32_t {
        if (in_slot >= 64 || out_slot >= 128) return -1;
        const int fi = feat2h(w, in_slot), fo3 = feat3h(w, out_slot);
        return (fi < 0 || fo3 < 0) ? -1 : I(W3 + (int64_t)fi * 4 * w + fo3);
      };
      auto w3fh = [&](int in_slot, int out_feat) -> int32_t {
        const int fi = feat2h(w, in_slot);
        return (fi < 0 || out_feat >= m1) ? -1 : I(W3 + (int64_t)fi * 4 * w + out_feat);
      };
      // the denser layout (FP64 force kernels)
      auto w2d = [&](int in_slot, int out_slot) -> int32_t {
        const int fi = wt1(w, in_slot), fo2 = val2(w, out_slot);
        return (fi < 0 || fo2 < 0) ? -1 : I(W2 + (int64_t)fi * 2 * w + fo2);
      };
      auto w3sd = [&](int in_slot, int out_slot) -> int32_t {
        if (in_slot >= 64 || out_slot >= 128) return -1;
        const int fi = wt2(w, in_slot), fo3 = val3(w, out_slot);
        return (fi < 0 || fo3 < 0) ? -1 : I(W3 + (int64_t)fi * 4 * w + fo3);
      };
      auto w3fd = [&](int in_slot, int out_feat) -> int32_t {
        const int fi = wt2(w, in_slot);
        return (fi < 0 || out_feat >= m1) ? -1 : I(W3 + (int64_t)fi * 4 * w + out_feat);
      };
      frag_block64(e64d, base + fo.F2, 4, 2, [&](int mo, int ki) { return w2d(ki, mo); }, true);
      frag_block64(e64d, base + fo.F3n, m->n3, 4, [&](int mo, int ki) { return w3fd(ki, mo); }, true);
      frag_block64(e64d, base + fo.F3t, 8, 4, [&](int mo, int ki) { return w3sd(ki, mo); }, true);
      frag_block64(e64d, base + fo.B3, 4, 8, [&](int mi, int ko) { return w3sd(mi, ko); }, true);
      frag_block64(e64d, base + fo.B2, 2, 4, [&](int mi, int ko) { return w2d(mi, ko); }, true);
      // forward (A operand W^T: m = out, k = in)
      frag_block64(e64, base + fo.F2, 4, 2, [&](int mo, int ki) { return w2(ki, mo); }, true);
      frag_block32(e32, base + fo.F2, 4, 1, [&](int mo, int ki) { return w2h(ki, mo); });
      frag_block64(e64, base + fo.F3n, m->n3, 4, [&](int mo, int ki) { return w3f(ki, mo); }, true);
      frag_block32(e32, base + fo.F3n, m->n3, 2, [&](int mo, int ki) { return w3fh(ki, mo); });
      frag_block64(e64, base + fo.F3t, 8, 4, [&](int mo, int ki) { return w3s(ki, mo); }, true);
      frag_block32(e32, base + fo.F3t, 8, 2, [&](int mo, int ki) { return w3sh(ki, mo); });
      // backward (A operand W: m = in, k = out)
      frag_block64(e64, base + fo.B3, 4, 8, [&](int mi, int ko) { return w3s(mi, ko); }, true);
      frag_block32(e32, base + fo.B3, 4, 4, [&](int mi, int ko) { return w3sh(mi, ko); });
      frag_block64(e64, base + fo.B2, 2, 4, [&](int mi, int ko) { return w2(mi, ko); }, true);
      frag_block32(e32, base + fo.B2, 2, 2, [&](int mi, int ko) { return w2h(mi, ko); });
    }
  // ---- fitting fragments
  const int fwp = ((fw + 31) / 32) * 32;
  FitFragOffsets& ff = m->ffo;
  FitFragOffsets& fl = m->ffo_lp;
  const int Kin[3] = {nd, fw, fw};
  {
    int64_t o = 0, ol = 0;
    for (int l = 0; l < 3; ++l) {
      ff.fwd[l] = o; o += (int64_t)fw * Kin[l];
      fl.fwd[l] = ol; ol += (int64_t)fw * (((Kin[l] + 31) / 32) * 32);
    }
    for (int l = 0; l < 3; ++l) {
      ff.bwd[l] = o; o += (int64_t)Kin[l] * fw;
      fl.bwd[l] = ol; ol += (int64_t)Kin[l] * fwp;
    }
    ff.per_type = o;
    fl.per_type = ol;
  }
  Map f64v((size_t)nt * ff.per_type, -1), f32v((size_t)nt * fl.per_type, -1);
  for (int t = 0; t < nt; ++t) {
    for (int l = 0; l < 3; ++l) {
      const int64_t W = L.fitW[t][l];  // [Kin][fw]
      const int K = Kin[l];
      auto wf = [&](int mo, int ki) -> int32_t { return (ki < K && mo < fw) ? I(W + (int64_t)ki * fw + mo) : -1; };
      auto wb = [&](int mi, int ko) -> int32_t { return (mi < K && ko < fw) ? I(W + (int64_t)mi * fw + ko) : -1; };
      frag_block64(f64v, t * ff.per_type + ff.fwd[l], fw / 16, K / 16, wf, false);
      frag_block32(f32v, t * fl.per_type + fl.fwd[l], fw / 16, (K + 31) / 32, wf);
      frag_block64(f64v, t * ff.per_type + ff.bwd[l], K / 16, fw / 16, wb, false);
      frag_block32(f32v, t * fl.per_type + fl.bwd[l], K / 16, fwp / 32, wb);
    }
  }
  // ---- fitting vectors: b1 b2 b3 wo | bo ebias
  m->fit_vec_per_type = 4 * fw + 2;
  Map fv((size_t)nt * m->fit_vec_per_type, -1);
  for (int t = 0; t < nt; ++t) {
    int32_t* v = &fv[(size_t)t * m->fit_vec_per_type];
    for (int l = 0; l < 3; ++l)
      for (int k = 0; k < fw; ++k) v[l * fw + k] = I(L.fitB[t][l] + k);
    for (int k = 0; k < fw; ++k) v[3 * fw + k] = I(L.wo[t] + k);
    v[4 * fw] = I(L.bo[t]);
    v[4 * fw + 1] = I(L.ebias + t);
  }
  // ---- device buffers and the gathers that fill them
  struct Target { const Map* map; void** dst; int kind; size_t esize; };
  const Target tg[] = {
      {&ev, (void**)&m->emb_vec64, 0, 8},      {&evh, (void**)&m->emb_vec32, 1, 4},
      {&e64, (void**)&m->emb_frag64, 0, 8},    {&evd, (void**)&m->emb_vec64d, 0, 8},
      {&e64d, (void**)&m->emb_frag64d, 0, 8},  {&e32, (void**)&m->emb_frag_bf16, 2, 2},
      {&e32, (void**)&m->emb_frag_f16, 3, 2},  {&e32, (void**)&m->emb_frag_f32, 1, 4},
      {&f64v, (void**)&m->fit_frag64, 0, 8},
      {&f32v, (void**)&m->fit_frag_bf16, 2, 2}, {&f32v, (void**)&m->fit_frag_f16, 3, 2},
      {&f32v, (void**)&m->fit_frag_f32, 1, 4},
      {&fv, (void**)&m->fit_vec64, 0, 8},      {&fv, (void**)&m->fit_vec32, 1, 4},
  };
  const Map* uploaded[16];
  int32_t* uploaded_dev[16];
  int nup = 0;
  m->n_maps = 0;
  for (const Target& t : tg) {
    int32_t* idx = nullptr;
    for (int k = 0; k < nup; ++k)
      if (uploaded[k] == t.map) idx = uploaded_dev[k];
    const bool own = idx == nullptr;
    if (own) {
      if ((rc = upload_vec(&idx, *t.map, "hipMalloc(parameter map)"))) return rc;
      uploaded[nup] = t.map;
      uploaded_dev[nup++] = idx;
    }
    if ((rc = dev_alloc((char**)t.dst, t.map->size() * t.esize, "hipMalloc(model copy)"))) return rc;
    ParamMap& pm = m->maps[m->n_maps++];
    pm.idx = own ? idx : nullptr;   // freed once, by its first user
    pm.idx_use = idx;
    pm.n = (int64_t)t.map->size();
    pm.kind = t.kind;
    pm.dst = *t.dst;
  }
  return dev_alloc(&m->params, (size_t)m->n_params, "hipMalloc(params)");
}

// Refreshes every device copy from m->params (stream-ordered).
void gather_all(dp_model* m, hipStream_t s) {
  for (int k = 0; k < m->n_maps; ++k) {
    const ParamMap& pm = m->maps[k];
    launch_param_gather(m->params, pm.idx_use, pm.n, pm.kind, pm.dst, s);
  }
  if (m->table) launch_tab_build(m, s);
}

// ------------------------------------------------------------ frames
int check_box(const double* box, double rc, double L[3]) {
  if (!box) { set_error("box is NULL"); return DP_ERR_BAD_ARG; }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (a != b && box[3 * a + b] != 0.0) {
        set_error("box must be orthorhombic (diagonal) for the GPU path");
        return DP_ERR_UNSUPPORTED;
      }
  for (int a = 0; a < 3; ++a) {
    L[a] = box[4 * a];
    if (!(L[a] > 0) || !std::isfinite(L[a])) { set_error("box edge %d not positive/finite", a); return DP_ERR_BAD_ARG; }
    if (!(rc < L[a])) { set_error("cut-off %.6g must be below every box edge (edge %d = %.6g)", rc, a, L[a]); return DP_ERR_UNSUPPORTED; }
  }
  return DP_OK;
}

// Fills the pinned frame table and queues its upload.  Returns the total
// number of cells in *ncells.
// Cells have edge >= rlist (the cut-off, or cut-off + skin for a Verlet list).
int stage_frames(dp_ctx* c, const double* boxes, const int64_t* off, int32_t nframes, hipStream_t s, int64_t* ncells,
                 double rlist) {
  if (nframes < 1 || nframes > c->max_frames) {
    set_error("nframes %d out of [1, %d]", nframes, c->max_frames);
    return DP_ERR_CAPACITY;
  }
  const double rc = rlist;
  int64_t cells = 0, chunks = 0;
  FrameInfo* F_new = c->frames_prev + c->max_frames;  // scratch half of the host copy
  for (int f = 0; f < nframes; ++f) {
    double L[3];
    int rcb = check_box(boxes + 9 * f, rc, L);
    if (rcb) return rcb;
    const int64_t a0 = off[f], a1 = off[f + 1];
    if (a0 < 0 || a1 < a0) { set_error("frame offsets must be non-decreasing from 0"); return DP_ERR_BAD_ARG; }
    FrameInfo& F = F_new[f];
    memset(&F, 0, sizeof(F));
    F.atom_off = (int32_t)a0;
    F.natoms = (int32_t)(a1 - a0);
    F.cell_off = (int32_t)cells;
    F.chunk_off = (int32_t)chunks;
    chunks += (F.natoms + kRedChunk - 1) / kRedChunk;
    int64_t nc = 1;
    for (int a = 0; a < 3; ++a) {
      int k = (int)std::floor(L[a] / (rc * (1.0 + 1e-10)));
      if (k < 1) k = 1;
      if (k > 1024) k = 1024;
      F.ncell[a] = k;
      F.L[a] = L[a];
      nc *= k;
    }
    cells += nc;
  }
  if (off[0] != 0) { set_error("frame_off[0] must be 0"); return DP_ERR_BAD_ARG; }
  if (off[nframes] > c->max_atoms) { set_error("%lld atoms exceed max_atoms %lld", (long long)off[nframes], (long long)c->max_atoms); return DP_ERR_CAPACITY; }
  if (cells > c->max_cells) { set_error("%lld cells exceed the context capacity %lld", (long long)cells, (long long)c->max_cells); return DP_ERR_CAPACITY; }
  // upload only when the table differs from the one already on the device
  if (nframes != c->nframes_dev || memcmp(F_new, c->frames_prev, sizeof(FrameInfo) * nframes) != 0) {
    if (c->frames_ev_pending) {
      HIPCHECK(hipEventSynchronize(c->frames_ev));
      c->frames_ev_pending = false;
    }
    memcpy(c->frames_host, F_new, sizeof(FrameInfo) * nframes);
    memcpy(c->frames_prev, F_new, sizeof(FrameInfo) * nframes);
    c->nframes_dev = nframes;
    c->frames_gen++;
    HIPCHECK(hipMemcpyAsync(c->frames_dev, c->frames_host, sizeof(FrameInfo) * nframes, hipMemcpyHostToDevice, s));
    HIPCHECK(hipEventRecord(c->frames_ev, s));
    c->frames_ev_pending = true;
  }
  c->nframes_last = nframes;
  c->nchunks_last = (int32_t)chunks;
  *ncells = cells;
  return DP_OK;
}

// ------------------------------------------------------------ stage timing
void prof_harvest(dp_ctx* c) {
  for (int k = 0; k < c->prof_n; ++k) {
    float ms = 0.f;
    (void)hipEventSynchronize(c->prof_ev[2 * k + 1]);
    if (hipEventElapsedTime(&ms, c->prof_ev[2 * k], c->prof_ev[2 * k + 1]) == hipSuccess) {
      c->prof_ms[c->prof_stage[k]] += ms;
      c->prof_cnt[c->prof_stage[k]] += 1;
    }
  }
  c->prof_n = 0;
}

struct StageScope {
  dp_ctx* c;
  int k;
  hipStream_t s;
  StageScope(dp_ctx* ctx, int stage, hipStream_t st) : c(ctx), k(-1), s(st) {
    if (!c->prof_ev || !((c->prof_mask >> stage) & 1)) return;
    if (c->prof_n == c->prof_cap) prof_harvest(c);
    k = c->prof_n++;
    c->prof_stage[k] = stage;
    (void)hipEventRecord(c->prof_ev[2 * k], s);
  }
  ~StageScope() {
    if (k >= 0) (void)hipEventRecord(c->prof_ev[2 * k + 1], s);
  }
};

int check_mode(int32_t mode) {
  if (mode < DP_FP64 || mode > DP_FP64_TAB) {
    set_error("mode %d is not one of DP_FP64, DP_MIX_BF16, DP_MIX_FP16, DP_MIX_FP32, DP_MIX_FP16_FIT1, DP_FP64_TAB",
              mode);
    return DP_ERR_BAD_ARG;
  }
  return DP_OK;
}

int set_device(int dev) {
  HIPCHECK(hipSetDevice(dev));
  return DP_OK;
}

// Column order by type (atom_at, col_of, type_meta, frame_of) depends only on
// the types, the atom count and the frame table.  A list is valid only for
// the types it was built with, so a compute on a list this context built or
// formatted keeps the order of the last sort when the types buffer, the
// count and the frame table are the ones that sort used; building a list
// (or a Verlet candidate list) always sorts anew, and a list from elsewhere
// always triggers a sort.
static void type_sort(dp_ctx* c, const int32_t* types, int64_t n, int32_t nframes, bool may_reuse, hipStream_t s) {
  if (may_reuse && c->ts_valid && c->ts_types == types && c->ts_n == n && c->ts_nframes == nframes &&
      c->ts_frames_gen == c->frames_gen)
    return;
  launch_type_sort(c, types, (int32_t)n, nframes, s);
  c->ts_valid = true;
  c->ts_types = types;
  c->ts_n = n;
  c->ts_nframes = nframes;
  c->ts_frames_gen = c->frames_gen;
}

int compute_impl(dp_ctx* c, const double* x, const int32_t* types, const double* boxes, const int64_t* off,
                 int32_t nframes, const int32_t* nlist, int32_t mode, double* energies, double* atom_energy,
                 double* forces, double* virials, hipStream_t s) {
  if (!c) { set_error("ctx is NULL"); return DP_ERR_BAD_ARG; }
  int rc = check_mode(mode);
  if (rc) return rc;
  const int64_t n = off ? off[nframes] : 0;
  if (n > 0 && (!x || !types || !nlist || !forces)) { set_error("coords/types/nlist/forces must be non-NULL"); return DP_ERR_BAD_ARG; }
  if (!energies || !virials) { set_error("energy/virial outputs must be non-NULL"); return DP_ERR_BAD_ARG; }
  if ((rc = set_device(c->device))) return rc;
  int64_t ncells = 0;
  if ((rc = stage_frames(c, boxes, off, nframes, s, &ncells, c->model->desc.rcut))) return rc;
  const bool tab = mode == DP_FP64_TAB;
  if (tab && !c->model->table) { set_error("DP_FP64_TAB needs dp_model_compress on the model"); return DP_ERR_STATE; }
  c->natoms_last = n;
  c->types_last = types;
  c->mode_last = mode;
  c->last_stream = s;
  // the tabulated form is the FP64 path with the embedding nets replaced
  if (tab) mode = DP_FP64;
  const int32_t ntot = (int32_t)n;
  const bool own_list = nlist == c->rev_list && n == c->natoms_rev;
  { StageScope p(c, DP_STAGE_TYPESORT, s); type_sort(c, types, n, nframes, own_list, s); }
  if (!own_list) {
    // list not built by this context: derive its reverse index now (slots
    // whose reverse is not found fall back to atomics in the force pass)
    StageScope p(c, DP_STAGE_NLIST, s);
    launch_nl_reverse(c, x, types, nlist, ntot, s);
    c->rev_list = nlist;
    c->natoms_rev = n;
  }
  { StageScope p(c, DP_STAGE_ENV, s); launch_env(c, x, types, nlist, ntot, forces, s); }
  c->act_used_last = !tab && c->act && mode == DP_FP64 && n * c->model->tpa * (int64_t)c->model->m1 * 16 * 8 <= c->act_bytes;
  c->grad_act = false;
  {
    StageScope p(c, DP_STAGE_EMBED_FWD, s);
    if (tab) launch_embed_tab(c, false, s);
    else launch_embed_fwd(c, types, mode, s);
  }
  { StageScope p(c, DP_STAGE_DESCRIPTOR, s); launch_descriptor(c, mode, s); }
  { StageScope p(c, DP_STAGE_FIT_FWD, s); launch_fit_forward(c, mode, c->train_h, s); }
  c->h_stored = c->train_h;
  { StageScope p(c, DP_STAGE_FIT_BWD, s); launch_fit_backward(c, mode, c->train_h, s); }
  { StageScope p(c, DP_STAGE_DESC_BWD, s); launch_desc_bwd(c, mode, s); }
  {
    StageScope p(c, DP_STAGE_EMBED_BWD, s);
    if (tab) launch_embed_tab(c, true, s);
    else launch_embed_bwd(c, types, mode, s);
  }
  { StageScope p(c, DP_STAGE_FORCE, s); launch_force(c, x, nlist, ntot, forces, s); }
  { StageScope p(c, DP_STAGE_REDUCE, s); launch_frame_reduce(c, nframes, energies, atom_energy, virials, s); }
  HIPCHECK(hipGetLastError());
  c->have_state = true;
  return DP_OK;
}

int nlist_impl(dp_ctx* c, const double* x, const int32_t* types, const double* boxes, const int64_t* off,
               int32_t nframes, int32_t* nlist, int32_t* overflow, hipStream_t s) {
  if (!c) { set_error("ctx is NULL"); return DP_ERR_BAD_ARG; }
  if (!overflow) { set_error("n_overflow_out must be non-NULL"); return DP_ERR_BAD_ARG; }
  const int64_t n = off[nframes];
  if (n > 0 && (!x || !types || !nlist)) { set_error("coords/types/nlist must be non-NULL"); return DP_ERR_BAD_ARG; }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  int64_t ncells = 0;
  if ((rc = stage_frames(c, boxes, off, nframes, s, &ncells, c->model->desc.rcut))) return rc;
  c->last_stream = s;
  const int32_t ntot = (int32_t)n;
  StageScope p(c, DP_STAGE_NLIST, s);
  launch_fill_i32(overflow, 0, 1, s);
  launch_nl_bin(c, x, ntot, nframes, s);  // cell counts are zero between builds (cleared by the scan)
  launch_nl_scan(c, (int32_t)ncells, s);
  launch_nl_scatter(c, ntot, s);
  launch_nl_search(c, x, types, ntot, nframes, nlist, overflow, s);
  type_sort(c, types, n, nframes, false, s);  // frame_of for the reverse index
  launch_nl_reverse(c, x, types, nlist, ntot, s);
  c->rev_list = nlist;
  c->natoms_rev = n;
  HIPCHECK(hipGetLastError());
  return DP_OK;
}

int skin_build_impl(dp_ctx* c, double* x, const int32_t* types, const double* box, int64_t n, double skin,
                    int32_t* images, hipStream_t s) {
  if (!c) { set_error("ctx is NULL"); return DP_ERR_BAD_ARG; }
  if (n < 0 || (n > 0 && (!x || !types))) { set_error("bad arguments"); return DP_ERR_BAD_ARG; }
  if (!(skin >= 0.0) || !std::isfinite(skin)) { set_error("skin must be finite and >= 0"); return DP_ERR_BAD_ARG; }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  const double rlist = c->model->desc.rcut + skin;
  double L[3];
  if ((rc = check_box(box, rlist, L))) return rc;
  int64_t ncells = 0;
  const int64_t off[2] = {0, n};
  if ((rc = stage_frames(c, box, off, 1, s, &ncells, rlist))) return rc;
  c->last_stream = s;
  c->skin = skin;
  for (int a = 0; a < 3; ++a) c->skin_L[a] = L[a];
  const int32_t ntot = (int32_t)n;
  StageScope p(c, DP_STAGE_NLIST, s);
  // the build's frame (box, grid of edge >= r_c + skin) is kept for the
  // rebuilds the device decides on later (dp_compute replaces the table)
  HIPCHECK(hipMemcpyAsync(c->skin_frame, c->frames_dev, sizeof(FrameInfo), hipMemcpyDeviceToDevice, s));
  c->skin_ncells = (int32_t)ncells;
  launch_nl_skin_build(c, x, types, ntot, (int32_t)ncells, images, s);
  c->skin_n = n;
  c->rev_list = nullptr;
  c->ts_valid = false;
  HIPCHECK(hipGetLastError());
  return DP_OK;
}

int skin_update_impl(dp_ctx* c, double* x, const int32_t* types, int64_t n, int32_t every, int32_t* images,
                     int32_t* nlist, int32_t* overflow, int32_t* rebuilds, hipStream_t s) {
  if (!c) { set_error("ctx is NULL"); return DP_ERR_BAD_ARG; }
  if (!overflow || n < 0 || every < 0 || (n > 0 && (!x || !types || !nlist))) { set_error("bad arguments"); return DP_ERR_BAD_ARG; }
  if (c->skin_n < 0 || n != c->skin_n) {
    set_error("no Verlet list built for %lld atoms on this context", (long long)n);
    return DP_ERR_STATE;
  }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  c->last_stream = s;
  StageScope p(c, DP_STAGE_NLIST, s);
  if (n == 0) launch_fill_i32(overflow, 0, 1, s);
  launch_nl_skin_update(c, x, types, (int32_t)n, every, images, rebuilds, s);
  launch_nl_skin_format(c, x, types, (int32_t)n, nlist, overflow, s);
  c->rev_list = nlist;
  c->natoms_rev = n;
  HIPCHECK(hipGetLastError());
  return DP_OK;
}

int skin_format_impl(dp_ctx* c, const double* x, const int32_t* types, int64_t n, int32_t* nlist, int32_t* overflow,
                     hipStream_t s) {
  if (!c) { set_error("ctx is NULL"); return DP_ERR_BAD_ARG; }
  if (!overflow || n < 0 || (n > 0 && (!x || !types || !nlist))) { set_error("bad arguments"); return DP_ERR_BAD_ARG; }
  if (c->skin_n < 0 || n != c->skin_n) {
    set_error("no Verlet list built for %lld atoms on this context", (long long)n);
    return DP_ERR_STATE;
  }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  c->last_stream = s;
  StageScope p(c, DP_STAGE_NLIST, s);
  if (n == 0) launch_fill_i32(overflow, 0, 1, s);  // otherwise written by the format's second pass
  launch_nl_skin_format(c, x, types, (int32_t)n, nlist, overflow, s);
  c->rev_list = nlist;
  c->natoms_rev = n;
  HIPCHECK(hipGetLastError());
  return DP_OK;
}


// ------------------------------------------------------------ no-allocation build
// Neighbour-list scratch of dp_build_nlist_noalloc: a file-scope device
// array (one copy per GPU, held until the process ends).  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): the device address is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_dev.
//   words [0, 16)    frame table (one FrameInfo)
//   words [16, 32)   status word of the call
//   then cell_count, cell_start, cell_fill [kNaMaxCells + 1] each and
//   cell_of, cell_atoms [kNaMaxAtoms] each.
constexpr int64_t kNaMaxAtoms = 1 << 16;
constexpr int64_t kNaMaxCells = 1 << 17;
constexpr int64_t kNaWords = 32 + 3 * (kNaMaxCells + 1) + 2 * kNaMaxAtoms;
static __device__ __align__(256) int32_t scratch[kNaWords];

constexpr int kNaMaxDevices = 64;
static std::mutex g_scratch_mu;
static int32_t* g_scratch_dev[kNaMaxDevices];

// Device address of this device's copy of the scratch array (the caller made
// the device current).
static int scratch_on_device(int dev, int32_t** out) {
  if (dev < 0 || dev >= kNaMaxDevices) { set_error("device %d beyond %d", dev, kNaMaxDevices); return DP_ERR_UNSUPPORTED; }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = (int32_t*)ptr;
  }
  *out = g_scratch_dev[dev];
  return DP_OK;
}

int nlist_noalloc_impl(const dp_model* m, const double* x, const int32_t* types, const double* box, int64_t n,
                       int32_t* nlist, int32_t* overflow, int32_t* flags_out, hipStream_t s) {
  if (!m) { set_error("model is NULL"); return DP_ERR_BAD_ARG; }
  if (!overflow || n < 0 || (n > 0 && (!x || !types || !nlist))) { set_error("bad arguments"); return DP_ERR_BAD_ARG; }
  if (n > kNaMaxAtoms) {
    set_error("%lld atoms exceed the %lld of the no-allocation scratch", (long long)n, (long long)kNaMaxAtoms);
    return DP_ERR_CAPACITY;
  }
  double L[3];
  int rc;
  if ((rc = check_box(box, m->desc.rcut, L))) return rc;
  FrameInfo F;
  memset(&F, 0, sizeof(F));
  F.natoms = (int32_t)n;
  int64_t ncells = 1;
  for (int a = 0; a < 3; ++a) {
    int k = (int)std::floor(L[a] / (m->desc.rcut * (1.0 + 1e-10)));
    if (k < 1) k = 1;
    if (k > 1024) k = 1024;
    F.ncell[a] = k;
    F.L[a] = L[a];
    ncells *= k;
  }
  if (ncells > kNaMaxCells) {
    set_error("%lld cells exceed the %lld of the no-allocation scratch", (long long)ncells, (long long)kNaMaxCells);
    return DP_ERR_CAPACITY;
  }
  if ((rc = set_device(m->device))) return rc;
  int32_t* base = nullptr;
  if ((rc = scratch_on_device(m->device, &base))) return rc;
  // a context view whose nlist buffers all lie in the scratch array
  dp_ctx v;
  memset(&v, 0, sizeof(v));
  v.model = m;
  v.device = m->device;
  v.frames_dev = reinterpret_cast<FrameInfo*>(base);
  v.flags_dev = base + 16;
  v.cell_count = base + 32;
  v.cell_start = v.cell_count + (kNaMaxCells + 1);
  v.cell_fill = v.cell_start + (kNaMaxCells + 1);
  v.cell_of = v.cell_fill + (kNaMaxCells + 1);
  v.cell_atoms = v.cell_of + kNaMaxAtoms;
  // the array keeps the last call's contents: the frame, the status word
  // and the cell counts are written or cleared first
  launch_set_frame(v.frames_dev, F, v.flags_dev, s);
  launch_fill_i32(v.cell_count, 0, ncells, s);
  launch_fill_i32(overflow, 0, 1, s);
  const int32_t ntot = (int32_t)n;
  launch_nl_bin(&v, x, ntot, 1, s);
  launch_nl_scan(&v, (int32_t)ncells, s);
  launch_nl_scatter(&v, ntot, s);
  launch_nl_search(&v, x, types, ntot, 1, nlist, overflow, s);
  if (flags_out) launch_copy_i32(v.flags_dev, flags_out, 1, s);
  HIPCHECK(hipGetLastError());
  return DP_OK;
}

}  // namespace

// ============================================================ C ABI
extern "C" {

const char* dp_last_error(void) { return g_err; }

int64_t dp_model_n_params(const dp_model_desc* desc) {
  if (!desc || desc->ntypes < 1 || desc->ntypes > DP_MAX_TYPES || desc->n_emb < 1 || desc->n_emb > DP_MAX_LAYERS ||
      desc->n_fit < 1 || desc->n_fit > DP_MAX_LAYERS) {
    set_error("bad descriptor");
    return DP_ERR_BAD_ARG;
  }
  return layout_of(desc).total;
}

int dp_model_create(const dp_model_desc* desc, const double* params_host, int64_t n_params, dp_model** out) {
  if (!out) { set_error("out is NULL"); return DP_ERR_BAD_ARG; }
  *out = nullptr;
  int rc = validate_desc(desc);
  if (rc) return rc;
  const int64_t need = layout_of(desc).total;
  if (!params_host || n_params != need) {
    set_error("params: expected %lld values, got %lld", (long long)need, (long long)n_params);
    return DP_ERR_BAD_ARG;
  }
  for (int64_t k = 0; k < n_params; ++k)
    if (!std::isfinite(params_host[k])) { set_error("parameter %lld is not finite", (long long)k); return DP_ERR_BAD_ARG; }
  dp_model* m = new dp_model;
  memset(m, 0, sizeof(*m));
  m->desc = *desc;
  m->nm = 0;
  m->sec[0] = 0;
  for (int t = 0; t < desc->ntypes; ++t) {
    m->sec[t + 1] = m->sec[t] + desc->sel[t];
    m->nm += desc->sel[t];
  }
  for (int t = desc->ntypes + 1; t <= DP_MAX_TYPES; ++t) m->sec[t] = m->nm;
  m->tpa = 0;
  for (int t = 0; t <= DP_MAX_TYPES; ++t) {
    m->toff[t] = m->tpa;
    if (t < desc->ntypes) m->tpa += (desc->sel[t] + 15) / 16;
  }
  m->w1 = desc->emb[0];
  m->m1 = desc->emb[2];
  m->n3 = (m->m1 + 15) / 16;
  m->nd = m->m1 * desc->m2;
  m->fw = desc->fit[0];
  m->n_params = n_params;
  hipError_t e = hipGetDevice(&m->device);
  if (e != hipSuccess) { delete m; return hip_fail(e, "hipGetDevice"); }
  rc = build_maps(m);
  if (rc == DP_OK) {
    e = hipMemcpy(m->params, params_host, (size_t)n_params * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
      gather_all(m, nullptr);
      e = hipStreamSynchronize(nullptr);
    }
    if (e != hipSuccess) rc = hip_fail(e, "model upload");
  }
  if (rc) { free_model(m); return rc; }
  *out = m;
  return DP_OK;
}

int dp_model_set_params(dp_model* m, const double* params_host, int64_t n_params) {
  if (!m || !params_host || n_params != m->n_params) { set_error("bad arguments"); return DP_ERR_BAD_ARG; }
  for (int64_t k = 0; k < n_params; ++k)
    if (!std::isfinite(params_host[k])) { set_error("parameter %lld is not finite", (long long)k); return DP_ERR_BAD_ARG; }
  int rc;
  if ((rc = set_device(m->device))) return rc;
  HIPCHECK(hipMemcpy(m->params, params_host, (size_t)n_params * 8, hipMemcpyHostToDevice));
  gather_all(m, nullptr);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(nullptr));
  return DP_OK;
}

int dp_model_set_params_device(dp_model* m, const double* params_dev, int64_t n_params, hipStream_t stream) {
  if (!m || !params_dev || n_params != m->n_params) { set_error("bad arguments"); return DP_ERR_BAD_ARG; }
  int rc;
  if ((rc = set_device(m->device))) return rc;
  if (params_dev != m->params)
    HIPCHECK(hipMemcpyAsync(m->params, params_dev, (size_t)n_params * 8, hipMemcpyDeviceToDevice, stream));
  gather_all(m, stream);
  HIPCHECK(hipGetLastError());
  return DP_OK;
}

int dp_model_compress(dp_model* m, double x_fine, double x_max, double h) {
  if (!m) { set_error("model is NULL"); return DP_ERR_BAD_ARG; }
  if (!(h > 0.0) || !(x_fine > 0.0) || !(x_max >= x_fine) || !std::isfinite(x_max)) {
    set_error("need h > 0, x_fine > 0, x_max >= x_fine (finite)");
    return DP_ERR_BAD_ARG;
  }
  TabGrid g;
  g.h = h;
  g.H = h * 10.0;
  const double n1d = std::ceil(x_fine / h);
  if (!(n1d <= 1e6)) { set_error("more than 10^6 table intervals"); return DP_ERR_BAD_ARG; }
  g.n1 = (int)n1d;
  g.X1 = (double)g.n1 * h;
  const double n2d = x_max > g.X1 ? std::ceil((x_max - g.X1) / g.H) : 0.0;
  if (!(n1d + n2d <= 1e6)) { set_error("more than 10^6 table intervals"); return DP_ERR_BAD_ARG; }
  g.n2 = (int)n2d;
  g.X2 = std::fma((double)g.n2, g.H, g.X1);
  g.nint = g.n1 + g.n2;
  int rc;
  if ((rc = set_device(m->device))) return rc;
  HIPCHECK(hipStreamSynchronize(nullptr));
  if (m->table) (void)hipFree(m->table);
  if (m->tab_nodes) (void)hipFree(m->tab_nodes);
  m->table = m->tab_nodes = nullptr;
  const int nnets = m->desc.ntypes * m->desc.ntypes;
  if ((rc = dev_alloc(&m->table, (size_t)nnets * g.nint * 6 * m->m1, "hipMalloc(table)"))) return rc;
  if ((rc = dev_alloc(&m->tab_nodes, (size_t)nnets * (g.nint + 1) * 3 * m->m1, "hipMalloc(table nodes)"))) {
    (void)hipFree(m->table);
    m->table = nullptr;
    return rc;
  }
  m->tab_grid = g;
  const ParamLayout L = layout_of(&m->desc);
  for (int a = 0; a < m->desc.ntypes; ++a)
    for (int b = 0; b < m->desc.ntypes; ++b)
      for (int l = 0; l < 3; ++l) {
        m->tab_off.W[a * m->desc.ntypes + b][l] = L.embW[a][b][l];
        m->tab_off.b[a * m->desc.ntypes + b][l] = L.embB[a][b][l];
      }
  launch_tab_build(m, nullptr);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(nullptr));
  return DP_OK;
}

int dp_model_copy_table(const dp_model* m, double* dst, int64_t* n_values) {
  if (!m || !n_values) { set_error("NULL argument"); return DP_ERR_BAD_ARG; }
  if (!m->table) { set_error("model not compressed"); return DP_ERR_STATE; }
  const int64_t nv = (int64_t)m->desc.ntypes * m->desc.ntypes * m->tab_grid.nint * 6 * m->m1;
  *n_values = nv;
  if (!dst) return DP_OK;
  int rc;
  if ((rc = set_device(m->device))) return rc;
  HIPCHECK(hipMemcpy(dst, m->table, (size_t)nv * 8, hipMemcpyDeviceToDevice));
  return DP_OK;
}

int dp_model_destroy(dp_model* m) {
  if (!m) return DP_OK;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  free_model(m);
  return DP_OK;
}

int dp_ctx_destroy(dp_ctx* c);

int dp_ctx_profile(dp_ctx* c, int32_t enable) {
  if (!c) { set_error("ctx is NULL"); return DP_ERR_BAD_ARG; }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  if (c->prof_ev) {
    (void)hipDeviceSynchronize();
    for (int k = 0; k < 2 * c->prof_cap; ++k) (void)hipEventDestroy(c->prof_ev[k]);
    delete[] c->prof_ev;
    delete[] c->prof_stage;
    c->prof_ev = nullptr;
    c->prof_stage = nullptr;
    c->prof_cap = c->prof_n = 0;
  }
  for (int k = 0; k < DP_NSTAGES; ++k) { c->prof_ms[k] = 0; c->prof_cnt[k] = 0; }
  c->prof_mask = enable;
  if (!enable) return DP_OK;
  const int cap = 4096;
  c->prof_ev = new hipEvent_t[2 * cap];
  c->prof_stage = new int32_t[cap];
  for (int k = 0; k < 2 * cap; ++k) HIPCHECK(hipEventCreate(&c->prof_ev[k]));
  c->prof_cap = cap;
  return DP_OK;
}

int dp_ctx_stage_times(dp_ctx* c, double* total_ms, int64_t* counts) {
  if (!c || !total_ms || !counts) { set_error("NULL argument"); return DP_ERR_BAD_ARG; }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  prof_harvest(c);
  for (int k = 0; k < DP_NSTAGES; ++k) {
    total_ms[k] = c->prof_ms[k];
    counts[k] = c->prof_cnt[k];
    c->prof_ms[k] = 0;
    c->prof_cnt[k] = 0;
  }
  return DP_OK;
}

int dp_ctx_create(const dp_model* m, int64_t max_atoms, int32_t max_frames, int64_t workspace_budget_bytes,
                  dp_ctx** out) {
  if (!out) { set_error("out is NULL"); return DP_ERR_BAD_ARG; }
  *out = nullptr;
  if (!m) { set_error("model is NULL"); return DP_ERR_BAD_ARG; }
  if (max_atoms < 1 || max_atoms > (int64_t)INT32_MAX / 27 - 1) { set_error("max_atoms out of range"); return DP_ERR_BAD_ARG; }
  // list slots and Verlet candidates are addressed with 32-bit indices
  // (atom * slots-per-atom + slot)
  if (max_atoms * (int64_t)(m->nm > kCandCap ? m->nm : kCandCap) > (int64_t)INT32_MAX) {
    set_error("max_atoms %lld times %d slots per atom exceeds the 32-bit slot index", (long long)max_atoms,
              m->nm > kCandCap ? m->nm : kCandCap);
    return DP_ERR_UNSUPPORTED;
  }
  if (max_frames < 1 || max_frames > 1 << 20) { set_error("max_frames out of range"); return DP_ERR_BAD_ARG; }
  if (workspace_budget_bytes < 0) { set_error("negative workspace budget"); return DP_ERR_BAD_ARG; }
  int rc;
  if ((rc = set_device(m->device))) return rc;
  dp_ctx* c = new dp_ctx;
  memset(c, 0, sizeof(*c));
  c->model = m;
  c->device = m->device;
  c->max_atoms = max_atoms;
  c->max_frames = max_frames;
  c->max_cols = max_atoms + (int64_t)m->desc.ntypes * kColPad;
  c->max_cells = max_atoms + 27LL * max_frames + 1024;
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || ncu <= 0)
      ncu = 256;
    c->ncu = ncu;
  }
  const int64_t N = max_atoms, C = c->max_cols;
  const int nm = m->nm, m1 = m->m1, nd = m->nd;
  const int fwp = ((m->fw + 31) / 32) * 32;
  const int nchunks = (int)((N + 1023) / 1024);
#define ALLOC(ptr, cnt)                                            \
  if ((rc = dev_alloc(&(ptr), (size_t)(cnt), "hipMalloc(ctx)"))) { \
    dp_ctx_destroy(c);                                             \
    return rc;                                                     \
  }
  ALLOC(c->frames_dev, max_frames);
  {
    hipError_t e = hipHostMalloc((void**)&c->frames_host, sizeof(FrameInfo) * max_frames, hipHostMallocDefault);
    if (e != hipSuccess) { dp_ctx_destroy(c); return hip_fail(e, "hipHostMalloc(frames)"); }
    c->frames_prev = new FrameInfo[2 * (size_t)max_frames];
    c->nframes_dev = -1;
    e = hipHostMalloc((void**)&c->flags_host, sizeof(int32_t), hipHostMallocDefault);
    if (e != hipSuccess) { dp_ctx_destroy(c); return hip_fail(e, "hipHostMalloc(flags)"); }
    e = hipEventCreateWithFlags(&c->frames_ev, hipEventDisableTiming);
    if (e != hipSuccess) { dp_ctx_destroy(c); return hip_fail(e, "hipEventCreate"); }
  }
  ALLOC(c->flags_dev, 1);
  ALLOC(c->cell_of, N);
  ALLOC(c->cell_count, c->max_cells + 1);
  ALLOC(c->cell_start, c->max_cells + 1);
  ALLOC(c->cell_fill, c->max_cells + 1);
  ALLOC(c->cell_atoms, N);
  ALLOC(c->chunk_counts, (int64_t)nchunks * kMaxT + kMaxT);
  ALLOC(c->type_meta, 2 * kMaxT);
  ALLOC(c->col_of, N);
  ALLOC(c->atom_at, C);
  ALLOC(c->frame_of, N);
  ALLOC(c->emb_ctr, (int64_t)kMaxT * kMaxT * 3 * c->ncu * 32);
  ALLOC(c->R, N * nm * 4);
  ALLOC(c->nnei, N * kMaxT);
  ALLOC(c->netd, N * nm * 4);
  ALLOC(c->rev, N * nm);
  ALLOC(c->skin_cand, N * kCandCap);
  ALLOC(c->skin_ncand, N);
  ALLOC(c->skin_crev, N * kCandCap);
  ALLOC(c->skin_slot, N * kCandCap);
  ALLOC(c->skin_cof, N * nm);
  ALLOC(c->skin_xref, N * 3);
  c->skin_n = -1;
  ALLOC(c->red_part, 10 * (N / kRedChunk + (int64_t)max_frames + 1));
  ALLOC(c->vatom, N * 9);
  ALLOC(c->ke_part, N / 256 + 2);
  ALLOC(c->ke_ctr, 32);
  ALLOC(c->frame_ctr, max_frames);
  ALLOC(c->ovf_ctr, 32);
  c->skin_gate = c->ovf_ctr + 8;
  ALLOC(c->skin_frame, 1);
  {
    hipError_t e = hipMemset(c->ke_ctr, 0, 32 * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(c->frame_ctr, 0, (size_t)max_frames * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(c->ovf_ctr, 0, 32 * sizeof(int32_t));
    // cell counts are zero between builds (each scan clears what it read)
    if (e == hipSuccess) e = hipMemset(c->cell_count, 0, (size_t)(c->max_cells + 1) * sizeof(int32_t));
    if (e != hipSuccess) {
      dp_ctx_destroy(c);
      return hip_fail(e, "hipMemset(ctx)");
    }
  }
  ALLOC(c->Ei_col, C);
  ALLOC(c->Ei_atom, N);
  ALLOC(c->gE_col, C);
  ALLOC(c->grad_tmp, m->n_params);
  {
    // parameter-gradient workspace: per-chunk partials of the fitting
    // reductions, per-work-group records of the embedding reductions
    int64_t fch = N / 1024, slots = N / 64;
    c->grad_chunks = (int32_t)(fch < 1 ? 1 : (fch > 16 ? 16 : fch));
    c->grad_slots = (int32_t)(slots < 1 ? 1 : (slots > 1024 ? 1024 : slots));
    const int64_t nt = m->desc.ntypes;
    const int64_t fit_w = nt * c->grad_chunks * (int64_t)nd * m->fw;
    const int64_t fit_b = nt * ((N + 255) / 256) * (int64_t)m->fw;  // bias sums: 256-column chunks
    const int64_t fit = fit_w > fit_b ? fit_w : fit_b;
    const int64_t emb = nt * nt * c->grad_slots * 10496LL;
    ALLOC(c->gpart, fit > emb ? fit : emb);
  }
  double* tmp = nullptr;
  ALLOC(tmp, (int64_t)m->desc.ntypes * C * m1 * 4); c->Tpart = tmp;
  ALLOC(tmp, C * m1 * 4); c->T = tmp;
  ALLOC(tmp, C * nd); c->D = tmp;
  ALLOC(tmp, C * nd); c->dD = tmp;
  ALLOC(tmp, C * m1 * 4); c->gT = tmp;
  for (int k = 0; k < 12; ++k) {
    ALLOC(tmp, C * fwp);
    c->fa[k] = tmp;
  }
  {
    const int64_t sc = kSplitCols + (int64_t)m->desc.ntypes * kColPad;
    c->split_cols = C < sc ? C : sc;
    ALLOC(tmp, (int64_t)kSplitMax * c->split_cols * fwp);
    c->split_part = tmp;
  }
  {
    // activation store: as much of the full [max_atoms, tpa, m1, 16] f64
    // store as the budget allows; each compute uses it when its atoms fit
    // (plus one record of slack: padding slots of the last record may be
    // read, and discarded, past its end)
    const int64_t full = N * m->tpa * (int64_t)m1 * 16 * 8;
    const int64_t bytes = workspace_budget_bytes < full ? workspace_budget_bytes : full;
    if (bytes >= (int64_t)m->tpa * m1 * 16 * 8) {
      ALLOC(tmp, bytes / 8 + (int64_t)m1 * 16);
      c->act = tmp;
      c->act_bytes = bytes;
    }
  }
#undef ALLOC
  // zero-initialise every buffer once: padding columns of the mixed-precision
  // activations (features fw..fwp) must hold finite zeros forever.
  {
    hipError_t e = hipSuccess;
    for (int k = 0; k < 12 && e == hipSuccess; ++k) e = hipMemset(c->fa[k], 0, (size_t)C * fwp * 8);
    if (e == hipSuccess) e = hipMemset(c->D, 0, (size_t)C * nd * 8);
    if (e == hipSuccess) e = hipMemset(c->flags_dev, 0, 4);
    if (e == hipSuccess) e = hipMemset(c->netd, 0, (size_t)N * nm * 4 * 8);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { dp_ctx_destroy(c); return hip_fail(e, "ctx init"); }
  }
  *out = c;
  return DP_OK;
}

int dp_ctx_destroy(dp_ctx* c) {
  if (!c) return DP_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  void* ptrs[] = {c->frames_dev, c->flags_dev, c->cell_of, c->cell_count, c->cell_start, c->cell_fill,
                  c->cell_atoms, c->chunk_counts, c->type_meta, c->col_of, c->atom_at, c->frame_of, c->emb_ctr, c->R, c->nnei,
                  c->netd, c->rev, c->red_part, c->vatom, c->ke_part, c->ke_ctr, c->frame_ctr, c->ovf_ctr, c->Ei_col, c->Ei_atom, c->gE_col, c->grad_tmp, c->Tpart, c->T, c->D, c->dD, c->gT, c->act,
                  c->skin_cand, c->skin_ncand, c->skin_crev, c->skin_slot, c->skin_cof, c->skin_xref, c->skin_frame,
                  c->gpart, c->split_part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int k = 0; k < 12; ++k)
    if (c->fa[k]) (void)hipFree(c->fa[k]);
  dp_ctx_profile(c, 0);
  if (c->frames_host) (void)hipHostFree(c->frames_host);
  delete[] c->frames_prev;
  if (c->flags_host) (void)hipHostFree(c->flags_host);
  if (c->frames_ev) (void)hipEventDestroy(c->frames_ev);
  delete c;
  return DP_OK;
}

int dp_build_nlist(dp_ctx* c, const double* coords, const int32_t* types, const double* box, int64_t n,
                   int32_t* nlist_out, int32_t* n_overflow_out, hipStream_t stream) {
  if (n < 0) { set_error("n < 0"); return DP_ERR_BAD_ARG; }
  const int64_t off[2] = {0, n};
  return nlist_impl(c, coords, types, box, off, 1, nlist_out, n_overflow_out, stream);
}

int dp_nlist_skin_build(dp_ctx* c, double* coords, const int32_t* types, const double* box, int64_t n, double skin,
                        int32_t* images, hipStream_t stream) {
  return skin_build_impl(c, coords, types, box, n, skin, images, stream);
}

int dp_nlist_skin_format(dp_ctx* c, const double* coords, const int32_t* types, int64_t n, int32_t* nlist_out,
                         int32_t* n_overflow_out, hipStream_t stream) {
  return skin_format_impl(c, coords, types, n, nlist_out, n_overflow_out, stream);
}

int dp_build_nlist_noalloc(const dp_model* model, const double* coords, const int32_t* types, const double* box,
                           int64_t n, int32_t* nlist_out, int32_t* n_overflow_out, int32_t* flags_out,
                           hipStream_t stream) {
  return nlist_noalloc_impl(model, coords, types, box, n, nlist_out, n_overflow_out, flags_out, stream);
}

int dp_nlist_skin_update(dp_ctx* c, double* coords, const int32_t* types, int64_t n, int32_t every, int32_t* images,
                         int32_t* nlist_out, int32_t* n_overflow_out, int32_t* rebuild_count, hipStream_t stream) {
  return skin_update_impl(c, coords, types, n, every, images, nlist_out, n_overflow_out, rebuild_count, stream);
}

int dp_build_nlist_batch(dp_ctx* c, const double* coords, const int32_t* types, const double* boxes,
                         const int64_t* frame_off, int32_t nframes, int32_t* nlist_out, int32_t* n_overflow_out,
                         hipStream_t stream) {
  if (!boxes || !frame_off) { set_error("boxes/frame_off are NULL"); return DP_ERR_BAD_ARG; }
  return nlist_impl(c, coords, types, boxes, frame_off, nframes, nlist_out, n_overflow_out, stream);
}

int dp_compute(dp_ctx* c, const double* coords, const int32_t* types, const double* box, int64_t n,
               const int32_t* nlist, int32_t mode, double* energy, double* atom_energy, double* forces,
               double* virial, hipStream_t stream) {
  if (n < 0) { set_error("n < 0"); return DP_ERR_BAD_ARG; }
  const int64_t off[2] = {0, n};
  return compute_impl(c, coords, types, box, off, 1, nlist, mode, energy, atom_energy, forces, virial, stream);
}

int dp_compute_batch(dp_ctx* c, const double* coords, const int32_t* types, const double* boxes,
                     const int64_t* frame_off, int32_t nframes, const int32_t* nlist, int32_t mode,
                     double* energies, double* forces, double* virials, hipStream_t stream) {
  if (!boxes || !frame_off) { set_error("boxes/frame_off are NULL"); return DP_ERR_BAD_ARG; }
  return compute_impl(c, coords, types, boxes, frame_off, nframes, nlist, mode, energies, nullptr, forces, virials,
                      stream);
}

int dp_backward_params(dp_ctx* c, const double* dL_dE, double* grad_params, hipStream_t stream) {
  if (!c || !dL_dE || !grad_params) { set_error("NULL argument"); return DP_ERR_BAD_ARG; }
  if (!c->have_state) { set_error("dp_backward_params needs a preceding dp_compute"); return DP_ERR_STATE; }
  if (c->mode_last == DP_FP64_TAB) { set_error("the tabulated model has no parameter gradient"); return DP_ERR_UNSUPPORTED; }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  const dp_model* m = c->model;
  const int fw = m->fw, nd = m->nd, fwp = ((fw + 31) / 32) * 32;
  // computes store h2, h3 and dz2 (read only here) once a gradient pass
  // has run on the context; the first time, the fitting forward and
  // backward run again to form them (same inputs, same values for
  // everything they rewrite)
  c->train_h = true;
  if (!c->h_stored) {
    launch_fit_forward(c, c->mode_last, true, stream);
    launch_fit_backward(c, c->mode_last, true, stream);
    c->h_stored = true;
  }
  ParamGradInputs in;
  in.ldz = fw;
  if (c->mode_last == DP_FP64) {
    launch_descriptor_ex(c, DP_FP64, true, stream);  // D is only formed inside the GEMM on the force path
    in.X[0] = (const double*)c->D;
    in.X[1] = (const double*)c->fa[0];
    in.X[2] = (const double*)c->fa[2];
    in.dz[0] = (const double*)c->fa[8];
    in.dz[1] = (const double*)c->fa[7];
    in.dz[2] = (const double*)c->fa[5];
    in.h3 = (const double*)c->fa[4];
    in.gT = (const double*)c->gT;
  } else {
    // mixed: the layer inputs, deltas and g_T of the mixed-precision passes,
    // widened to FP64 into buffers the force path no longer needs; the
    // weight-gradient reductions then run in FP64
    // launch_widen kinds: 0 FP32, 1 BF16, 2 FP16
    const MixKinds mk = mix_kinds(c->mode_last);
    const int k1 = mk.fit1 == 3 ? 0 : mk.fit1, k23 = mk.fit23 == 3 ? 0 : mk.fit23;
    const int64_t cols = c->natoms_last + (int64_t)m->desc.ntypes * kColPad;
    // the embedding gradient recomputes the FP64 activations of the frame;
    // when the workspace holds them, the FP64 embedding forward with its
    // store runs first (same inputs, same values) and the gradient reads the
    // last layer back, which costs less than recomputing it there.  The
    // forward also writes Tpart, which the widened g_T takes below.
    if (!c->grad_act && c->act &&
        (int64_t)c->natoms_last * m->tpa * (int64_t)m->m1 * 16 * 8 <= c->act_bytes) {
      c->grad_act = true;
      launch_embed_fwd(c, nullptr, DP_FP64, stream);
    }
    double* D64 = (double*)c->dD;
    double* f64[6] = {(double*)c->fa[1], (double*)c->fa[3], (double*)c->fa[10],
                      (double*)c->fa[11], (double*)c->fa[5], (double*)c->fa[6]};
    launch_widen(c->D, k1, nd, D64, nd, nd, cols, stream);
    launch_widen(c->fa[0], 0, fwp, f64[0], fw, fw, cols, stream);  // h1
    launch_widen(c->fa[2], 0, fwp, f64[1], fw, fw, cols, stream);  // h2
    launch_widen(c->fa[4], 0, fwp, f64[2], fw, fw, cols, stream);  // h3
    launch_widen(c->fa[9], k1, fwp, f64[3], fw, fw, cols, stream);  // dz1
    launch_widen(c->fa[8], k23, fwp, f64[4], fw, fw, cols, stream);  // dz2
    launch_widen(c->fa[7], k23, fwp, f64[5], fw, fw, cols, stream);  // dz3
    double* gT64 = (double*)c->Tpart;
    launch_widen(c->gT, 0, m->m1 * 4, gT64, m->m1 * 4, m->m1 * 4, cols, stream);
    in.X[0] = D64;
    in.X[1] = f64[0];
    in.X[2] = f64[1];
    in.h3 = f64[2];
    in.dz[0] = f64[3];
    in.dz[1] = f64[4];
    in.dz[2] = f64[5];
    in.gT = gT64;
  }
  in.ldx[0] = nd;
  in.ldx[1] = fw;
  in.ldx[2] = fw;
  launch_param_grads(c, in, dL_dE, grad_params, stream);
  HIPCHECK(hipGetLastError());
  return DP_OK;
}

int dp_md_kick_drift(dp_ctx* c, double* coords, double* vel, const double* forces, const int32_t* types,
                     const double* box, int64_t n, double dt, int32_t wrap, int32_t* images, hipStream_t stream) {
  if (!c || n < 0 || (n > 0 && (!coords || !vel || !forces || !types))) { set_error("bad arguments"); return DP_ERR_BAD_ARG; }
  if (n > c->max_atoms) { set_error("n exceeds max_atoms"); return DP_ERR_CAPACITY; }
  if (!std::isfinite(dt)) { set_error("dt not finite"); return DP_ERR_BAD_ARG; }
  double L[3];
  int rc;
  if (wrap && (rc = check_box(box, c->model->desc.rcut, L))) return rc;
  if ((rc = set_device(c->device))) return rc;
  StageScope p(c, DP_STAGE_MD, stream);
  launch_kick_drift(c, coords, vel, forces, types, (int32_t)n, dt, wrap ? L : nullptr, images, stream);
  HIPCHECK(hipGetLastError());
  return DP_OK;
}

int dp_md_kick(dp_ctx* c, double* vel, const double* forces, const int32_t* types, int64_t n, double dt, double* ke,
               hipStream_t stream) {
  if (!c || n < 0 || !ke || (n > 0 && (!vel || !forces || !types))) { set_error("bad arguments"); return DP_ERR_BAD_ARG; }
  if (n > c->max_atoms) { set_error("n exceeds max_atoms"); return DP_ERR_CAPACITY; }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  StageScope p(c, DP_STAGE_MD, stream);
  launch_kick(c, vel, forces, types, (int32_t)n, dt, ke, stream);
  HIPCHECK(hipGetLastError());
  return DP_OK;
}

int dp_ctx_status(dp_ctx* c, int32_t* flags) {
  if (!c || !flags) { set_error("NULL argument"); return DP_ERR_BAD_ARG; }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  HIPCHECK(hipStreamSynchronize(c->last_stream));
  HIPCHECK(hipMemcpy(c->flags_host, c->flags_dev, 4, hipMemcpyDeviceToHost));
  *flags = *c->flags_host;
  launch_fill_i32(c->flags_dev, 0, 1, c->last_stream);
  HIPCHECK(hipStreamSynchronize(c->last_stream));
  return DP_OK;
}

int dp_ctx_store_info(dp_ctx* c, int64_t* capacity_bytes, int32_t* last_used) {
  if (!c) { set_error("ctx is NULL"); return DP_ERR_BAD_ARG; }
  if (capacity_bytes) *capacity_bytes = c->act_bytes;
  if (last_used) *last_used = c->act_used_last ? 1 : (c->grad_act ? 2 : 0);
  return DP_OK;
}

int dp_ctx_copy_buffer(dp_ctx* c, int32_t which, void* dst, int64_t* nbytes, hipStream_t stream) {
  if (!c || !nbytes) { set_error("NULL argument"); return DP_ERR_BAD_ARG; }
  const dp_model* m = c->model;
  const int64_t n = c->natoms_last;
  int64_t bytes;
  switch (which) {
    case 0: case 4: bytes = n * m->nm * 4 * 8; break;
    case 1: case 5: bytes = n * m->m1 * 4 * 8; break;
    case 2: case 3: bytes = n * m->nd * 8; break;
    default: set_error("which %d out of range", which); return DP_ERR_BAD_ARG;
  }
  *nbytes = bytes;
  if (!dst) return DP_OK;
  if (!c->have_state) { set_error("no compute on this context yet"); return DP_ERR_STATE; }
  int rc;
  if ((rc = set_device(c->device))) return rc;
  if (which == 0) HIPCHECK(hipMemcpyAsync(dst, c->R, bytes, hipMemcpyDeviceToDevice, stream));
  else if (which == 4) HIPCHECK(hipMemcpyAsync(dst, c->netd, bytes, hipMemcpyDeviceToDevice, stream));
  else {
    const int32_t md = c->mode_last == DP_FP64_TAB ? DP_FP64 : c->mode_last;
    // buffers the compute did not form: D on the FP64 path (built inside
    // the GEMM), D and dE/dD with the fused half-precision first layer (which
    // writes D only on contexts that keep the layer inputs for gradients)
    if (which == 2 && (md == DP_FP64 || (fit1_fused(c, md) && !c->h_stored))) launch_descriptor_ex(c, md, true, stream);
    if (which == 3 && fit1_fused(c, md)) launch_fit1_bwd_gemm(c, md, stream);
    launch_gather_cols(c, which, md, (int32_t)n, (double*)dst, stream);
  }
  HIPCHECK(hipGetLastError());
  return DP_OK;
}

}  // extern "C"
