// Parameter gradients of an energy loss, sum_f dL/dE_f dE_f/dtheta, from the
// state of the last FP64 compute (energy-loss training of the model; the
// paper's model is trained this way, its Background section cites the
// training papers).  Everything downstream of E_f is linear in the seed, so
// each centre-atom column is weighted by w_col = dL/dE of its frame and the
// unit-seed deltas stored by the force backward are reused where they exist.
//
// Fitting weights:   dW_l = sum_col X_l[col]^T w_col dz_l[col]  (column
//   reduction; MFMA with columns along K, split over column chunks whose
//   partial sums are written to a workspace and summed in chunk order).
// Embedding weights: the backward of each neighbour row is recomputed (as in
//   the force path, with g_T scaled by w_col; the last layer's tanh is read
//   from the forward's activation store when that was kept); per 16-row tile
//   the activations and deltas are transposed through LDS so that the
//   reduction over rows is an MFMA product, accumulated in per-work-group LDS
//   sums that are written to the workspace and summed in work-group order.
//   No global atomics.  The fitting gradients are bitwise deterministic; in
//   the embedding gradients the LDS sums of a work-group take its waves'
//   contributions in arrival order, so they can differ in the last bits
//   from run to run (the work-group records are added in a fixed order).
#include "dp_internal.h"
#include "dp_device.h"

namespace dpse {

// ------------------------------------------------------------ column weights
__global__ void k_col_weights(const int32_t* __restrict__ atom_at, const int32_t* __restrict__ frame_of,
                              const double* __restrict__ dLdE, double* __restrict__ w, int ncols) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int i = atom_at[c];
  w[c] = i >= 0 ? dLdE[frame_of[i]] : 0.0;
}

// ------------------------------------------------------------ fitting grads
// out[m][n] += sum_{col in chunk} X[col][m] w[col] Y[col][n]; m < M, n < N
// (multiples of 16).  Block: 4 waves; wave w handles m-tile (blockIdx.y*4+w),
// all n-tiles; blockIdx.x = column chunk; blockIdx.z = type.
struct WGradArgs {
  const double* X;  int ldx;
  const double* Y;  int ldy;
  const double* w;
  const int32_t* meta;
  int M, N, chunk, nchunks;
  double* part;     // [type][chunk][M][N] partial sums
};

// Work-group blockIdx.y owns MT m-tiles of out; its wave w owns n-tiles
// NT w ... NT w + NT - 1 (slots past the last tile repeat it and are not
// stored), so the four waves read the same X values (served once from L1)
// and different Y; blockIdx.x = column chunk, blockIdx.z = type.  Per
// k-step of 4 columns a lane loads one value of X (scaled by w) per m-tile
// and one of Y per n-tile; the next step's operands are requested before
// the current products issue (two register buffers used alternately).
template <int MT, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_wgrad_cols(WGradArgs a) {
  const int t = blockIdx.z;
  const int n_t = a.meta[2 * t], cb = a.meta[2 * t + 1];
  const int c0 = blockIdx.x * a.chunk;
  if (c0 >= n_t) return;
  const int c1 = min(n_t, c0 + a.chunk);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int mtiles = a.M / 16, ntiles = a.N / 16;
  const int mg = blockIdx.y, ng = wv;
  if (ng * NT >= ntiles) return;
  int mt[MT], nt[NT];
#pragma unroll
  for (int j = 0; j < MT; ++j) mt[j] = min(mg * MT + j, mtiles - 1);
#pragma unroll
  for (int i = 0; i < NT; ++i) nt[i] = min(ng * NT + i, ntiles - 1);
  d4 acc[MT][NT];
#pragma unroll
  for (int j = 0; j < MT; ++j)
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[j][i] = d4{0.0, 0.0, 0.0, 0.0};
  // raw operands and the column weight are buffered and the weight is
  // applied when the step consumes them; columns past the chunk load the
  // chunk's last column (no branch around a load, so nothing forces an
  // early wait) and get weight 0
  double xA[MT], yA[NT], xB[MT], yB[NT], wA, wB;
  auto load = [&](int c, double* xv, double* yv, double& wv_) {
    const int64_t col = cb + min(c + g, c1 - 1);
    wv_ = a.w[col];
#pragma unroll
    for (int j = 0; j < MT; ++j) xv[j] = a.X[col * a.ldx + mt[j] * 16 + r16];
#pragma unroll
    for (int i = 0; i < NT; ++i) yv[i] = a.Y[col * a.ldy + nt[i] * 16 + r16];
  };
  auto step = [&](int c, const double* xv, const double* yv, double wl) {
    const double wc = c + g < c1 ? wl : 0.0;
    double ys[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) ys[i] = yv[i] * wc;
#pragma unroll
    for (int j = 0; j < MT; ++j)
#pragma unroll
      for (int i = 0; i < NT; ++i) acc[j][i] = mfma_f64(xv[j], ys[i], acc[j][i]);
  };
  load(c0, xA, yA, wA);
  int c = c0;
  for (; c + 4 < c1; c += 8) {
    load(c + 4, xB, yB, wB);
    __builtin_amdgcn_sched_barrier(0);
    step(c, xA, yA, wA);
    __builtin_amdgcn_sched_barrier(0);
    load(c + 8, xA, yA, wA);  // past c1: weight 0
    __builtin_amdgcn_sched_barrier(0);
    step(c + 4, xB, yB, wB);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (c < c1) step(c, xA, yA, wA);
  double* out = a.part + ((int64_t)t * a.nchunks + blockIdx.x) * a.M * a.N;
#pragma unroll
  for (int j = 0; j < MT; ++j) {
    if (mg * MT + j >= mtiles) continue;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
      if (ng * NT + i >= ntiles) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = mt[j] * 16 + 4 * v + g;
        const int n = nt[i] * 16 + r16;
        out[(int64_t)m * a.N + n] = acc[j][i][v];
      }
    }
  }
}

// out[t][e] = sum over the chunks that hold columns of type t of part[t][c][e]
__global__ void k_sum_chunks(const double* __restrict__ part, const int32_t* __restrict__ meta, int chunk,
                             int nchunks, int E, double* __restrict__ out, int64_t out_type_stride, int64_t out_off) {
  const int t = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int used = (meta[2 * t] + chunk - 1) / chunk;
  const double* p = part + (int64_t)t * nchunks * E + e;
  double acc = 0.0;
  for (int c = 0; c < used; ++c) acc += p[(int64_t)c * E];
  out[t * out_type_stride + out_off + e] = acc;
}

// bias-type reductions: out[n] += sum_col w[col] Y[col][n] (Y == nullptr: 1)
// bias-type partial sums: part[t][chunk][n] = sum_col w[col] Y[col][n]
// (Y == nullptr: 1); a work-group of 4 waves splits the chunk's columns
// four ways and adds the quarters in LDS in a fixed order
__global__ __launch_bounds__(256) void k_bgrad_cols(const double* __restrict__ Y, int ldy, const double* __restrict__ w,
                                                    const int32_t* __restrict__ meta, int N, int chunk, int nchunks,
                                                    double* __restrict__ part) {
  __shared__ double red[4][256];
  const int t = blockIdx.z;
  const int n_t = meta[2 * t], cb = meta[2 * t + 1];
  const int c0 = blockIdx.x * chunk;
  if (c0 >= n_t) return;
  const int c1 = min(n_t, c0 + chunk);
  const int q = threadIdx.x >> 6, l = threadIdx.x & 63;
  double* out = part + ((int64_t)t * nchunks + blockIdx.x) * N;
  for (int n0 = 0; n0 < N; n0 += 64) {
    const int n = n0 + l;
    double acc = 0.0;
    if (n < N)
      for (int c = c0 + q; c < c1; c += 4) {
        const int64_t col = cb + c;
        acc += w[col] * (Y ? Y[col * ldy + n] : 1.0);
      }
    red[q][l] = acc;
    __syncthreads();
    if (q == 0 && n < N) out[n] = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
    __syncthreads();
  }
}

// ------------------------------------------------------------ embedding grads
struct EGradArgs {
  const int32_t* atom_at;
  const int32_t* meta;
  const double* R;
  const int32_t* nnei;
  const double* frag64;
  const double* vec64;
  int64_t vec_per_net;
  EmbFragOffsets fo;
  const double* gT;
  const double* wcol;
  double* grad;
  double* part;     // [net][slot][kEgRec] partial records
  int nslots;
  int64_t offW[kMaxT * kMaxT][3], offB[kMaxT * kMaxT][3];
  int ntypes, nm;
  int ngroups;      // work-groups per net (contiguous column ranges)
  int32_t* ctr;     // [nets][ngroups][32] per-work-group column counters
  int sec[kMaxT + 1];
  double inv_nm;
  // last embedding layer's tanh per 16-row tile of the forward pass
  // ([N, tpa, m1, 16]) when it was stored, else null (recomputed)
  const double* act;
  int tpa;
  int toff[kMaxT + 1];
};

template <int W>
__device__ __forceinline__ int e_feat1(int p) { return p < W ? p : -1; }
template <int W>
__device__ __forceinline__ int e_feat2(int p) { return (p & 31) < W ? (p >> 5) * W + (p & 31) : -1; }
template <int W>
__device__ __forceinline__ int e_feat3(int p) {
  const int f = e_feat2<W>(p & 63);
  return f < 0 ? -1 : (p >> 6) * 2 * W + f;
}

// waves per work-group of the embedding-gradient kernel: one work-group per
// CU holds the slot-indexed accumulators (82 KB) and per-wave buffers
// (16.5 KB + 32 B per feature); four waves fit in 160 KB up to M1 = 100.
template <int W>
constexpr int egw() { return 4 * W <= 100 ? 4 : 3; }
// k-step (t, v) of 16 t + 4 v + {0..3} holds only padding (w = 25: slots
// 28..31 mod 32); such products and activations are skipped
template <int W>
__device__ __forceinline__ constexpr bool g_kpad(int t, int v) {
  return W <= 28 && (t & 1) && v == 3;
}
// With padding in every 32-slot group, slot 31 of the layer inputs h1 and
// h2 holds 1.0 in the transposed buffers: the weight-gradient products then
// also yield the bias gradients (row 31 of dW2 and dW3), with no products
// of their own.
template <int W>
constexpr bool kBiasRow = W <= 28;
// partial record of one work-group (slot-indexed): W3 | W2 | b3 | b2 | b1 | W1
constexpr int kEgW3 = 0, kEgW2 = 64 * 128, kEgB3 = kEgW2 + 32 * 64, kEgB2 = kEgB3 + 128, kEgB1 = kEgB2 + 64,
              kEgW1 = kEgB1 + 32, kEgRec = kEgW1 + 32;

template <int W, bool ST>
__global__ __launch_bounds__(256) void k_embed_grad_f64(EGradArgs A) {
  constexpr int M1 = 4 * W, GW = egw<W>();
  // per-block accumulators (slot-indexed)
  __shared__ double aW3[64 * 128];
  __shared__ double aW2[32 * 64];
  __shared__ double aW1[32], aB1[32], aB2[64], aB3[128];
  // per-wave transposition buffers [row][slot]: h2 | one half of dz3, then
  // h1 | dz2 | dz1 | s
  __shared__ double tb[GW][16][129];
  __shared__ d4 gts[GW][M1];  // feature-indexed
  const int net = blockIdx.y;
  const int ti = net / A.ntypes, tj = net - ti * A.ntypes;
  const int n_t = A.meta[2 * ti], cb = A.meta[2 * ti + 1];
  // contiguous column range of this work-group; its waves take the columns
  // from a counter that only this work-group uses (next one requested ahead)
  const int c_lo = (int)((int64_t)n_t * blockIdx.x / gridDim.x);
  const int c_hi = (int)((int64_t)n_t * (blockIdx.x + 1) / gridDim.x);
  double* pr = A.part + ((int64_t)net * A.nslots + blockIdx.x) * kEgRec;
  if (c_lo >= c_hi) {
    for (int k = threadIdx.x; k < kEgRec; k += 64 * GW) pr[k] = 0.0;
    return;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  int* const next_col = A.ctr + (net * gridDim.x + blockIdx.x) * 32;
  if (threadIdx.x == 0) atomicExch(next_col, c_lo);
  auto take = [&]() {
    int k = 0;
    if (lane == 0) k = atomicAdd(next_col, 1);
    return k;
  };
  for (int k = threadIdx.x; k < 64 * 128; k += 64 * GW) aW3[k] = 0.0;
  for (int k = threadIdx.x; k < 32 * 64; k += 64 * GW) aW2[k] = 0.0;
  for (int k = threadIdx.x; k < 128; k += 64 * GW) {
    aB3[k] = 0.0;
    if (k < 64) aB2[k] = 0.0;
    if (k < 32) { aB1[k] = 0.0; aW1[k] = 0.0; }
  }
  __syncthreads();
  const double* base = A.frag64 + net * A.fo.per_net;
  const double* vec = A.vec64 + net * A.vec_per_net;
  double w1s[2][4], b1s[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      w1s[mt][v] = vec[16 * mt + 4 * v + g];
      b1s[mt][v] = vec[32 + 16 * mt + 4 * v + g];
    }
  double (*T)[129] = tb[wv];
  for (int c_next = take();;) {
    const int c = __builtin_amdgcn_readfirstlane(c_next);
    if (c >= c_hi) break;
    c_next = take();
    const int col = cb + c;
    const int i = A.atom_at[col];
    const double wc = A.wcol[col];
    {
      const double* gT = A.gT + (int64_t)col * (4 * W) * 4;
      wave_lds_sync();
      for (int a = lane; a < M1; a += 64) gts[wv][a] = *reinterpret_cast<const d4*>(gT + a * 4) * (A.inv_nm * wc);
      wave_lds_sync();
    }
    const int nn = A.nnei[i * kMaxT + tj];
    const double* Rs = A.R + ((int64_t)i * A.nm + A.sec[tj]) * 4;
    const env_rsrc_t Rb = env_rsrc(Rs, nn);
    d4 R_next = env_row(Rb, r16);  // row of the next tile is always in flight
    for (int r0 = 0; r0 < nn; r0 += 16) {
      const double* F2 = opaque(base + A.fo.F2);
      const double* F3 = opaque(base + A.fo.F3t);
      const double* B3 = opaque(base + A.fo.B3);
      const double* B2 = opaque(base + A.fo.B2);
      const int row = r0 + r16;
      const d4 Rrow = R_next;  // zero past the section's real rows
      R_next = env_row(Rb, row + 16);
      const double s = Rrow[0];
      double t1[2][4];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) t1[mt][v] = g_kpad<W>(mt, v) ? 0.0 : tanh_d(fma(s, w1s[mt][v], b1s[mt][v]));
      double t2[4][4], h2[4][4];
      // weight fragments are requested one group ahead of their products
      // (one wave per SIMD: nothing else hides their latency)
      double f2[2][8];
      auto ld_f2 = [&](int ot, double* f) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            f[mt * 4 + v] = g_kpad<W>(mt, v) ? 0.0 : F2[((ot * 2 + mt) * 4 + v) * 64 + lane];
      };
      ld_f2(0, f2[0]);
#pragma unroll
      for (int ot = 0; ot < 4; ++ot) {
        if (ot + 1 < 4) ld_f2(ot + 1, f2[(ot + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        d4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (!g_kpad<W>(mt, v)) z = mfma_f64(f2[ot & 1][mt * 4 + v], t1[mt][v], z);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          t2[ot][v] = g_kpad<W>(ot, v) ? 0.0 : tanh_d(z[v] + vec[64 + 16 * ot + 4 * v + g]);
          h2[ot][v] = t1[ot & 1][v] + t2[ot][v];
        }
      }
      wave_lds_sync();
      // h2 -> T[row][0..64) (slot 31: 1.0 for the bias gradient)
#pragma unroll
      for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int v = 0; v < 4; ++v) T[r16][16 * ot + 4 * v + g] = h2[ot][v];
      if (kBiasRow<W> && g == 3) T[r16][31] = 1.0;
      double skip2[4][4];
      d4 dh2a[4];
#pragma unroll
      for (int ot = 0; ot < 4; ++ot) {
        dh2a[ot] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int v = 0; v < 4; ++v) skip2[ot][v] = 0.0;
      }
      // stored t3 of the tile: slot p = 64 oo + 16 o4 + 4 v + g holds feature
      // 2W oo + W (o4 / 2) + 16 (o4 % 2) + 4 v + g when 16 (o4 % 2) + 4 v + g
      // < W; a padding slot may read past its record (one record of slack at
      // the end of the store) and its value is not used
      const double* rec =
          ST ? A.act + ((int64_t)i * A.tpa + A.toff[tj] + (r0 >> 4)) * (M1 * 16) + g * 16 + r16 : nullptr;
#pragma unroll 1
      for (int oo = 0; oo < 2; ++oo) {
        const double* F3o = opaque(F3 + oo * 4 * 16 * 64);
        const double* B3o = opaque(B3 + oo * 4 * 4 * 64);
        double t3v[16];
        if constexpr (ST) {
#pragma unroll
          for (int o4 = 0; o4 < 4; ++o4)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int lo = 16 * (o4 & 1) + 4 * v;
              t3v[o4 * 4 + v] = (lo < W) ? rec[(oo * 2 * W + (o4 >> 1) * W + lo) * 16] : 0.0;
            }
        }
        double fb[2][16];
        auto ld_b3 = [&](int o4, double* f) {
#pragma unroll
          for (int i2 = 0; i2 < 4; ++i2)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              f[i2 * 4 + v] = g_kpad<W>(o4, v) ? 0.0 : B3o[((i2 * 8 + o4) * 4 + v) * 64 + lane];
        };
        ld_b3(0, fb[0]);
#pragma unroll
        for (int o4 = 0; o4 < 4; ++o4) {
          if (o4 + 1 < 4) ld_b3(o4 + 1, fb[(o4 + 1) & 1]);
          __builtin_amdgcn_sched_barrier(0);
          d4 z = {0.0, 0.0, 0.0, 0.0};
          if constexpr (!ST) {
            const double* b3 = vec + 128 + 16 * (4 * oo + o4) + g;
            z = d4{b3[0], b3[4], b3[8], b3[12]};
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
              for (int v = 0; v < 4; ++v) z = mfma_f64(F3o[((o4 * 4 + mt) * 4 + v) * 64 + lane], h2[mt][v], z);
          }
          double dz3[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int a = e_feat3<W>(16 * (4 * oo + o4) + 4 * v + g);
            const double t3 = ST ? t3v[o4 * 4 + v] : tanh_d(z[v]);
            double dG = 0.0;
            if (a >= 0) {
              const d4 gt = gts[wv][a];
              dG = gt[0] * Rrow[0] + gt[1] * Rrow[1] + gt[2] * Rrow[2] + gt[3] * Rrow[3];
            }
            dz3[v] = a >= 0 ? dG * (1.0 - t3 * t3) : 0.0;
            skip2[o4][v] += dG;
            T[r16][64 + 16 * o4 + 4 * v + g] = dz3[v];
          }
#pragma unroll
          for (int i2 = 0; i2 < 4; ++i2)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (!g_kpad<W>(o4, v)) dh2a[i2] = mfma_f64(fb[o4 & 1][i2 * 4 + v], dz3[v], dh2a[i2]);
        }
        wave_lds_sync();
        // dW3[p][q] += sum_row h2[row][p] dz3[row][q];  db3[q] += sum_row dz3[row][q]  (q in this half)
        const double one = 1.0;
        // the h2 operands are the same for every q tile: read once
        double hA[4][4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
          for (int pt = 0; pt < 4; ++pt) hA[ks][pt] = T[4 * ks + g][16 * pt + r16];
#pragma unroll 1
        for (int qh = 0; qh < 4; ++qh) {
          const int qt = 4 * oo + qh;
          d4 acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
          d4 bacc = {0, 0, 0, 0};
          double bqv[4];
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) bqv[ks] = T[4 * ks + g][64 + 16 * qh + r16];
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const double bq = bqv[ks];
#pragma unroll
            for (int pt = 0; pt < 4; ++pt) acc[pt] = mfma_f64(hA[ks][pt], bq, acc[pt]);
            if constexpr (!kBiasRow<W>) bacc = mfma_f64(one, bq, bacc);
          }
#pragma unroll
          for (int pt = 0; pt < 4; ++pt)
#pragma unroll
            for (int v = 0; v < 4; ++v) atomicAdd(&aW3[(16 * pt + 4 * v + g) * 128 + 16 * qt + r16], acc[pt][v]);
          if (!kBiasRow<W> && g == 0) atomicAdd(&aB3[16 * qt + r16], bacc[0]);
        }
        wave_lds_sync();  // the next half overwrites dz3
      }
      // dz2 = (dh2 + skip)(1 - t2^2); dh1 = W2 dz2 + skip; dz1 = dh1 (1 - t1^2)
      double dz2[4][4], skip1[2][4];
      double fb2[2][16];
      auto ld_b2 = [&](int i2, double* f) {
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            f[o * 4 + v] = g_kpad<W>(o, v) ? 0.0 : B2[((i2 * 4 + o) * 4 + v) * 64 + lane];
      };
      ld_b2(0, fb2[0]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
        for (int v = 0; v < 4; ++v) skip1[i2][v] = 0.0;
#pragma unroll
      for (int i2 = 0; i2 < 4; ++i2)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double dh2 = dh2a[i2][v] + skip2[i2][v];
          dz2[i2][v] = dh2 * (1.0 - t2[i2][v] * t2[i2][v]);
          skip1[i2 & 1][v] += dh2;
        }
      double dz1[2][4];
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2) {
        if (i2 == 0) ld_b2(1, fb2[1]);
        __builtin_amdgcn_sched_barrier(0);
        d4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (!g_kpad<W>(o, v)) z = mfma_f64(fb2[i2][o * 4 + v], dz2[o][v], z);
#pragma unroll
        for (int v = 0; v < 4; ++v) dz1[i2][v] = (z[v] + skip1[i2][v]) * (1.0 - t1[i2][v] * t1[i2][v]);
      }
      wave_lds_sync();
      // buffer: h1 [0,32), dz2 [32,96), dz1 [96,128), s at 128
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T[r16][16 * mt + 4 * v + g] = t1[mt][v];
          T[r16][96 + 16 * mt + 4 * v + g] = dz1[mt][v];
        }
#pragma unroll
      for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int v = 0; v < 4; ++v) T[r16][32 + 16 * ot + 4 * v + g] = dz2[ot][v];
      if (g == 0) T[r16][128] = row < nn ? s : 0.0;
      if (kBiasRow<W> && g == 3) T[r16][31] = 1.0;  // h1 slot 31 (padding)
      wave_lds_sync();
      {
        const double one = 1.0;
        double h1A[4][2];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
          for (int pt = 0; pt < 2; ++pt) h1A[ks][pt] = T[4 * ks + g][16 * pt + r16];
#pragma unroll 1
        for (int qt = 0; qt < 4; ++qt) {
          d4 acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
          d4 bacc = {0, 0, 0, 0};
          double bqv[4];
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) bqv[ks] = T[4 * ks + g][32 + 16 * qt + r16];
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const double bq = bqv[ks];
#pragma unroll
            for (int pt = 0; pt < 2; ++pt) acc[pt] = mfma_f64(h1A[ks][pt], bq, acc[pt]);
            if constexpr (!kBiasRow<W>) bacc = mfma_f64(one, bq, bacc);
          }
#pragma unroll
          for (int pt = 0; pt < 2; ++pt)
#pragma unroll
            for (int v = 0; v < 4; ++v) atomicAdd(&aW2[(16 * pt + 4 * v + g) * 64 + 16 * qt + r16], acc[pt][v]);
          if (!kBiasRow<W> && g == 0) atomicAdd(&aB2[16 * qt + r16], bacc[0]);
        }
        // dW1[q] = sum_row s dz1[q] and db1[q] = sum_row dz1[q] as rows 0
        // and 1 of one product (A row 0: s, row 1: 1)
#pragma unroll
        for (int qt = 0; qt < 2; ++qt) {
          d4 wacc = {0, 0, 0, 0};
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const int rr = 4 * ks + g;
            const double bq = T[rr][96 + 16 * qt + r16];
            const double sr = T[rr][128];  // read by every lane, then selected
            wacc = mfma_f64(r16 == 0 ? sr : (r16 == 1 ? one : 0.0), bq, wacc);
          }
          if (g == 0) atomicAdd(&aW1[16 * qt + r16], wacc[0]);
          if (g == 1) atomicAdd(&aB1[16 * qt + r16], wacc[0]);
        }
      }
    }
  }
  __syncthreads();
  // slot-indexed block sums -> this work-group's partial record
  for (int k = threadIdx.x; k < 64 * 128; k += 64 * GW) pr[kEgW3 + k] = aW3[k];
  for (int k = threadIdx.x; k < 32 * 64; k += 64 * GW) pr[kEgW2 + k] = aW2[k];
  for (int k = threadIdx.x; k < 128; k += 64 * GW) {
    pr[kEgB3 + k] = kBiasRow<W> ? aW3[31 * 128 + k] : aB3[k];
    if (k < 64) pr[kEgB2 + k] = kBiasRow<W> ? aW2[31 * 64 + k] : aB2[k];
    if (k < 32) {
      pr[kEgB1 + k] = aB1[k];
      pr[kEgW1 + k] = aW1[k];
    }
  }
}

// sums the partial records of the work-groups that held columns, in
// work-group order, and maps slots to the flat parameter layout
template <int W>
__global__ void k_egrad_reduce(EGradArgs A) {
  const int net = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kEgRec) return;
  const int used = A.ngroups;
  int dst = -1;
  if (k < kEgW2) {
    const int fi = e_feat2<W>(k >> 7), fo = e_feat3<W>(k & 127);
    if (fi >= 0 && fo >= 0) dst = (int)A.offW[net][2] + fi * 4 * W + fo;
  } else if (k < kEgB3) {
    const int kk = k - kEgW2, fi = e_feat1<W>(kk >> 6), fo = e_feat2<W>(kk & 63);
    if (fi >= 0 && fo >= 0) dst = (int)A.offW[net][1] + fi * 2 * W + fo;
  } else if (k < kEgB2) {
    const int f3 = e_feat3<W>(k - kEgB3);
    if (f3 >= 0) dst = (int)A.offB[net][2] + f3;
  } else if (k < kEgB1) {
    const int f2 = e_feat2<W>(k - kEgB2);
    if (f2 >= 0) dst = (int)A.offB[net][1] + f2;
  } else if (k < kEgW1) {
    if (k - kEgB1 < W) dst = (int)A.offB[net][0] + (k - kEgB1);
  } else {
    if (k - kEgW1 < W) dst = (int)A.offW[net][0] + (k - kEgW1);
  }
  if (dst < 0) return;
  const double* p = A.part + (int64_t)net * A.nslots * kEgRec + k;
  double acc = 0.0;
  for (int c = 0; c < used; ++c) acc += p[(int64_t)c * kEgRec];
  A.grad[dst] = acc;
}

// ------------------------------------------------------------ launcher
__global__ void k_widen(const void* __restrict__ src, int kind, int ld_src, double* __restrict__ dst, int ld_dst,
                        int width, int64_t rows) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rows * width) return;
  const int64_t r = q / width;
  const int k = (int)(q - r * width);
  const int64_t si = r * ld_src + k;
  double v;
  if (kind == 0) v = (double)static_cast<const float*>(src)[si];
  else if (kind == 1) v = (double)PrecBF16::tof(static_cast<const uint16_t*>(src)[si]);
  else v = (double)PrecF16::tof(static_cast<const uint16_t*>(src)[si]);
  dst[r * ld_dst + k] = v;
}

void launch_widen(const void* src, int kind, int ld_src, double* dst, int ld_dst, int width, int64_t rows,
                  hipStream_t s) {
  const int64_t n = rows * width;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, kind, ld_src, dst, ld_dst, width,
                     rows);
}

void launch_param_grads(dp_ctx* c, const ParamGradInputs& in, const double* dLdE, double* grad, hipStream_t s) {
  const dp_model* m = c->model;
  const int n = (int)c->natoms_last;
  const int nt = m->desc.ntypes;
  const int ncols = (int)(c->natoms_last + nt * kColPad);
  launch_fill_f64(grad, 0.0, m->n_params, s);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_col_weights, dim3((ncols + 255) / 256), dim3(256), 0, s, c->atom_at, c->frame_of, dLdE,
                     c->gE_col, ncols);
  // ---- fitting: per layer dW = X^T diag(w) dz, db = sum w dz; w_out, b_out, e_bias
  // Column chunks of a type write partial sums into the workspace, which the
  // next kernel sums in chunk order; launches on one stream reuse it in turn.
  const int fw = m->fw, nd = m->nd;
  const int Kin[3] = {nd, fw, fw};
  auto sum_chunks = [&](int E, int chunk, int nch, int64_t stride, int64_t off) {
    hipLaunchKernelGGL(k_sum_chunks, dim3((E + 255) / 256, nt), dim3(256), 0, s, c->gpart, c->type_meta, chunk, nch,
                       E, grad, stride, off);
  };
  // bias-type sums have tiny partials: short chunks, many work-groups
  const int bchunk = 256;
  const int bnch = (n + bchunk - 1) / bchunk;
  auto bgrad = [&](const double* Y, int N, int64_t stride, int64_t off) {
    hipLaunchKernelGGL(k_bgrad_cols, dim3(bnch, 1, nt), dim3(256), 0, s, Y, in.ldz, c->gE_col, c->type_meta, N, bchunk,
                       bnch, c->gpart);
    hipLaunchKernelGGL(k_sum_chunks, dim3((N + 255) / 256, nt), dim3(256), 0, s, c->gpart, c->type_meta, bchunk, bnch,
                       N, grad, stride, off);
  };
  // column chunks per layer: about two waves per SIMD in one round (4 x 4
  // tiles per wave, four waves per work-group cover 16 n-tiles), within the
  // workspace (sized for grad_chunks chunks of the first layer), chunks of
  // at least 64 columns
  constexpr int WMT = 4, WNT = 4;
  const int64_t cap = (int64_t)c->grad_chunks * nd * fw;  // per type
  for (int l = 0; l < 3; ++l) {
    const int mgroups = (Kin[l] / 16 + WMT - 1) / WMT;
    int64_t want = (2LL * c->ncu) / ((int64_t)mgroups * nt);
    if (want < 1) want = 1;
    const int64_t fit = cap / ((int64_t)Kin[l] * fw);
    const int64_t most = (n + 63) / 64;
    if (want > fit) want = fit;
    if (want > most) want = most;
    const int nch = (int)(want < 1 ? 1 : want);
    const int chunk = (n + nch - 1) / nch;
    WGradArgs a = {};
    a.X = in.X[l];
    a.ldx = in.ldx[l];
    a.Y = in.dz[l];
    a.ldy = in.ldz;
    a.w = c->gE_col;
    a.meta = c->type_meta;
    a.M = Kin[l];
    a.N = fw;
    a.chunk = chunk;
    a.nchunks = nch;
    a.part = c->gpart;
    dim3 grid(nch, mgroups, nt);
    hipLaunchKernelGGL((k_wgrad_cols<WMT, WNT>), grid, dim3(256), 0, s, a);
    sum_chunks(Kin[l] * fw, chunk, nch, m->fit_param_stride, m->fit_param_off[l]);
    bgrad(in.dz[l], fw, m->fit_param_stride, m->fit_param_off[3 + l]);
  }
  // w_out: sum w h3; b_out and e_bias: sum w
  bgrad(in.h3, fw, m->fit_param_stride, m->fit_param_off[6]);
  bgrad(nullptr, 1, m->fit_param_stride, m->fit_param_off[7]);
  bgrad(nullptr, 1, 1, m->ebias_off);
  // ---- embedding nets
  EGradArgs A = {};
  A.atom_at = c->atom_at;
  A.meta = c->type_meta;
  A.R = c->R;
  A.nnei = c->nnei;
  A.frag64 = m->emb_frag64;
  A.vec64 = m->emb_vec64;
  A.vec_per_net = m->emb_vec_per_net;
  A.fo = m->efo;
  A.gT = in.gT;
  A.wcol = c->gE_col;
  A.grad = grad;
  A.part = c->gpart;
  A.nslots = c->grad_slots;
  for (int k = 0; k < nt * nt; ++k)
    for (int l = 0; l < 3; ++l) {
      A.offW[k][l] = m->emb_param_off[k][2 * l];
      A.offB[k][l] = m->emb_param_off[k][2 * l + 1];
    }
  A.ntypes = nt;
  A.nm = m->nm;
  // one work-group per CU and net (at most nslots records per net)
  const int gw = m->w1 == 25 ? egw<25>() : egw<32>();
  int groups = c->ncu < A.nslots ? c->ncu : A.nslots;
  if ((int64_t)groups * gw > n) groups = (int)((n + gw - 1) / gw);
  A.ngroups = groups < 1 ? 1 : groups;
  A.ctr = c->emb_ctr;
  for (int t = 0; t <= kMaxT; ++t) A.sec[t] = t <= nt ? m->sec[t] : m->nm;
  A.inv_nm = 1.0 / (double)m->nm;
  dim3 grid(A.ngroups, nt * nt);
  dim3 rgrid((kEgRec + 255) / 256, nt * nt);
  // the forward's stored last-layer activations (FP64 computes that fit the
  // workspace) replace the recomputation of the last embedding layer
  A.act = c->act_used_last || c->grad_act ? (const double*)c->act : nullptr;
  A.tpa = m->tpa;
  for (int t = 0; t <= kMaxT; ++t) A.toff[t] = t <= nt ? m->toff[t] : m->tpa;
  if (m->w1 == 25) {
    if (A.act) hipLaunchKernelGGL((k_embed_grad_f64<25, true>), grid, dim3(64 * gw), 0, s, A);
    else hipLaunchKernelGGL((k_embed_grad_f64<25, false>), grid, dim3(64 * gw), 0, s, A);
    hipLaunchKernelGGL(k_egrad_reduce<25>, rgrid, dim3(256), 0, s, A);
  } else {
    if (A.act) hipLaunchKernelGGL((k_embed_grad_f64<32, true>), grid, dim3(64 * gw), 0, s, A);
    else hipLaunchKernelGGL((k_embed_grad_f64<32, false>), grid, dim3(64 * gw), 0, s, A);
    hipLaunchKernelGGL(k_egrad_reduce<32>, rgrid, dim3(256), 0, s, A);
  }
}

}  // namespace dpse
