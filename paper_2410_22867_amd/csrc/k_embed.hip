// Embedding nets and the G^T R contraction (Background section: the smoothed
// first column of R_i passes through the three-layer embedding net; the
// descriptor preserves the symmetries), forward and backward.
//
// Work layout.  One wavefront owns one centre atom (one fitting column) and
// walks its neighbour sections t_j = 0..ntypes-1 in tiles of 16 neighbour
// rows (only the real rows of a section: sections are sorted and padded at
// their end).  Inside a tile the activations live in registers in the MFMA
// output layout with features along M and the 16 rows along N ("transposed"
// layout): lane n + 16g holds features 16t + 4v + g (FP64) or 16t + 4g + v
// (16x16x32 forms) of row n, element v.  That tile is
// directly the B operand of the next layer (weights are the A operand, stored
// pre-arranged per lane at model load), so layers chain without LDS traffic.
//
// Slot layout (widths w, 2w, 4w with w <= 32): layer 1 uses 32 slots
// (feature f at slot f), layer 2 uses 64 (features [0, w) at slots [0, w),
// [w, 2w) at [32, 32 + w)), layer 3 uses 128 (two copies of the layer-2
// layout).  With that layout the identity skips of width-doubling layers,
// h_l = [h_{l-1}, h_{l-1}] + tanh(z_l), stay inside a lane.  The
// half-precision kernels order the layer-1 slots so that, for w <= 28, a
// whole register of each odd tile is padding (kpadh below).
//
// Forward: layer 3 is evaluated with rows along M instead (the layer-2 tile
// is a valid A operand as it is), so the contraction T = G^T R / nm reduces
// over 4 rows inside a lane and over the 4 lane groups once per atom; the
// layer-2 values needed by the layer-3 skip are exchanged through a
// wave-private LDS tile.  Backward recomputes layers 1-3 in the transposed
// layout, forms dE/dG = g_T R / nm and the direct term g_T^T G / nm, and
// back-propagates with the transposed-weight fragments to dE/ds.
//
// Activation store (ST, FP64 only): when the context's workspace budget holds
// it, the forward also writes the last layer's tanh output t3 = G - [h2, h2]
// of every 16-row tile as a [m1][16] record, and the backward reads it back
// instead of recomputing layer 3 (the widest layer: 4/5 of the net's
// products).  Layers 1 and 2 are always recomputed.  The mixed forms always
// recompute: their half-precision layer 3 costs less than the store's HBM
// round trip.
#include "dp_internal.h"
#include "dp_device.h"

namespace dpse {

struct EmbArgs {
  const int32_t* atom_at;
  const int32_t* meta;   // n_t, cbase_t per centre type
  const double* R;
  const int32_t* nnei;
  const double* frag64;
  const void* fraglp;     // mixed forms: fragments in the form's element type
  const double* vec64;
  const float* vec32;
  int64_t vec_per_net;
  EmbFragOffsets fo;
  void* Tpart;           // forward: [ntypes][cols][m1][4] partial T per neighbour section
  int64_t tpart_stride;  // elements between sections
  const void* gT;        // backward: [cols][m1][4]
  double* netd;
  void* act;             // last-layer tanh store [N][tpa][m1][16] (f64 / f32), or NULL
  int tpa;
  int toff[kMaxT];
  int ntypes, nm;
  int sec[kMaxT + 1];
  double inv_nm;
  int32_t* ctr;          // [nets][gridDim.x][32] per-work-group column counters
};

// Returns 0 in a register the optimiser cannot see through; added to LDS
// indices inside the neighbour-tile loop it keeps fragment loads in the loop.
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+v"(z));
  return z;
}

// per-net vector block: W1s[32] | b1s[32] | b2s[64] | b3s[128] | b3f[128]
constexpr int kV_W1 = 0, kV_B1 = 32, kV_B2 = 64, kV_B3S = 128, kV_B3F = 256, kVecPerNet = 384;

template <int W>
__device__ __forceinline__ int slot2_of_feat(int f) {  // f in [0, 2W)
  return (f / W) * 32 + (f % W);
}
template <int W>
__device__ __forceinline__ int feat3_of_slot(int p) {  // -1 for padding slots
  const int q = p & 63;
  if ((q & 31) >= W) return -1;
  return (p >> 6) * 2 * W + (q >> 5) * W + (q & 31);
}

// Slot order of the half-precision kernels (lane group g, element v hold
// slot 16t + 4g + v of tile t): for w <= 28 the layer-1 slots 16 + 4g + 3
// and their copies in the wider layers are padding, so element 3 of every
// odd tile is padding in all four lane groups and its activation is not
// evaluated; the features fill the other slots in order.
template <int W>
__device__ __forceinline__ constexpr bool kpadh(int t, int v) {
  return W <= 28 && (t & 1) && v == 3;
}
template <int W>
__device__ __forceinline__ int feat3h_of_slot(int p) {  // -1 for padding slots
  const int q = p & 31;
  int f = q;
  if (W <= 28 && q >= 16) f = (q & 3) == 3 ? W : 16 + 3 * ((q - 16) >> 2) + ((q - 16) & 3);
  if (f >= W) return -1;
  return (p >> 6) * 2 * W + ((p >> 5) & 1) * W + f;
}

// 2^(j/32), j = 0..31, correctly rounded (the table of tanh_d_tab)
__constant__ double kExp2Frac32[32] = {
    1.0, 1.0218971486541166, 1.0442737824274138, 1.0671404006768237, 1.0905077326652577, 1.1143867425958924,
    1.1387886347566916, 1.1637248587775775, 1.189207115002721, 1.215247359980469, 1.241857812073484,
    1.2690509571917332, 1.2968395546510096, 1.3252366431597413, 1.3542555469368927, 1.383909881963832,
    1.4142135623730951, 1.4451808069770467, 1.4768261459394993, 1.5091644275934228, 1.5422108254079407,
    1.5759808451078865, 1.6104903319492543, 1.645755478153965, 1.681792830507429, 1.718619298122478,
    1.7562521603732995, 1.7947090750031072, 1.8340080864093424, 1.8741676341103, 1.9152065613971474,
    1.9571441241754002};

// The net that work-group row y serves: the nets in decreasing order of
// their work, the centre type's columns times the neighbour section's row
// tiles (ceil(sel / 16)), ties in net order.  Rows are dispatched in order,
// so the heaviest net's work-groups start first and the lighter ones fill
// the end of the launch.
__device__ __forceinline__ int net_of_row(const int32_t* meta, const int* sec, int ntypes, int y) {
  const int nnets = ntypes * ntypes;
  int64_t wt[kMaxT * kMaxT];
  for (int k = 0; k < nnets; ++k) {
    const int kti = k / ntypes, ktj = k - kti * ntypes;
    wt[k] = (int64_t)meta[2 * kti] * ((sec[ktj + 1] - sec[ktj] + 15) / 16);
  }
  for (int k = 0; k < nnets; ++k) {
    int rank = 0;
    for (int q = 0; q < nnets; ++q) rank += wt[q] > wt[k] || (wt[q] == wt[k] && q < k);
    if (rank == y) return k;
  }
  return 0;
}

// Common prologue of the per-net kernels: net = t_i * ntypes + t_j (centre
// type t_i, neighbour section t_j) from net_of_group (one-row grid) or
// net_of_row (one grid row per net).  Work assignment: the
// net's columns are split into contiguous ranges, one per
// work-group; inside its range a wavefront takes the next column from the
// work-group's counter (a word in global memory that no other work-group
// touches, set by the work-group itself before its first barrier; the next
// column is requested one column ahead so the atomic's latency hides behind
// the current column) until the range is exhausted.  Each column's work is
// done by one wavefront (or, in group mode, by the work-group's waves in a
// fixed split), so results do not depend on the assignment; the waves of a
// work-group end within about one column of each other, whatever the spread
// of neighbour counts.
#define DPSE_NET_PROLOGUE(WPB)                                            \
  int grp = blockIdx.x, ngrp = gridDim.x;                                 \
  const int net = gridDim.y == 1                                          \
                      ? net_of_group(A.meta, A.sec, A.ntypes, gridDim.x, blockIdx.x, &grp, &ngrp) \
                      : net_of_row(A.meta, A.sec, A.ntypes, blockIdx.y);  \
  if (net < 0) return;                                                    \
  const int ti = net / A.ntypes, tj = net - ti * A.ntypes;                \
  const int n_t = A.meta[2 * ti], cb = A.meta[2 * ti + 1];                \
  const int c_lo = (int)((int64_t)n_t * grp / ngrp);                      \
  const int c_hi = (int)((int64_t)n_t * (grp + 1) / ngrp);                \
  if (c_lo >= c_hi) return;                                               \
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;              \
  const int r16 = lane & 15, g = lane >> 4;                               \
  (void)wv;                                                               \
  int* const next_col = A.ctr + (blockIdx.y * gridDim.x + blockIdx.x) * 32; \
  if (threadIdx.x == 0) atomicExch(next_col, c_lo);                       \
  auto take = [&]() {                                                     \
    int k = 0;                                                            \
    if (lane == 0) k = atomicAdd(next_col, 1);                            \
    return k;                                                             \
  };

// FP64 k-step (t, v) covers slots 16t + 4v + {0..3}; with w = 25 the slot
// groups 28..31 (mod 32) hold only padding, so those k-steps are skipped and
// the activations of those slots (tanh(0) = 0) are not evaluated.
//
// The FP64 kernels use a denser layout of the width-2w layer for w = 25
// (the mixed kernels, whose k-steps are 32 wide, keep the plain one).  Each
// half of the layer ends in a k-step (slots 24..27, 56..59) holding a
// single feature; both halves' last features (24 and 49) go to slots 24 and
// 25, and slots 26 and 27 hold copies of them, so that slots 56..59 are
// padding and their k-steps drop out.  A copy is computed like a feature
// (its layer-1 slot partner, slots 25..27 of layer 1, holds a copy of
// feature 24 of layer 1) but has no outgoing weights: the layer above
// reads only the original, and a copy reaches the output only through the
// identity skip.  That skip pairs layer-3 slot 64 zo + q with layer-2 slot
// q, so slots 24..27 of the first layer-3 half hold features 24, 49, 74
// and 99 (whose skip partners are 24, 49, 24, 49), and slots 24..27 of the
// second half are padding.  Gradients flow through the copies like
// through any other unit.
template <int W>
constexpr bool kDense2 = (W == 25);
template <int W>
__device__ __forceinline__ constexpr bool kpad(int t, int v) {  // layer-1 slots
  return W <= 28 && (t & 1) && v == 3;
}
template <int W>
__device__ __forceinline__ constexpr bool kpad2(int t, int v) {  // layer-2 slots, FP64 layout
  return kpad<W>(t, v) || (kDense2<W> && t == 3 && v == 2);
}
template <int W>
__device__ __forceinline__ constexpr bool kpad3(int zo, int t, int v) {  // layer-3 slots 64 zo + 16 t + 4 v + g
  return kpad2<W>(t, v) || (kDense2<W> && zo == 1 && t == 1 && v == 2);
}
template <int W>
__device__ __forceinline__ int slot2d_of_feat(int f) {  // f in [0, 2W), FP64 layout
  if (kDense2<W> && f == 2 * W - 1) return W;
  return slot2_of_feat<W>(f);
}
template <int W>
__device__ __forceinline__ int feat3d_of_slot(int p) {  // FP64 layout; -1 for padding slots
  if constexpr (kDense2<W>) {
    const int q = p & 63;
    if (q >= W - 1 && q < W + 3) return p < 64 ? (W - 1) + W * (q - (W - 1)) : -1;
    if (q >= 32 + W - 1) return -1;
  }
  return feat3_of_slot<W>(p);
}

// ============================================================== FP64 forward
// Group mode (GM, frames of few atoms): the work-group's waves share one
// column at a time, wave w taking its tiles w, w + WPB, ...; the waves'
// partial T are added in wave order through LDS.  Without it each wave owns
// a column and walks its tiles alone, which leaves most of the chip idle
// when there are fewer columns than wave slots.
template <int W, int WPB, bool ST, bool GM>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_embed_fwd_f64(EmbArgs A) {
  constexpr int M1 = 4 * W;
  constexpr int N3 = (M1 + 15) / 16;
  constexpr int NF2 = 2048, NF3 = N3 * 1024;
  // A last feature tile with at most 4 real features (w = 25: features
  // 96..99) is evaluated transposed, features along M: its real outputs are
  // then element 0 of every lane (one tanh per lane instead of four), and
  // its contraction runs over the lane's own row
  constexpr int REM = M1 % 16;
  constexpr bool TLAST = REM > 0 && REM <= 4;
  __shared__ double fr[NF2 + NF3];
  __shared__ double h2s[WPB][16][kP2 + 1];
  __shared__ double vs[kVecPerNet];
  __shared__ double etab[32];  // tanh_d_tab's table
  __shared__ int col_sh;  // group mode: the work-group's column
  DPSE_NET_PROLOGUE(WPB)
  {
    const double* src = A.frag64 + net * A.fo.per_net;
    for (int k = threadIdx.x; k < NF2; k += 64 * WPB) fr[k] = src[A.fo.F2 + k];
    for (int k = threadIdx.x; k < NF3; k += 64 * WPB) fr[NF2 + k] = src[A.fo.F3n + k];
    const double* vsrc = A.vec64 + net * A.vec_per_net;
    for (int k = threadIdx.x; k < kVecPerNet; k += 64 * WPB) vs[k] = vsrc[k];
    if (threadIdx.x < 32) etab[threadIdx.x] = kExp2Frac32[threadIdx.x];
  }
  __syncthreads();
  constexpr int RSTEP = GM ? 16 * WPB : 16;  // rows between a wave's tiles
  const int rfirst = GM ? 16 * wv : 0;

  for (int c_next = GM ? 0 : take();;) {
    int c;
    if constexpr (GM) {
      if (threadIdx.x == 0) col_sh = atomicAdd(next_col, 1);
      __syncthreads();
      c = __builtin_amdgcn_readfirstlane(col_sh);
    } else {
      c = __builtin_amdgcn_readfirstlane(c_next);
    }
    if (c >= c_hi) break;
    if constexpr (!GM) c_next = take();
    const int col = cb + c;
    const int i = A.atom_at[col];
    double accT[N3][4];
#pragma unroll
    for (int o = 0; o < N3; ++o)
#pragma unroll
      for (int k = 0; k < 4; ++k) accT[o][k] = 0.0;
    double accL[4] = {0.0, 0.0, 0.0, 0.0};  // last tile when transposed: feature 16 (N3 - 1) + g, over rows r16
    const int nn = A.nnei[i * kMaxT + tj];
    const double* Rs = A.R + ((int64_t)i * A.nm + A.sec[tj]) * 4;
    double s_next = rfirst + r16 < nn ? Rs[(rfirst + r16) * 4] : 0.0;  // s of the next tile is always in flight
    for (int r0 = rfirst; r0 < nn; r0 += RSTEP) {
      const int z0 = opaque_zero();
      const double* vec = vs + z0;  // per-tile LDS reads instead of hoisted registers
      const int row = r0 + r16;
      const double s = s_next;
      s_next = row + RSTEP < nn ? Rs[(row + RSTEP) * 4] : 0.0;
      double* const recb =
          ST ? static_cast<double*>(A.act) + ((int64_t)i * A.tpa + A.toff[tj] + (r0 >> 4)) * (M1 * 16) : nullptr;
      double* const rec = ST ? recb + r16 * 16 + g : nullptr;
      // the lane's own row (contraction of a transposed last tile)
      d4 Rown = {0.0, 0.0, 0.0, 0.0};
      if (TLAST && row < nn) Rown = *reinterpret_cast<const d4*>(Rs + row * 4);
      // rows of the contraction, requested before layers 1-2 run
      double Rr[4][4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = r0 + 4 * v + g;
        d4 x = {0.0, 0.0, 0.0, 0.0};
        if (rr < nn) x = *reinterpret_cast<const d4*>(Rs + rr * 4);
#pragma unroll
        for (int k = 0; k < 4; ++k) Rr[v][k] = x[k];
      }
      double h1[2][4];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          h1[mt][v] = kpad<W>(mt, v) ? 0.0 : tanh_d_tab(fma(s, vec[kV_W1 + 16 * mt + 4 * v + g], vec[kV_B1 + 16 * mt + 4 * v + g]), etab);
      double h2[4][4];
#pragma unroll
      for (int ot = 0; ot < 4; ++ot) {
        const double* b2 = vec + kV_B2 + 16 * ot + g;
        d4 z = {b2[0], b2[4], b2[8], b2[12]};
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (!kpad<W>(mt, v)) z = mfma_f64(fr[z0 + ((ot * 2 + mt) * 4 + v) * 64 + lane], h1[mt][v], z);
#pragma unroll
        for (int v = 0; v < 4; ++v) h2[ot][v] = kpad2<W>(ot, v) ? 0.0 : h1[ot & 1][v] + tanh_d_tab(z[v], etab);
      }
      wave_lds_sync();
#pragma unroll
      for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int v = 0; v < 4; ++v) h2s[wv][r16][16 * ot + 4 * v + g] = h2[ot][v];
      wave_lds_sync();
#pragma unroll
      for (int o = 0; o < N3; ++o) {
        if (TLAST && o == N3 - 1) {
          // features 16 o + 4 v + g along M, rows along N: element 0 holds
          // feature 16 o + g of row r0 + r16
          const int f = 16 * o + g;
          d4 z = {vec[kV_B3F + f], 0.0, 0.0, 0.0};
#pragma unroll
          for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (!kpad2<W>(mt, v)) z = mfma_f64(fr[z0 + NF2 + ((o * 4 + mt) * 4 + v) * 64 + lane], h2[mt][v], z);
          if (g < REM) {
            const double t3 = tanh_d_tab(z[0], etab);
            if constexpr (ST) recb[f * 16 + r16] = t3;
            const double G = h2s[wv][r16][slot2d_of_feat<W>(f % (2 * W))] + t3;
#pragma unroll
            for (int k = 0; k < 4; ++k) accL[k] = fma(G, Rown[k], accL[k]);
          }
          continue;
        }
        const int feat = 16 * o + r16;
        const double b3 = vec[kV_B3F + feat];  // the table spans kP3 features
        d4 z = {b3, b3, b3, b3};
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (!kpad2<W>(mt, v))
              z = mfma_f64(h2[mt][v], fr[z0 + NF2 + ((o * 4 + mt) * 4 + v) * 64 + lane], z);
        if (feat < M1) {
          const int src = slot2d_of_feat<W>(feat % (2 * W));
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double t3 = tanh_d_tab(z[v], etab);
            if constexpr (ST) rec[o * 256 + 4 * v] = t3;
            const double G = h2s[wv][4 * v + g][src] + t3;
#pragma unroll
            for (int k = 0; k < 4; ++k) accT[o][k] = fma(G, Rr[v][k], accT[o][k]);
          }
        }
      }
    }
    constexpr int NR = TLAST ? N3 - 1 : N3;  // tiles in the row-sum layout
#pragma unroll
    for (int o = 0; o < NR; ++o)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double x = accT[o][k];
        x += shfl_xor_d(x, 16);
        x += shfl_xor_d(x, 32);
        accT[o][k] = x * A.inv_nm;
      }
    double* T = reinterpret_cast<double*>(A.Tpart) + tj * A.tpart_stride + (int64_t)col * M1 * 4;
    if constexpr (TLAST) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double x = accL[k];
#pragma unroll
        for (int msk = 1; msk < 16; msk <<= 1) x += shfl_xor_d(x, msk);
        accL[k] = x * A.inv_nm;
      }
    }
    // group mode: each wave's partial T to LDS (the h2s tiles, free once
    // every wave has left its tile loop), then the sum in wave order
    double* const dst = GM ? &h2s[0][0][0] + wv * M1 * 4 : T;
    if constexpr (GM) __syncthreads();
    if (g == 0) {
#pragma unroll
      for (int o = 0; o < NR; ++o) {
        const int feat = 16 * o + r16;
        if (feat < M1) *reinterpret_cast<d4*>(dst + feat * 4) = d4{accT[o][0], accT[o][1], accT[o][2], accT[o][3]};
      }
    }
    if constexpr (TLAST) {
      if (r16 == 0 && g < REM)
        *reinterpret_cast<d4*>(dst + (16 * (N3 - 1) + g) * 4) = d4{accL[0], accL[1], accL[2], accL[3]};
    }
    if constexpr (GM) {
      static_assert(WPB * M1 * 4 <= WPB * 16 * (kP2 + 1), "partials fit the h2s tiles");
      __syncthreads();
      const double* red = &h2s[0][0][0];
      for (int e = threadIdx.x; e < M1 * 4; e += 64 * WPB) {
        double x = red[e];
        for (int w = 1; w < WPB; ++w) x += red[w * M1 * 4 + e];
        T[e] = x;
      }
      __syncthreads();  // h2s and col_sh are reused by the next column
    }
  }
}

// ============================================================== FP64 backward
// GM: group mode as in the forward (the waves share the column's g_T tile).
template <int W, int WPB, bool ST, bool GM>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_embed_bwd_f64(EmbArgs A) {
  constexpr int M1 = 4 * W;
  // F3t | B3; with the activation store F3t is not needed and its space
  // holds F2 | B2 | the vector block instead (no global operand loads)
  __shared__ double fr[8192 + 8192];
  __shared__ d4 gts[GM ? 1 : WPB][kP3];
  __shared__ int col_sh;  // group mode: the work-group's column
  DPSE_NET_PROLOGUE(WPB)
  const double* gsrc = A.frag64 + net * A.fo.per_net;
  const double* vecg = A.vec64 + net * A.vec_per_net;
  for (int k = threadIdx.x; k < 8192; k += 64 * WPB) {
    if constexpr (!ST) {
      fr[k] = gsrc[A.fo.F3t + k];
    } else {
      if (k < 2048) fr[k] = gsrc[A.fo.F2 + k];
      else if (k < 4096) fr[k] = gsrc[A.fo.B2 + k - 2048];
      else if (k < 4096 + kVecPerNet) fr[k] = vecg[k - 4096];
      else if (k < 4096 + kVecPerNet + 32) fr[k] = kExp2Frac32[k - 4096 - kVecPerNet];  // tanh_d_tab's table
    }
    fr[8192 + k] = gsrc[A.fo.B3 + k];
  }
  __syncthreads();
  // layers 1-2: the table form of the FP64 tanh where the store leaves LDS
  // room for its table
  const double* etab = fr + 4096 + kVecPerNet;
  auto tanh_l = [&](double x) { return ST ? tanh_d_tab(x, etab) : tanh_d(x); };
  const int gw = GM ? 0 : wv;  // this wave's g_T tile
  constexpr int RSTEP = GM ? 16 * WPB : 16;
  const int rfirst = GM ? 16 * wv : 0;
  for (int c_next = GM ? 0 : take();;) {
    int c;
    if constexpr (GM) {
      if (threadIdx.x == 0) col_sh = atomicAdd(next_col, 1);
      __syncthreads();
      c = __builtin_amdgcn_readfirstlane(col_sh);
    } else {
      c = __builtin_amdgcn_readfirstlane(c_next);
    }
    if (c >= c_hi) break;
    if constexpr (!GM) c_next = take();
    const int col = cb + c;
    const int i = A.atom_at[col];
    {
      const double* gT = reinterpret_cast<const double*>(A.gT) + (int64_t)col * M1 * 4;
      if constexpr (!GM) wave_lds_sync();
      for (int p = GM ? (int)threadIdx.x : lane; p < kP3; p += GM ? 64 * WPB : 64) {
        const int a = feat3d_of_slot<W>(p);
        d4 x = {0.0, 0.0, 0.0, 0.0};
        if (a >= 0) x = *reinterpret_cast<const d4*>(gT + a * 4) * A.inv_nm;
        gts[gw][p] = x;
      }
      if constexpr (GM) __syncthreads();
      else wave_lds_sync();
    }
    const int nn = A.nnei[i * kMaxT + tj];
    const int64_t rbase = (int64_t)i * A.nm + A.sec[tj];
    const double* Rs = A.R + rbase * 4;
    d4 R_next = {0.0, 0.0, 0.0, 0.0};  // row of the next tile is always in flight
    if (rfirst + r16 < nn) R_next = *reinterpret_cast<const d4*>(Rs + (rfirst + r16) * 4);
    for (int r0 = rfirst; r0 < nn; r0 += RSTEP) {
      const int z0 = opaque_zero();
      const double* F2 = ST ? fr + z0 : opaque(gsrc + A.fo.F2);
      const double* B2 = ST ? fr + 2048 + z0 : opaque(gsrc + A.fo.B2);
      const double* vec = ST ? fr + 4096 + z0 : opaque(vecg);
      const int row = r0 + r16;
      const bool valid = row < nn;
      const d4 Rrow = R_next;
      R_next = d4{0.0, 0.0, 0.0, 0.0};
      if (row + RSTEP < nn) R_next = *reinterpret_cast<const d4*>(Rs + (row + RSTEP) * 4);
      const double s = Rrow[0];
      const double* rec =
          ST ? static_cast<const double*>(A.act) + ((int64_t)i * A.tpa + A.toff[tj] + (r0 >> 4)) * (M1 * 16) + g * 16 + r16
             : nullptr;
      // stored t3 of the whole tile, requested before layers 1-2 are
      // recomputed so that the loads are in flight meanwhile.  Slot
      // p = 64 zo + 16 o4 + 4 v + g holds feature 2W zo + W (o4 / 2) +
      // 16 (o4 % 2) + 4 v + g when 16 (o4 % 2) + 4 v + g < W, except the
      // slots of the denser layout (features W - 1 + W g in the first half's
      // k-step W - 1); a padding slot may read past its record (the store
      // has one record of slack at its end) and its value is discarded.
      double t3v[2][16];
      if constexpr (ST) {
#pragma unroll
        for (int oo = 0; oo < 2; ++oo)
#pragma unroll
          for (int o4 = 0; o4 < 4; ++o4)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int lo = 16 * (o4 & 1) + 4 * v;
              if (kpad3<W>(oo, o4, v)) {
                t3v[oo][o4 * 4 + v] = 0.0;
              } else if (kDense2<W> && oo == 0 && o4 == 1 && v == 2) {
                t3v[oo][o4 * 4 + v] = rec[((W - 1) + (W - 1) * g) * 16];  // feature W - 1 + W g
              } else {
                t3v[oo][o4 * 4 + v] = (lo < W) ? rec[(oo * 2 * W + (o4 >> 1) * W + lo) * 16] : 0.0;
              }
            }
      }
      double t1[2][4];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          t1[mt][v] = kpad<W>(mt, v) ? 0.0 : tanh_l(fma(s, vec[kV_W1 + 16 * mt + 4 * v + g], vec[kV_B1 + 16 * mt + 4 * v + g]));
      double h2[4][4];  // t2 = h2 - t1 is re-derived where needed
#pragma unroll
      for (int ot = 0; ot < 4; ++ot) {
        const double* b2 = vec + kV_B2 + 16 * ot + g;
        d4 z = {b2[0], b2[4], b2[8], b2[12]};
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (!kpad<W>(mt, v)) z = mfma_f64(F2[((ot * 2 + mt) * 4 + v) * 64 + lane], t1[mt][v], z);
#pragma unroll
        for (int v = 0; v < 4; ++v) h2[ot][v] = kpad2<W>(ot, v) ? 0.0 : t1[ot & 1][v] + tanh_l(z[v]);
      }
      // layer 3 per output tile o, folded immediately into dh2 = W3 dz3
      double skip2[4][4];
      double dRd[4] = {0.0, 0.0, 0.0, 0.0};
      d4 dh2a[4];
#pragma unroll
      for (int ot = 0; ot < 4; ++ot) {
        dh2a[ot] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int v = 0; v < 4; ++v) skip2[ot][v] = 0.0;
      }
#pragma unroll 1
      for (int oo = 0; oo < 2; ++oo) {
        const int zo = opaque_zero() + oo;
#pragma unroll
        for (int o4 = 0; o4 < 4; ++o4) {
          d4 z = {0.0, 0.0, 0.0, 0.0};
          if constexpr (!ST) {
            const double* b3 = vec + kV_B3S + 16 * (4 * zo + o4) + g;
            z = d4{b3[0], b3[4], b3[8], b3[12]};
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                if (!kpad2<W>(mt, v)) z = mfma_f64(fr[z0 + zo * 4096 + ((o4 * 4 + mt) * 4 + v) * 64 + lane], h2[mt][v], z);
          }
          double dz3[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            dz3[v] = 0.0;
            if (kpad2<W>(o4, v)) continue;  // padding slots: G = 0 and no weights
            if (kDense2<W> && o4 == 1 && v == 2 && oo != 0) continue;
            const int p = 16 * (4 * zo + o4) + 4 * v + g;
            double t3;
            if constexpr (ST) {
              const double x = oo == 0 ? t3v[0][o4 * 4 + v] : t3v[1][o4 * 4 + v];
              t3 = (kDense2<W> && o4 == 1 && v == 2) || 16 * (o4 & 1) + 4 * v + g < W ? x : 0.0;
            } else {
              t3 = tanh_d(z[v]);
            }
            const double G = h2[o4][v] + t3;
            const d4 gt = gts[gw][p];
            const double dG = gt[0] * Rrow[0] + gt[1] * Rrow[1] + gt[2] * Rrow[2] + gt[3] * Rrow[3];
#pragma unroll
            for (int k = 0; k < 4; ++k) dRd[k] = fma(gt[k], G, dRd[k]);
            dz3[v] = dG * (1.0 - t3 * t3);
            skip2[o4][v] += dG;
          }
#pragma unroll
          for (int i2 = 0; i2 < 4; ++i2)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (!kpad2<W>(o4, v) && !(kDense2<W> && o4 == 1 && v == 2 && oo != 0))
                dh2a[i2] = mfma_f64(fr[z0 + 8192 + zo * 1024 + ((i2 * 8 + o4) * 4 + v) * 64 + lane], dz3[v], dh2a[i2]);
        }
      }
      double dz2[4][4];
      double skip1[2][4];
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
        for (int v = 0; v < 4; ++v) skip1[i2][v] = 0.0;
#pragma unroll
      for (int i2 = 0; i2 < 4; ++i2)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          dz2[i2][v] = 0.0;
          if (kpad2<W>(i2, v)) continue;
          const double dh2 = dh2a[i2][v] + skip2[i2][v];
          const double t2 = h2[i2][v] - t1[i2 & 1][v];
          dz2[i2][v] = dh2 * (1.0 - t2 * t2);
          skip1[i2 & 1][v] += dh2;
        }
      double dsp = 0.0;
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2) {
        d4 z = {skip1[i2][0], skip1[i2][1], skip1[i2][2], skip1[i2][3]};
#pragma unroll
        for (int o = 0; o < 4; ++o)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (!kpad2<W>(o, v)) z = mfma_f64(B2[((i2 * 4 + o) * 4 + v) * 64 + lane], dz2[o][v], z);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double dh1 = z[v];
          dsp = fma(vec[kV_W1 + 16 * i2 + 4 * v + g], dh1 * (1.0 - t1[i2][v] * t1[i2][v]), dsp);
        }
      }
      dsp += shfl_xor_d(dsp, 16);
      dsp += shfl_xor_d(dsp, 32);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        dRd[k] += shfl_xor_d(dRd[k], 16);
        dRd[k] += shfl_xor_d(dRd[k], 32);
      }
      if (g == 0 && valid) *reinterpret_cast<d4*>(A.netd + (rbase + row) * 4) = d4{dRd[0] + dsp, dRd[1], dRd[2], dRd[3]};
    }
    if constexpr (GM) __syncthreads();  // the g_T tile and col_sh are reused by the next column
  }
}

// ============================================================== mixed forward
// Layer 1 in FP32 on the vector ALUs (K = 1), layers 2 and 3 on 16x16x32
// MFMA with BF16/FP16 operands and FP32 accumulation, tanh and skips in FP32.
// The contraction T = G^T R~ of the 16-bit forms is a matrix-core product
// too, a 16x16x16 one with FP16 operands in both 16-bit forms (BF16's 8-bit
// mantissa raised the BF16 form's copper force error by half; G and R~ are
// well inside FP16's range) and FP32 accumulation: per 16-feature tile o,
// T[feature][k] += sum over the tile's 16 rows of G[row][feature] R~[row][k],
// with M = feature, N = k (4 of 16 used) and K = rows (lane group g carries
// rows 4g..4g+3, which is where layer 3's output puts them), so neither
// operand moves between lanes and the per-atom T needs no cross-lane
// reduction.  The FP32 form keeps the vector contraction (its 16x16x4
// products would cost more than the multiply-adds they replace).
// GM: group mode as in the FP64 kernels (a work-group's waves share a column).
template <class P, int W, int WPB, bool GM>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(4))) void k_embed_fwd_lp(EmbArgs A) {
  constexpr int M1 = 4 * W;
  constexpr int N3 = (M1 + 15) / 16;
  constexpr int NF2 = 2048, NF3 = N3 * 1024;
  typedef typename P::store_t ST;
  typedef typename P::raw8 R8;
  __shared__ __attribute__((aligned(16))) ST fr[NF2 + NF3];
  __shared__ float h2s[WPB][16][kP2 + 1];
  __shared__ float vs[kVecPerNet];
  __shared__ int col_sh;  // group mode: the work-group's column
  DPSE_NET_PROLOGUE(WPB)
  {
    const ST* src = reinterpret_cast<const ST*>(A.fraglp) + net * A.fo.per_net;
    for (int k = threadIdx.x; k < NF2 / 8; k += 64 * WPB)
      reinterpret_cast<R8*>(fr)[k] = reinterpret_cast<const R8*>(src + A.fo.F2)[k];
    for (int k = threadIdx.x; k < NF3 / 8; k += 64 * WPB)
      reinterpret_cast<R8*>(fr + NF2)[k] = reinterpret_cast<const R8*>(src + A.fo.F3n)[k];
  }
  __syncthreads();
  {
    const float* vsrc = A.vec32 + net * A.vec_per_net;
    // 16-bit forms: the biases pre-scaled by 2/ln 2 (they enter only tanh
    // arguments, as fma(z, 2/ln 2, b'), which saves the accumulator set-up
    // of every product); the layer-1 weights as they are
    for (int k = threadIdx.x; k < kVecPerNet; k += 64 * WPB)
      vs[k] = P::kind != 3 && k >= kV_B1 ? vsrc[k] * kTanhScale : vsrc[k];
  }
  __syncthreads();
  constexpr bool MC = P::kind != 3;  // contraction on the matrix cores
  constexpr bool PS = P::kind != 3;  // biases pre-scaled (see the staging above)
  // tanh of a product's output z plus its bias b (PS: b pre-scaled and added
  // in the argument's multiply-add; otherwise z already holds the bias)
  auto act = [](float z, float b) { return PS ? tanh_f_pre(fmaf(z, kTanhScale, b)) : tanh_f(z); };
  constexpr int RSTEP = GM ? 16 * WPB : 16;  // rows between a wave's tiles
  const int rfirst = GM ? 16 * wv : 0;
  for (int c_next = GM ? 0 : take();;) {
    int c;
    if constexpr (GM) {
      if (threadIdx.x == 0) col_sh = atomicAdd(next_col, 1);
      __syncthreads();
      c = __builtin_amdgcn_readfirstlane(col_sh);
    } else {
      c = __builtin_amdgcn_readfirstlane(c_next);
    }
    if (c >= c_hi) break;
    if constexpr (!GM) c_next = take();
    const int col = cb + c;
    const int i = A.atom_at[col];
    float accT[N3][4];
#pragma unroll
    for (int o = 0; o < N3; ++o)
#pragma unroll
      for (int k = 0; k < 4; ++k) accT[o][k] = 0.f;
    const int nn = A.nnei[i * kMaxT + tj];
    const double* Rs = A.R + ((int64_t)i * A.nm + A.sec[tj]) * 4;
    const env_rsrc_t Rb = env_rsrc(Rs, nn);
    double s_next = env_elt(Rb, rfirst + r16, 0);  // s of the next tile is always in flight
    // 16-bit forms: column r16 % 4 of rows 4g..4g+3 of the next tile, also in
    // flight (row indices clamped into the section, unused values discarded)
    double rc_next[4];
    if constexpr (MC) {
#pragma unroll
      for (int v = 0; v < 4; ++v) rc_next[v] = Rs[max(min(rfirst + 4 * g + v, nn - 1), 0) * 4 + (r16 & 3)];
    }
    for (int r0 = rfirst; r0 < nn; r0 += RSTEP) {
      // the per-net vectors are read from LDS for every tile (the opaque
      // offset keeps the reads inside the loop): held in registers they
      // would cost the 40 registers that a fourth wave per SIMD needs
      const int z0 = opaque_zero();
      const float* vec = vs + z0;
      float w1s[8], b1s[8], b2s[4][4];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        w1s[j] = kpadh<W>(j >> 2, j & 3) ? 0.f : vec[kV_W1 + 16 * (j >> 2) + 4 * g + (j & 3)];
        b1s[j] = kpadh<W>(j >> 2, j & 3) ? 0.f : vec[kV_B1 + 16 * (j >> 2) + 4 * g + (j & 3)];
      }
#pragma unroll
      for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int v = 0; v < 4; ++v) b2s[ot][v] = kpadh<W>(ot, v) ? 0.f : vec[kV_B2 + 16 * ot + 4 * g + v];
      const int row = r0 + r16;
      const float sK = (float)s_next * (PS ? kTanhScale : 1.f);
      s_next = env_elt(Rb, row + RSTEP, 0);
      // rows of the contraction, requested before layers 1-2 run: the vector
      // form needs all four columns of rows 4g..4g+3, the matrix form column
      // r16 (< 4) of them as its B operand
      float Rr[4][4];
      h16x4 bR;
      if constexpr (MC) {
        float rv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          float x = (float)rc_next[v];
          asm volatile("" : "+v"(x));  // FP64 -> FP32 -> FP16, as the FP32 form sees it
          rv[v] = r16 < 4 && r0 + 4 * g + v < nn ? x : 0.f;
          rc_next[v] = Rs[max(min(r0 + RSTEP + 4 * g + v, nn - 1), 0) * 4 + (r16 & 3)];
        }
        bR = pack4_f16(rv);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const d4 x = env_row(Rb, r0 + 4 * g + v);
#pragma unroll
          for (int k = 0; k < 4; ++k) Rr[v][k] = (float)x[k];
        }
      }

      float h1[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float y = fmaf(sK, w1s[j], b1s[j]);  // PS: (s w + b) 2/ln 2
        h1[j] = kpadh<W>(j >> 2, j & 3) ? 0.f : PS ? tanh_f_pre(y) : tanh_f(y);
      }
      const typename P::vec8 b1v = pack8<P>(h1);
      float h2[4][4];
#pragma unroll
      for (int ot = 0; ot < 4; ++ot) {
        f4 z = PS ? f4{0.f, 0.f, 0.f, 0.f} : f4{b2s[ot][0], b2s[ot][1], b2s[ot][2], b2s[ot][3]};
        z = P::mfma(load8<P>(fr + z0 + (ot * 64 + lane) * 8), b1v, z);
#pragma unroll
        for (int v = 0; v < 4; ++v) h2[ot][v] = kpadh<W>(ot, v) ? 0.f : h1[4 * (ot & 1) + v] + act(z[v], b2s[ot][v]);
      }
      // the layer-2 tile to LDS in feature order (column f of row r16): the
      // feature of slot 16 ot + 4g + v is linear in g, so every store is one
      // base address plus a constant; the padding slots are left out
      wave_lds_sync();
#pragma unroll
      for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (kpadh<W>(ot, v)) continue;
          const int f1 = (ot & 1) ? 16 + (W <= 28 ? 3 : 4) * g + v : 4 * g + v;  // feature within the half
          if ((ot & 1) == 0 || f1 < W) h2s[wv][r16][(ot >> 1) * W + f1] = h2[ot][v];
        }
      wave_lds_sync();
      typename P::vec8 a3[2];
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {
        float tmp[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) tmp[j] = h2[2 * kt + (j >> 2)][j & 3];
        a3[kt] = pack8<P>(tmp);
      }
#pragma unroll
      for (int o = 0; o < N3; ++o) {
        const int feat = 16 * o + r16;
        const float b3 = vec[kV_B3F + feat];  // the table spans kP3 features
        f4 z = PS ? f4{0.f, 0.f, 0.f, 0.f} : f4{b3, b3, b3, b3};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) z = P::mfma(a3[kt], load8<P>(fr + z0 + NF2 + ((o * 2 + kt) * 64 + lane) * 8), z);
        if constexpr (MC) {
          // A operand: G of rows 4g..4g+3 of this lane's feature (0 past m1)
          float gv[4] = {0.f, 0.f, 0.f, 0.f};
          if (feat < M1) {
            const int src = feat < 2 * W ? feat : feat - 2 * W;  // the skip partner's feature
#pragma unroll
            for (int v = 0; v < 4; ++v) gv[v] = h2s[wv][4 * g + v][src] + act(z[v], b3);
          }
          const f4 t4 = mfma_f16k16(pack4_f16(gv), bR, f4{accT[o][0], accT[o][1], accT[o][2], accT[o][3]});
#pragma unroll
          for (int k = 0; k < 4; ++k) accT[o][k] = t4[k];
        } else if (feat < M1) {
          const int src = feat < 2 * W ? feat : feat - 2 * W;  // the skip partner's feature
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float G = h2s[wv][4 * g + v][src] + act(z[v], b3);
#pragma unroll
            for (int k = 0; k < 4; ++k) accT[o][k] = fmaf(G, Rr[v][k], accT[o][k]);
          }
        }
      }
    }
    const float inv_nm = (float)A.inv_nm;
    float* T = reinterpret_cast<float*>(A.Tpart) + tj * A.tpart_stride + (int64_t)col * M1 * 4;
    // group mode: each wave's partial T to LDS (the h2s tiles, free once every
    // wave has left its tile loop), then the sum in wave order
    float* const dst = GM ? &h2s[0][0][0] + wv * M1 * 4 : T;
    if constexpr (GM) __syncthreads();
    if constexpr (MC) {
      // lane (k = r16 < 4, g) holds T[16 o + 4 g + e][k] in element e
      if (r16 < 4) {
#pragma unroll
        for (int o = 0; o < N3; ++o)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int feat = 16 * o + 4 * g + e;
            if (feat < M1) dst[feat * 4 + r16] = accT[o][e] * inv_nm;
          }
      }
    } else {
#pragma unroll
      for (int o = 0; o < N3; ++o)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float x = accT[o][k];
          x += shfl_xor_f(x, 16);
          x += shfl_xor_f(x, 32);
          accT[o][k] = x * inv_nm;
        }
      if (g == 0) {
#pragma unroll
        for (int o = 0; o < N3; ++o) {
          const int feat = 16 * o + r16;
          if (feat < M1) *reinterpret_cast<f4*>(dst + feat * 4) = f4{accT[o][0], accT[o][1], accT[o][2], accT[o][3]};
        }
      }
    }
    if constexpr (GM) {
      static_assert(WPB * M1 * 4 <= WPB * 16 * (kP2 + 1), "partials fit the h2s tiles");
      __syncthreads();
      const float* red = &h2s[0][0][0];
      for (int e = threadIdx.x; e < M1 * 4; e += 64 * WPB) {
        float x = red[e];
        for (int w = 1; w < WPB; ++w) x += red[w * M1 * 4 + e];
        T[e] = x;
      }
      __syncthreads();  // h2s and col_sh are reused by the next column
    }
  }
}

// ============================================================== mixed backward
// Every quantity of the backward is linear in g_T, so g_T enters unscaled
// and the 1/nm factor is applied once to each output row (g_T / nm sits
// below FP16's normal range for most slots).
// The 16-bit forms run the two per-row contractions with g_T on the matrix
// cores, as 16x16x16 products with FP16 operands and FP32 accumulation:
//  * dE/dG[slot][row] = g_T[slot] . R~[row]: M = slot (16 per tile o),
//    N = row, K = the 4 columns of R~ (lane group 0; the B elements of the
//    other groups are zero, so their A elements may hold anything finite).
//    The result lands in layer 3's output layout.
//  * the direct term dE/dR~[row][k] = sum_slot g_T[slot][k] G[slot][row]:
//    M = k (4 of 16 used), N = row, K = the 16 slots of tile o (lane group
//    g, element v: slot 16o + 4g + v), so G is the B operand as layer 3
//    leaves it; column k of each row ends in lane group 0, element k, with
//    no cross-lane reduction.
// g_T is kept in LDS as FP16 per slot (A of the first product) and
// transposed per column k (A of the second, built once per centre atom).
// The FP32 form keeps the vector multiply-adds.
template <class P, int W, int WPB, bool GM>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(4))) void k_embed_bwd_lp(EmbArgs A) {
  constexpr int M1 = 4 * W;
  constexpr int NFR = 2048 + 8192 + 8192 + 2048;  // F2 | F3t | B3 | B2
  constexpr bool MC = P::kind != 3;  // contractions on the matrix cores
  typedef typename P::store_t ST;
  typedef typename P::raw8 R8;
  __shared__ __attribute__((aligned(16))) ST fr[NFR];
  constexpr int NG = GM ? 1 : WPB;                // g_T tiles (group mode: one, shared)
  __shared__ f4 gts[MC ? 1 : NG][kP3];            // FP32 form: g_T per slot
  __shared__ u16x4 gth[MC ? NG : 1][kP3];         // 16-bit forms: g_T per slot, FP16
  __shared__ u16x4 gtt[MC ? NG : 1][4][kP3 / 4];   // 16-bit forms: column k of g_T, FP16
  __shared__ float vs[kVecPerNet];
  __shared__ int col_sh;  // group mode: the work-group's column
  DPSE_NET_PROLOGUE(WPB)
  {
    const ST* src = reinterpret_cast<const ST*>(A.fraglp) + net * A.fo.per_net;
    const int64_t offs[4] = {A.fo.F2, A.fo.F3t, A.fo.B3, A.fo.B2};
    const int lens[4] = {2048, 8192, 8192, 2048};
    int dst = 0;
    for (int b = 0; b < 4; ++b) {
      for (int k = threadIdx.x; k < lens[b] / 8; k += 64 * WPB)
        reinterpret_cast<R8*>(fr + dst)[k] = reinterpret_cast<const R8*>(src + offs[b])[k];
      dst += lens[b];
    }
  }
  __syncthreads();
  constexpr int oF2 = 0, oF3 = 2048, oB3 = 2048 + 8192, oB2 = 2048 + 8192 + 8192;
  {
    const float* vsrc = A.vec32 + net * A.vec_per_net;
    for (int k = threadIdx.x; k < kVecPerNet; k += 64 * WPB) vs[k] = vsrc[k];
  }
  __syncthreads();
  const int gw = GM ? 0 : wv;  // this wave's g_T tile
  constexpr int RSTEP = GM ? 16 * WPB : 16;
  const int rfirst = GM ? 16 * wv : 0;
  for (int c_next = GM ? 0 : take();;) {
    int c;
    if constexpr (GM) {
      if (threadIdx.x == 0) col_sh = atomicAdd(next_col, 1);
      __syncthreads();
      c = __builtin_amdgcn_readfirstlane(col_sh);
    } else {
      c = __builtin_amdgcn_readfirstlane(c_next);
    }
    if (c >= c_hi) break;
    if constexpr (!GM) c_next = take();
    const int col = cb + c;
    const int i = A.atom_at[col];
    {
      const float* gT = reinterpret_cast<const float*>(A.gT) + (int64_t)col * M1 * 4;
      if constexpr (!GM) wave_lds_sync();
      for (int p = GM ? (int)threadIdx.x : lane; p < kP3; p += GM ? 64 * WPB : 64) {
        const int a = feat3h_of_slot<W>(p);
        f4 x = {0.f, 0.f, 0.f, 0.f};
        if (a >= 0) x = *reinterpret_cast<const f4*>(gT + a * 4);
        if constexpr (MC) {
          u16x4 h;
#pragma unroll
          for (int k = 0; k < 4; ++k) h[k] = PrecF16::bits(x[k]);
          gth[gw][p] = h;
          uint16_t* tk = reinterpret_cast<uint16_t*>(&gtt[gw][0][0]);
#pragma unroll
          for (int k = 0; k < 4; ++k) tk[k * kP3 + p] = h[k];
        } else {
          gts[gw][p] = x;
        }
      }
      if constexpr (GM) __syncthreads();
      else wave_lds_sync();
    }
    // A operands of the direct-term product, per centre atom: lane (m, g),
    // tile o, element v holds g_T[16o + 4g + v][m % 4]
    const int nn = A.nnei[i * kMaxT + tj];
    const int64_t rbase = (int64_t)i * A.nm + A.sec[tj];
    const double* Rs = A.R + rbase * 4;
    const env_rsrc_t Rb = env_rsrc(Rs, nn);
    d4 R_next = env_row(Rb, rfirst + r16);  // row of the next tile is always in flight
    for (int r0 = rfirst; r0 < nn; r0 += RSTEP) {
      const int z0 = opaque_zero();
      const float* vec = vs + z0;  // per-net vectors re-read per tile, as in the forward
      float w1s[8], b1s[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        w1s[j] = kpadh<W>(j >> 2, j & 3) ? 0.f : vec[kV_W1 + 16 * (j >> 2) + 4 * g + (j & 3)];
        b1s[j] = kpadh<W>(j >> 2, j & 3) ? 0.f : vec[kV_B1 + 16 * (j >> 2) + 4 * g + (j & 3)];
      }
      const int row = r0 + r16;
      const bool valid = row < nn;
      const d4 Rd = R_next;
      R_next = env_row(Rb, row + RSTEP);
      const float Rrow[4] = {(float)Rd[0], (float)Rd[1], (float)Rd[2], (float)Rd[3]};
      const float s = Rrow[0];
      float t1[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) t1[j] = kpadh<W>(j >> 2, j & 3) ? 0.f : tanh_f(fmaf(s, w1s[j], b1s[j]));
      const typename P::vec8 b1v = pack8<P>(t1);
      float t2[4][4], h2[4][4];
#pragma unroll
      for (int ot = 0; ot < 4; ++ot) {
        const float* b2 = vec + kV_B2 + 16 * ot + 4 * g;
        f4 z = {b2[0], b2[1], b2[2], kpadh<W>(ot, 3) ? 0.f : b2[3]};
        z = P::mfma(load8<P>(fr + z0 + oF2 + (ot * 64 + lane) * 8), b1v, z);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          t2[ot][v] = kpadh<W>(ot, v) ? 0.f : tanh_f(z[v]);
          h2[ot][v] = kpadh<W>(ot, v) ? 0.f : t1[4 * (ot & 1) + v] + t2[ot][v];
        }
      }
      typename P::vec8 b2v[2];
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {
        float tmp[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) tmp[j] = h2[2 * kt + (j >> 2)][j & 3];
        b2v[kt] = pack8<P>(tmp);
      }
      // B operand of the dE/dG product: R~[row][0..3] in lane group 0
      h16x4 bR;
      if constexpr (MC) {
        // the FP32 values are rounded to FP16 (the empty asm keeps the
        // compiler from fusing both roundings into one from FP64)
        float v4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float x = Rrow[k];
          asm volatile("" : "+v"(x));
          v4[k] = g == 0 ? x : 0.f;
        }
        bR = pack4_f16(v4);
      }
      float skip2[4][4];
      float dRd[4] = {0.f, 0.f, 0.f, 0.f};
      f4 accD = {0.f, 0.f, 0.f, 0.f};
      typename P::vec8 bz3[4];
#pragma unroll
      for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int v = 0; v < 4; ++v) skip2[ot][v] = 0.f;
      float dz3p[8];  // k-step pairs of tiles (2t, 2t + 1)
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const float* b3 = vec + kV_B3S + 16 * o + 4 * g;
        f4 z = {b3[0], b3[1], b3[2], kpadh<W>(o, 3) ? 0.f : b3[3]};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) z = P::mfma(load8<P>(fr + z0 + oF3 + ((o * 2 + kt) * 64 + lane) * 8), b2v[kt], z);
        f4 dGv;
        if constexpr (MC) {
          dGv = mfma_f16k16(__builtin_bit_cast(h16x4, gth[gw][16 * o + r16]), bR, f4{0.f, 0.f, 0.f, 0.f});
        }
        float G4[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (kpadh<W>(o, v)) {  // padding slot: G = 0 and g_T = 0, no gradient
            G4[v] = 0.f;
            dz3p[4 * (o & 1) + v] = 0.f;
            continue;
          }
          const float t3 = tanh_f(z[v]);
          const float G = h2[o & 3][v] + t3;
          float dG;
          if constexpr (MC) {
            dG = dGv[v];
            G4[v] = G;
          } else {
            const f4 gt = gts[gw][16 * o + 4 * g + v];
            dG = gt[0] * Rrow[0] + gt[1] * Rrow[1] + gt[2] * Rrow[2] + gt[3] * Rrow[3];
#pragma unroll
            for (int k = 0; k < 4; ++k) dRd[k] = fmaf(gt[k], G, dRd[k]);
          }
          dz3p[4 * (o & 1) + v] = dG * (1.f - t3 * t3);
          skip2[o & 3][v] += dG;
        }
        // direct term: A operand lane (m, g), element v = g_T[16 o + 4 g + v][m % 4]
        // (read for every tile: kept in registers for the atom it would take
        // 16 of the 128 registers of four waves per SIMD)
        if constexpr (MC) accD = mfma_f16k16(__builtin_bit_cast(h16x4, gtt[gw][r16 & 3][4 * o + g + z0]), pack4_f16(G4), accD);
        if (o & 1) bz3[o >> 1] = pack8<P>(dz3p);
      }
      float dz2[4][4], skip1[2][4];
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
        for (int v = 0; v < 4; ++v) skip1[i2][v] = 0.f;
#pragma unroll
      for (int i2 = 0; i2 < 4; ++i2) {
        f4 z = {skip2[i2][0], skip2[i2][1], skip2[i2][2], skip2[i2][3]};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) z = P::mfma(load8<P>(fr + z0 + oB3 + ((i2 * 4 + kt) * 64 + lane) * 8), bz3[kt], z);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (kpadh<W>(i2, v)) {
            dz2[i2][v] = 0.f;
            continue;
          }
          const float dh2 = z[v];
          dz2[i2][v] = dh2 * (1.f - t2[i2][v] * t2[i2][v]);
          skip1[i2 & 1][v] += dh2;
        }
      }
      typename P::vec8 bz2[2];
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) {
        float tmp[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) tmp[j] = dz2[2 * kt + (j >> 2)][j & 3];
        bz2[kt] = pack8<P>(tmp);
      }
      float dsp = 0.f;
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2) {
        f4 z = {skip1[i2][0], skip1[i2][1], skip1[i2][2], skip1[i2][3]};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) z = P::mfma(load8<P>(fr + z0 + oB2 + ((i2 * 2 + kt) * 64 + lane) * 8), bz2[kt], z);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (kpadh<W>(i2, v)) continue;
          const float dh1 = z[v];
          const float tt = t1[4 * i2 + v];
          dsp = fmaf(w1s[4 * i2 + v], dh1 * (1.f - tt * tt), dsp);
        }
      }
      dsp += shfl_xor_f(dsp, 16);
      dsp += shfl_xor_f(dsp, 32);
      if constexpr (MC) {
#pragma unroll
        for (int k = 0; k < 4; ++k) dRd[k] = accD[k];
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          dRd[k] += shfl_xor_f(dRd[k], 16);
          dRd[k] += shfl_xor_f(dRd[k], 32);
        }
      }
      const double inv_nm = A.inv_nm;
      if (g == 0 && valid)
        *reinterpret_cast<d4*>(A.netd + (rbase + row) * 4) =
            d4{((double)dRd[0] + (double)dsp) * inv_nm, (double)dRd[1] * inv_nm, (double)dRd[2] * inv_nm,
               (double)dRd[3] * inv_nm};
    }
    if constexpr (GM) __syncthreads();  // the g_T tile and col_sh are reused by the next column
  }
}

// ============================================================== launchers
// FP64 kernels run 2 waves per SIMD: 8-wave work-groups share one LDS copy
// of the net's fragments.  The mixed kernels fit 3 work-groups of 4 waves.
constexpr int kWPB64 = 8, kWPBlp = 4;

static EmbArgs emb_args(dp_ctx* c, int32_t mode) {
  const dp_model* m = c->model;
  EmbArgs A;
  A.atom_at = c->atom_at;
  A.meta = c->type_meta;
  A.R = c->R;
  A.nnei = c->nnei;
  A.frag64 = m->emb_frag64d;
  A.fraglp = mode == DP_FP64 ? nullptr : frag_of(m->emb_frag_bf16, m->emb_frag_f16, m->emb_frag_f32, mix_kinds(mode).emb);
  A.vec64 = m->emb_vec64d;
  A.vec32 = m->emb_vec32;
  A.vec_per_net = m->emb_vec_per_net;
  A.fo = m->efo;
  A.Tpart = c->Tpart;
  A.tpart_stride = c->max_cols * m->m1 * 4;
  A.gT = c->gT;
  A.netd = c->netd;
  A.act = c->act_used_last || c->grad_act ? c->act : nullptr;
  A.tpa = m->tpa;
  for (int t = 0; t < kMaxT; ++t) A.toff[t] = m->toff[t];
  A.ntypes = m->desc.ntypes;
  A.nm = m->nm;
  for (int t = 0; t <= kMaxT; ++t) A.sec[t] = t <= m->desc.ntypes ? m->sec[t] : m->nm;
  A.inv_nm = 1.0 / (double)m->nm;
  A.ctr = c->emb_ctr;
  return A;
}

// Work-groups: one-row grid (flat) as many as the CUs hold at once (per_cu
// per CU), fewer when the columns (one per atom and neighbour section) are
// fewer than that many waves, at least one per net, shared out among the
// nets by net_of_group; otherwise one row per net, each with as many
// work-groups as the CUs hold at once (fewer when the net has fewer columns
// than that many waves), so that the work-groups of the lighter nets take
// over the slots of the heavier ones as they finish.
static dim3 emb_grid(dp_ctx* c, int wpb, int per_cu, int ntypes, bool flat) {
  const int nnets = ntypes * ntypes;
  const int64_t res = (int64_t)c->ncu * per_cu;
  if (flat) {
    const int64_t need = (c->natoms_last * ntypes + wpb - 1) / wpb;
    const int64_t g = need < res ? need : res;
    return dim3((unsigned)(g > nnets ? g : nnets), 1);
  }
  const int64_t need = (c->natoms_last + wpb - 1) / wpb;
  return dim3((unsigned)(need < res ? need : res), (unsigned)nnets);
}

template <int W, bool ST, bool GM>
static void launch_embed_f64(bool bwd, dim3 grid, dim3 block, const EmbArgs& A, hipStream_t s) {
  if (bwd) hipLaunchKernelGGL((k_embed_bwd_f64<W, kWPB64, ST, GM>), grid, block, 0, s, A);
  else hipLaunchKernelGGL((k_embed_fwd_f64<W, kWPB64, ST, GM>), grid, block, 0, s, A);
}

// Mixed kernels: the forward with WPBF waves per work-group, the backward
// with WPBB; GM selects group mode.
template <class P, int W, int WPBF, int WPBB>
static void launch_embed_lp_gm(bool bwd, bool gm, dim3 grid, const EmbArgs& A, hipStream_t s) {
  if (bwd) {
    if (gm) hipLaunchKernelGGL((k_embed_bwd_lp<P, W, WPBB, true>), grid, dim3(64 * WPBB), 0, s, A);
    else hipLaunchKernelGGL((k_embed_bwd_lp<P, W, WPBB, false>), grid, dim3(64 * WPBB), 0, s, A);
  } else {
    if (gm) hipLaunchKernelGGL((k_embed_fwd_lp<P, W, WPBF, true>), grid, dim3(64 * WPBF), 0, s, A);
    else hipLaunchKernelGGL((k_embed_fwd_lp<P, W, WPBF, false>), grid, dim3(64 * WPBF), 0, s, A);
  }
}

// Resident work-groups per CU: FP64 one 8-wave group; the 16-bit forms
// four 4-wave groups forward (37 KB of LDS each) and two 8-wave groups
// backward (59 KB: the 40 KB of fragments shared by eight waves), four
// waves per SIMD in both; the FP32 form holds its fragments in twice the
// LDS: the forward two 8-wave groups (72 KB each), the backward one 16-wave
// group (80 KB of fragments and 32 KB of g_T tiles), so that four waves per
// SIMD share the LDS copies (forward 274 -> 256 us, backward 536 -> 519 us
// at water12k against 4- and 8-wave groups).
template <int W>
static void launch_embed(dp_ctx* c, int32_t mode, bool bwd, hipStream_t s) {
  const int kind = mode == DP_FP64 ? 0 : mix_kinds(mode).emb;
  const int wpb = mode == DP_FP64 ? 8 : (bwd ? (kind == 3 ? 16 : 8) : (kind == 3 ? 8 : kWPBlp));
  EmbArgs A = emb_args(c, mode);
  const int per_cu = mode == DP_FP64 ? 1 : (kind == 3 ? (bwd ? 1 : 2) : (bwd ? 2 : 4));
  const int nnets = A.ntypes * A.ntypes;
  // one-row grid for the FP64 kernels and the FP32 form's backward (water12k:
  // FP64 forward 547 -> 516 us, backward with stored activations 589 -> 561
  // us, FP32 backward 504 -> 458 us); the other kernels keep one row per net
  // (the 16-bit forward one-row: 97 -> 103 us)
  const bool flat = mode == DP_FP64 || (kind == 3 && bwd);
  dim3 grid = emb_grid(c, wpb, per_cu, A.ntypes, flat);
  dim3 block(64 * wpb);
  if (mode == DP_FP64) {
    // group mode when the columns (one per atom and neighbour section) are
    // fewer than the chip's wave slots: about one work-group per CU in all,
    // each taking whole columns with all its waves
    const bool gm = c->natoms_last * A.ntypes < (int64_t)c->ncu * wpb;
    if (gm) {  // row y: the y-th heaviest net
      const int64_t per = c->ncu / nnets > 0 ? c->ncu / nnets : 1;
      grid = dim3((unsigned)(c->natoms_last < per ? c->natoms_last : per), (unsigned)nnets);
      if (A.act) launch_embed_f64<W, true, true>(bwd, grid, block, A, s);
      else launch_embed_f64<W, false, true>(bwd, grid, block, A, s);
    } else {
      if (A.act) launch_embed_f64<W, true, false>(bwd, grid, block, A, s);
      else launch_embed_f64<W, false, false>(bwd, grid, block, A, s);
    }
  } else {
    // group mode on the same rule as FP64 (columns fewer than wave slots)
    const bool gm = c->natoms_last * A.ntypes < (int64_t)c->ncu * wpb * per_cu;
    if (gm) {  // row y: the y-th heaviest net
      const int64_t per = (int64_t)c->ncu * per_cu / nnets > 0 ? (int64_t)c->ncu * per_cu / nnets : 1;
      grid = dim3((unsigned)(c->natoms_last < per ? c->natoms_last : per), (unsigned)nnets);
    }
    if (kind == 1) launch_embed_lp_gm<PrecBF16, W, kWPBlp, 8>(bwd, gm, grid, A, s);
    else if (kind == 2) launch_embed_lp_gm<PrecF16, W, kWPBlp, 8>(bwd, gm, grid, A, s);
    else launch_embed_lp_gm<PrecF32, W, 8, 16>(bwd, gm, grid, A, s);
  }
}

void launch_embed_fwd(dp_ctx* c, const int32_t* types, int32_t mode, hipStream_t s) {
  (void)types;
  if (c->natoms_last <= 0) return;
  if (c->model->w1 == 25) launch_embed<25>(c, mode, false, s);
  else launch_embed<32>(c, mode, false, s);
}

void launch_embed_bwd(dp_ctx* c, const int32_t* types, int32_t mode, hipStream_t s) {
  (void)types;
  if (c->natoms_last <= 0) return;
  if (c->model->w1 == 25) launch_embed<25>(c, mode, true, s);
  else launch_embed<32>(c, mode, true, s);
}

}  // namespace dpse
