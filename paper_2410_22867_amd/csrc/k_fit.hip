// Descriptor D = T T<^T, the per-type fitting net (forward and backward) and
// the descriptor backward (Background section: the fitting net maps D_i to
// E_i; Computation Optimization section: the fitting GEMMs dominate, weights
// are transposed once at start-up so every product is a plain one, mixed
// precision runs the GEMMs in half precision).
//
// Fitting activations are stored atom-major, [column][feature], one column
// per centre atom, columns bucketed by centre type into segments padded to
// kColPad.  A GEMM computes out[col][m] = epi(sum_k X[col][k] W[k][m]) for
// all columns of every type (blockIdx.z), with the weight operand stored in
// per-lane fragment order (A operand, features along M) and X as the B
// operand: FP64 reads it straight from memory (lane n + 16g reads 4
// consecutive features of its column); the half-precision GEMM stages it
// through LDS in fragment order.
#include "dp_internal.h"
#include "dp_device.h"

#include <type_traits>

namespace dpse {

enum { EPI_TANH = 0, EPI_PLAIN = 1 };

struct GemmArgs {
  const void* Afr;       // fragments of this layer for type 0
  int64_t a_type_stride; // elements between types
  const void* X;         // [cols][ldx]
  int ldx;
  int K;                 // reduction length (multiple of 16 for f64, padded to 32 for lp)
  int Kreal;             // real reduction length (multiple of 16); lp columns beyond it are ignored
  int M;                 // output features (multiple of 16)
  const int32_t* meta;   // n_t, cbase_t
  int epi;
  const void* vec;       // per-type fitting vectors (b1 b2 b3 wo | bo ebias)
  int64_t vec_type_stride;
  int bias_off;          // offset of the bias of this layer inside the vector block
  void* out0;            // EPI_TANH: tanh(acc + bias); EPI_PLAIN: acc  (f64 or f32, [cols][ld0])
  int ld0;
  const double* T;       // FP64 layer 1: X[col][a*16 + b] = sum_k T[col][a][k] T[col][b][k] built on the fly
  int m1;
  // split-K form: work-group row blockIdx.y = m-block * nsplit + split; split
  // s covers k-steps [KS s / nsplit, KS (s + 1) / nsplit) and writes its raw
  // sums to part[s][col][M] (FP64, or FP32 for the half-precision GEMM)
  void* part;
  int nsplit;
  int64_t part_cols;
};

// ---------------------------------------------------------------- FP64 GEMM
template <int MT, int NT, bool XT, bool SPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_fit_gemm_f64(GemmArgs g) {
  const int t = blockIdx.z;
  const int n_t = g.meta[2 * t], cb = g.meta[2 * t + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, gq = lane >> 4;
  const int c0 = (blockIdx.x * 4 + wv) * NT * 16;
  if (c0 >= n_t) return;
  const int mtiles = g.M / 16;
  const int mb = SPLIT ? (int)blockIdx.y / g.nsplit : (int)blockIdx.y;
  const int sp = SPLIT ? (int)blockIdx.y - mb * g.nsplit : 0;
  const int mt0 = mb * MT;
  const int KS = g.K / 16;
  // k-steps of this work-group: all of them, or one split's range
  const int S0 = SPLIT ? (int)((int64_t)KS * sp / g.nsplit) : 0;
  const int S1 = SPLIT ? (int)((int64_t)KS * (sp + 1) / g.nsplit) : KS;
  const double* Afr = reinterpret_cast<const double*>(g.Afr) + t * g.a_type_stride;
  const double* X = reinterpret_cast<const double*>(g.X);
  d4 acc[MT][NT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const double* xrow[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) xrow[nt] = X + (int64_t)(cb + c0 + nt * 16 + r16) * g.ldx + 4 * gq;
  int mtv[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) mtv[mt] = (mt0 + mt) < mtiles ? (mt0 + mt) : (mtiles - 1);
  // descriptor from T: lane group g needs D[a = S][b = 4g + v], v = 0..3
  d4 Tb[NT][4];
  const double* trow[NT];
  if constexpr (XT) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      trow[nt] = g.T + (int64_t)(cb + c0 + nt * 16 + r16) * g.m1 * 4;
#pragma unroll
      for (int v = 0; v < 4; ++v) Tb[nt][v] = *reinterpret_cast<const d4*>(trow[nt] + (4 * gq + v) * 4);
    }
  }
  // Operands of k-step S + 1 are requested before the products of step S
  // issue: two register buffers used alternately (the loop is unrolled by
  // two, so no copy between them forces an early wait); an odd last step
  // runs after the loop on the buffer the loop filled last.
  d4 xA[NT], xB[NT];
  double aA[MT][4], aB[MT][4];
  auto load = [&](int S, d4* xv, double (*av)[4]) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      xv[nt] = *reinterpret_cast<const d4*>(XT ? trow[nt] + S * 4 : xrow[nt] + 16 * S);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const d4 q = *reinterpret_cast<const d4*>(Afr + (((int64_t)mtv[mt] * KS + S) * 64 + lane) * 4);
#pragma unroll
      for (int v = 0; v < 4; ++v) av[mt][v] = q[v];
    }
  };
  auto step = [&](const d4* xv, const double (*av)[4]) {
    d4 xb[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      if constexpr (XT) {
        const d4 ta = xv[nt];
#pragma unroll
        for (int v = 0; v < 4; ++v)
          xb[nt][v] = ta[0] * Tb[nt][v][0] + ta[1] * Tb[nt][v][1] + ta[2] * Tb[nt][v][2] + ta[3] * Tb[nt][v][3];
      } else {
        xb[nt] = xv[nt];
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma_f64(av[mt][v], xb[nt][v], acc[mt][nt]);
  };
  // (scheduling barriers keep each phase's loads ahead of the products)
  load(S0, xA, aA);
  int S = S0;
  for (; S + 1 < S1; S += 2) {
    load(S + 1, xB, aB);
    __builtin_amdgcn_sched_barrier(0);
    step(xA, aA);
    __builtin_amdgcn_sched_barrier(0);
    load(S + 2 < S1 ? S + 2 : S1 - 1, xA, aA);
    __builtin_amdgcn_sched_barrier(0);
    step(xB, aB);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (S < S1) step(xA, aA);
  if constexpr (SPLIT) {
    double* part = static_cast<double*>(g.part) + (int64_t)sp * g.part_cols * g.M;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      if (mt0 + mt >= mtiles) break;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int64_t col = cb + c0 + nt * 16 + r16;
#pragma unroll
        for (int v = 0; v < 4; ++v) part[col * g.M + (mt0 + mt) * 16 + gq + 4 * v] = acc[mt][nt][v];
      }
    }
    return;
  }
  const double* vec = reinterpret_cast<const double*>(g.vec) + t * g.vec_type_stride;
  // D layout of the f64 MFMA: element v of lane n + 16g is row m = 16 mt + g + 4v.
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    if (mt0 + mt >= mtiles) break;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int64_t col = cb + c0 + nt * 16 + r16;
      const d4 a = acc[mt][nt];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = (mt0 + mt) * 16 + gq + 4 * v;
        if (g.epi == EPI_PLAIN) {
          reinterpret_cast<double*>(g.out0)[col * g.ld0 + m] = a[v];
        } else {
          reinterpret_cast<double*>(g.out0)[col * g.ld0 + m] = tanh_d(a[v] + vec[g.bias_off + m]);
        }
      }
    }
  }
}

// ------------------------------------------------- FP64 fitting layer pairs
// The two equal-width hidden layers after the first, for 16 NCT columns of
// one centre type per work-group, with the activation tile resident in LDS
// between them.  Forward: h2 = h1 + tanh(h1 W2 + b2), h3 = h2 +
// tanh(h2 W3 + b3), E_i = h3 . w_o + b_o + e_bias, plus dz3 = w_o (1 - t3^2)
// for the backward.  Backward: dh2 = w_o + W3 dz3, dz2 = dh2 (1 - t2^2),
// dh1 = dh2 + W2 dz2, dz1 = dh1 (1 - t1^2).  Wave w owns m-tiles w, w + 4,
// ...; operands as in k_fit_gemm_f64 (weight fragments lane-major from
// memory, requested one k-step ahead; activations from LDS).
struct PairArgs {
  const int32_t* meta;
  const int32_t* atom_at;
  int fw;
  const double* in;        // forward: h1; backward: dz3   [cols][fw]
  const double* A[2];      // fragments of the first and second layer, type 0
  int64_t a_type_stride;
  const double* vec;       // per-type fitting vectors (b1 b2 b3 wo | bo ebias)
  int64_t vec_type_stride;
  const double* tprev[2];  // backward: t2, t1
  double* out[4];          // forward: t2, h2, h3, dz3; backward: dz2, dz1
  double* Ei_col;
  double* Ei_atom;
};

template <bool BWD, int NCT, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 4 ? 3 : (NW == 8 ? 6 : 4)))) void k_fit_pair_f64(PairArgs p) {
  constexpr int MW = 16 / NW;      // m-tile slots per wave (fw <= 256)
  constexpr int NC = 16 * NCT;    // columns of the work-group
  extern __shared__ double hs[];  // [NC][fw + 2]
  const int t = blockIdx.z;
  const int n_t = p.meta[2 * t], cb = p.meta[2 * t + 1];
  const int c0 = blockIdx.x * NC;
  if (c0 >= n_t) return;
  const int lane = threadIdx.x & 63, r16 = lane & 15, gq = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int fw = p.fw, KS = fw / 16, mtiles = fw / 16, ldh = fw + 2;
  const double* vec = p.vec + t * p.vec_type_stride;
  for (int e = threadIdx.x; e < NC * fw; e += 64 * NW) {
    const int c = e / fw, k = e - c * fw;
    hs[c * ldh + k] = p.in[(int64_t)(cb + c0 + c) * fw + k];
  }
  // m-tile slots past the last tile (wave 3 when fw = 240) repeat the last
  // tile in the products, which keeps the k-loop free of branches; their
  // results are dropped
  bool own[MW];
  int mtj[MW];
#pragma unroll
  for (int j = 0; j < MW; ++j) {
    own[j] = wv + NW * j < mtiles;
    mtj[j] = own[j] ? wv + NW * j : mtiles - 1;
  }
  // element v of m-tile slot j, column tile nt: feature 16 mtj[j] + gq + 4 v
  // of column c0 + 16 nt + r16
  auto feat = [&](int j, int v) { return 16 * mtj[j] + gq + 4 * v; };
  auto colof = [&](int nt) { return (int64_t)cb + c0 + 16 * nt + r16; };
  auto hrow = [&](int nt) { return hs + (16 * nt + r16) * ldh; };
  d4 acc[MW][NCT];
  auto init = [&](int off) {
#pragma unroll
    for (int j = 0; j < MW; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double b = vec[off + feat(j, v)];
#pragma unroll
        for (int nt = 0; nt < NCT; ++nt) acc[j][nt][v] = b;
      }
  };
  auto layer = [&](const double* Afr) {
    d4 aA[MW], aB[MW];
    auto load = [&](int S, d4* a) {
#pragma unroll
      for (int j = 0; j < MW; ++j)
        a[j] = *reinterpret_cast<const d4*>(Afr + (((int64_t)mtj[j] * KS + S) * 64 + lane) * 4);
    };
    auto step = [&](int S, const d4* a) {
      d4 x[NCT];
#pragma unroll
      for (int nt = 0; nt < NCT; ++nt) x[nt] = *reinterpret_cast<const d4*>(hrow(nt) + 16 * S + 4 * gq);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < MW; ++j)
#pragma unroll
          for (int nt = 0; nt < NCT; ++nt) acc[j][nt] = mfma_f64(a[j][v], x[nt][v], acc[j][nt]);
    };
    load(0, aA);
    int S = 0;
    for (; S + 1 < KS; S += 2) {
      load(S + 1, aB);
      step(S, aA);
      load(S + 2 < KS ? S + 2 : KS - 1, aA);
      step(S + 1, aB);
    }
    if (S < KS) step(S, aA);
  };
  const double* A0 = p.A[0] + t * p.a_type_stride;
  const double* A1 = p.A[1] + t * p.a_type_stride;
  if constexpr (!BWD) {
    // second (LAST false) or third layer with its epilogue: t2 and h2, or h3
    // and dz3
    auto fwd_layer = [&](const double* Afr, int bias_off, auto last_tag) {
      constexpr bool LAST = decltype(last_tag)::value;
      init(bias_off);
      __syncthreads();  // the tile (input or previous layer) is complete
      layer(Afr);
      __syncthreads();  // every wave has read the tile
#pragma unroll
      for (int j = 0; j < MW; ++j) {
        if (!own[j]) continue;
#pragma unroll
        for (int nt = 0; nt < NCT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int m = feat(j, v);
            const int64_t col = colof(nt);
            const double tv = tanh_d(acc[j][nt][v]);
            const double h = hrow(nt)[m] + tv;
            hrow(nt)[m] = h;
            if constexpr (!LAST) {
              p.out[0][col * fw + m] = tv;
              if (p.out[1]) p.out[1][col * fw + m] = h;
            } else {
              if (p.out[2]) p.out[2][col * fw + m] = h;
              p.out[3][col * fw + m] = vec[3 * fw + m] * (1.0 - tv * tv);
            }
          }
      }
    };
    fwd_layer(A0, fw, std::false_type{});
    fwd_layer(A1, 2 * fw, std::true_type{});
    __syncthreads();
    // E_i: TPC threads per column, partial dots over features part, part + TPC, ...
    constexpr int TPC = 64 * NW / NC;
    const int c = threadIdx.x / TPC, part = threadIdx.x % TPC;
    double e = 0.0;
    for (int m = part; m < fw; m += TPC) e += hs[c * ldh + m] * vec[3 * fw + m];
#pragma unroll
    for (int o = TPC / 2; o >= 1; o >>= 1) e += __shfl_xor(e, o, 64);
    if (part == 0) {
      const int64_t cc = cb + c0 + c;
      const int i = p.atom_at[cc];
      if (i >= 0) {
        const double E = e + vec[4 * fw] + vec[4 * fw + 1];
        p.Ei_col[cc] = E;
        p.Ei_atom[i] = E;
      }
    }
  } else {
    // tanh of the layers below, requested before the products
    double tp[MW][NCT][4];
    auto load_t = [&](const double* src) {
#pragma unroll
      for (int j = 0; j < MW; ++j)
#pragma unroll
        for (int nt = 0; nt < NCT; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) tp[j][nt][v] = src[colof(nt) * fw + feat(j, v)];
    };
    load_t(p.tprev[0]);
    init(3 * fw);  // w_o
    __syncthreads();
    layer(A0);     // acc = dh2
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      if (!own[j]) continue;
#pragma unroll
      for (int nt = 0; nt < NCT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = feat(j, v);
          const double dz = acc[j][nt][v] * (1.0 - tp[j][nt][v] * tp[j][nt][v]);
          hrow(nt)[m] = dz;
          if (p.out[0]) p.out[0][colof(nt) * fw + m] = dz;
        }
    }
    load_t(p.tprev[1]);
    __syncthreads();
    layer(A1);     // acc = dh1 = dh2 + W2 dz2
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      if (!own[j]) continue;
#pragma unroll
      for (int nt = 0; nt < NCT; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          p.out[1][colof(nt) * fw + feat(j, v)] = acc[j][nt][v] * (1.0 - tp[j][nt][v] * tp[j][nt][v]);
    }
  }
}

// One 16-column tile per work-group and four waves of four m-tile slots
// (32 columns, or eight waves of two slots, measured no faster).  Frames
// too small to give every CU a work-group (few atoms) take sixteen waves of
// one slot each instead: the same work in a quarter of the serial chain.
template <int NW>
static void launch_pair_f64_t(dp_ctx* c, bool bwd, const PairArgs& p, hipStream_t s) {
  constexpr int NCT = 1;
  const dp_model* m = c->model;
  dim3 grid((unsigned)((c->natoms_last + 16 * NCT - 1) / (16 * NCT)), 1, (unsigned)m->desc.ntypes);
  const size_t lds = (size_t)16 * NCT * (m->fw + 2) * sizeof(double);
  if (grid.x == 0) return;
  if (bwd) hipLaunchKernelGGL((k_fit_pair_f64<true, NCT, NW>), grid, dim3(64 * NW), lds, s, p);
  else hipLaunchKernelGGL((k_fit_pair_f64<false, NCT, NW>), grid, dim3(64 * NW), lds, s, p);
}

static void launch_pair_f64(dp_ctx* c, bool bwd, const PairArgs& p, hipStream_t s) {
  const int64_t wgs = (c->natoms_last + 15) / 16 + c->model->desc.ntypes - 1;
  if (wgs < c->ncu) launch_pair_f64_t<16>(c, bwd, p, s);
  else launch_pair_f64_t<4>(c, bwd, p, s);
}

// ---------------------------------------------------------------- mixed GEMM
// Epilogue of one 16x16 output tile row group: lane holds features m0..m0+3
// of column col.
template <class P>
__device__ __forceinline__ void epi_lp(const GemmArgs& g, const float* vec, int64_t col, int m0, const f4 a) {
  float* out = reinterpret_cast<float*>(g.out0) + col * g.ld0 + m0;
  if (g.epi == EPI_PLAIN) {
    *reinterpret_cast<f4*>(out) = a;
  } else {
    float tv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) tv[v] = tanh_f(a[v] + vec[g.bias_off + m0 + v]);
    *reinterpret_cast<f4*>(out) = f4{tv[0], tv[1], tv[2], tv[3]};
  }
}

// Half-precision GEMM, 2D-tiled through LDS.  A work-group of 4 waves
// (2 along M x 2 along N) computes a (32 MTW) x (32 NTW) output tile: wave
// (wm, wn) owns MTW m-tiles x NTW n-tiles.  Each 32-wide k-step of the
// weight tile (pre-arranged fragments, copied as they are) and of the X tile
// (rearranged into B-fragment order on the way) is loaded once per
// work-group into double-buffered LDS, so a weight fragment serves 2 NTW
// n-tiles and an X fragment 2 MTW m-tiles.
template <class P, int MTW, int NTW, int PF, bool SPLIT>
__global__ __launch_bounds__(256) void k_fit_gemm_lp(GemmArgs g) {
  constexpr int MB = 2 * MTW, NB = 2 * NTW;  // m-tiles, n-tiles per work-group
  constexpr int BN = 16 * NB;
  typedef typename P::store_t ST;
  typedef typename P::raw8 R8;
  typedef typename P::raw4 R4;
  __shared__ __attribute__((aligned(16))) ST as[2][MB * 512];
  __shared__ __attribute__((aligned(16))) ST xs[2][NB * 512];
  const int t = blockIdx.z;
  const int n_t = g.meta[2 * t], cb = g.meta[2 * t + 1];
  const int c0 = blockIdx.x * BN;
  if (c0 >= n_t) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int r16 = lane & 15, gq = lane >> 4;
  const int mtiles = g.M / 16;
  const int mb = SPLIT ? (int)blockIdx.y / g.nsplit : (int)blockIdx.y;
  const int sp = SPLIT ? (int)blockIdx.y - mb * g.nsplit : 0;
  const int mb0 = mb * MB;
  const int KTall = g.K / 32;
  // k-steps of this work-group: [kt0, kt0 + KT)
  const int kt0 = SPLIT ? (int)((int64_t)KTall * sp / g.nsplit) : 0;
  const int KT = SPLIT ? (int)((int64_t)KTall * (sp + 1) / g.nsplit) - kt0 : KTall;
  const ST* Afr = reinterpret_cast<const ST*>(g.Afr) + t * g.a_type_stride;
  const ST* X = reinterpret_cast<const ST*>(g.X);
  // weight copy: MB fragments of 64 lanes x 16 B per k-step; thread tid
  // moves lane tid % 64 of fragments tid / 64 + 4u
  constexpr int AU = (MB + 3) / 4;
  // X copy: thread (col, q) moves X[col][32 kt + 8q .. +7] into lane
  // (col % 16) + 16 (2 (q % 2) + h), elements 4 (q / 2) .. +3, of n-tile
  // col / 16 (the k order of the fragments); BN * 4 / 256 columns each
  constexpr int XU = (BN * 4 + 255) / 256;
  // Operands travel global -> registers -> LDS.  Loads run PF k-steps
  // ahead of the products through a ring of register buffers (PF = 8 for
  // long reductions, 2 for short ones, where the ring's re-reads past the
  // end would cost more than they hide); they have no
  // branches around them (m-tiles past the last repeat it, their results
  // are dropped), so no wait is forced before the ring slot is consumed.
  static_assert((MB + 3) / 4 == 1 && (BN * 4 + 255) / 256 == 1, "one weight and one X vector per thread");
  const int fA = tid >> 6;
  const int mA = min(mb0 + fA, mtiles - 1);
  const int colX = tid >> 2, qX = tid & 3;
  const ST* aSrc = Afr + ((int64_t)mA * KTall * 64 + lane) * 8 + (int64_t)kt0 * 512;
  const ST* xSrc = X + (int64_t)(cb + c0 + colX) * g.ldx + 8 * qX + 32 * kt0;
  auto load = [&](int kt, R8& av, R8& xv) {
    av = *reinterpret_cast<const R8*>(aSrc + (int64_t)kt * 512);
    xv = *reinterpret_cast<const R8*>(xSrc + 32 * kt);
  };
  auto store = [&](int buf, int kt, const R8& av, R8 xv) {
    // the padded upper half of the last k-step may hold stale bits: zeros
    if (!(qX < 2 || 32 * (kt0 + kt) + 16 < g.Kreal)) xv = zero8<P>();
    if (fA < MB) *reinterpret_cast<R8*>(&as[buf][(fA * 64 + lane) * 8]) = av;
    const int d0 = (((colX >> 4) * 64 + 32 * (qX & 1) + (colX & 15)) * 8) + 4 * (qX >> 1);
    R4 lo, hi;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      lo[j] = xv[j];
      hi[j] = xv[4 + j];
    }
    *reinterpret_cast<R4*>(&xs[buf][d0]) = lo;
    *reinterpret_cast<R4*>(&xs[buf][d0 + 128]) = hi;
  };
  f4 acc[MTW][NTW];
#pragma unroll
  for (int a = 0; a < MTW; ++a)
#pragma unroll
    for (int b = 0; b < NTW; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  R8 ar[PF], xr[PF];
#pragma unroll
  for (int d = 0; d < PF; ++d)
    if (d < KT) load(d, ar[d], xr[d]);
  store(0, 0, ar[0], xr[0]);
  __syncthreads();
  // one k-step: products from LDS buffer kt & 1, ring slot d refilled with
  // k-step kt + PF (past the end the last k-step is read again and never
  // stored, so neither the load nor the store needs a branch: the other LDS
  // buffer after the last step is simply not read)
  auto iter = [&](int kt, int d) {
    const int buf = kt & 1;
    load(min(kt + PF, KT - 1), ar[d], xr[d]);
    R8 aa[MTW], bb[NTW];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) aa[mt] = *reinterpret_cast<const R8*>(&as[buf][((wm * MTW + mt) * 64 + lane) * 8]);
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) bb[nt] = *reinterpret_cast<const R8*>(&xs[buf][((wn * NTW + nt) * 64 + lane) * 8]);
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
      for (int nt = 0; nt < NTW; ++nt)
        acc[mt][nt] = P::mfma(__builtin_bit_cast(typename P::vec8, aa[mt]), __builtin_bit_cast(typename P::vec8, bb[nt]),
                              acc[mt][nt]);
    store(buf ^ 1, min(kt + 1, KT - 1), ar[(d + 1) % PF], xr[(d + 1) % PF]);
    __syncthreads();
  };
  int kb = 0;
  for (; kb + PF <= KT; kb += PF)
#pragma unroll
    for (int d = 0; d < PF; ++d) iter(kb + d, d);
#pragma unroll
  for (int d = 0; d < PF; ++d)
    if (kb + d < KT) iter(kb + d, d);
  const float* vec = reinterpret_cast<const float*>(g.vec) + t * g.vec_type_stride;
#pragma unroll
  for (int mt = 0; mt < MTW; ++mt) {
    const int m = mb0 + wm * MTW + mt;
    if (m >= mtiles) break;
    const int m0 = m * 16 + 4 * gq;
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
      const int cl = c0 + (wn * NTW + nt) * 16;
      if (cl >= n_t) continue;
      const int64_t col = cb + cl + r16;
      if constexpr (SPLIT) {
        float* part = static_cast<float*>(g.part) + (int64_t)sp * g.part_cols * g.M;
        *reinterpret_cast<f4*>(part + col * g.M + m0) = acc[mt][nt];
      } else {
        epi_lp<P>(g, vec, col, m0, acc[mt][nt]);
      }
    }
  }
}

// Completion of the split-K form: out[col][m] = epi(sum over the splits, in
// split order, of part[s][col][m] (+ bias)) for the columns and features the
// unsplit GEMM writes (16-column tiles of each type's segment).
template <typename T>
__global__ __launch_bounds__(256) void k_split_finish(GemmArgs g) {
  const int t = blockIdx.y;
  const int n_t = g.meta[2 * t], cb = g.meta[2 * t + 1];
  const int ncol = (n_t + 15) & ~15;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= (int64_t)ncol * g.M) return;
  const int64_t col = cb + k / g.M;
  const int m = (int)(k % g.M);
  const T* part = static_cast<const T*>(g.part);
  T acc = 0;
  for (int s = 0; s < g.nsplit; ++s) acc += part[((int64_t)s * g.part_cols + col) * g.M + m];
  T* out = static_cast<T*>(g.out0) + col * g.ld0 + m;
  if (g.epi == EPI_PLAIN) {
    *out = acc;
  } else {
    const T b = static_cast<const T*>(g.vec)[t * g.vec_type_stride + g.bias_off + m];
    if constexpr (sizeof(T) == 8) *out = tanh_d(acc + b);
    else *out = tanh_f(acc + b);
  }
}

// --------------------------------------------- mixed fitting layer pairs
// The layer pair of k_fit_pair_f64 in the mixed forms: BF16/FP16 operands,
// FP32 accumulation, tanh and skips.  The 16-column tile stays in LDS: FP32
// activations in the forward (the skips add in FP32; each k-step's B operand
// is converted from them), half-precision deltas in the backward (the B
// operand as the unfused GEMM reads it).  K is padded to fwp = 32-multiple
// with zeros.  Forward writes t2, h2, h3 (FP32), dz3 (half) and E_i;
// backward writes dz2 and dz1 (half).
struct PairArgsLp {
  const int32_t* meta;
  const int32_t* atom_at;
  int fw, fwp;
  const void* in;          // forward: h1 (FP32, ld fwp); backward: dz3 (the form's element type, ld fwp)
  const void* A[2];        // fragments of the first and second layer, type 0
  int64_t a_type_stride;
  const float* vec;        // per-type fitting vectors (b1 b2 b3 wo | bo ebias)
  int64_t vec_type_stride;
  const float* tprev[2];   // backward: t2, t1 (FP32)
  float* out[3];           // forward: t2, h2, h3
  void* outlp[2];          // forward: dz3; backward: dz2 (element type of P), dz1 (of PO)
  double* Ei_col;
  double* Ei_atom;
};

// PO: element type of dz1, the X operand of the first layer's backward GEMM
// (the same as P except in the paper's MIX-fp16 recipe).
template <class P, class PO, bool BWD, int NCT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NCT > 1 ? 2 : 3))) void k_fit_pair_lp(PairArgsLp p) {
  constexpr int NC = 16 * NCT, NW = 4, MW = 4;
  typedef typename P::store_t ST;
  typedef typename P::raw8 R8;
  typedef typename P::raw4 R4;
  // forward: FP32 tile [NC][fwp + 4]; backward: tile of ST [NC][fwp + 8]
  extern __shared__ __attribute__((aligned(16))) float hsf[];
  ST* const hsh = reinterpret_cast<ST*>(hsf);
  const int t = blockIdx.z;
  const int n_t = p.meta[2 * t], cb = p.meta[2 * t + 1];
  const int c0 = blockIdx.x * NC;
  if (c0 >= n_t) return;
  const int lane = threadIdx.x & 63, r16 = lane & 15, gq = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int fw = p.fw, fwp = p.fwp, KT = fwp / 32, mtiles = fw / 16;
  const int ldf = fwp + 4, ldh = fwp + 8;
  const float* vec = p.vec + t * p.vec_type_stride;
  for (int e = threadIdx.x; e < NC * fwp; e += 64 * NW) {
    const int c = e / fwp, k = e - c * fwp;
    const int64_t src = (int64_t)(cb + c0 + c) * fwp + k;
    if constexpr (BWD) hsh[c * ldh + k] = k < fw ? reinterpret_cast<const ST*>(p.in)[src] : (ST)0;
    else hsf[c * ldf + k] = k < fw ? reinterpret_cast<const float*>(p.in)[src] : 0.f;
  }
  bool own[MW];
  int mtj[MW];
#pragma unroll
  for (int j = 0; j < MW; ++j) {
    own[j] = wv + NW * j < mtiles;
    mtj[j] = own[j] ? wv + NW * j : mtiles - 1;
  }
  // element v of m-tile slot j, column tile n: feature 16 mtj[j] + 4 gq + v
  // of column c0 + 16 n + r16
  auto feat = [&](int j, int v) { return 16 * mtj[j] + 4 * gq + v; };
  auto colof = [&](int n) { return (int64_t)(cb + c0 + 16 * n + r16); };
  f4 acc[MW][NCT];
  auto layer = [&](const ST* Afr) {
    R8 aA[MW], aB[MW];
    auto load = [&](int kt, R8* a) {
#pragma unroll
      for (int j = 0; j < MW; ++j)
        a[j] = *reinterpret_cast<const R8*>(Afr + (((int64_t)mtj[j] * KT + kt) * 64 + lane) * 8);
    };
    auto step = [&](int kt, const R8* a) {
#pragma unroll
      for (int n = 0; n < NCT; ++n) {
        // B operand: features 32 kt + 4 gq + {0..3} and 32 kt + 16 + 4 gq + {0..3}
        const int rc = 16 * n + r16;
        typename P::vec8 x;
        if constexpr (BWD) {
          const ST* rowp = hsh + rc * ldh + 32 * kt + 4 * gq;
          const R4 lo = *reinterpret_cast<const R4*>(rowp);
          const R4 hi = *reinterpret_cast<const R4*>(rowp + 16);
          x = __builtin_bit_cast(typename P::vec8, join8<P>(lo, hi));
        } else {
          const float* rowp = hsf + rc * ldf + 32 * kt + 4 * gq;
          const f4 lo = *reinterpret_cast<const f4*>(rowp);
          const f4 hi = *reinterpret_cast<const f4*>(rowp + 16);
          const float v8[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
          x = pack8<P>(v8);
        }
#pragma unroll
        for (int j = 0; j < MW; ++j) acc[j][n] = P::mfma(__builtin_bit_cast(typename P::vec8, a[j]), x, acc[j][n]);
      }
    };
    load(0, aA);
    int kt = 0;
    for (; kt + 1 < KT; kt += 2) {
      load(kt + 1, aB);
      step(kt, aA);
      load(kt + 2 < KT ? kt + 2 : KT - 1, aA);
      step(kt + 1, aB);
    }
    if (kt < KT) step(kt, aA);
  };
  const ST* A0 = reinterpret_cast<const ST*>(p.A[0]) + t * p.a_type_stride;
  const ST* A1 = reinterpret_cast<const ST*>(p.A[1]) + t * p.a_type_stride;
  if constexpr (!BWD) {
    auto fwd_layer = [&](const ST* Afr, int bias_off, auto last_tag) {
      constexpr bool LAST = decltype(last_tag)::value;
#pragma unroll
      for (int j = 0; j < MW; ++j)
#pragma unroll
        for (int n = 0; n < NCT; ++n)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[j][n][v] = vec[bias_off + feat(j, v)];
      __syncthreads();  // the tile (input or previous layer) is complete
      layer(Afr);
      __syncthreads();  // every wave has read the tile
#pragma unroll
      for (int j = 0; j < MW; ++j)
#pragma unroll
      for (int n = 0; n < NCT; ++n) {
        if (!own[j]) continue;
        const int m0 = feat(j, 0);
        const int64_t col = colof(n);
        float* hrow = hsf + (16 * n + r16) * ldf + m0;
        const f4 hprev = *reinterpret_cast<const f4*>(hrow);
        float tv[4], hv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          tv[v] = tanh_f(acc[j][n][v]);
          hv[v] = hprev[v] + tv[v];
        }
        *reinterpret_cast<f4*>(hrow) = f4{hv[0], hv[1], hv[2], hv[3]};
        if constexpr (!LAST) {
          *reinterpret_cast<f4*>(p.out[0] + col * fwp + m0) = f4{tv[0], tv[1], tv[2], tv[3]};
          if (p.out[1]) *reinterpret_cast<f4*>(p.out[1] + col * fwp + m0) = f4{hv[0], hv[1], hv[2], hv[3]};
        } else {
          if (p.out[2]) *reinterpret_cast<f4*>(p.out[2] + col * fwp + m0) = f4{hv[0], hv[1], hv[2], hv[3]};
          float dz[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) dz[v] = vec[3 * fw + m0 + v] * (1.f - tv[v] * tv[v]);
          store4<P>(reinterpret_cast<ST*>(p.outlp[0]) + col * fwp + m0, dz);
        }
      }
    };
    fwd_layer(A0, fw, std::false_type{});
    fwd_layer(A1, 2 * fw, std::true_type{});
    __syncthreads();
    // E_i (summed in FP64 over the FP32 h3 w_o products): 16 threads per column
    const int part = threadIdx.x & 15;
#pragma unroll
    for (int n = 0; n < NCT; ++n) {
      const int c = 16 * n + (threadIdx.x >> 4);
      double e = 0.0;
      for (int m = part; m < fw; m += 16) e += (double)(hsf[c * ldf + m] * vec[3 * fw + m]);
#pragma unroll
      for (int o = 8; o >= 1; o >>= 1) e += __shfl_xor(e, o, 64);
      if (part == 0) {
        const int64_t cc = cb + c0 + c;
        const int i = p.atom_at[cc];
        if (i >= 0) {
          const double E = e + (double)vec[4 * fw] + (double)vec[4 * fw + 1];
          p.Ei_col[cc] = E;
          p.Ei_atom[i] = E;
        }
      }
    }
  } else {
    float tp[MW][NCT][4];
    auto load_t = [&](const float* src) {
#pragma unroll
      for (int j = 0; j < MW; ++j)
#pragma unroll
        for (int n = 0; n < NCT; ++n) {
          const f4 x = *reinterpret_cast<const f4*>(src + colof(n) * fwp + feat(j, 0));
#pragma unroll
          for (int v = 0; v < 4; ++v) tp[j][n][v] = x[v];
        }
    };
    load_t(p.tprev[0]);
#pragma unroll
    for (int j = 0; j < MW; ++j)
#pragma unroll
      for (int n = 0; n < NCT; ++n)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[j][n][v] = vec[3 * fw + feat(j, v)];  // w_o
    __syncthreads();
    layer(A0);  // acc = dh2
    __syncthreads();
#pragma unroll
    for (int j = 0; j < MW; ++j)
#pragma unroll
      for (int n = 0; n < NCT; ++n) {
        if (!own[j]) continue;
        const int m0 = feat(j, 0);
        float dz[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) dz[v] = acc[j][n][v] * (1.f - tp[j][n][v] * tp[j][n][v]);
        store4<P>(hsh + (16 * n + r16) * ldh + m0, dz);
        if (p.outlp[0]) store4<P>(reinterpret_cast<ST*>(p.outlp[0]) + colof(n) * fwp + m0, dz);
      }
    load_t(p.tprev[1]);
    __syncthreads();
    layer(A1);  // acc = dh1 = dh2 + W2 dz2
#pragma unroll
    for (int j = 0; j < MW; ++j)
#pragma unroll
      for (int n = 0; n < NCT; ++n) {
        if (!own[j]) continue;
        const int m0 = feat(j, 0);
        float dz[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) dz[v] = acc[j][n][v] * (1.f - tp[j][n][v] * tp[j][n][v]);
        store4<PO>(reinterpret_cast<typename PO::store_t*>(p.outlp[1]) + colof(n) * fwp + m0, dz);
      }
  }
}

// Column tiles per work-group of the half-precision layer pairs (each
// weight fragment a wave loads serves that many products): one, measured
// faster than two or four (water12k BF16 forward 57 / 62 / 82 us) — the
// kernel gains more from the work-groups than from the weight reuse.
constexpr int kPairNCT = 1;

template <class P, class PO>
static void launch_pair_lp_t(bool bwd, dim3 grid, size_t lds, const PairArgsLp& p, hipStream_t s) {
  if (bwd) hipLaunchKernelGGL((k_fit_pair_lp<P, PO, true, kPairNCT>), grid, dim3(256), lds, s, p);
  else hipLaunchKernelGGL((k_fit_pair_lp<P, P, false, kPairNCT>), grid, dim3(256), lds, s, p);
}

static void launch_pair_lp(dp_ctx* c, bool bwd, int mode, const PairArgsLp& p, hipStream_t s) {
  const dp_model* m = c->model;
  const MixKinds mk = mix_kinds(mode);
  constexpr int NC = 16 * kPairNCT;
  dim3 grid((unsigned)((c->natoms_last + NC - 1) / NC), 1, (unsigned)m->desc.ntypes);
  const size_t esz = mk.fit23 == 3 ? 4 : 2;
  const size_t lds = bwd ? (size_t)NC * (p.fwp + 8) * esz : (size_t)NC * (p.fwp + 4) * 4;
  if (grid.x == 0) return;
  if (mk.fit23 == 1) launch_pair_lp_t<PrecBF16, PrecBF16>(bwd, grid, lds, p, s);
  else if (mk.fit23 == 2) launch_pair_lp_t<PrecF16, PrecF16>(bwd, grid, lds, p, s);
  else if (mk.fit1 == 2) launch_pair_lp_t<PrecF32, PrecF16>(bwd, grid, lds, p, s);
  else launch_pair_lp_t<PrecF32, PrecF32>(bwd, grid, lds, p, s);
}

// ---------------------------------------------------------------- fused first fitting layer
// Half-precision forms (16-bit operands, FP32 accumulation) of the first
// fitting layer with the descriptor folded in on both sides:
//   forward : h1[col][m] = tanh(sum_k D[col][k] W1[k][m] + b1[m]), D built
//             from T = sum of the section partials inside the GEMM;
//   backward: dE/dD = dz1 W1^T is contracted with T in the GEMM's epilogue,
//             g_T[a][k] = sum_b dD[a][b] T[b][k] + [a < m2] sum_a' dD[a'][a] T[a'][k],
//             so neither D nor dE/dD passes through HBM.
// The k order of a 32-wide step is the fragments' (lane group g, element j:
// k = 32 kt + 16 (j / 4) + 4 g + j % 4), so a lane of a D fragment always
// holds b = 4 g .. 4 g + 3 and a = 2 kt + j / 4: the four T rows b are kept
// in registers and one row a is read per step.
constexpr int kFit1MaxM1 = 128;  // LDS copy of T: 16 B per column and row

struct Fit1Args {
  const int32_t* meta;   // n_t, cbase_t per centre type
  const float* Tpart;    // forward: [sections][cols][m1][4] partial T
  int64_t tstride;       // elements between sections
  int ntypes;
  float* T;              // [cols][m1][4]: written by the forward, read by the backward
  void* D;               // forward: D in the operand type [cols][16 m1], or NULL
  const void* Afr;       // layer-1 fragments of type 0 (forward W1^T, backward W1)
  int64_t a_type_stride;
  const float* vec;      // fitting vectors per type (b1 at offset 0)
  int64_t vec_type_stride;
  void* X;               // forward: h1 out, FP32 [cols][ldx]; backward: dz1 in, operand type [cols][ldx]
  int ldx;
  float* gT;             // backward: [cols][m1][4]
  int m1, fw;
};

// Forward.  A work-group of NW waves owns 16 NB columns of one type and all
// output features (at most 16 m-tiles): wave w computes m-tiles w + NW i,
// i < 16 / NW (a tile past the last repeats it; its results are dropped),
// for the NB column tiles.  Per 32-wide k-step the work-group forms the D
// fragments of its columns into double-buffered LDS (8 NB / NW values per
// thread) from an LDS copy of T, and each wave reads its weight fragments
// from memory, PF k-steps ahead through a ring of registers.
template <class P, int NB, int NW, int PF>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2))) void k_fit1_fwd_lp(Fit1Args f) {
  typedef typename P::store_t ST;
  typedef typename P::raw8 R8;
  typedef typename P::raw4 R4;
  constexpr int NT = 64 * NW;      // threads
  constexpr int CW = 16 * NB;
  constexpr int MPW = 16 / NW;     // m-tiles per wave
  constexpr int EPT = 8 * NB / NW; // D elements per thread and k-step
  static_assert(EPT == 1 || EPT == 2 || EPT == 4, "D elements of a thread share one half of a lane's fragment");
  __shared__ f4 Ts[CW * kFit1MaxM1];  // [CW][m1]
  __shared__ __attribute__((aligned(16))) ST bfr[2][NB][64 * 8];
  const int t = blockIdx.z;
  const int n_t = f.meta[2 * t], cb = f.meta[2 * t + 1];
  const int c0 = blockIdx.x * CW;
  if (c0 >= n_t) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r16 = lane & 15, gq = lane >> 4;
  const int m1 = f.m1, nd = 16 * m1, KT = nd / 32;
  // T of the work-group's columns (zero past the type's atoms): thread tid
  // sums rows e = tid + NT u of the column-major [CW][m1] tile; every load
  // of a section is issued before any is used
  {
    constexpr int U = (CW * kFit1MaxM1 + NT - 1) / NT;
    const float* base = f.Tpart + (int64_t)(cb + c0) * m1 * 4;
    const int lim = min(CW, n_t - c0) * m1;  // rows of real columns
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = f4{0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < f.ntypes; ++s) {
      f4 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = tid + NT * u;
        x[u] = e < lim ? *reinterpret_cast<const f4*>(base + s * f.tstride + (int64_t)e * 4) : f4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] += x[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + NT * u;
      if (e < CW * m1) Ts[e] = v[u];
    }
  }
  __syncthreads();
  // this thread's D elements: column tile dq, fragment lane dl, elements
  // dj0 .. dj0 + EPT - 1, all with j / 4 = dh (a = 2 kt + dh):
  // tid = dq 64 (8 / EPT) + dl (8 / EPT) + dj0 / EPT
  constexpr int TPL = 8 / EPT;  // threads per fragment lane
  const int dq = tid / (64 * TPL);
  const int dl = (tid / TPL) & 63;
  const int dj0 = (tid % TPL) * EPT;
  const int dh = dj0 >> 2;
  const int dcol = dq * 16 + (dl & 15);
  f4 Tb[EPT];
#pragma unroll
  for (int u = 0; u < EPT; ++u) Tb[u] = Ts[dcol * m1 + 4 * (dl >> 4) + ((dj0 + u) & 3)];
  ST* const dglob = f.D ? static_cast<ST*>(f.D) + (int64_t)(cb + c0 + dcol) * nd + 4 * (dl >> 4) + (dj0 & 3) : nullptr;
  auto form = [&](int buf, int kt) {
    const int a = 2 * kt + dh;
    const f4 Ta = Ts[dcol * m1 + a];
    float d[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) d[u] = Ta[0] * Tb[u][0] + Ta[1] * Tb[u][1] + Ta[2] * Tb[u][2] + Ta[3] * Tb[u][3];
    ST* dst = &bfr[buf][dq][dl * 8 + dj0];
    if constexpr (EPT == 4) {
      R4 u4;
#pragma unroll
      for (int u = 0; u < 4; ++u) u4[u] = P::bits(d[u]);
      *reinterpret_cast<R4*>(dst) = u4;
      if (dglob) *reinterpret_cast<R4*>(dglob + 16 * a) = u4;
    } else {
#pragma unroll
      for (int u = 0; u < EPT; ++u) {
        dst[u] = P::bits(d[u]);
        if (dglob) dglob[16 * a + u] = P::bits(d[u]);
      }
    }
  };
  const int mtiles = f.fw / 16;
  const ST* Afr = static_cast<const ST*>(f.Afr) + t * f.a_type_stride;
  const ST* aSrc[MPW];
#pragma unroll
  for (int i = 0; i < MPW; ++i) aSrc[i] = Afr + ((int64_t)min(wv + NW * i, mtiles - 1) * KT * 64 + lane) * 8;
  f4 acc[MPW][NB];
#pragma unroll
  for (int i = 0; i < MPW; ++i)
#pragma unroll
    for (int n = 0; n < NB; ++n) acc[i][n] = f4{0.f, 0.f, 0.f, 0.f};
  R8 ar[PF][MPW];
  auto load = [&](int kt, R8* r) {
#pragma unroll
    for (int i = 0; i < MPW; ++i) r[i] = *reinterpret_cast<const R8*>(aSrc[i] + (int64_t)kt * 512);
  };
#pragma unroll
  for (int d = 0; d < PF; ++d) load(min(d, KT - 1), ar[d]);
  form(0, 0);
  __syncthreads();
  // one k-step: products from buffer kt & 1 with ring slot d, which is then
  // refilled with step kt + PF (the last step again past the end); the D
  // fragments of step kt + 1 go to the other buffer
  auto iter = [&](int kt, int d) {
    const int buf = kt & 1;
    R8 bb[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) bb[n] = *reinterpret_cast<const R8*>(&bfr[buf][n][lane * 8]);
#pragma unroll
    for (int i = 0; i < MPW; ++i)
#pragma unroll
      for (int n = 0; n < NB; ++n)
        acc[i][n] = P::mfma(__builtin_bit_cast(typename P::vec8, ar[d][i]), __builtin_bit_cast(typename P::vec8, bb[n]),
                            acc[i][n]);
    load(min(kt + PF, KT - 1), ar[d]);
    if (kt + 1 < KT) form(buf ^ 1, kt + 1);
    __syncthreads();
  };
  int kb = 0;
  for (; kb + PF <= KT; kb += PF)
#pragma unroll
    for (int d = 0; d < PF; ++d) iter(kb + d, d);
#pragma unroll
  for (int d = 0; d < PF; ++d)
    if (kb + d < KT) iter(kb + d, d);
  // T to HBM from the LDS copy (the tile's columns are contiguous there)
  {
    f4* const dst = reinterpret_cast<f4*>(f.T + (int64_t)(cb + c0) * m1 * 4);
    for (int e = tid; e < CW * m1; e += NT) dst[e] = Ts[e];
  }
  const float* vec = f.vec + t * f.vec_type_stride;
#pragma unroll
  for (int i = 0; i < MPW; ++i) {
    const int mt = wv + NW * i;
    if (mt >= mtiles) break;
    const int m0 = 16 * mt + 4 * gq;
#pragma unroll
    for (int n = 0; n < NB; ++n) {
      if (c0 + 16 * n >= n_t) continue;
      float* out = static_cast<float*>(f.X) + (int64_t)(cb + c0 + 16 * n + r16) * f.ldx + m0;
      float tv[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) tv[v] = tanh_f(acc[i][n][v] + vec[m0 + v]);
      *reinterpret_cast<f4*>(out) = f4{tv[0], tv[1], tv[2], tv[3]};
    }
  }
}

// Backward.  A work-group of 4 NCG waves owns 16 NT NCG columns of one
// type: wave (cg, ch) takes the NT column tiles of column group cg and the
// quarter ch of the m1 rows a of dE/dD (m-tile a = dD[a][0..15]), so each
// weight fragment it loads serves NT products (the kept form: NT = 2,
// NCG = 1).  Its dz1 fragments (the whole reduction, fw <= 256) stay in
// registers; per m-tile it runs the fw/32 products per column tile, then
// folds each 16 x 16 result tile into g_T at once: lane (column n, group g)
// holds dD[a][4 g + e] in element e, so the first term sums the lane's four
// elements against its T rows 4 g + e and the four lane groups (two
// exchanges), and the second term accumulates dD[a][4 g + e] T[a][k] into
// the lane's rows 4 g + e.  The first terms go to an LDS copy of the
// work-group's g_T tile (its columns are contiguous in HBM, so the tile is
// written out at the end with whole 16-byte vectors per lane); the quarters'
// second terms are then added into its rows a < m2 one quarter after the
// other.
template <class P, int NT, int NCG, int KT, int R>
__global__ __launch_bounds__(256 * NCG) __attribute__((amdgpu_waves_per_eu(R > 2 ? 1 : 2))) void k_fit1_bwd_lp(Fit1Args f) {
  typedef typename P::store_t ST;
  typedef typename P::raw8 R8;
  typedef typename P::raw4 R4;
  constexpr int CW = 16 * NT * NCG;
  __shared__ f4 gtile[CW * kFit1MaxM1];          // g_T of the work-group's columns, [CW][m1]
  const int t = blockIdx.z;
  const int n_t = f.meta[2 * t], cb = f.meta[2 * t + 1];
  const int c0 = blockIdx.x * CW;
  if (c0 >= n_t) return;
  const int tid = threadIdx.x, lane = tid & 63, ch = (tid >> 6) & 3;
  const int r16 = lane & 15, gq = lane >> 4;
  const int m1 = f.m1;
  // the wave's first column: column group tid / 256 holds tiles NT cg .. NT cg + NT - 1
  const int cw0 = 16 * NT * (tid >> 8);
  // dz1 fragments of column tile n: lane elements j < 4 are
  // dz1[32 kt + 4 g ..], j >= 4 dz1[32 kt + 16 + 4 g ..]; entries at or past
  // fw are zero (the buffer's padding, inside its 32 KT-wide rows, may hold
  // stale bits)
  R8 bz[NT][KT];
  f4 Tlo[NT][4], q[NT][4];
#pragma unroll
  for (int n = 0; n < NT; ++n) {
    const int64_t col = cb + c0 + cw0 + 16 * n + r16;
    const ST* src = static_cast<const ST*>(f.X) + col * f.ldx + 4 * gq;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      R4 l4 = *reinterpret_cast<const R4*>(src + 32 * kt);
      R4 h4 = *reinterpret_cast<const R4*>(src + 32 * kt + 16);
      const R4 z4 = {};
      if (32 * kt + 4 * gq >= f.fw) l4 = z4;
      if (32 * kt + 16 + 4 * gq >= f.fw) h4 = z4;
      bz[n][kt] = join8<P>(l4, h4);
    }
    const float* Tc = f.T + col * m1 * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Tlo[n][e] = *reinterpret_cast<const f4*>(Tc + (4 * gq + e) * 4);
      q[n][e] = f4{0.f, 0.f, 0.f, 0.f};
    }
  }
  const int a_lo = m1 * ch / 4, a_hi = m1 * (ch + 1) / 4;
  const ST* Afr = static_cast<const ST*>(f.Afr) + t * f.a_type_stride + (int64_t)lane * 8;
  // T rows of the lane's column in tile 0; tile n is 16 n columns on
  const int64_t cstride = 16 * (int64_t)m1 * 4;
  const float* const Tcol0 = f.T + (cb + c0 + cw0 + r16) * (int64_t)m1 * 4;
  // operands of m-tile a, R - 1 m-tiles ahead through a ring of R register
  // sets: the weight fragments and the T row a of each column, requested
  // together so that waiting for one m-tile's operands never waits for a
  // later one's
  R8 Ar[R][KT];
  f4 Tar[R][NT];
  auto load = [&](int a, R8* r, f4* ta) {
    const int aa = min(a, a_hi - 1);
    const ST* p = Afr + (int64_t)aa * (KT * 512);
#pragma unroll
    for (int n = 0; n < NT; ++n) ta[n] = *reinterpret_cast<const f4*>(Tcol0 + n * cstride + aa * 4);
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) r[kt] = *reinterpret_cast<const R8*>(p + kt * 512);
  };
  const bool odd = gq & 1, high = gq & 2;
  auto tile = [&](int a, const R8* r, const f4* ta) {
    // the column tiles' product chains interleaved
    f4 accs[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) accs[n] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int n = 0; n < NT; ++n)
        accs[n] = P::mfma(__builtin_bit_cast(typename P::vec8, r[kt]), __builtin_bit_cast(typename P::vec8, bz[n][kt]), accs[n]);
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const f4 acc = accs[n];
      // first term: the lane's partial over its four elements, then summed
      // over the four lane groups by halving (exchange with g ^ 1 keeps the
      // columns k of g's parity, exchange with g ^ 2 leaves k = g)
      float p[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float s = acc[0] * Tlo[n][0][k];
#pragma unroll
        for (int e = 1; e < 4; ++e) s = fmaf(acc[e], Tlo[n][e][k], s);
        p[k] = s;
      }
      const float u0 = (odd ? p[1] : p[0]) + shfl_xor_f(odd ? p[0] : p[1], 16);
      const float u1 = (odd ? p[3] : p[2]) + shfl_xor_f(odd ? p[2] : p[3], 16);
      const float mine = (high ? u1 : u0) + shfl_xor_f(high ? u0 : u1, 32);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int k = 0; k < 4; ++k) q[n][e][k] = fmaf(acc[e], ta[n][k], q[n][e][k]);
      reinterpret_cast<float*>(&gtile[(cw0 + 16 * n + r16) * m1 + a])[gq] = mine;
    }
  };
#pragma unroll
  for (int d = 0; d + 1 < R; ++d) load(a_lo + d, Ar[d], Tar[d]);
  // m-tile a_lo + i uses slot i % R; slot (i - 1) % R, just consumed, takes
  // m-tile a_lo + i + R - 1 (past the end the last m-tile again, unused)
  for (int a = a_lo; a < a_hi; a += R)
#pragma unroll
    for (int d = 0; d < R; ++d)
      if (a + d < a_hi) {
        load(a + d + R - 1, Ar[(d + R - 1) % R], Tar[(d + R - 1) % R]);
        tile(a + d, Ar[d], Tar[d]);
      }
  // second-term partials, quarter by quarter: lane (n, g) holds rows 4 g + e
  for (int h = 0; h < 4; ++h) {
    __syncthreads();
    if (ch == h) {
#pragma unroll
      for (int n = 0; n < NT; ++n)
#pragma unroll
        for (int e = 0; e < 4; ++e) gtile[(cw0 + 16 * n + r16) * m1 + 4 * gq + e] += q[n][e];
    }
  }
  __syncthreads();
  // the real columns' rows, in order: one contiguous block of HBM
  const int rows = min(CW, n_t - c0) * m1;
  f4* const dst = reinterpret_cast<f4*>(f.gT + (int64_t)(cb + c0) * m1 * 4);
  for (int e = tid; e < rows; e += 256 * NCG) dst[e] = gtile[e];
}

// ---------------------------------------------------------------- descriptor
// D[a*m2 + b] = sum_k T[a][k] T[b][k], a < m1, b < m2 (m2 = 16).  One
// work-group per column, thread a writes 16 consecutive entries.
template <typename TT, typename DT>
__global__ __launch_bounds__(128) void k_descriptor(const int32_t* __restrict__ atom_at, const TT* __restrict__ Tpart,
                                                    int64_t tstride, int ntypes, TT* __restrict__ T,
                                                    DT* __restrict__ D, int m1, int mode_lp_f16) {
  // D == nullptr: only the section sum T is formed (FP64 builds D inside the
  // fitting GEMM)
  __shared__ TT Ts[128][4];
  const int col = blockIdx.x;
  const bool real = atom_at[col] >= 0;
  const int a = threadIdx.x;
  if (a < m1) {
    TT v[4] = {(TT)0, (TT)0, (TT)0, (TT)0};
    if (real)
      for (int t = 0; t < ntypes; ++t) {
        const TT* p = Tpart + t * tstride + ((int64_t)col * m1 + a) * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += p[k];
      }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      Ts[a][k] = v[k];
      T[((int64_t)col * m1 + a) * 4 + k] = v[k];  // zeros on padding columns
    }
  }
  if (D == nullptr) return;
  __syncthreads();
  // consecutive threads write consecutive entries e = a*16 + b
  DT* out = D + (int64_t)col * m1 * 16;
  for (int e = threadIdx.x; e < m1 * 16; e += 128) {
    const int aa = e >> 4, b = e & 15;
    const TT acc = Ts[aa][0] * Ts[b][0] + Ts[aa][1] * Ts[b][1] + Ts[aa][2] * Ts[b][2] + Ts[aa][3] * Ts[b][3];
    if constexpr (sizeof(DT) == 2) {
      out[e] = mode_lp_f16 ? PrecF16::bits((float)acc) : PrecBF16::bits((float)acc);
    } else {
      out[e] = (DT)acc;  // FP64, or FP32 for an FP32 first fitting layer
    }
  }
}

// g_T[a][k] = sum_b dD[a][b] T[b][k] + [a < m2] sum_a' dD[a'][a] T[a'][k]
template <typename TT>
__global__ __launch_bounds__(128) void k_desc_bwd(const int32_t* __restrict__ atom_at, const TT* __restrict__ T,
                                                  const TT* __restrict__ dD, TT* __restrict__ gT, int m1) {
  __shared__ TT Ts[128][4];
  __shared__ TT dDs[128 * 16 + 1];
  const int col = blockIdx.x;
  if (atom_at[col] < 0) return;
  const int a = threadIdx.x;
  if (a < m1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) Ts[a][k] = T[((int64_t)col * m1 + a) * 4 + k];
#pragma unroll
    for (int b = 0; b < 16; ++b) dDs[a * 16 + b] = dD[((int64_t)col * m1 + a) * 16 + b];
  }
  __syncthreads();
  // second term by the first wave: lane group q = a / 16 sums a' = q, q + 4,
  // ..., then the four groups are added across lanes
  TT s2[4] = {0, 0, 0, 0};
  if (a < 64) {
    const int c16 = a & 15;
    for (int a2 = a >> 4; a2 < m1; a2 += 4) {
      const TT w = dDs[a2 * 16 + c16];
#pragma unroll
      for (int k = 0; k < 4; ++k) s2[k] += w * Ts[a2][k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s2[k] += __shfl_xor(s2[k], 16, 64);
      s2[k] += __shfl_xor(s2[k], 32, 64);
    }
  }
  if (a >= m1) return;
  TT acc[4] = {0, 0, 0, 0};
  for (int b = 0; b < 16; ++b) {
    const TT w = dDs[a * 16 + b];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += w * Ts[b][k];
  }
  if (a < 16)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += s2[k];
#pragma unroll
  for (int k = 0; k < 4; ++k) gT[((int64_t)col * m1 + a) * 4 + k] = acc[k];
}

// ---------------------------------------------------------------- launchers
// Pointer to element `off` of a fragment array of element kind (1, 2: 2 B;
// 3: 4 B).
static const void* elem_offset(const void* base, int kind, int64_t off) {
  return kind == 3 ? (const void*)((const float*)base + off) : (const void*)((const uint16_t*)base + off);
}

// Activation buffer slots in dp_ctx::fa (FP64 / mixed):
//   FP64 : 0 t1(=h1) 1 t2 2 h2 4 h3 5 dz3 7 dz2 8 dz1 [cols][fw]
//   mixed: 0 t1 1 t2 2 h2 4 h3 (f32 [cols][fwp]); 7 dz3 8 dz2 9 dz1 (half
//          [cols][fwp])
// The other slots are free; the parameter gradients after a mixed compute
// use them for FP64 copies.
// Tile shapes (m-tiles x n-tiles per wave, 4 waves along the columns).
// Small-M form (the paper's concern with GEMMs of few rows, here few atoms
// per type): when the unsplit grid would leave most of the chip idle and the
// reduction is long, the k-steps are split over up to kSplitMax work-groups
// per tile (at least 8 k-steps each) and k_split_finish adds the partial
// sums in a fixed order.  Returns the split count (1: no split).
static int split_count(const dp_ctx* c, int64_t wgs_unsplit, int ksteps) {
  const int64_t cols = c->natoms_last + (int64_t)c->model->desc.ntypes * kColPad;
  if (cols > c->split_cols || wgs_unsplit <= 0) return 1;
  int64_t ns = (int64_t)c->ncu / wgs_unsplit;  // about one work-group per CU
  if (ns > kSplitMax) ns = kSplitMax;
  if (ns > ksteps / 8) ns = ksteps / 8;
  return ns >= 2 ? (int)ns : 1;
}

// Work-groups of the unsplit grid that have columns to do (per-type counts
// live on the device; the types' columns sum to natoms_last, and each type
// may end in a partial tile).
static int64_t unsplit_wgs(const dp_ctx* c, int BN, int mblocks) {
  return ((c->natoms_last + BN - 1) / BN + c->model->desc.ntypes - 1) * mblocks;
}

template <typename T>
static void split_finish(dp_ctx* c, const GemmArgs& g, hipStream_t s) {
  // each type's columns are at most natoms_last (bounded per type on the device)
  const int64_t work = ((c->natoms_last + 15) & ~15) * (int64_t)g.M;
  dim3 grid((unsigned)((work + 255) / 256), (unsigned)c->model->desc.ntypes);
  if (work > 0) hipLaunchKernelGGL((k_split_finish<T>), grid, dim3(256), 0, s, g);
}

template <int MT, int NT>
static void gemm_launch_f64(dp_ctx* c, const GemmArgs& g0, hipStream_t s) {
  const int ntypes = c->model->desc.ntypes;
  const int BN = 4 * NT * 16;
  const int mtiles = g0.M / 16;
  const int mblocks = (mtiles + MT - 1) / MT;
  dim3 grid((unsigned)((c->natoms_last + BN - 1) / BN), (unsigned)mblocks, (unsigned)ntypes);
  if (grid.x == 0) return;
  GemmArgs g = g0;
  g.nsplit = split_count(c, unsplit_wgs(c, BN, mblocks), g.K / 16);
  if (g.nsplit > 1) {
    g.part = c->split_part;
    g.part_cols = c->split_cols;
    grid.y = (unsigned)(mblocks * g.nsplit);
    if (g.T) hipLaunchKernelGGL((k_fit_gemm_f64<MT, NT, true, true>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_fit_gemm_f64<MT, NT, false, true>), grid, dim3(256), 0, s, g);
    split_finish<double>(c, g, s);
    return;
  }
  if (g.T) hipLaunchKernelGGL((k_fit_gemm_f64<MT, NT, true, false>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((k_fit_gemm_f64<MT, NT, false, false>), grid, dim3(256), 0, s, g);
}

template <class P, int MTW, int NTW, bool SPLIT>
static void gemm_launch_lp_t(dim3 grid, bool deep, const GemmArgs& g, hipStream_t s) {
  if (deep) hipLaunchKernelGGL((k_fit_gemm_lp<P, MTW, NTW, 8, SPLIT>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((k_fit_gemm_lp<P, MTW, NTW, 2, SPLIT>), grid, dim3(256), 0, s, g);
}

template <class P, int MTW, int NTW>
static void gemm_launch_lp_k(dim3 grid, bool deep, const GemmArgs& g, hipStream_t s) {
  if (g.nsplit > 1) gemm_launch_lp_t<P, MTW, NTW, true>(grid, deep, g, s);
  else gemm_launch_lp_t<P, MTW, NTW, false>(grid, deep, g, s);
}

// kind: element kind of the first fitting layer (the only GEMM launched here)
template <int MTW, int NTW>
static void gemm_launch_lp(dp_ctx* c, const GemmArgs& g0, int kind, hipStream_t s) {
  const int ntypes = c->model->desc.ntypes;
  const int BN = 32 * NTW;
  const int mtiles = g0.M / 16;
  const int mblocks = (mtiles + 2 * MTW - 1) / (2 * MTW);
  dim3 grid((unsigned)((c->natoms_last + BN - 1) / BN), (unsigned)mblocks, (unsigned)ntypes);
  if (grid.x == 0) return;
  GemmArgs g = g0;
  g.nsplit = split_count(c, unsplit_wgs(c, BN, mblocks), g.K / 32);
  if (g.nsplit > 1) {
    g.part = c->split_part;
    g.part_cols = c->split_cols;
    grid.y = (unsigned)(mblocks * g.nsplit);
  }
  // the ring depth follows the k-steps one work-group walks
  const bool deep = g.K / 32 / g.nsplit >= 16;
  if (kind == 1) gemm_launch_lp_k<PrecBF16, MTW, NTW>(grid, deep, g, s);
  else if (kind == 2) gemm_launch_lp_k<PrecF16, MTW, NTW>(grid, deep, g, s);
  else gemm_launch_lp_k<PrecF32, MTW, NTW>(grid, deep, g, s);
  if (g.nsplit > 1) split_finish<float>(c, g, s);
}

// Tile shapes picked by sweeps on the 12,288-atom water model: FP64 MFMA
// wants a 3x2 tile per wave (48 features x 32 columns; 5x2 and 3x1 were
// slower: too few or too many work-groups for these sizes, and a 48-column
// tile would cross the 128-column type segments); the half-precision GEMM
// 2x2 per wave (64 x 64 per work-group).
static void gemm_launch(dp_ctx* c, const GemmArgs& g, int mode, hipStream_t s) {
  if (mode != DP_FP64) gemm_launch_lp<2, 2>(c, g, mix_kinds(mode).fit1, s);
  else gemm_launch_f64<3, 2>(c, g, s);
}

static GemmArgs gemm_base(dp_ctx* c, int mode) {
  const dp_model* m = c->model;
  GemmArgs g = {};
  g.meta = c->type_meta;
  g.vec = mode == DP_FP64 ? (const void*)m->fit_vec64 : (const void*)m->fit_vec32;
  g.vec_type_stride = m->fit_vec_per_type;
  return g;
}

// The fused first layer (k_fit1_fwd_lp / k_fit1_bwd_lp) serves the BF16 and
// FP16 first layers once a frame has enough atoms to give every compute unit
// a 32-column work-group; frames of few atoms keep the split-K GEMM with the
// separate descriptor passes.
bool fit1_fused(const dp_ctx* c, int32_t mode) {
  if (mode == DP_FP64 || mode == DP_FP64_TAB) return false;
  const dp_model* m = c->model;
  const int k1 = mix_kinds(mode).fit1;
  if (k1 != 1 && k1 != 2) return false;
  // the backward's reduction is 8 steps of 32 (224 < fw <= 256, as the
  // paper's 240-wide fitting net)
  if (m->m1 < 16 || m->m1 > kFit1MaxM1 || (m->m1 & 1) || m->fw % 16 || m->fw <= 224 || m->fw > 256) return false;
  return (c->natoms_last + 31) / 32 >= c->ncu;
}

static Fit1Args fit1_base(dp_ctx* c, int32_t mode, bool bwd) {
  const dp_model* m = c->model;
  const MixKinds mk = mix_kinds(mode);
  Fit1Args f = {};
  f.meta = c->type_meta;
  f.Tpart = (const float*)c->Tpart;
  f.tstride = c->max_cols * m->m1 * 4;
  f.ntypes = m->desc.ntypes;
  f.T = (float*)c->T;
  const void* frag1 = frag_of(m->fit_frag_bf16, m->fit_frag_f16, m->fit_frag_f32, mk.fit1);
  f.Afr = elem_offset(frag1, mk.fit1, bwd ? m->ffo_lp.bwd[0] : m->ffo_lp.fwd[0]);
  f.a_type_stride = m->ffo_lp.per_type;
  f.vec = m->fit_vec32;
  f.vec_type_stride = m->fit_vec_per_type;
  f.ldx = ((m->fw + 31) / 32) * 32;
  f.gT = (float*)c->gT;
  f.m1 = m->m1;
  f.fw = m->fw;
  return f;
}

// h1 = tanh(D W1 + b1) with D formed from the section partials of T (T is
// written too; D only when write_d, for the parameter gradients)
static void launch_fit1_fwd(dp_ctx* c, int32_t mode, bool write_d, hipStream_t s) {
  Fit1Args f = fit1_base(c, mode, false);
  f.D = write_d ? c->D : nullptr;
  f.X = c->fa[0];
  constexpr int NB = 2, NW = 4;
  dim3 grid((unsigned)((c->natoms_last + 16 * NB - 1) / (16 * NB)), 1, (unsigned)c->model->desc.ntypes);
  if (mix_kinds(mode).fit1 == 1) hipLaunchKernelGGL((k_fit1_fwd_lp<PrecBF16, NB, NW, 4>), grid, dim3(64 * NW), 0, s, f);
  else hipLaunchKernelGGL((k_fit1_fwd_lp<PrecF16, NB, NW, 4>), grid, dim3(64 * NW), 0, s, f);
}

// g_T from dz1 (the first layer's backward product with the descriptor
// backward in its epilogue)
static void launch_fit1_bwd(dp_ctx* c, int32_t mode, hipStream_t s) {
  constexpr int NT = 2, NCG = 1, RING = 2, CW = 16 * NT * NCG;
  Fit1Args f = fit1_base(c, mode, true);
  f.X = c->fa[9];
  dim3 grid((unsigned)((c->natoms_last + CW - 1) / CW), 1, (unsigned)c->model->desc.ntypes);
  if (mix_kinds(mode).fit1 == 1) hipLaunchKernelGGL((k_fit1_bwd_lp<PrecBF16, NT, NCG, 8, RING>), grid, dim3(256 * NCG), 0, s, f);
  else hipLaunchKernelGGL((k_fit1_bwd_lp<PrecF16, NT, NCG, 8, RING>), grid, dim3(256 * NCG), 0, s, f);
}

void launch_descriptor(dp_ctx* c, int32_t mode, hipStream_t s) {
  if (fit1_fused(c, mode)) return;  // formed inside the first fitting layer
  launch_descriptor_ex(c, mode, mode != DP_FP64, s);
}

void launch_descriptor_ex(dp_ctx* c, int32_t mode, bool write_d, hipStream_t s) {
  const dp_model* m = c->model;
  const int ncols = (int)(c->natoms_last + m->desc.ntypes * kColPad);
  if (c->natoms_last <= 0) return;
  const int64_t ts = c->max_cols * m->m1 * 4;
  if (mode == DP_FP64)
    hipLaunchKernelGGL((k_descriptor<double, double>), dim3(ncols), dim3(128), 0, s, c->atom_at,
                       (const double*)c->Tpart, ts, m->desc.ntypes, (double*)c->T,
                       write_d ? (double*)c->D : (double*)nullptr, m->m1, 0);
  else if (mix_kinds(mode).fit1 == 3)
    hipLaunchKernelGGL((k_descriptor<float, float>), dim3(ncols), dim3(128), 0, s, c->atom_at,
                       (const float*)c->Tpart, ts, m->desc.ntypes, (float*)c->T, (float*)c->D, m->m1, 0);
  else
    hipLaunchKernelGGL((k_descriptor<float, uint16_t>), dim3(ncols), dim3(128), 0, s, c->atom_at,
                       (const float*)c->Tpart, ts, m->desc.ntypes, (float*)c->T, (uint16_t*)c->D, m->m1,
                       mix_kinds(mode).fit1 == 2 ? 1 : 0);
}

void launch_desc_bwd(dp_ctx* c, int32_t mode, hipStream_t s) {
  if (fit1_fused(c, mode)) return;  // folded into the first layer's backward product
  const dp_model* m = c->model;
  const int ncols = (int)(c->natoms_last + m->desc.ntypes * kColPad);
  if (c->natoms_last <= 0) return;
  if (mode == DP_FP64)
    hipLaunchKernelGGL((k_desc_bwd<double>), dim3(ncols), dim3(128), 0, s, c->atom_at, (const double*)c->T,
                       (const double*)c->dD, (double*)c->gT, m->m1);
  else
    hipLaunchKernelGGL((k_desc_bwd<float>), dim3(ncols), dim3(128), 0, s, c->atom_at, (const float*)c->T,
                       (const float*)c->dD, (float*)c->gT, m->m1);
}

// keep_h: also store h2 and h3, which only the parameter gradients read.
void launch_fit_forward(dp_ctx* c, int32_t mode, bool keep_h, hipStream_t s) {
  const dp_model* m = c->model;
  if (c->natoms_last <= 0) return;
  const int fw = m->fw;
  const int fwp = ((fw + 31) / 32) * 32;
  GemmArgs g = gemm_base(c, mode);
  const bool f64 = mode == DP_FP64;
  const MixKinds mk = mix_kinds(mode);
  const void* frag1 = f64 ? (const void*)m->fit_frag64 : frag_of(m->fit_frag_bf16, m->fit_frag_f16, m->fit_frag_f32, mk.fit1);
  const void* frag = f64 ? (const void*)m->fit_frag64 : frag_of(m->fit_frag_bf16, m->fit_frag_f16, m->fit_frag_f32, mk.fit23);
  const int64_t* off_fwd = f64 ? m->ffo.fwd : m->ffo_lp.fwd;
  const int64_t tstride = f64 ? m->ffo.per_type : m->ffo_lp.per_type;
  // layer 1: X = D [cols][nd] (FP64: built from T inside the GEMM)
  if (fit1_fused(c, mode)) {
    launch_fit1_fwd(c, mode, keep_h, s);
  } else {
  g.a_type_stride = tstride;
  g.Afr = f64 ? (const void*)((const double*)frag1 + off_fwd[0]) : elem_offset(frag1, mk.fit1, off_fwd[0]);
  g.X = c->D;
  g.ldx = m->nd;
  g.K = m->nd;
  g.Kreal = m->nd;
  g.T = f64 ? (const double*)c->T : nullptr;
  g.m1 = m->m1;
  g.M = fw;
  g.epi = EPI_TANH;
  g.bias_off = 0;
  g.out0 = c->fa[0];
  g.ld0 = f64 ? fw : fwp;
  gemm_launch(c, g, mode, s);
  }
  // layers 2, 3 and the output layer
  if (f64) {
    PairArgs p = {};
    p.meta = c->type_meta;
    p.atom_at = c->atom_at;
    p.fw = fw;
    p.in = (const double*)c->fa[0];
    p.A[0] = (const double*)frag + off_fwd[1];
    p.A[1] = (const double*)frag + off_fwd[2];
    p.a_type_stride = tstride;
    p.vec = m->fit_vec64;
    p.vec_type_stride = m->fit_vec_per_type;
    p.out[0] = (double*)c->fa[1];
    p.out[1] = keep_h ? (double*)c->fa[2] : nullptr;
    p.out[2] = keep_h ? (double*)c->fa[4] : nullptr;
    p.out[3] = (double*)c->fa[5];
    p.Ei_col = c->Ei_col;
    p.Ei_atom = c->Ei_atom;
    launch_pair_f64(c, false, p, s);
  } else {
    PairArgsLp p = {};
    p.meta = c->type_meta;
    p.atom_at = c->atom_at;
    p.fw = fw;
    p.fwp = fwp;
    p.in = c->fa[0];
    p.A[0] = elem_offset(frag, mk.fit23, off_fwd[1]);
    p.A[1] = elem_offset(frag, mk.fit23, off_fwd[2]);
    p.a_type_stride = tstride;
    p.vec = m->fit_vec32;
    p.vec_type_stride = m->fit_vec_per_type;
    p.out[0] = (float*)c->fa[1];
    p.out[1] = keep_h ? (float*)c->fa[2] : nullptr;
    p.out[2] = keep_h ? (float*)c->fa[4] : nullptr;
    p.outlp[0] = c->fa[7];
    p.Ei_col = c->Ei_col;
    p.Ei_atom = c->Ei_atom;
    launch_pair_lp(c, false, mode, p, s);
  }
}

// keep_dz2: also store dz2, which only the parameter gradients read.
void launch_fit_backward(dp_ctx* c, int32_t mode, bool keep_dz2, hipStream_t s) {
  const dp_model* m = c->model;
  if (c->natoms_last <= 0) return;
  const int fw = m->fw;
  const int fwp = ((fw + 31) / 32) * 32;
  const bool f64 = mode == DP_FP64;
  const MixKinds mk = mix_kinds(mode);
  const void* frag1 = f64 ? (const void*)m->fit_frag64 : frag_of(m->fit_frag_bf16, m->fit_frag_f16, m->fit_frag_f32, mk.fit1);
  const void* frag = f64 ? (const void*)m->fit_frag64 : frag_of(m->fit_frag_bf16, m->fit_frag_f16, m->fit_frag_f32, mk.fit23);
  const int64_t* off_bwd = f64 ? m->ffo.bwd : m->ffo_lp.bwd;
  const int64_t tstride = f64 ? m->ffo.per_type : m->ffo_lp.per_type;
  // layers 3 and 2: dh2 = w_out + W3 dz3, dz2 = dh2 (1 - t2^2), dh1 = dh2 +
  // W2 dz2, dz1 = dh1 (1 - t1^2)
  if (f64) {
    PairArgs p = {};
    p.meta = c->type_meta;
    p.fw = fw;
    p.in = (const double*)c->fa[5];
    p.A[0] = (const double*)frag + off_bwd[2];
    p.A[1] = (const double*)frag + off_bwd[1];
    p.a_type_stride = tstride;
    p.vec = m->fit_vec64;
    p.vec_type_stride = m->fit_vec_per_type;
    p.tprev[0] = (const double*)c->fa[1];
    p.tprev[1] = (const double*)c->fa[0];
    p.out[0] = keep_dz2 ? (double*)c->fa[7] : nullptr;
    p.out[1] = (double*)c->fa[8];
    launch_pair_f64(c, true, p, s);
  } else {
    PairArgsLp p = {};
    p.meta = c->type_meta;
    p.fw = fw;
    p.fwp = fwp;
    p.in = c->fa[7];
    p.A[0] = elem_offset(frag, mk.fit23, off_bwd[2]);
    p.A[1] = elem_offset(frag, mk.fit23, off_bwd[1]);
    p.a_type_stride = tstride;
    p.vec = m->fit_vec32;
    p.vec_type_stride = m->fit_vec_per_type;
    p.tprev[0] = (const float*)c->fa[1];
    p.tprev[1] = (const float*)c->fa[0];
    p.outlp[0] = keep_dz2 ? c->fa[8] : nullptr;
    p.outlp[1] = c->fa[9];
    launch_pair_lp(c, true, mode, p, s);
  }
  // layer 1: dD = W1 dz1
  if (fit1_fused(c, mode)) launch_fit1_bwd(c, mode, s);
  else launch_fit1_bwd_gemm(c, mode, s);
}

// dD = W1 dz1 as a plain GEMM (FP64, FP32, few atoms; also dE/dD on request
// where the fused form does not write it)
void launch_fit1_bwd_gemm(dp_ctx* c, int32_t mode, hipStream_t s) {
  const dp_model* m = c->model;
  if (c->natoms_last <= 0) return;
  const int fw = m->fw;
  const int fwp = ((fw + 31) / 32) * 32;
  const bool f64 = mode == DP_FP64;
  const MixKinds mk = mix_kinds(mode);
  const void* frag1 = f64 ? (const void*)m->fit_frag64 : frag_of(m->fit_frag_bf16, m->fit_frag_f16, m->fit_frag_f32, mk.fit1);
  const int64_t* off_bwd = f64 ? m->ffo.bwd : m->ffo_lp.bwd;
  const int64_t tstride = f64 ? m->ffo.per_type : m->ffo_lp.per_type;
  GemmArgs g = gemm_base(c, mode);
  g.a_type_stride = tstride;
  g.Afr = f64 ? (const void*)((const double*)frag1 + off_bwd[0]) : elem_offset(frag1, mk.fit1, off_bwd[0]);
  g.X = f64 ? c->fa[8] : c->fa[9];
  g.ldx = f64 ? fw : fwp;
  g.K = f64 ? fw : fwp;
  g.Kreal = fw;
  g.M = m->nd;
  g.epi = EPI_PLAIN;
  g.out0 = c->dD;
  g.ld0 = m->nd;
  gemm_launch(c, g, mode, s);
}

// ---------------------------------------------------------------- inspection
// Copies a column-ordered per-atom buffer into atom order as f64.
__global__ void k_gather_cols(const int32_t* __restrict__ col_of, const void* __restrict__ src, int kind_f32,
                              int kind_lp, int width, double* __restrict__ dst, int ntot) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ntot * width) return;
  const int i = (int)(idx / width), k = (int)(idx % width);
  const int64_t s = (int64_t)col_of[i] * width + k;
  double v;
  if (kind_lp == 1) v = PrecBF16::tof(reinterpret_cast<const uint16_t*>(src)[s]);
  else if (kind_lp == 2) v = PrecF16::tof(reinterpret_cast<const uint16_t*>(src)[s]);
  else if (kind_f32) v = reinterpret_cast<const float*>(src)[s];
  else v = reinterpret_cast<const double*>(src)[s];
  dst[idx] = v;
}

void launch_gather_cols(dp_ctx* c, int32_t which, int32_t mode, int32_t ntot, double* dst, hipStream_t s) {
  const dp_model* m = c->model;
  const void* src = which == 1 ? c->T : (which == 2 ? c->D : (which == 5 ? c->gT : c->dD));
  const int width = which == 1 || which == 5 ? m->m1 * 4 : m->nd;
  const bool f64 = mode == DP_FP64;
  int kind_lp = 0;
  if (!f64 && which == 2 && mix_kinds(mode).fit1 != 3) kind_lp = mix_kinds(mode).fit1;
  const int64_t tot = (int64_t)ntot * width;
  if (tot > 0)
    hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, c->col_of, src,
                       f64 ? 0 : 1, kind_lp, width, dst, ntot);
}

}  // namespace dpse
