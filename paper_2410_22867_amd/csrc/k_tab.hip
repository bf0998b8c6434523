// DP-compress: the embedding nets as tables of piecewise quintics (the
// compression of the embedding net that the Background section cites), built
// on the device from the model's parameters and evaluated, fused with the
// G^T R contraction, in the FP64 force path.
//
// Grid (shared with the documentation of dp_model_compress): a fine stride
// h on [0, X1) with n1 intervals (X1 = n1 h) and a coarse stride H = 10 h on
// [X1, X2) with n2 intervals.  Node n is at n h for n <= n1 and at
// X1 + (n - n1) H beyond.  On interval k the quintic in t = x - x_k matches
// G, dG/dx and d2G/dx2 at both ends.  Table layout [net][k][p][a]: for a
// power p the m1 features are contiguous, so 16 lanes that evaluate 16
// consecutive features of one row read 128 contiguous bytes.
//
// Inputs x >= X2 take G(X2) with zero slope and raise DP_FLAG_TABLE_RANGE.
#include "dp_internal.h"
#include "dp_device.h"

namespace dpse {

// ------------------------------------------------------------ table build
// Node values: one work-group per (net, node), one thread per feature.
// Forward-mode derivatives through the layers: z = h W + b, z' = h' W,
// z'' = h'' W, tau = tanh z, tau' = (1 - tau^2) z',
// tau'' = (1 - tau^2)(z'' - 2 tau z'^2); the identity skips carry h, h', h''.
__global__ __launch_bounds__(128) void k_tab_nodes(const double* __restrict__ P, TabGrid g, int ntypes, int w1,
                                                   TabNetOffsets off, double* __restrict__ nodes) {
  const int net = blockIdx.y, node = blockIdx.x;
  const int m1 = 4 * w1;
  __shared__ double hv[3][128];  // value, slope, curvature of the layer's outputs
  const double x = node <= g.n1 ? (double)node * g.h : fma((double)(node - g.n1), g.H, g.X1);
  const int q = threadIdx.x;
  const double* W[3] = {P + off.W[net][0], P + off.W[net][1], P + off.W[net][2]};
  const double* B[3] = {P + off.b[net][0], P + off.b[net][1], P + off.b[net][2]};
  // layer 1: input x with x' = 1, x'' = 0 (width w1, no skip)
  double v = 0.0, v1 = 0.0, v2 = 0.0;
  if (q < w1) {
    const double z = fma(x, W[0][q], B[0][q]), z1 = W[0][q];
    const double tt = tanh_d(z), gg = 1.0 - tt * tt;
    v = tt;
    v1 = gg * z1;
    v2 = gg * (-2.0 * tt * z1 * z1);
  }
  int wp = w1;
  for (int l = 1; l < 3; ++l) {
    __syncthreads();
    if (q < wp) {
      hv[0][q] = v;
      hv[1][q] = v1;
      hv[2][q] = v2;
    }
    __syncthreads();
    const int w = 2 * wp;
    if (q < w) {
      double z = B[l][q], z1 = 0.0, z2 = 0.0;
      for (int p = 0; p < wp; ++p) {
        const double wt = W[l][(int64_t)p * w + q];
        z = fma(hv[0][p], wt, z);
        z1 = fma(hv[1][p], wt, z1);
        z2 = fma(hv[2][p], wt, z2);
      }
      const double tt = tanh_d(z), gg = 1.0 - tt * tt;
      const int s = q % wp;  // [h, h] skip of a doubled width
      v = hv[0][s] + tt;
      v1 = hv[1][s] + gg * z1;
      v2 = hv[2][s] + gg * (z2 - 2.0 * tt * z1 * z1);
    }
    wp = w;
  }
  if (q < m1) {
    double* o = nodes + ((int64_t)net * (g.nint + 1) + node) * 3 * m1;
    o[q] = v;
    o[m1 + q] = v1;
    o[2 * m1 + q] = v2;
  }
}

// Coefficients: one thread per (net, interval, feature).  With
// A = y1 - y0 - d0 L - s0 L^2/2, B = d1 - d0 - s0 L, C = s1 - s0:
// c0 = y0, c1 = d0, c2 = s0/2, c3 = (20A - 8BL + CL^2)/(2L^3),
// c4 = (-30A + 14BL - 2CL^2)/(2L^4), c5 = (12A - 6BL + CL^2)/(2L^5).
__global__ void k_tab_coef(const double* __restrict__ nodes, TabGrid g, int m1, int nnets, double* __restrict__ table) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)nnets * g.nint * m1;
  if (id >= total) return;
  const int a = (int)(id % m1);
  const int64_t nk = id / m1;
  const int k = (int)(nk % g.nint), net = (int)(nk / g.nint);
  const double L = k < g.n1 ? g.h : g.H;
  const double* n0 = nodes + ((int64_t)net * (g.nint + 1) + k) * 3 * m1;
  const double* n1 = n0 + 3 * m1;
  const double y0 = n0[a], d0 = n0[m1 + a], s0 = n0[2 * m1 + a];
  const double y1 = n1[a], d1 = n1[m1 + a], s1 = n1[2 * m1 + a];
  const double A = y1 - y0 - d0 * L - 0.5 * s0 * L * L;
  const double B = d1 - d0 - s0 * L;
  const double C = s1 - s0;
  const double L2 = L * L, L3 = L2 * L;
  double* c = table + ((int64_t)net * g.nint + k) * 6 * m1 + a;
  c[0] = y0;
  c[m1] = d0;
  c[2 * m1] = 0.5 * s0;
  c[3 * m1] = (20.0 * A - 8.0 * B * L + C * L2) / (2.0 * L3);
  c[4 * m1] = (-30.0 * A + 14.0 * B * L - 2.0 * C * L2) / (2.0 * L3 * L);
  c[5 * m1] = (12.0 * A - 6.0 * B * L + C * L2) / (2.0 * L3 * L2);
}

void launch_tab_build(const dp_model* m, hipStream_t s) {
  const TabGrid& g = m->tab_grid;
  const int nnets = m->desc.ntypes * m->desc.ntypes;
  hipLaunchKernelGGL(k_tab_nodes, dim3((unsigned)(g.nint + 1), (unsigned)nnets), dim3(128), 0, s,
                     (const double*)m->params, g, m->desc.ntypes, m->w1, m->tab_off, m->tab_nodes);
  const int64_t total = (int64_t)nnets * g.nint * m->m1;
  hipLaunchKernelGGL(k_tab_coef, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const double*)m->tab_nodes,
                     g, m->m1, nnets, m->table);
}

// ------------------------------------------------------------ evaluation
// Interval and offset of input x (the same operations as the checking
// implementation: IEEE division and floor pick the interval, one fused
// multiply-add gives t).
__device__ __forceinline__ int tab_interval(const TabGrid& g, double x, double& t, bool& clip) {
  clip = false;
  if (x < g.X1) {
    int k = (int)floor(x / g.h);
    k = k >= g.n1 ? g.n1 - 1 : (k < 0 ? 0 : k);
    t = fma(-(double)k, g.h, x);
    return k;
  }
  if (x < g.X2) {
    int m = (int)floor((x - g.X1) / g.H);
    m = m >= g.n2 ? g.n2 - 1 : m;
    t = fma(-(double)m, g.H, x - g.X1);
    return g.n1 + m;
  }
  clip = true;
  t = g.n2 > 0 ? g.H : g.h;
  return g.nint - 1;
}

struct TabArgs {
  const int32_t* atom_at;
  const int32_t* meta;
  const double* R;
  const int32_t* nnei;
  const double* table;
  TabGrid g;
  double* Tpart;          // forward: [ntypes][cols][m1][4]
  int64_t tpart_stride;
  const double* gT;       // backward: [cols][m1][4]
  double* netd;
  int ntypes, nm;
  int sec[kMaxT + 1];
  double inv_nm;
  int32_t* ctr;
  int32_t* flags;
};

// Work layout: one wavefront per centre atom and neighbour section (columns
// of the net taken from a per-work-group counter as in the MLP kernels);
// lanes 16 r + f work on row r of a group of four rows and on features
// f, f + 16, ... (NF = m1 / 16 rounded up per lane), so a coefficient load
// of 16 lanes is 128 contiguous bytes and every row's sums over features
// reduce over 16 lanes.
#define DPSE_TAB_PROLOGUE                                                  \
  int grp = 0, ngrp = 1;                                                  \
  const int net = net_of_group(A.meta, A.sec, A.ntypes, gridDim.x, blockIdx.x, &grp, &ngrp); \
  if (net < 0) return;                                                    \
  const int ti = net / A.ntypes, tj = net - ti * A.ntypes;                \
  const int n_t = A.meta[2 * ti], cb = A.meta[2 * ti + 1];                \
  const int c_lo = (int)((int64_t)n_t * grp / ngrp);                      \
  const int c_hi = (int)((int64_t)n_t * (grp + 1) / ngrp);                \
  if (c_lo >= c_hi) return;                                               \
  const int lane = threadIdx.x & 63;                                      \
  const int fl = lane & 15, rg = lane >> 4;                               \
  int* const next_col = A.ctr + blockIdx.x * 32;                          \
  if (threadIdx.x == 0) atomicExch(next_col, c_lo);                       \
  __syncthreads();                                                        \
  auto take = [&]() {                                                     \
    int k = 0;                                                            \
    if (lane == 0) k = atomicAdd(next_col, 1);                            \
    return k;                                                             \
  };                                                                      \
  const double* tabnet = A.table + (int64_t)net * A.g.nint * 6 * M1;

template <int M1>
__global__ __launch_bounds__(256) void k_embed_fwd_tab(TabArgs A) {
  constexpr int NF = (M1 + 15) / 16;
  DPSE_TAB_PROLOGUE
  bool clipped = false;
  for (int c_next = take();;) {
    const int c = __builtin_amdgcn_readfirstlane(__shfl(c_next, 0, 64));
    if (c >= c_hi) break;
    c_next = take();
    const int col = cb + c;
    const int i = A.atom_at[col];
    const int nn = A.nnei[i * kMaxT + tj];
    const double* Rs = A.R + ((int64_t)i * A.nm + A.sec[tj]) * 4;
    double acc[NF][4];
#pragma unroll
    for (int u = 0; u < NF; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[u][k] = 0.0;
    const env_rsrc_t Rb = env_rsrc(Rs, nn);
    d4 Rn = env_row(Rb, rg);
    for (int r0 = 0; r0 < nn; r0 += 4) {
      const int row = r0 + rg;
      const d4 Rv = Rn;  // zero past the section's real rows
      Rn = env_row(Rb, row + 4);
      double t;
      bool cl;
      const int k = tab_interval(A.g, Rv[0], t, cl);
      clipped |= cl && row < nn;
      const double* cf = tabnet + (int64_t)k * 6 * M1 + fl;
#pragma unroll
      for (int u = 0; u < NF; ++u) {
        if (M1 % 16 != 0 && fl + 16 * u >= M1) break;
        const double* cu = cf + 16 * u;
        double G = cu[5 * M1];
        G = fma(G, t, cu[4 * M1]);
        G = fma(G, t, cu[3 * M1]);
        G = fma(G, t, cu[2 * M1]);
        G = fma(G, t, cu[M1]);
        G = fma(G, t, cu[0]);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[u][q] = fma(G, Rv[q], acc[u][q]);
      }
    }
    // sum the four row groups; lanes of row group 0 write T (scaled 1/nm)
    double* T = A.Tpart + tj * A.tpart_stride + (int64_t)col * M1 * 4;
#pragma unroll
    for (int u = 0; u < NF; ++u) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double v = acc[u][q];
        v += shfl_xor_d(v, 16);
        v += shfl_xor_d(v, 32);
        acc[u][q] = v * A.inv_nm;
      }
      const int a = fl + 16 * u;
      if (rg == 0 && a < M1) *reinterpret_cast<d4*>(T + a * 4) = d4{acc[u][0], acc[u][1], acc[u][2], acc[u][3]};
    }
  }
  if (__ballot(clipped) && lane == 0) set_flag(A.flags, DP_FLAG_TABLE_RANGE);
}

// Backward: per row, dE/dG_a = g_T[a] . R~ / nm, the direct term
// dE/dR~ = sum_a g_T[a] G_a / nm and dE/dx = sum_a dE/dG_a dG_a/dx.
template <int M1>
__global__ __launch_bounds__(256) void k_embed_bwd_tab(TabArgs A) {
  constexpr int NF = (M1 + 15) / 16;
  DPSE_TAB_PROLOGUE
  for (int c_next = take();;) {
    const int c = __builtin_amdgcn_readfirstlane(__shfl(c_next, 0, 64));
    if (c >= c_hi) break;
    c_next = take();
    const int col = cb + c;
    const int i = A.atom_at[col];
    const int nn = A.nnei[i * kMaxT + tj];
    const int64_t rbase = (int64_t)i * A.nm + A.sec[tj];
    const double* Rs = A.R + rbase * 4;
    double gt[NF][4];
    const double* gcol = A.gT + (int64_t)col * M1 * 4;
#pragma unroll
    for (int u = 0; u < NF; ++u) {
      const int a = fl + 16 * u;
      d4 v = {0.0, 0.0, 0.0, 0.0};
      if (a < M1) v = *reinterpret_cast<const d4*>(gcol + a * 4);
#pragma unroll
      for (int q = 0; q < 4; ++q) gt[u][q] = v[q] * A.inv_nm;
    }
    const env_rsrc_t Rb = env_rsrc(Rs, nn);
    d4 Rn = env_row(Rb, rg);
    for (int r0 = 0; r0 < nn; r0 += 4) {
      const int row = r0 + rg;
      const d4 Rv = Rn;
      Rn = env_row(Rb, row + 4);
      double t;
      bool cl;
      const int k = tab_interval(A.g, Rv[0], t, cl);
      const double* cf = tabnet + (int64_t)k * 6 * M1 + fl;
      double ds = 0.0, dr[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < NF; ++u) {
        if (M1 % 16 != 0 && fl + 16 * u >= M1) break;
        const double* cu = cf + 16 * u;
        const double c5 = cu[5 * M1], c4 = cu[4 * M1], c3 = cu[3 * M1], c2 = cu[2 * M1], c1 = cu[M1], c0 = cu[0];
        double G = fma(fma(fma(fma(fma(c5, t, c4), t, c3), t, c2), t, c1), t, c0);
        double Gp = fma(fma(fma(fma(5.0 * c5, t, 4.0 * c4), t, 3.0 * c3), t, 2.0 * c2), t, c1);
        if (cl) Gp = 0.0;
        const double dG = fma(gt[u][0], Rv[0], fma(gt[u][1], Rv[1], fma(gt[u][2], Rv[2], gt[u][3] * Rv[3])));
        ds = fma(dG, Gp, ds);
#pragma unroll
        for (int q = 0; q < 4; ++q) dr[q] = fma(gt[u][q], G, dr[q]);
      }
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) {
        ds += shfl_xor_d(ds, m);
#pragma unroll
        for (int q = 0; q < 4; ++q) dr[q] += shfl_xor_d(dr[q], m);
      }
      if (fl == 0 && row < nn)
        *reinterpret_cast<d4*>(A.netd + (rbase + row) * 4) = d4{dr[0] + ds, dr[1], dr[2], dr[3]};
    }
  }
}

void launch_embed_tab(dp_ctx* c, bool bwd, hipStream_t s) {
  const dp_model* m = c->model;
  if (c->natoms_last <= 0) return;
  TabArgs A;
  A.atom_at = c->atom_at;
  A.meta = c->type_meta;
  A.R = c->R;
  A.nnei = c->nnei;
  A.table = m->table;
  A.g = m->tab_grid;
  A.Tpart = (double*)c->Tpart;
  A.tpart_stride = c->max_cols * m->m1 * 4;
  A.gT = (const double*)c->gT;
  A.netd = c->netd;
  A.ntypes = m->desc.ntypes;
  A.nm = m->nm;
  for (int t = 0; t <= kMaxT; ++t) A.sec[t] = t <= m->desc.ntypes ? m->sec[t] : m->nm;
  A.inv_nm = 1.0 / (double)m->nm;
  A.ctr = c->emb_ctr;
  A.flags = c->flags_dev;
  // 4-wave work-groups, three per CU, on one grid row shared out among the
  // nets by their work (net_of_group), all resident at once
  const int nnets = A.ntypes * A.ntypes;
  const int64_t need = (c->natoms_last * A.ntypes + 3) / 4, res = (int64_t)c->ncu * 3;
  const int64_t groups = need < res ? need : res;
  dim3 grid((unsigned)(groups > nnets ? groups : nnets), 1);
  if (m->m1 == 100) {
    if (bwd) hipLaunchKernelGGL(k_embed_bwd_tab<100>, grid, dim3(256), 0, s, A);
    else hipLaunchKernelGGL(k_embed_fwd_tab<100>, grid, dim3(256), 0, s, A);
  } else {
    if (bwd) hipLaunchKernelGGL(k_embed_bwd_tab<128>, grid, dim3(256), 0, s, A);
    else hipLaunchKernelGGL(k_embed_fwd_tab<128>, grid, dim3(256), 0, s, A);
  }
}

}  // namespace dpse
