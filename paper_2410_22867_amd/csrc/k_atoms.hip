// Per-atom kernels: type bucketing of centre atoms, environment matrix,
// force/virial scatter, per-frame reductions, velocity-Verlet halves.
//
// Environment matrix and forces follow the Background section (Fig. 1): the
// smoothed first column s(r) of R_i, and forces by back-propagation of the
// atomic energies.  The switching function is the quintic C2 switch of the
// DP se_a papers cited there:
//   u = (r - rs)/(rc - rs);  s = 1/r (r < rs);
//   s = (u^3(-6u^2 + 15u - 10) + 1)/r (rs <= r < rc);  s = 0 (r >= rc),
// and R_ij = [s/std_s, s x/(r std_v), s y/(r std_v), s z/(r std_v)].
#include "dp_internal.h"
#include "dp_device.h"

namespace dpse {

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_set_frame(FrameInfo* dst, FrameInfo F, int32_t* flags) {
  if (threadIdx.x == 0) {
    *dst = F;
    *flags = 0;
  }
}
__global__ void k_copy_i32(const int32_t* a, int32_t* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}
template <int KIND>
__global__ void k_param_gather(const double* __restrict__ P, const int32_t* __restrict__ idx, int64_t n, void* dst) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t q = idx[k];
    const double v = q >= 0 ? P[q] : 0.0;
    if (KIND == 0) reinterpret_cast<double*>(dst)[k] = v;
    else if (KIND == 1) reinterpret_cast<float*>(dst)[k] = (float)v;
    else if (KIND == 2) reinterpret_cast<__bf16*>(dst)[k] = (__bf16)(float)v;
    else reinterpret_cast<_Float16*>(dst)[k] = (_Float16)(float)v;
  }
}
void launch_param_gather(const double* P, const int32_t* idx, int64_t n, int kind, void* dst, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  if (kind == 0) hipLaunchKernelGGL(k_param_gather<0>, dim3(g), dim3(256), 0, s, P, idx, n, dst);
  else if (kind == 1) hipLaunchKernelGGL(k_param_gather<1>, dim3(g), dim3(256), 0, s, P, idx, n, dst);
  else if (kind == 2) hipLaunchKernelGGL(k_param_gather<2>, dim3(g), dim3(256), 0, s, P, idx, n, dst);
  else hipLaunchKernelGGL(k_param_gather<3>, dim3(g), dim3(256), 0, s, P, idx, n, dst);
}
void launch_set_frame(FrameInfo* dst, const FrameInfo& F, int32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_set_frame, dim3(1), dim3(64), 0, s, dst, F, flags);
}
void launch_copy_i32(const int32_t* a, int32_t* b, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
}
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
}
void launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
}

__device__ __forceinline__ int frame_lookup(const FrameInfo* fr, int nframes, int i) {
  int lo = 0, hi = nframes - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (fr[mid].atom_off <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- type sort
// Centre atoms are bucketed by type (Computation Optimization section: the
// environment matrix is pre-classified by atom type) into column segments of
// the fitting GEMMs: segment t holds the atoms of type t in atom order and is
// padded to a multiple of kColPad columns.
constexpr int kChunk = 1024;

__device__ __forceinline__ int clamp_type(int t, int ntypes, int32_t* flags) {
  if (t < 0 || t >= ntypes) {
    set_flag(flags, DP_FLAG_BAD_INPUT);
    t = t < 0 ? 0 : ntypes - 1;
  }
  return t;
}

__global__ __launch_bounds__(1024) void k_type_count(const int32_t* __restrict__ types, int ntot, int ntypes,
                                                     int32_t* __restrict__ chunk_counts, int32_t* flags) {
  __shared__ int32_t cnt[kMaxT];
  if (threadIdx.x < kMaxT) cnt[threadIdx.x] = 0;
  __syncthreads();
  int i = blockIdx.x * kChunk + threadIdx.x;
  if (i < ntot) atomicAdd(&cnt[clamp_type(types[i], ntypes, flags)], 1);
  __syncthreads();
  if (threadIdx.x < kMaxT) chunk_counts[blockIdx.x * kMaxT + threadIdx.x] = cnt[threadIdx.x];
}

// One thread per type: turns per-chunk counts into per-chunk offsets and
// writes n_t and the segment bases.
__global__ void k_type_scan(int32_t* __restrict__ chunk_counts, int nchunks, int ntypes,
                            int32_t* __restrict__ meta) {
  __shared__ int32_t tot[kMaxT];
  int t = threadIdx.x;
  if (t < kMaxT) {
    int acc = 0;
    if (t < ntypes)
      for (int c = 0; c < nchunks; ++c) {
        int v = chunk_counts[c * kMaxT + t];
        chunk_counts[c * kMaxT + t] = acc;
        acc += v;
      }
    tot[t] = acc;
  }
  __syncthreads();
  if (t == 0) {
    int base = 0;
    for (int u = 0; u < kMaxT; ++u) {
      meta[2 * u] = tot[u];
      meta[2 * u + 1] = base;
      base += ((tot[u] + kColPad - 1) / kColPad) * kColPad;
    }
  }
}

__global__ __launch_bounds__(1024) void k_type_assign(const int32_t* __restrict__ types, int ntot, int ntypes,
                                                      const int32_t* __restrict__ chunk_off,
                                                      const int32_t* __restrict__ meta,
                                                      const FrameInfo* __restrict__ fr, int nframes,
                                                      int32_t* __restrict__ col_of, int32_t* __restrict__ atom_at,
                                                      int32_t* __restrict__ frame_of) {
  __shared__ int32_t wave_cnt[16][kMaxT];
  const int i = blockIdx.x * kChunk + threadIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = i < ntot ? (types[i] < 0 ? 0 : (types[i] >= ntypes ? ntypes - 1 : types[i])) : -1;
  int before = 0;
  for (int u = 0; u < kMaxT; ++u) {
    uint64_t m = __ballot(t == u);
    if (t == u)
      before = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
    if (lane == 0) wave_cnt[w][u] = __popcll(m);
  }
  __syncthreads();
  if (t >= 0) {
    int off = 0;
    for (int ww = 0; ww < w; ++ww) off += wave_cnt[ww][t];
    const int col = meta[2 * t + 1] + chunk_off[blockIdx.x * kMaxT + t] + off + before;
    col_of[i] = col;
    atom_at[col] = i;
    frame_of[i] = frame_lookup(fr, nframes, i);
  }
}

void launch_type_sort(dp_ctx* c, const int32_t* types, int32_t ntot, int32_t nframes, hipStream_t s) {
  const int ntypes = c->model->desc.ntypes;
  const int nchunks = (ntot + kChunk - 1) / kChunk;
  launch_fill_i32(c->atom_at, -1, c->max_cols, s);
  if (ntot > 0)
    hipLaunchKernelGGL(k_type_count, dim3(nchunks), dim3(kChunk), 0, s, types, ntot, ntypes, c->chunk_counts,
                       c->flags_dev);
  hipLaunchKernelGGL(k_type_scan, dim3(1), dim3(64), 0, s, c->chunk_counts, nchunks, ntypes, c->type_meta);
  if (ntot > 0)
    hipLaunchKernelGGL(k_type_assign, dim3(nchunks), dim3(kChunk), 0, s, types, ntot, ntypes, c->chunk_counts,
                       c->type_meta, c->frames_dev, nframes, c->col_of, c->atom_at, c->frame_of);
}

// ---------------------------------------------------------------- env matrix
struct EnvArgs {
  const double* x;
  const int32_t* types;
  const int32_t* nlist;
  const int32_t* frame_of;
  const FrameInfo* fr;
  double* R;
  int32_t* nnei;
  int32_t* flags;
  double* F;  // forces, cleared here for the force pass (which accumulates)
  int ntot, nm, ntypes;
  int sec[kMaxT + 1];
  double rs, rc, inv_std_s, inv_std_v;
};

__device__ __forceinline__ void switch_fn(double r, double rs, double rc, double& s, double& ds) {
  if (r < rs) {
    s = 1.0 / r;
    ds = -1.0 / (r * r);
  } else if (r < rc) {
    const double w = rc - rs;
    const double u = (r - rs) / w;
    const double poly = u * u * u * (-6.0 * u * u + 15.0 * u - 10.0) + 1.0;
    const double dpoly = -30.0 * u * u * (1.0 - u) * (1.0 - u) / w;
    s = poly / r;
    ds = dpoly / r - poly / (r * r);
  } else {
    s = 0.0;
    ds = 0.0;
  }
}

// One wavefront per atom, lanes over neighbour slots.
__global__ __launch_bounds__(256) void k_env(EnvArgs A) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= A.ntot) return;
  const FrameInfo& F = A.fr[A.frame_of[i]];
  const double xi = A.x[3 * i], yi = A.x[3 * i + 1], zi = A.x[3 * i + 2];
  if (lane < 3) A.F[3 * i + lane] = 0.0;
  int cnt[kMaxT] = {0, 0, 0, 0};
  bool overlap = false;
  for (int q = lane; q < A.nm; q += 64) {
    const int e = A.nlist[(int64_t)i * A.nm + q];
    d4 out = {0.0, 0.0, 0.0, 0.0};
    if (e >= 0 && e / 27 >= A.ntot) set_flag(A.flags, DP_FLAG_BAD_INPUT);
    if (e >= 0 && e / 27 < A.ntot) {
      const int j = e / 27, sc = e - 27 * (e / 27);
      const double dx = (A.x[3 * j] - xi) + (double)(sc % 3 - 1) * F.L[0];
      const double dy = (A.x[3 * j + 1] - yi) + (double)((sc / 3) % 3 - 1) * F.L[1];
      const double dz = (A.x[3 * j + 2] - zi) + (double)(sc / 9 - 1) * F.L[2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (r == 0.0) overlap = true;
      double s, ds;
      switch_fn(r, A.rs, A.rc, s, ds);
      const double sv = s / r * A.inv_std_v;
      out[0] = s * A.inv_std_s;
      out[1] = sv * dx;
      out[2] = sv * dy;
      out[3] = sv * dz;
#pragma unroll
      for (int t = 0; t < kMaxT; ++t) cnt[t] += (q >= A.sec[t] && q < A.sec[t + 1]);
    }
    *reinterpret_cast<d4*>(A.R + ((int64_t)i * A.nm + q) * 4) = out;
  }
  for (int t = 0; t < A.ntypes; ++t) {
    int v = cnt[t];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0) A.nnei[i * kMaxT + t] = v;
  }
  if (overlap) set_flag(A.flags, DP_FLAG_OVERLAP);
}

void launch_env(dp_ctx* c, const double* x, const int32_t* types, const int32_t* nlist, int32_t ntot,
                double* forces, hipStream_t s) {
  if (ntot <= 0) return;
  const dp_model* m = c->model;
  EnvArgs A;
  A.x = x;
  A.types = types;
  A.nlist = nlist;
  A.frame_of = c->frame_of;
  A.fr = c->frames_dev;
  A.R = c->R;
  A.nnei = c->nnei;
  A.flags = c->flags_dev;
  A.F = forces;
  A.ntot = ntot;
  A.nm = m->nm;
  A.ntypes = m->desc.ntypes;
  for (int t = 0; t <= kMaxT; ++t) A.sec[t] = t <= m->desc.ntypes ? m->sec[t] : m->nm;
  A.rs = m->desc.rcut_smth;
  A.rc = m->desc.rcut;
  A.inv_std_s = 1.0 / m->desc.std_s;
  A.inv_std_v = 1.0 / m->desc.std_v;
  hipLaunchKernelGGL(k_env, dim3((ntot + 3) / 4), dim3(256), 0, s, A);
}

// ---------------------------------------------------------------- forces
// g_ij = sum_k n_ij[k] dR_ij[k]/dd (d = x_j + s L - x_i), one pass with
// one wavefront per atom i: for every own slot q, g_iq from n(i, q) adds to
// F_i and to the atom's virial row -sum d (x) g; for the reverse entry r of
// the slot ((i, -s) in j's list) the pair's g_ji is recomputed from n(r) and
// d_ji = -d_ij, which is bit-identical to j's own g at r (fl(a - b) =
// -fl(b - a) and the shift changes sign exactly), and subtracted from F_i.
// F_i is therefore summed in a fixed order with no g buffer in HBM.  A slot
// whose reverse entry is missing (j's section was truncated) subtracts g_iq
// from F_j with an atomic; the atom's own total is added atomically too, so
// the two never race (forces were cleared by the environment pass, and with
// a symmetric list each F_i receives exactly one addition).
struct ForceArgs {
  const double* x;
  const int32_t* nlist;
  const int32_t* rev;
  const int32_t* frame_of;
  const FrameInfo* fr;
  const double* netd;
  double* F;
  double* vatom;
  int ntot, nm;
  double rs, rc, inv_std_s, inv_std_v;
};

__device__ __forceinline__ void pair_g(const double d[3], const d4 n, const ForceArgs& A, double g[3]) {
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double s, ds;
  switch_fn(r, A.rs, A.rc, s, ds);
  const double ir = 1.0 / r;
  // dR0/dd_a = ds d_a / r (scaled); dRc/dd_a = ds d_a d_c / r^2 + s (delta_ca / r - d_c d_a / r^3)
  const double n0 = n[0] * A.inv_std_s;
  const double nv[3] = {n[1] * A.inv_std_v, n[2] * A.inv_std_v, n[3] * A.inv_std_v};
  const double ndot = nv[0] * d[0] + nv[1] * d[1] + nv[2] * d[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ua = d[a] * ir;
    g[a] = n0 * ds * ua + ndot * (ds * ua * ir) + s * (nv[a] * ir - ndot * ua * ir * ir);
  }
}

__global__ __launch_bounds__(256) void k_force(ForceArgs A) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= A.ntot) return;
  const FrameInfo& F = A.fr[A.frame_of[i]];
  const double xi = A.x[3 * i], yi = A.x[3 * i + 1], zi = A.x[3 * i + 2];
  double vir[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double f[3] = {0.0, 0.0, 0.0};
  for (int q = lane; q < A.nm; q += 64) {
    const int64_t slot = (int64_t)i * A.nm + q;
    const int e = A.nlist[slot];
    if (e < 0 || e / 27 >= A.ntot) continue;
    const int j = e / 27, sc = e - 27 * (e / 27);
    // the reverse entry is used only when it lies in j's row and holds
    // (i, -s) in the list passed in, so an index derived for another list
    // of the same size (a buffer rewritten in place) is never trusted.  Every
    // reverse index is built as an involution over the slots of one list
    // (rev[rev[q]] = q wherever rev[q] >= 0), so when this slot passes the
    // test, the entry at r points back here and passes it too: both slots of
    // a pair take the same path.
    int r = A.rev[slot];
    if (r >= 0 && ((unsigned)(r - j * A.nm) >= (unsigned)A.nm || A.nlist[r] != 27 * i + 26 - sc)) r = -1;
    const d4 n = *reinterpret_cast<const d4*>(A.netd + slot * 4);
    d4 nr = {0.0, 0.0, 0.0, 0.0};
    if (r >= 0) nr = *reinterpret_cast<const d4*>(A.netd + (int64_t)r * 4);
    const double d[3] = {(A.x[3 * j] - xi) + (double)(sc % 3 - 1) * F.L[0],
                         (A.x[3 * j + 1] - yi) + (double)((sc / 3) % 3 - 1) * F.L[1],
                         (A.x[3 * j + 2] - zi) + (double)(sc / 9 - 1) * F.L[2]};
    double g[3];
    pair_g(d, n, A, g);
    f[0] += g[0];
    f[1] += g[1];
    f[2] += g[2];
    if (r >= 0) {
      const double dm[3] = {-d[0], -d[1], -d[2]};
      double gb[3];
      pair_g(dm, nr, A, gb);
      f[0] -= gb[0];
      f[1] -= gb[1];
      f[2] -= gb[2];
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) atomicAdd(&A.F[3 * j + a], -g[a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) vir[3 * a + b] -= d[a] * g[b];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) vir[k] = wave_sum_d(vir[k]);
#pragma unroll
  for (int a = 0; a < 3; ++a) f[a] = wave_sum_d(f[a]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) A.vatom[(int64_t)i * 9 + k] = vir[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) atomicAdd(&A.F[3 * i + a], f[a]);
  }
}

void launch_force(dp_ctx* c, const double* x, const int32_t* nlist, int32_t ntot, double* forces, hipStream_t s) {
  if (ntot <= 0) return;
  const dp_model* m = c->model;
  ForceArgs A;
  A.x = x;
  A.nlist = nlist;
  A.rev = c->rev;
  A.frame_of = c->frame_of;
  A.fr = c->frames_dev;
  A.netd = c->netd;
  A.F = forces;
  A.vatom = c->vatom;
  A.ntot = ntot;
  A.nm = m->nm;
  A.rs = m->desc.rcut_smth;
  A.rc = m->desc.rcut;
  A.inv_std_s = 1.0 / m->desc.std_s;
  A.inv_std_v = 1.0 / m->desc.std_v;
  // forces were cleared by the environment pass of the same compute
  hipLaunchKernelGGL(k_force, dim3((ntot + 3) / 4), dim3(256), 0, s, A);
}

// ---------------------------------------------------------------- reductions
// Per-frame E_f = sum of E_i and W_f = sum of per-atom virial rows in two
// fixed-order stages (deterministic): one block per chunk of kRedChunk atoms
// of a frame (one atom per thread, wave shuffle trees, the four waves in
// order), then the frame's chunks (lane l of one wave adds chunks l, l + 64,
// ..., then a shuffle tree).  With a counter array
// (no empty frame) the second stage is done by the frame's last chunk block
// to finish, which resets the frame's counter; otherwise by k_frame_reduce.
__global__ __launch_bounds__(256) void k_chunk_reduce(const FrameInfo* __restrict__ fr, int nframes,
                                                      const double* __restrict__ Ei, const double* __restrict__ vatom,
                                                      double* __restrict__ part, int32_t* __restrict__ ctr,
                                                      double* __restrict__ E, double* __restrict__ W,
                                                      int32_t* __restrict__ flags) {
  static_assert(kRedChunk == 256, "one atom per thread");
  __shared__ double red[4][10];
  __shared__ bool last;
  const int b = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int lo = 0, hi = nframes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fr[mid].chunk_off <= b) lo = mid; else hi = mid - 1;
  }
  const FrameInfo F = fr[lo];
  const int a0 = F.atom_off + (b - F.chunk_off) * kRedChunk;
  const int a1 = min(F.atom_off + F.natoms, a0 + kRedChunk);
  const int k = a0 + (int)threadIdx.x;
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (k < a1) {
    acc[0] = Ei[k];
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[1 + c] = vatom[(int64_t)k * 9 + c];
  }
  // wave sums (a fixed shuffle tree), then the four waves in order
#pragma unroll
  for (int c = 0; c < 10; ++c) acc[c] = wave_sum_d(acc[c]);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 10; ++c) red[wv][c] = acc[c];
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    part[(int64_t)b * 10 + threadIdx.x] =
        ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    if (ctr != nullptr) __threadfence();
  }
  if (ctr == nullptr) return;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nc = (F.natoms + kRedChunk - 1) / kRedChunk;
    last = atomicAdd(ctr + lo, 1) == nc - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  // the frame's chunks: lane l of the first wave sums chunks l, l + 64, ...
  // (a fixed order), then a shuffle tree
  if (wv == 0) {
    const int nc = (F.natoms + kRedChunk - 1) / kRedChunk;
    double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = lane; c < nc; c += 64)
#pragma unroll
      for (int q = 0; q < 10; ++q) s[q] += part[(int64_t)(F.chunk_off + c) * 10 + q];
#pragma unroll
    for (int q = 0; q < 10; ++q) s[q] = wave_sum_d(s[q]);
    if (lane == 0) {
      E[lo] = s[0];
      if (!isfinite(s[0])) set_flag(flags, DP_FLAG_NONFINITE);
      ctr[lo] = 0;
#pragma unroll
      for (int q = 0; q < 9; ++q) W[9 * lo + q] = s[1 + q];
    }
  }
}

__global__ __launch_bounds__(64) void k_frame_reduce(const FrameInfo* __restrict__ fr, const double* __restrict__ part,
                                                     double* __restrict__ E, double* __restrict__ W, int32_t* flags) {
  // the same order as the last chunk block's sum in k_chunk_reduce
  const int f = blockIdx.x, lane = threadIdx.x;
  const int c0 = fr[f].chunk_off, nc = (fr[f].natoms + kRedChunk - 1) / kRedChunk;
  double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = lane; c < nc; c += 64)
#pragma unroll
    for (int q = 0; q < 10; ++q) s[q] += part[(int64_t)(c0 + c) * 10 + q];
#pragma unroll
  for (int q = 0; q < 10; ++q) s[q] = wave_sum_d(s[q]);
  if (lane == 0) {
    E[f] = s[0];
    if (!isfinite(s[0])) set_flag(flags, DP_FLAG_NONFINITE);
#pragma unroll
    for (int q = 0; q < 9; ++q) W[9 * f + q] = s[1 + q];
  }
}

__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

void launch_frame_reduce(dp_ctx* c, int32_t nframes, double* energies, double* atom_energy, double* virials,
                         hipStream_t s) {
  bool empty = false;  // host copy of the table the kernels read
  for (int f = 0; f < nframes; ++f) empty |= c->frames_prev[f].natoms == 0;
  if (c->nchunks_last > 0)
    hipLaunchKernelGGL(k_chunk_reduce, dim3(c->nchunks_last), dim3(256), 0, s, c->frames_dev, nframes, c->Ei_atom,
                       c->vatom, c->red_part, empty ? nullptr : c->frame_ctr, energies, virials, c->flags_dev);
  if (empty || c->nchunks_last == 0)
    hipLaunchKernelGGL(k_frame_reduce, dim3(nframes), dim3(64), 0, s, c->frames_dev, c->red_part, energies, virials,
                       c->flags_dev);
  if (atom_energy && c->natoms_last > 0)
    hipLaunchKernelGGL(k_copy_f64, dim3((c->natoms_last + 255) / 256), dim3(256), 0, s, c->Ei_atom, atom_energy,
                       (int)c->natoms_last);
}

// ---------------------------------------------------------------- integrator
// Velocity Verlet in metal units: a = F/m * 9.64853321e-3 A/fs^2.
constexpr double kFtm2v = 9.64853321e-3;

struct MdArgs {
  double* x;
  double* v;
  const double* f;
  const int32_t* types;
  int32_t* images;
  double* ke;
  int n;
  int wrap;
  double dt;
  double L[3];
  double mass[kMaxT];
};

__global__ void k_kick_drift(MdArgs A) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const double inv_m = kFtm2v / A.mass[A.types[i]];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v = A.v[3 * i + a] + 0.5 * A.dt * A.f[3 * i + a] * inv_m;
    A.v[3 * i + a] = v;
    double x = A.x[3 * i + a] + A.dt * v;
    if (A.wrap) {
      const double L = A.L[a];
      int im = 0;
      if (x >= L) { x -= L; im = 1; }
      else if (x < 0.0) { x += L; im = -1; if (x >= L) x -= L; }
      if (A.images) A.images[3 * i + a] += im;
    }
    A.x[3 * i + a] = x;
  }
}

// Wraps positions into [0, L) by whole box lengths (any distance), counting
// the lengths moved in the image counters.
__global__ void k_wrap(MdArgs A) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double x = A.x[3 * i + a];
    const double L = A.L[a];
    if (x >= 0.0 && x < L) continue;
    const double k = floor(x / L);
    x -= k * L;
    if (x >= L) x -= L;  // rounding of x - k L
    if (x < 0.0) x += L;
    if (x >= L) x = 0.0;
    A.x[3 * i + a] = x;
    if (A.images) A.images[3 * i + a] += (int32_t)k;
  }
}

// Second half-kick; each block writes its partial kinetic energy, a second
// single-block kernel sums the partials in a fixed order.
// Second half-kick and kinetic energy: each block writes its partial sum;
// the block that finishes last (counted by an atomic that it resets) adds
// the partials in block order.
__global__ __launch_bounds__(256) void k_kick(MdArgs A, double* __restrict__ part, int32_t* __restrict__ ctr,
                                              double scale) {
  // block and grid sums in a fixed order: wave shuffle trees, the four
  // waves in order, then the blocks' partials lane-strided in the last block
  __shared__ double red[4];
  __shared__ bool last;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc = 0.0;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < A.n) {
    const double m = A.mass[A.types[i]];
    const double h = 0.5 * A.dt * kFtm2v / m;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double v = A.v[3 * i + a] + h * A.f[3 * i + a];
      A.v[3 * i + a] = v;
      acc += 0.5 * m * v * v;
    }
  }
  acc = wave_sum_d(acc);
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
    __threadfence();
    last = atomicAdd(ctr, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!last || wv != 0) return;
  __threadfence();
  const int nb = (int)gridDim.x;
  double a2 = 0.0;
  for (int k = lane; k < nb; k += 64) a2 += part[k];
  a2 = wave_sum_d(a2);
  if (lane == 0) {
    A.ke[0] = a2 * scale;
    *ctr = 0;
  }
}

__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int n, double scale,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) acc += part[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

static MdArgs md_args(dp_ctx* c, double* x, double* v, const double* f, const int32_t* types, int32_t n, double dt) {
  MdArgs A;
  A.x = x;
  A.v = v;
  A.f = f;
  A.types = types;
  A.images = nullptr;
  A.ke = nullptr;
  A.n = n;
  A.wrap = 0;
  A.dt = dt;
  for (int a = 0; a < 3; ++a) A.L[a] = 0;
  for (int t = 0; t < kMaxT; ++t) A.mass[t] = t < c->model->desc.ntypes ? c->model->desc.masses[t] : 1.0;
  return A;
}

void launch_kick_drift(dp_ctx* c, double* x, double* v, const double* f, const int32_t* types, int32_t n, double dt,
                       const double* L, int32_t* images, hipStream_t s) {
  if (n <= 0) return;
  MdArgs A = md_args(c, x, v, f, types, n, dt);
  A.wrap = L != nullptr;
  if (L)
    for (int a = 0; a < 3; ++a) A.L[a] = L[a];
  A.images = images;
  hipLaunchKernelGGL(k_kick_drift, dim3((n + 255) / 256), dim3(256), 0, s, A);
}

void launch_wrap(dp_ctx* c, double* x, int32_t n, const double L[3], int32_t* images, hipStream_t s) {
  if (n <= 0) return;
  MdArgs A = md_args(c, x, nullptr, nullptr, nullptr, n, 0.0);
  for (int a = 0; a < 3; ++a) A.L[a] = L[a];
  A.images = images;
  hipLaunchKernelGGL(k_wrap, dim3((n + 255) / 256), dim3(256), 0, s, A);
}

void launch_kick(dp_ctx* c, double* v, const double* f, const int32_t* types, int32_t n, double dt, double* ke,
                 hipStream_t s) {
  MdArgs A = md_args(c, nullptr, v, f, types, n, dt);
  A.ke = ke;
  const int nb = (n + 255) / 256;
  if (nb > 0) hipLaunchKernelGGL(k_kick, dim3(nb), dim3(256), 0, s, A, c->ke_part, c->ke_ctr, 1.0 / kFtm2v);
  else hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, c->ke_part, 0, 1.0 / kFtm2v, ke);
}

}  // namespace dpse
