// Neighbour list (Background section, Fig. 1(a); Evaluation section:
// per-type neighbour counts sel): cell binning + 27-cell stencil search +
// per-type sorted, truncated, -1-padded sections.
//
// Work layout: binning is one thread per atom (counting sort by cell with
// global atomics); the search is one wavefront per centre atom: lanes walk
// the atoms of each stencil cell 64 at a time, survivors of r^2 < rc^2 are
// appended to a wave-private LDS candidate list with ballot/prefix counts,
// then every candidate's rank within its type section is counted against all
// candidates (a deterministic total order on (r^2, packed)), so the written
// list does not depend on the nondeterministic order of binning.
#include "dp_internal.h"
#include "dp_device.h"

// Every floating-point operation of this file is rounded on its own (no fused
// multiply-add): the cut-off test and the sort key must reproduce the plain
// expression bit for bit.
#pragma clang fp contract(off)

namespace dpse {

// r^2 = (dx*dx + dy*dy) + dz*dz, each operation rounded separately.
__device__ __forceinline__ double r2_nofma(double dx, double dy, double dz) {
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ int find_frame(const FrameInfo* fr, int nframes, int i) {
  int lo = 0, hi = nframes - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (fr[mid].atom_off <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int cell_coord(double x, double L, int nc) {
  int k = (int)floor(x / L * (double)nc);
  return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

__global__ void k_nl_bin(const double* __restrict__ x, const FrameInfo* __restrict__ fr, int nframes, int ntot,
                         int32_t* __restrict__ cell_of, int32_t* __restrict__ cell_count, int32_t* flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  int f = find_frame(fr, nframes, i);
  const FrameInfo F = fr[f];
  int c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double xa = x[3 * i + a];
    if (!(xa >= 0.0 && xa < F.L[a])) set_flag(flags, DP_FLAG_NOT_WRAPPED);
    c[a] = cell_coord(xa, F.L[a], F.ncell[a]);
  }
  int cid = F.cell_off + c[0] + F.ncell[0] * (c[1] + F.ncell[1] * c[2]);
  cell_of[i] = cid;
  atomicAdd(&cell_count[cid], 1);
}

// Exclusive scan of cell counts with one work-group (cells number in the
// thousands); also clears the fill counters.
__global__ __launch_bounds__(1024) void k_nl_scan(const int32_t* __restrict__ count, int32_t* __restrict__ start,
                                                  int32_t* __restrict__ fill, int ncells) {
  __shared__ int32_t part[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ncells; base += 1024) {
    int k = base + threadIdx.x;
    int v = k < ncells ? count[k] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (k < ncells) {
      start[k] = carry + part[threadIdx.x] - v;
      fill[k] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 1023) carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) start[ncells] = carry;
}

__global__ void k_nl_scatter(const int32_t* __restrict__ cell_of, const int32_t* __restrict__ start,
                             int32_t* __restrict__ fill, int32_t* __restrict__ cell_atoms, int ntot) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  int c = cell_of[i];
  int p = atomicAdd(&fill[c], 1);
  cell_atoms[start[c] + p] = i;
}

struct SearchArgs {
  const double* x;
  const int32_t* types;
  const FrameInfo* fr;
  const int32_t* cell_start;
  const int32_t* cell_atoms;
  int32_t* nlist;
  int32_t* overflow;
  int32_t* flags;
  int nframes, ntot, ntypes, nm;
  int sel[kMaxT];
  int sec[kMaxT + 1];
  double rc2;
};

constexpr int kSearchWaves = 4;

__global__ __launch_bounds__(256) void k_nl_search(SearchArgs A) {
  __shared__ double cr2[kSearchWaves][kCandCap];
  __shared__ int32_t cpk[kSearchWaves][kCandCap];
  __shared__ int8_t ctp[kSearchWaves][kCandCap];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * kSearchWaves + w;
  if (i >= A.ntot) return;
  const int f = find_frame(A.fr, A.nframes, i);
  const FrameInfo F = A.fr[f];
  const double xi = A.x[3 * i], yi = A.x[3 * i + 1], zi = A.x[3 * i + 2];
  const int ci[3] = {cell_coord(xi, F.L[0], F.ncell[0]), cell_coord(yi, F.L[1], F.ncell[1]),
                     cell_coord(zi, F.L[2], F.ncell[2])};
  int ncand = 0;
  bool capacity = false;
  // Lane c < 27 describes stencil cell c (dx, dy, dz in {-1,0,1}): first
  // atom, atom count and image code; a wave prefix sum over the counts turns
  // the 27 cell loops into one flat loop over all candidates.
  int c_start = 0, c_cnt = 0, c_code = 13;
  if (lane < 27) {
    const int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
    int cc[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
    int sh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sh[a] = 0;
      if (cc[a] < 0) { cc[a] += F.ncell[a]; sh[a] = -1; }
      else if (cc[a] >= F.ncell[a]) { cc[a] -= F.ncell[a]; sh[a] = 1; }
    }
    const int cid = F.cell_off + cc[0] + F.ncell[0] * (cc[1] + F.ncell[1] * cc[2]);
    c_start = A.cell_start[cid];
    c_cnt = A.cell_start[cid + 1] - c_start;
    c_code = (sh[0] + 1) + 3 * (sh[1] + 1) + 9 * (sh[2] + 1);
  }
  int c_end = c_cnt;  // inclusive prefix sum
#pragma unroll
  for (int off = 1; off < 32; off <<= 1) {
    const int y = __shfl_up(c_end, off, 64);
    if (lane >= off) c_end += y;
  }
  const int total = __shfl(c_end, 26, 64);
  for (int t0 = 0; t0 < total; t0 += 64) {
    const int t = t0 + lane;
    // cell holding flat index t (all lanes run the lookup and the shuffles)
    const int tt = t < total ? t : total - 1;
    int c = 0;
#pragma unroll
    for (int step = 16; step >= 1; step >>= 1) {
      const int probe = c + step - 1;
      const int e = __shfl(c_end, probe < 27 ? probe : 26, 64);
      if (probe < 27 && e <= tt) c += step;
    }
    const int cstart = __shfl(c_start, c, 64);
    const int cbeg = __shfl(c_end - c_cnt, c, 64);
    const int scode = __shfl(c_code, c, 64);
    bool keep = false;
    double r2 = 0.0;
    int j = -1;
    if (t < total) {
      j = A.cell_atoms[cstart + (t - cbeg)];
      if (!(scode == 13 && j == i)) {
        const double shx = (double)(scode % 3 - 1) * F.L[0];
        const double shy = (double)((scode / 3) % 3 - 1) * F.L[1];
        const double shz = (double)(scode / 9 - 1) * F.L[2];
        const double ddx = (A.x[3 * j] - xi) + shx;
        const double ddy = (A.x[3 * j + 1] - yi) + shy;
        const double ddz = (A.x[3 * j + 2] - zi) + shz;
        r2 = r2_nofma(ddx, ddy, ddz);
        keep = r2 < A.rc2;
      }
    }
    const uint64_t mask = __ballot(keep);
    const int before = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
    const int slot = ncand + before;
    if (keep && slot < kCandCap) {
      cr2[w][slot] = r2;
      cpk[w][slot] = 27 * j + scode;
      int tj = A.types[j];
      if (tj < 0 || tj >= A.ntypes) {
        set_flag(A.flags, DP_FLAG_BAD_INPUT);
        tj = tj < 0 ? 0 : A.ntypes - 1;
      }
      ctp[w][slot] = (int8_t)tj;
    }
    ncand += __popcll(mask);
  }
  if (ncand > kCandCap) {
    capacity = true;
    ncand = kCandCap;
  }
  wave_lds_sync();
  // rank of each candidate inside its type section
  int cnt[kMaxT] = {0, 0, 0, 0};
  int32_t* row = A.nlist + (int64_t)i * A.nm;
  for (int c = lane; c < ncand; c += 64) {
    const double r2 = cr2[w][c];
    const int pk = cpk[w][c];
    const int t = ctp[w][c];
    int rank = 0;
    for (int o = 0; o < ncand; ++o) {
      const double r2o = cr2[w][o];
      const int pko = cpk[w][o];
      rank += (ctp[w][o] == t) && (r2o < r2 || (r2o == r2 && pko < pk));
    }
    if (rank < A.sel[t]) row[A.sec[t] + rank] = pk;
#pragma unroll
    for (int u = 0; u < kMaxT; ++u) cnt[u] += (t == u);
  }
  int ovf = 0;
  for (int t = 0; t < A.ntypes; ++t) {
    int n_t = cnt[t];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) n_t += __shfl_xor(n_t, m, 64);
    const int kept = n_t < A.sel[t] ? n_t : A.sel[t];
    for (int q = kept + lane; q < A.sel[t]; q += 64) row[A.sec[t] + q] = -1;
    ovf += n_t - kept;
  }
  if (lane == 0) {
    if (ovf) {
      atomicAdd(A.overflow, ovf);
      set_flag(A.flags, DP_FLAG_SEL_OVERFLOW);
    }
    if (capacity) set_flag(A.flags, DP_FLAG_CAND_CAPACITY);
  }
}

// Reverse index of a symmetric list: for entry q' of atom i pointing to
// (j, s), the slot q of j's list holding (i, -s), stored as j*nm + q
// (-1 when j's section was truncated before i).  The key (r^2, packed) of
// the reverse entry is bit-identical (fl(a - b) = -fl(b - a) and the shift
// changes sign exactly), so a binary search over j's sorted section finds
// it; a pair missing from j's list is never matched to a wrong slot.
struct RevArgs {
  const double* x;
  const int32_t* types;
  const int32_t* nlist;
  const int32_t* frame_of;
  const FrameInfo* fr;
  int32_t* rev;
  int ntot, nm, ntypes;
  int sel[kMaxT];
  int sec[kMaxT + 1];
};

__device__ __forceinline__ double pair_r2(const double* x, int a, int e, const double* L) {
  const int b = e / 27, sc = e - 27 * (e / 27);
  const double dx = (x[3 * b] - x[3 * a]) + (double)(sc % 3 - 1) * L[0];
  const double dy = (x[3 * b + 1] - x[3 * a + 1]) + (double)((sc / 3) % 3 - 1) * L[1];
  const double dz = (x[3 * b + 2] - x[3 * a + 2]) + (double)(sc / 9 - 1) * L[2];
  return r2_nofma(dx, dy, dz);
}

__global__ __launch_bounds__(256) void k_nl_reverse(RevArgs A) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= A.ntot) return;
  int ti = A.types[i];
  ti = ti < 0 ? 0 : (ti >= A.ntypes ? A.ntypes - 1 : ti);
  const double* L = A.fr[A.frame_of[i]].L;
  for (int q = lane; q < A.nm; q += 64) {
    const int e = A.nlist[(int64_t)i * A.nm + q];
    int out = -1;
    if (e >= 0 && e / 27 < A.ntot) {
      const int j = e / 27;
      const int target = 27 * i + (26 - (e - 27 * j));
      const double r2 = pair_r2(A.x, i, e, L);
      const int32_t* row = A.nlist + (int64_t)j * A.nm + A.sec[ti];
      int lo = 0, hi = A.sel[ti];  // first position with key >= (r2, target)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int em = row[mid];
        bool less;
        if (em < 0 || em / 27 >= A.ntot) less = false;  // padding sorts last
        else {
          const double rm = pair_r2(A.x, j, em, L);
          less = rm < r2 || (rm == r2 && em < target);
        }
        if (less) lo = mid + 1; else hi = mid;
      }
      if (lo < A.sel[ti] && row[lo] == target) out = j * A.nm + A.sec[ti] + lo;
    }
    A.rev[(int64_t)i * A.nm + q] = out;
  }
}

void launch_nl_reverse(dp_ctx* c, const double* x, const int32_t* types, const int32_t* nlist, int32_t ntot,
                       hipStream_t s) {
  if (ntot <= 0) return;
  const dp_model* m = c->model;
  RevArgs A;
  A.x = x;
  A.types = types;
  A.nlist = nlist;
  A.frame_of = c->frame_of;
  A.fr = c->frames_dev;
  A.rev = c->rev;
  A.ntot = ntot;
  A.nm = m->nm;
  A.ntypes = m->desc.ntypes;
  for (int t = 0; t < kMaxT; ++t) A.sel[t] = t < m->desc.ntypes ? m->desc.sel[t] : 0;
  for (int t = 0; t <= kMaxT; ++t) A.sec[t] = t <= m->desc.ntypes ? m->sec[t] : m->nm;
  hipLaunchKernelGGL(k_nl_reverse, dim3((ntot + 3) / 4), dim3(256), 0, s, A);
}

void launch_nl_bin(dp_ctx* c, const double* x, int32_t ntot, int32_t nframes, hipStream_t s) {
  if (ntot <= 0) return;
  hipLaunchKernelGGL(k_nl_bin, dim3((ntot + 255) / 256), dim3(256), 0, s, x, c->frames_dev, nframes, ntot,
                     c->cell_of, c->cell_count, c->flags_dev);
}

void launch_nl_scan(dp_ctx* c, int32_t ncells, hipStream_t s) {
  hipLaunchKernelGGL(k_nl_scan, dim3(1), dim3(1024), 0, s, c->cell_count, c->cell_start, c->cell_fill, ncells);
}

void launch_nl_scatter(dp_ctx* c, int32_t ntot, hipStream_t s) {
  if (ntot <= 0) return;
  hipLaunchKernelGGL(k_nl_scatter, dim3((ntot + 255) / 256), dim3(256), 0, s, c->cell_of, c->cell_start,
                     c->cell_fill, c->cell_atoms, ntot);
}

void launch_nl_search(dp_ctx* c, const double* x, const int32_t* types, int32_t ntot, int32_t nframes,
                      int32_t* nlist, int32_t* overflow, hipStream_t s) {
  if (ntot <= 0) return;
  const dp_model* m = c->model;
  SearchArgs A;
  A.x = x;
  A.types = types;
  A.fr = c->frames_dev;
  A.cell_start = c->cell_start;
  A.cell_atoms = c->cell_atoms;
  A.nlist = nlist;
  A.overflow = overflow;
  A.flags = c->flags_dev;
  A.nframes = nframes;
  A.ntot = ntot;
  A.ntypes = m->desc.ntypes;
  A.nm = m->nm;
  for (int t = 0; t < kMaxT; ++t) A.sel[t] = t < m->desc.ntypes ? m->desc.sel[t] : 0;
  for (int t = 0; t <= kMaxT; ++t) A.sec[t] = t <= m->desc.ntypes ? m->sec[t] : m->nm;
  A.rc2 = m->desc.rcut * m->desc.rcut;
  hipLaunchKernelGGL(k_nl_search, dim3((ntot + kSearchWaves - 1) / kSearchWaves), dim3(64 * kSearchWaves), 0, s, A);
}

}  // namespace dpse
