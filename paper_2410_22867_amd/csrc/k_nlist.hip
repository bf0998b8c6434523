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

// With xw != NULL (a Verlet build) the positions are first wrapped into
// [0, L) in place by whole box lengths, the lengths moved being added to the
// image counters (when non-NULL).  gate: see launch_nl_skin_update.
__global__ void k_nl_bin(const double* __restrict__ x, const FrameInfo* __restrict__ fr, int nframes, int ntot,
                         int32_t* __restrict__ cell_of, int32_t* __restrict__ cell_count, int32_t* flags,
                         double* xw, int32_t* images, const int32_t* gate) {
  if (gate && *gate == 0) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntot) return;
  int f = find_frame(fr, nframes, i);
  const FrameInfo F = fr[f];
  int c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double xa = x[3 * i + a];
    if (xw && !(xa >= 0.0 && xa < F.L[a])) {
      const double L = F.L[a];
      const double k = floor(xa / L);
      xa -= k * L;
      if (xa >= L) xa -= L;  // rounding of x - k L
      if (xa < 0.0) xa += L;
      if (xa >= L) xa = 0.0;
      xw[3 * i + a] = xa;
      if (images) images[3 * i + a] += (int32_t)k;
    }
    if (!(xa >= 0.0 && xa < F.L[a])) set_flag(flags, DP_FLAG_NOT_WRAPPED);
    c[a] = cell_coord(xa, F.L[a], F.ncell[a]);
  }
  int cid = F.cell_off + c[0] + F.ncell[0] * (c[1] + F.ncell[1] * c[2]);
  cell_of[i] = cid;
  atomicAdd(&cell_count[cid], 1);
}

// Exclusive scan of cell counts with one work-group (cells number in the
// thousands); also clears the fill counters, and the counts once read, so
// that the next binning starts from zero.
__global__ __launch_bounds__(1024) void k_nl_scan(int32_t* __restrict__ count, int32_t* __restrict__ start,
                                                  int32_t* __restrict__ fill, int ncells, const int32_t* gate) {
  if (gate && *gate == 0) return;
  __shared__ int32_t part[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ncells; base += 1024) {
    int k = base + threadIdx.x;
    int v = k < ncells ? count[k] : 0;
    if (k < ncells) count[k] = 0;
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
                             int32_t* __restrict__ fill, int32_t* __restrict__ cell_atoms, int ntot,
                             const int32_t* gate) {
  if (gate && *gate == 0) return;
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

// Wave-private candidate buffers in LDS: one 16-byte record per candidate.
struct CandRec {
  double r2;
  int32_t pk;
  int16_t k;  // position in the Verlet candidate list (format only)
  int8_t t;
  int8_t pad;
};
// CAP records per wave: kCandCap for the Verlet build (every pair within
// r_c + skin); for the search and the format, which keep pairs within r_c
// only, 256 when the sections hold at most 256 neighbours (half the LDS,
// twice the resident work-groups), kCandCap otherwise.  More kept pairs
// than CAP raise DP_FLAG_CAND_CAPACITY.
constexpr int kKeepCapSmall = 256;
template <int CAP>
struct CandLds {
  CandRec r[kSearchWaves][CAP];
};

__device__ __forceinline__ int clamp_type(const int32_t* types, int j, int ntypes, int32_t* flags) {
  int tj = types[j];
  if (tj < 0 || tj >= ntypes) {
    set_flag(flags, DP_FLAG_BAD_INPUT);
    tj = tj < 0 ? 0 : ntypes - 1;
  }
  return tj;
}

// Walks the 27 stencil cells of atom i (one wavefront) and appends every
// (j, s) with r^2 < rad2 to the LDS buffers of wave w, in a fixed order.
// Returns the candidate count (capped at CAP; *capacity set beyond).
template <int CAP>
__device__ __forceinline__ int gather_cells(const SearchArgs& A, CandLds<CAP>& L, int w, int lane, int i, const FrameInfo& F, double rad2,
                            bool* capacity) {
  const double xi = A.x[3 * i], yi = A.x[3 * i + 1], zi = A.x[3 * i + 2];
  const int ci[3] = {cell_coord(xi, F.L[0], F.ncell[0]), cell_coord(yi, F.L[1], F.ncell[1]),
                     cell_coord(zi, F.L[2], F.ncell[2])};
  int ncand = 0;
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
        keep = r2 < rad2;
      }
    }
    const uint64_t mask = __ballot(keep);
    const int before = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
    const int slot = ncand + before;
    if (keep && slot < CAP) {
      CandRec rec;
      rec.r2 = r2;
      rec.pk = 27 * j + scode;
      rec.k = 0;
      rec.t = (int8_t)clamp_type(A.types, j, A.ntypes, A.flags);
      rec.pad = 0;
      L.r[w][slot] = rec;
    }
    ncand += __popcll(mask);
  }
  if (ncand > CAP) {
    *capacity = true;
    ncand = CAP;
  }
  return ncand;
}

// Ranks the ncand LDS candidates of wave w inside their type sections by
// (r^2, packed) -- a total order, so the result does not depend on the order
// of the buffer -- writes the first sel[t] of each section to row i of the
// list, pads with -1 and counts what was dropped.  The buffer is first
// regrouped by type (through registers), so each candidate is compared only
// with its own section.  With cof != NULL (Verlet format) it also records,
// per written slot, the candidate it came from and, per kept candidate, its
// slot (-1 when truncated).
template <int CAP>
__device__ __forceinline__ void rank_and_write(const SearchArgs& A, CandLds<CAP>& L, int w, int lane, int i, int ncand, bool capacity,
                               int32_t* cof, int32_t* slot_of) {
  constexpr int kPer = CAP / 64;
  // records move as 16-byte vectors (r^2 bits | packed | k, type)
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4* R = reinterpret_cast<u32x4*>(&L.r[w][0]);
  u32x4 mine[kPer];
  int pos[kPer], mt[kPer];
  int cnt[kMaxT] = {0, 0, 0, 0};
#pragma clang loop unroll(full)
  for (int m = 0; m < kPer; ++m) {
    pos[m] = -1;
    mt[m] = -1;
    if (m * 64 < ncand) {
      const int c = m * 64 + lane;
      if (c < ncand) {
        mine[m] = R[c];
        mt[m] = (int)((mine[m][3] >> 16) & 0xff);
      }
#pragma unroll
      for (int u = 0; u < kMaxT; ++u) {
        if (u < A.ntypes) {
          const uint64_t bal = __ballot(mt[m] == u);
          const int before = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
          if (mt[m] == u) pos[m] = cnt[u] + before;
          cnt[u] += __popcll(bal);
        }
      }
    }
  }
  int off[kMaxT];
  {
    int acc = 0;
#pragma unroll
    for (int u = 0; u < kMaxT; ++u) {
      off[u] = acc;
      acc += cnt[u];
    }
  }
  wave_lds_sync();
#pragma clang loop unroll(full)
  for (int m = 0; m < kPer; ++m)
    if (pos[m] >= 0) {
      int base = 0;  // off[t] without a dynamically indexed register array
#pragma unroll
      for (int u = 1; u < kMaxT; ++u) base = mt[m] == u ? off[u] : base;
      R[base + pos[m]] = mine[m];
    }
  wave_lds_sync();
  int32_t* row = A.nlist + (int64_t)i * A.nm;
  int ovf = 0;
#pragma unroll
  for (int u = 0; u < kMaxT; ++u) {
    if (u >= A.ntypes) break;
    const CandRec* sec = &L.r[w][off[u]];
    const int n_u = cnt[u];
    const int sel = A.sel[u];
    // Rank of each candidate in its section on (r^2, packed).  Exact ties in
    // r^2 are rare, so each candidate first counts the candidates whose r^2
    // is <= its own (one compare per pair).  Without ties these counts are
    // a permutation of 1..n_u; with T pairs of equal r^2 they sum to
    // n_u (n_u + 1) / 2 + T, so one wave sum tells whether the section
    // needs the full comparison with the packed-index tie-break.
    int rk[kPer];
    int sum = 0;
#pragma clang loop unroll(full)
    for (int m = 0; m < kPer; ++m) {
      rk[m] = 0;
      if (64 * m < n_u) {
        const int c = 64 * m + lane;
        if (c < n_u) {
          const double r2 = sec[c].r2;
          int le = 0;
#pragma unroll 4
          for (int o = 0; o < n_u; ++o) le += sec[o].r2 <= r2;
          rk[m] = le;
          sum += le;
        }
      }
    }
#pragma unroll
    for (int x = 32; x >= 1; x >>= 1) sum += __shfl_xor(sum, x, 64);
    const bool ties = sum != n_u * (n_u + 1) / 2;
#pragma clang loop unroll(full)
    for (int m = 0; m < kPer; ++m) {
      if (64 * m >= n_u) break;
      const int c = 64 * m + lane;
      if (c >= n_u) continue;
      const CandRec me = sec[c];
      int rank = rk[m] - 1;
      if (ties) {
        rank = 0;
        for (int o = 0; o < n_u; ++o) {
          const CandRec ot = sec[o];
          rank += (ot.r2 < me.r2 || (ot.r2 == me.r2 && ot.pk < me.pk));
        }
      }
      const bool kept = rank < sel;
      if (kept) row[A.sec[u] + rank] = me.pk;
      if (cof) {
        if (kept) cof[(int64_t)i * A.nm + A.sec[u] + rank] = me.k;
        slot_of[(int64_t)i * kCandCap + me.k] = kept ? i * A.nm + A.sec[u] + rank : -1;
      }
    }
    const int kept = n_u < sel ? n_u : sel;
    for (int q = kept + lane; q < sel; q += 64) row[A.sec[u] + q] = -1;
    ovf += n_u - kept;
  }
  if (lane == 0) {
    if (ovf) {
      atomicAdd(A.overflow, ovf);
      set_flag(A.flags, DP_FLAG_SEL_OVERFLOW);
    }
    if (capacity) set_flag(A.flags, DP_FLAG_CAND_CAPACITY);
  }
}

template <int CAP>
__global__ __launch_bounds__(256) void k_nl_search(SearchArgs A) {
  __shared__ CandLds<CAP> L;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * kSearchWaves + w;
  if (i >= A.ntot) return;
  const FrameInfo F = A.fr[find_frame(A.fr, A.nframes, i)];
  bool capacity = false;
  const int ncand = gather_cells(A, L, w, lane, i, F, A.rc2, &capacity);
  wave_lds_sync();
  rank_and_write(A, L, w, lane, i, ncand, capacity, nullptr, nullptr);
}

// ------------------------------------------------------------ Verlet list
// Build: every (j, s) with r^2 < (r_c + skin)^2 on the wrapped positions,
// stored per atom sorted by packed value (so a pair's reverse entry is found
// by binary search), with the positions of the build.
struct SkinArgs {
  int32_t* cand;    // [n, kCandCap]
  int32_t* ncand;   // [n]
  int32_t* crev;    // [n, kCandCap]
  int32_t* slot_of; // [n, kCandCap]
  int32_t* cof;     // [n, nm]
  double* xref;     // [n, 3]
  double L[3];
  double half_skin2;
  // rebuild decided on the device (launch_nl_skin_update): gate[0] != 0
  // when the kernels of a build run, gate[1] counts formats since the last
  // build; NULL for a build the host asked for
  int32_t* gate;
  int32_t* rebuilds;  // incremented by every gated build (nullable)
};

// One wavefront per atom, atoms taken in a grid-stride loop (the grid is
// sized to the resident capacity, so a gated launch that does nothing is
// cheap).
__global__ __launch_bounds__(256) void k_nl_skin_build(SearchArgs A, SkinArgs S, double rl2) {
  if (S.gate && S.gate[0] == 0) return;
  __shared__ CandLds<kCandCap> L;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  if (S.gate && blockIdx.x == 0 && threadIdx.x == 0) {
    S.gate[1] = 0;
    if (S.rebuilds) *S.rebuilds += 1;
  }
  for (int i = blockIdx.x * kSearchWaves + w; i < A.ntot; i += gridDim.x * kSearchWaves) {
    const FrameInfo F = A.fr[find_frame(A.fr, A.nframes, i)];
    bool capacity = false;
    const int ncand = gather_cells(A, L, w, lane, i, F, rl2, &capacity);
    wave_lds_sync();
    // rank of each candidate by its packed key (keys are distinct): one pass
    // over the list serves all of a lane's candidates, each record read once
    constexpr int M = kCandCap / 64;
    const int mmax = (ncand + 63) / 64;  // wave-uniform
    int pkm[M], rank[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int c = 64 * m + lane;
      pkm[m] = c < ncand ? L.r[w][c].pk : 0x7fffffff;
      rank[m] = 0;
    }
    for (int o = 0; o < ncand; ++o) {
      const int v = L.r[w][o].pk;
#pragma unroll
      for (int m = 0; m < M; ++m)
        if (m < mmax) rank[m] += v < pkm[m];
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int c = 64 * m + lane;
      if (c < ncand) S.cand[(int64_t)i * kCandCap + rank[m]] = pkm[m];
    }
    if (lane < 3) S.xref[3 * i + lane] = A.x[3 * i + lane];
    if (lane == 0) {
      S.ncand[i] = ncand;
      if (capacity) set_flag(A.flags, DP_FLAG_CAND_CAPACITY);
    }
    wave_lds_sync();  // the wave's LDS records are rewritten by its next atom
  }
}

// Position of each candidate's reverse pair (i, -s) in j's candidate list.
// One wave per atom i (atoms in a grid-stride loop over a grid of the
// resident capacity, so that a gated launch with nothing to do is cheap);
// lane l takes candidates l, l + 64, ... of i's list, four at a time, and
// runs their binary searches in j's sorted candidate list in lockstep (a
// fixed ten halvings cover the 512-entry capacity), so that four
// dependent-load chains are in flight per lane instead of one.
__global__ __launch_bounds__(256) void k_nl_skin_crev(SkinArgs S, int ntot) {
  if (S.gate && S.gate[0] == 0) return;
  const int lane = threadIdx.x & 63;
  for (int i = blockIdx.x * 4 + (threadIdx.x >> 6); i < ntot; i += gridDim.x * 4) {
    const int nc = S.ncand[i];
    const int32_t* ci = S.cand + (int64_t)i * kCandCap;
    constexpr int M = kCandCap / 64, U = 4;
    static_assert(kCandCap <= 1024, "ten halvings cover the list");
    for (int m0 = 0; m0 < M && 64 * m0 < nc; m0 += U) {
      int lo[U], hi[U], nj[U], tgt[U];
      const int32_t* cj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = 64 * (m0 + u) + lane;
        lo[u] = 0;
        hi[u] = 0;
        nj[u] = 0;
        tgt[u] = 0;
        cj[u] = ci;
        if (m0 + u < M && k < nc) {
          const int e = ci[k];
          const int j = e / 27;
          tgt[u] = 27 * i + (26 - (e - 27 * j));
          cj[u] = S.cand + (int64_t)j * kCandCap;
          nj[u] = S.ncand[j];
          hi[u] = nj[u];
        }
      }
#pragma unroll
      for (int it = 0; it < 10; ++it)
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (lo[u] < hi[u]) {
            const int mid = (lo[u] + hi[u]) >> 1;
            if (cj[u][mid] < tgt[u]) lo[u] = mid + 1;
            else hi[u] = mid;
          }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = 64 * (m0 + u) + lane;
        if (m0 + u < M && k < nc) S.crev[(int64_t)i * kCandCap + k] = (lo[u] < nj[u] && cj[u][lo[u]] == tgt[u]) ? lo[u] : -1;
      }
    }
  }
}

// After a build the host asked for: no rebuild pending, no format since.
__global__ void k_fill_gate(int32_t* gate) {
  if (threadIdx.x < 2) gate[threadIdx.x] = 0;
}

// Rebuild decision of a Verlet update: gate[0] is set when an atom has moved
// more than skin/2 since the build (the format's exactness condition) or
// when `every` > 0 updates have passed since it.  gate[0] was cleared by the
// previous format's second pass.
__global__ __launch_bounds__(256) void k_nl_skin_check(const double* __restrict__ x, const double* __restrict__ xref,
                                                       int ntot, double half_skin2, int every, int32_t* gate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool moved = false;
  if (i < ntot) {
    const double ex = x[3 * i] - xref[3 * i], ey = x[3 * i + 1] - xref[3 * i + 1], ez = x[3 * i + 2] - xref[3 * i + 2];
    moved = !((ex * ex + ey * ey) + ez * ez <= half_skin2);
  }
  if (__ballot(moved) && (threadIdx.x & 63) == 0) atomicOr(gate, 1);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int k = gate[1] + 1;
    gate[1] = k;
    if (every > 0 && k >= every) atomicOr(gate, 1);
  }
}

// Small frames: the cell binning of a gated Verlet build (wrap in place,
// cell counts, their scan, the scatter) in one work-group, one launch
// instead of three; a step with no rebuild returns at once.  Counts and
// fill counters stay in LDS (the global ones, which the multi-work-group
// binning uses, stay zero).  The skin check stays a kernel of its own: one
// compute unit alone reads the positions several times slower.
constexpr int kPrepSmallAtoms = 1 << 17, kPrepSmallCells = 4096;
__global__ __launch_bounds__(1024) void k_nl_bin_small(double* __restrict__ x, const FrameInfo* __restrict__ fr,
                                                      int ntot, int ncells, const int32_t* gate,
                                                      int32_t* __restrict__ cell_of, int32_t* __restrict__ cell_start,
                                                      int32_t* __restrict__ cell_atoms, int32_t* flags,
                                                      int32_t* images) {
  if (*gate == 0) return;
  __shared__ int32_t cnt[kPrepSmallCells];  // counts, then fill counters
  __shared__ int32_t st[kPrepSmallCells];   // cell starts
  __shared__ int32_t part[1024];
  const int tid = threadIdx.x;
  for (int c = tid; c < ncells; c += 1024) cnt[c] = 0;
  __syncthreads();
  const FrameInfo F = fr[0];
  for (int i = tid; i < ntot; i += 1024) {
    int cc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double xa = x[3 * i + a];
      if (!(xa >= 0.0 && xa < F.L[a])) {
        const double L = F.L[a];
        const double k = floor(xa / L);
        xa -= k * L;
        if (xa >= L) xa -= L;  // rounding of x - k L
        if (xa < 0.0) xa += L;
        if (xa >= L) xa = 0.0;
        x[3 * i + a] = xa;
        if (images) images[3 * i + a] += (int32_t)k;
      }
      if (!(xa >= 0.0 && xa < F.L[a])) set_flag(flags, DP_FLAG_NOT_WRAPPED);
      cc[a] = cell_coord(xa, F.L[a], F.ncell[a]);
    }
    const int cid = cc[0] + F.ncell[0] * (cc[1] + F.ncell[1] * cc[2]);
    cell_of[i] = F.cell_off + cid;
    atomicAdd(&cnt[cid], 1);
  }
  __syncthreads();
  // exclusive scan: thread t sums its run of cells, a scan of the 1024 sums,
  // then the run's starts
  constexpr int kRun = kPrepSmallCells / 1024;
  const int c0 = tid * kRun;
  int run = 0;
#pragma unroll
  for (int q = 0; q < kRun; ++q) run += c0 + q < ncells ? cnt[c0 + q] : 0;
  part[tid] = run;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int t = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += t;
    __syncthreads();
  }
  int acc = part[tid] - run;
#pragma unroll
  for (int q = 0; q < kRun; ++q)
    if (c0 + q < ncells) {
      st[c0 + q] = acc;
      cell_start[F.cell_off + c0 + q] = acc;
      acc += cnt[c0 + q];
      cnt[c0 + q] = 0;
    }
  if (tid == 1023) cell_start[F.cell_off + ncells] = part[1023];
  __syncthreads();
  for (int i = tid; i < ntot; i += 1024) {
    const int cid = cell_of[i] - F.cell_off;
    const int p = atomicAdd(&cnt[cid], 1);
    cell_atoms[st[cid] + p] = i;
  }
}

// Format: the sorted, truncated list on the current positions from the
// candidates of the last build (same test and order as the cell search).
template <int CAP>
__global__ __launch_bounds__(256) void k_nl_skin_format(SearchArgs A, SkinArgs S) {
  __shared__ CandLds<CAP> L;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * kSearchWaves + w;
  if (i >= A.ntot) return;
  const double xi = A.x[3 * i], yi = A.x[3 * i + 1], zi = A.x[3 * i + 2];
  if (lane == 0) {
    const double ex = xi - S.xref[3 * i], ey = yi - S.xref[3 * i + 1], ez = zi - S.xref[3 * i + 2];
    if (!((ex * ex + ey * ey) + ez * ez <= S.half_skin2)) set_flag(A.flags, DP_FLAG_SKIN_EXCEEDED);
  }
  const int nc = S.ncand[i];
  const int32_t* ci = S.cand + (int64_t)i * kCandCap;
  // all loads of a lane's candidates are issued before any is used
  constexpr int kPer = kCandCap / 64;
  int e[kPer], tj[kPer];
  double r2[kPer];
#pragma unroll
  for (int m = 0; m < kPer; ++m) e[m] = (64 * m < nc && 64 * m + lane < nc) ? ci[64 * m + lane] : -1;
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    r2[m] = 0.0;
    tj[m] = 0;
    if (e[m] >= 0) {
      const int j = e[m] / 27, sc = e[m] - 27 * j;
      const double ddx = (A.x[3 * j] - xi) + (double)(sc % 3 - 1) * S.L[0];
      const double ddy = (A.x[3 * j + 1] - yi) + (double)((sc / 3) % 3 - 1) * S.L[1];
      const double ddz = (A.x[3 * j + 2] - zi) + (double)(sc / 9 - 1) * S.L[2];
      r2[m] = r2_nofma(ddx, ddy, ddz);
      tj[m] = A.types[j];
    }
  }
  int ncand = 0;
#pragma unroll
  for (int m = 0; m < kPer; ++m) {
    if (64 * m >= nc) break;
    const int k = 64 * m + lane;
    const bool keep = e[m] >= 0 && r2[m] < A.rc2;
    if (e[m] >= 0 && !keep) S.slot_of[(int64_t)i * kCandCap + k] = -1;
    const uint64_t mask = __ballot(keep);
    const int before = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
    if (keep && ncand + before >= CAP) S.slot_of[(int64_t)i * kCandCap + k] = -1;  // beyond capacity (flagged)
    if (keep && ncand + before < CAP) {
      int t = tj[m];
      if (t < 0 || t >= A.ntypes) {
        set_flag(A.flags, DP_FLAG_BAD_INPUT);
        t = t < 0 ? 0 : A.ntypes - 1;
      }
      CandRec rec;
      rec.r2 = r2[m];
      rec.pk = e[m];
      rec.k = (int16_t)k;
      rec.t = (int8_t)t;
      rec.pad = 0;
      L.r[w][ncand + before] = rec;
    }
    ncand += __popcll(mask);
  }
  const bool capacity = ncand > CAP;
  if (capacity) ncand = CAP;
  wave_lds_sync();
  rank_and_write(A, L, w, lane, i, ncand, capacity, S.cof, S.slot_of);
}

// Reverse index from the candidate bookkeeping of the format (same meaning
// as the index built by binary search below).  Its first thread also moves
// the format's truncation count to the caller's buffer and clears the
// internal counter for the next format (stream order: every format block
// has finished, and the next format has not started).
__global__ void k_nl_skin_revmap(const int32_t* __restrict__ nlist, SkinArgs S, int32_t* __restrict__ rev, int ntot,
                                 int nm, int32_t* __restrict__ ovf_ctr, int32_t* __restrict__ overflow,
                                 int32_t* __restrict__ gate) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q == 0) {
    *overflow = *ovf_ctr;
    *ovf_ctr = 0;
    gate[0] = 0;  // the next update decides again
  }
  if (q >= (int64_t)ntot * nm) return;
  const int e = nlist[q];
  int out = -1;
  if (e >= 0) {
    const int i = (int)(q / nm);
    const int kr = S.crev[(int64_t)i * kCandCap + S.cof[q]];
    if (kr >= 0) out = S.slot_of[(int64_t)(e / 27) * kCandCap + kr];
  }
  rev[q] = out;
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
                     c->cell_of, c->cell_count, c->flags_dev, (double*)nullptr, (int32_t*)nullptr,
                     (const int32_t*)nullptr);
}

void launch_nl_scan(dp_ctx* c, int32_t ncells, hipStream_t s) {
  hipLaunchKernelGGL(k_nl_scan, dim3(1), dim3(1024), 0, s, c->cell_count, c->cell_start, c->cell_fill, ncells,
                     (const int32_t*)nullptr);
}

void launch_nl_scatter(dp_ctx* c, int32_t ntot, hipStream_t s) {
  if (ntot <= 0) return;
  hipLaunchKernelGGL(k_nl_scatter, dim3((ntot + 255) / 256), dim3(256), 0, s, c->cell_of, c->cell_start,
                     c->cell_fill, c->cell_atoms, ntot, (const int32_t*)nullptr);
}

static SearchArgs search_args(dp_ctx* c, const double* x, const int32_t* types, int32_t ntot, int32_t nframes,
                              int32_t* nlist, int32_t* overflow) {
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
  return A;
}

static SkinArgs skin_args(dp_ctx* c) {
  SkinArgs S;
  S.cand = c->skin_cand;
  S.ncand = c->skin_ncand;
  S.crev = c->skin_crev;
  S.slot_of = c->skin_slot;
  S.cof = c->skin_cof;
  S.xref = c->skin_xref;
  for (int a = 0; a < 3; ++a) S.L[a] = c->skin_L[a];
  S.half_skin2 = 0.25 * c->skin * c->skin;
  S.gate = nullptr;
  S.rebuilds = nullptr;
  return S;
}

void launch_nl_search(dp_ctx* c, const double* x, const int32_t* types, int32_t ntot, int32_t nframes,
                      int32_t* nlist, int32_t* overflow, hipStream_t s) {
  if (ntot <= 0) return;
  SearchArgs A = search_args(c, x, types, ntot, nframes, nlist, overflow);
  const dim3 grid((ntot + kSearchWaves - 1) / kSearchWaves), block(64 * kSearchWaves);
  if (A.nm <= kKeepCapSmall) hipLaunchKernelGGL(k_nl_search<kKeepCapSmall>, grid, block, 0, s, A);
  else hipLaunchKernelGGL(k_nl_search<kCandCap>, grid, block, 0, s, A);
}

// Verlet build from the binned wrapped positions.  The frame (box, cell
// grid of edge >= r_c + skin) is the context's copy made at the last
// dp_nlist_skin_build: dp_compute replaces the general frame table.
static void skin_build_kernels(dp_ctx* c, const double* x, const int32_t* types, int32_t ntot, int32_t* gate,
                               int32_t* rebuilds, hipStream_t s) {
  SearchArgs A = search_args(c, x, types, ntot, 1, nullptr, nullptr);
  A.fr = c->skin_frame;
  SkinArgs S = skin_args(c);
  S.gate = gate;
  S.rebuilds = rebuilds;
  const double rl = c->model->desc.rcut + c->skin;
  // 4-wave work-groups with 32 KB of LDS records: 5 resident per CU
  const int64_t gb = (ntot + kSearchWaves - 1) / kSearchWaves, gbmax = 5LL * c->ncu;
  hipLaunchKernelGGL(k_nl_skin_build, dim3((unsigned)(gb < gbmax ? gb : gbmax)), dim3(64 * kSearchWaves), 0, s, A, S,
                     rl * rl);
  const int64_t gq = (ntot + 3) / 4, gqmax = 8LL * c->ncu;  // a wave per atom, resident grid
  hipLaunchKernelGGL(k_nl_skin_crev, dim3((unsigned)(gq < gqmax ? gq : gqmax)), dim3(256), 0, s, S, ntot);
}

void launch_nl_skin_build(dp_ctx* c, double* x, const int32_t* types, int32_t ntot, int32_t ncells, int32_t* images,
                          hipStream_t s) {
  if (ntot <= 0) return;
  hipLaunchKernelGGL(k_nl_bin, dim3((ntot + 255) / 256), dim3(256), 0, s, (const double*)x, c->skin_frame, 1, ntot,
                     c->cell_of, c->cell_count, c->flags_dev, x, images, (const int32_t*)nullptr);
  launch_nl_scan(c, ncells, s);
  launch_nl_scatter(c, ntot, s);
  skin_build_kernels(c, x, types, ntot, nullptr, nullptr, s);
  hipLaunchKernelGGL(k_fill_gate, dim3(1), dim3(64), 0, s, c->skin_gate);
}

void launch_nl_skin_update(dp_ctx* c, double* x, const int32_t* types, int32_t ntot, int32_t every, int32_t* images,
                           int32_t* rebuilds, hipStream_t s) {
  if (ntot <= 0) return;
  int32_t* gate = c->skin_gate;
  hipLaunchKernelGGL(k_nl_skin_check, dim3((ntot + 255) / 256), dim3(256), 0, s, (const double*)x,
                     (const double*)c->skin_xref, ntot, 0.25 * c->skin * c->skin, every, gate);
  if (ntot <= kPrepSmallAtoms && c->skin_ncells <= kPrepSmallCells) {
    hipLaunchKernelGGL(k_nl_bin_small, dim3(1), dim3(1024), 0, s, x, c->skin_frame, ntot, c->skin_ncells,
                       (const int32_t*)gate, c->cell_of, c->cell_start, c->cell_atoms, c->flags_dev, images);
  } else {
    hipLaunchKernelGGL(k_nl_bin, dim3((ntot + 255) / 256), dim3(256), 0, s, (const double*)x, c->skin_frame, 1, ntot,
                       c->cell_of, c->cell_count, c->flags_dev, x, images, (const int32_t*)gate);
    hipLaunchKernelGGL(k_nl_scan, dim3(1), dim3(1024), 0, s, c->cell_count, c->cell_start, c->cell_fill,
                       c->skin_ncells, (const int32_t*)gate);
    hipLaunchKernelGGL(k_nl_scatter, dim3((ntot + 255) / 256), dim3(256), 0, s, c->cell_of, c->cell_start,
                       c->cell_fill, c->cell_atoms, ntot, (const int32_t*)gate);
  }
  skin_build_kernels(c, x, types, ntot, gate, rebuilds, s);
}

void launch_nl_skin_format(dp_ctx* c, const double* x, const int32_t* types, int32_t ntot, int32_t* nlist,
                           int32_t* overflow, hipStream_t s) {
  if (ntot <= 0) return;
  SearchArgs A = search_args(c, x, types, ntot, 1, nlist, c->ovf_ctr);
  SkinArgs S = skin_args(c);
  const dim3 grid((ntot + kSearchWaves - 1) / kSearchWaves), block(64 * kSearchWaves);
  if (A.nm <= kKeepCapSmall) hipLaunchKernelGGL(k_nl_skin_format<kKeepCapSmall>, grid, block, 0, s, A, S);
  else hipLaunchKernelGGL(k_nl_skin_format<kCandCap>, grid, block, 0, s, A, S);
  const int64_t q = (int64_t)ntot * A.nm;
  hipLaunchKernelGGL(k_nl_skin_revmap, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, nlist, S, c->rev, ntot,
                     A.nm, c->ovf_ctr, overflow, c->skin_gate);
}

}  // namespace dpse
