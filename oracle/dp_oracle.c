/*
 * FP64 CPU oracle for Deep Potential smooth-edition (se_a) energy, forces and
 * virial.  TEST INFRASTRUCTURE ONLY: it is called by the tests, by smoke() and
 * by the cpu_baseline leg of the bench, never by the product path.  It shares
 * no code, header or table with the GPU library.
 *
 * What it computes follows the Background section (DeePMD-kit subsection and
 * Fig. 1): a neighbour list within the cut-off, the environment matrix R_i
 * whose smoothed first column feeds a three-layer embedding net, the
 * symmetry-preserving descriptor D_i, a three-layer fitting net giving the
 * atomic energy E_i, E = sum_i E_i, and forces as the gradient of E obtained
 * by back-propagation.  The paper does not print the formulas; the readings
 * used here (quintic switch, DeePMD skip connections, 1/N_m scaling,
 * environment normalisation with mean 0 and a per-column sigma, strict
 * r^2 < rc^2 cut-off, per-type sections sorted by (r^2, packed index)) are
 * the standard DP se_a definitions from the DeepPot-SE / DeePMD-kit papers
 * the Background section cites.
 *
 * Plain loops in natural order, no BLAS, no blocking; OpenMP only runs
 * independent atoms in parallel.  Build with -O2 -ffp-contract=off so that
 * the r^2 used by the cut-off test is the un-contracted expression.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXT 4
#define OR_MAXL 8

typedef struct {
  int ntypes;
  double rc, rs;
  double inv_std[2]; /* 1/sigma of the radial column and of the three vector columns */
  int sel[OR_MAXT];
  int sec[OR_MAXT + 1]; /* section offsets into the nm slots */
  int nm;
  int nemb, emb[OR_MAXL];
  int m1, m2, nd;
  int nfit, fit[OR_MAXL];
  /* parameter offsets into the flat vector */
  int64_t emb_w[OR_MAXT][OR_MAXT][OR_MAXL], emb_b[OR_MAXT][OR_MAXT][OR_MAXL];
  int64_t fit_w[OR_MAXT][OR_MAXL], fit_b[OR_MAXT][OR_MAXL];
  int64_t fit_wo[OR_MAXT], fit_bo[OR_MAXT], ebias;
  int64_t nparams;
} or_model;

/* idesc = {ntypes, sel[ntypes], nemb, emb[nemb], m2, nfit, fit[nfit]} ;
 * ddesc = {rcut, rcut_smth, sigma_radial, sigma_vector}.  Returns 0 or -1. */
static int or_parse(const int32_t* idesc, const double* ddesc, or_model* m) {
  memset(m, 0, sizeof(*m));
  int p = 0;
  m->ntypes = idesc[p++];
  if (m->ntypes < 1 || m->ntypes > OR_MAXT) return -1;
  m->sec[0] = 0;
  for (int t = 0; t < m->ntypes; t++) {
    m->sel[t] = idesc[p++];
    m->sec[t + 1] = m->sec[t] + m->sel[t];
  }
  m->nm = m->sec[m->ntypes];
  m->nemb = idesc[p++];
  if (m->nemb < 1 || m->nemb > OR_MAXL) return -1;
  for (int l = 0; l < m->nemb; l++) m->emb[l] = idesc[p++];
  m->m2 = idesc[p++];
  m->nfit = idesc[p++];
  if (m->nfit < 1 || m->nfit > OR_MAXL) return -1;
  for (int l = 0; l < m->nfit; l++) m->fit[l] = idesc[p++];
  m->m1 = m->emb[m->nemb - 1];
  if (m->m2 > m->m1) return -1;
  m->nd = m->m1 * m->m2;
  m->rc = ddesc[0];
  m->rs = ddesc[1];
  if (!(ddesc[2] > 0.0) || !(ddesc[3] > 0.0)) return -1;
  m->inv_std[0] = 1.0 / ddesc[2];
  m->inv_std[1] = 1.0 / ddesc[3];
  int64_t off = 0;
  for (int a = 0; a < m->ntypes; a++)
    for (int b = 0; b < m->ntypes; b++) {
      int prev = 1;
      for (int l = 0; l < m->nemb; l++) {
        m->emb_w[a][b][l] = off; off += (int64_t)prev * m->emb[l];
        m->emb_b[a][b][l] = off; off += m->emb[l];
        prev = m->emb[l];
      }
    }
  for (int t = 0; t < m->ntypes; t++) {
    int prev = m->nd;
    for (int l = 0; l < m->nfit; l++) {
      m->fit_w[t][l] = off; off += (int64_t)prev * m->fit[l];
      m->fit_b[t][l] = off; off += m->fit[l];
      prev = m->fit[l];
    }
    m->fit_wo[t] = off; off += prev;
    m->fit_bo[t] = off; off += 1;
  }
  m->ebias = off; off += m->ntypes;
  m->nparams = off;
  return 0;
}

int64_t or_nparams(const int32_t* idesc, const double* ddesc) {
  or_model m;
  if (or_parse(idesc, ddesc, &m)) return -1;
  return m.nparams;
}

/* ------------------------------------------------------------------------ */
/* Neighbour list.
 * For atom i, every image (j, s), s in {-1,0,1}^3, except (i, 0), with
 *   d = (x_j - x_i) + (s0*h0 + s1*h1 + s2*h2)     (component-wise)
 *   r2 = (dx*dx + dy*dy) + dz*dz                  (no fused multiply-add)
 * is a neighbour when r2 < rc^2.  Neighbours are split by their type into
 * sections of sel[t] slots, sorted within a section by r2 ascending then by
 * packed = 27*j + (s0+1) + 3*(s1+1) + 9*(s2+1), truncated to sel[t] (the
 * excess is counted as overflow) and padded with -1.                        */

typedef struct { double r2; int64_t packed; } or_cand;

static int or_cand_cmp(const void* a, const void* b) {
  const or_cand* x = (const or_cand*)a;
  const or_cand* y = (const or_cand*)b;
  if (x->r2 < y->r2) return -1;
  if (x->r2 > y->r2) return 1;
  return (x->packed > y->packed) - (x->packed < y->packed);
}

static double or_sq_sum(double dx, double dy, double dz) {
  volatile double a = dx * dx; /* volatile keeps each product rounded */
  volatile double b = dy * dy;
  volatile double c = dz * dz;
  volatile double ab = a + b;
  return ab + c;
}

/* Candidate enumeration for one atom: brute force over all j and 27 images
 * (use_cells == 0), or only over the 27 neighbouring cells of an
 * orthorhombic cell grid (use_cells == 1).  Both evaluate the same r2
 * expression; tests check that they produce identical lists.              */
typedef struct {
  int ncell[3];
  int* head; /* [ncells+1] */
  int* idx;  /* [n] */
} or_cells;

static int or_build_cells(int64_t n, const double* x, const double* h, double rc, or_cells* c) {
  for (int d = 0; d < 3; d++) {
    double L = h[4 * d];
    int nc = (int)floor(L / rc);
    if (nc < 1) nc = 1;
    c->ncell[d] = nc;
  }
  int64_t nct = (int64_t)c->ncell[0] * c->ncell[1] * c->ncell[2];
  c->head = (int*)calloc((size_t)nct + 1, sizeof(int));
  c->idx = (int*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
  int* cell = (int*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
  int* fill = (int*)calloc((size_t)nct + 1, sizeof(int));
  for (int64_t i = 0; i < n; i++) {
    int ci[3];
    for (int d = 0; d < 3; d++) {
      double L = h[4 * d];
      int k = (int)floor(x[3 * i + d] / L * c->ncell[d]);
      if (k < 0) k = 0;
      if (k >= c->ncell[d]) k = c->ncell[d] - 1;
      ci[d] = k;
    }
    cell[i] = ci[0] + c->ncell[0] * (ci[1] + c->ncell[1] * ci[2]);
    c->head[cell[i] + 1]++;
  }
  for (int64_t k = 0; k < nct; k++) c->head[k + 1] += c->head[k];
  for (int64_t i = 0; i < n; i++) c->idx[c->head[cell[i]] + fill[cell[i]]++] = (int)i;
  free(cell);
  free(fill);
  return 0;
}

static int64_t or_one_row(int64_t i, int64_t n, const double* x, const int32_t* type, const double* h,
                          const or_model* m, const or_cells* cells, or_cand* buf, int64_t cap,
                          int32_t* row, int64_t* overflow) {
  double rc2 = m->rc * m->rc;
  int64_t nc[OR_MAXT];
  or_cand* sec[OR_MAXT];
  for (int t = 0; t < m->ntypes; t++) { nc[t] = 0; sec[t] = buf + t * cap; }
  int64_t total = 0;
  if (!cells) {
    for (int64_t j = 0; j < n; j++)
      for (int sz = -1; sz <= 1; sz++)
        for (int sy = -1; sy <= 1; sy++)
          for (int sx = -1; sx <= 1; sx++) {
            if (j == i && sx == 0 && sy == 0 && sz == 0) continue;
            double d[3];
            for (int a = 0; a < 3; a++) {
              double sh = (double)sx * h[0 + a] + (double)sy * h[3 + a] + (double)sz * h[6 + a];
              d[a] = (x[3 * j + a] - x[3 * i + a]) + sh;
            }
            double r2 = or_sq_sum(d[0], d[1], d[2]);
            if (r2 < rc2) {
              int t = type[j];
              if (nc[t] >= cap) return -1;
              sec[t][nc[t]].r2 = r2;
              sec[t][nc[t]].packed = 27 * j + (sx + 1) + 3 * (sy + 1) + 9 * (sz + 1);
              nc[t]++;
            }
          }
  } else {
    int ci[3];
    for (int a = 0; a < 3; a++) {
      double L = h[4 * a];
      int k = (int)floor(x[3 * i + a] / L * cells->ncell[a]);
      if (k < 0) k = 0;
      if (k >= cells->ncell[a]) k = cells->ncell[a] - 1;
      ci[a] = k;
    }
    for (int dz = -1; dz <= 1; dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
          int cc[3] = {ci[0] + dx, ci[1] + dy, ci[2] + dz};
          int s[3];
          for (int a = 0; a < 3; a++) {
            s[a] = 0;
            if (cc[a] < 0) { cc[a] += cells->ncell[a]; s[a] = -1; }
            else if (cc[a] >= cells->ncell[a]) { cc[a] -= cells->ncell[a]; s[a] = 1; }
          }
          int cid = cc[0] + cells->ncell[0] * (cc[1] + cells->ncell[1] * cc[2]);
          for (int q = cells->head[cid]; q < cells->head[cid + 1]; q++) {
            int64_t j = cells->idx[q];
            if (j == i && s[0] == 0 && s[1] == 0 && s[2] == 0) continue;
            double d[3];
            for (int a = 0; a < 3; a++) {
              double sh = (double)s[0] * h[0 + a] + (double)s[1] * h[3 + a] + (double)s[2] * h[6 + a];
              d[a] = (x[3 * j + a] - x[3 * i + a]) + sh;
            }
            double r2 = or_sq_sum(d[0], d[1], d[2]);
            if (r2 < rc2) {
              int t = type[j];
              if (nc[t] >= cap) return -1;
              sec[t][nc[t]].r2 = r2;
              sec[t][nc[t]].packed = 27 * j + (s[0] + 1) + 3 * (s[1] + 1) + 9 * (s[2] + 1);
              nc[t]++;
            }
          }
        }
  }
  int64_t ov = 0;
  for (int t = 0; t < m->ntypes; t++) {
    qsort(sec[t], (size_t)nc[t], sizeof(or_cand), or_cand_cmp);
    for (int q = 0; q < m->sel[t]; q++)
      row[m->sec[t] + q] = q < nc[t] ? (int32_t)sec[t][q].packed : -1;
    if (nc[t] > m->sel[t]) ov += nc[t] - m->sel[t];
    total += nc[t];
  }
  *overflow = ov;
  return total;
}

/* Neighbour rows for the atoms rows[0..nrows) (rows == NULL: all atoms).
 * nlist_out is [nrows, nm].  Returns 0, or -1 on bad input / capacity.   */
int or_nlist(int64_t n, const double* x, const int32_t* type, const double* h,
             const int32_t* idesc, const double* ddesc, const int64_t* rows, int64_t nrows,
             int use_cells, int32_t* nlist_out, int64_t* overflow_out) {
  or_model m;
  if (or_parse(idesc, ddesc, &m)) return -1;
  for (int64_t i = 0; i < n; i++)
    if (type[i] < 0 || type[i] >= m.ntypes) return -1;
  if (use_cells && (h[1] != 0 || h[2] != 0 || h[3] != 0 || h[5] != 0 || h[6] != 0 || h[7] != 0)) return -1;
  or_cells cells;
  if (use_cells) or_build_cells(n, x, h, m.rc, &cells);
  int64_t cap = 4096;
  int64_t ovtot = 0;
  int err = 0;
#pragma omp parallel
  {
    or_cand* buf = (or_cand*)malloc(sizeof(or_cand) * (size_t)cap * m.ntypes);
#pragma omp for schedule(dynamic, 16) reduction(+ : ovtot)
    for (int64_t r = 0; r < nrows; r++) {
      int64_t i = rows ? rows[r] : r;
      int64_t ov = 0;
      if (or_one_row(i, n, x, type, h, &m, use_cells ? &cells : NULL, buf, cap, nlist_out + r * m.nm, &ov) < 0)
        err = 1;
      ovtot += ov;
    }
    free(buf);
  }
  if (use_cells) { free(cells.head); free(cells.idx); }
  *overflow_out = ovtot;
  return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Smooth switching (quintic reading):
 *   u = (r - rs)/(rc - rs);  s = 1/r for r < rs,
 *   s = (u^3 (-6u^2 + 15u - 10) + 1)/r for rs <= r < rc,  s = 0 for r >= rc. */
static void or_switch(double r, double rs, double rc, double* s, double* ds) {
  if (r < rs) {
    *s = 1.0 / r;
    *ds = -1.0 / (r * r);
  } else if (r < rc) {
    double u = (r - rs) / (rc - rs);
    double poly = u * u * u * (-6.0 * u * u + 15.0 * u - 10.0) + 1.0;
    double dpoly = -30.0 * u * u * (1.0 - u) * (1.0 - u) / (rc - rs);
    *s = poly / r;
    *ds = dpoly / r - poly / (r * r);
  } else {
    *s = 0.0;
    *ds = 0.0;
  }
}

void or_switch_fn(int64_t n, const double* r, double rs, double rc, double* s, double* ds) {
  for (int64_t k = 0; k < n; k++) or_switch(r[k], rs, rc, &s[k], &ds[k]);
}

/* Per-layer forward of a DP dense net: z = h_prev W + b, then
 *   h = tanh(z)                      if w != w_prev and w != 2 w_prev,
 *   h = h_prev + tanh(z)             if w == w_prev,
 *   h = [h_prev, h_prev] + tanh(z)   if w == 2 w_prev.
 * t receives tanh(z).                                                      */
static void or_dense_fwd(const double* hp, int wp, const double* W, const double* b, int w, double* t, double* h) {
  for (int q = 0; q < w; q++) {
    double z = b[q];
    for (int p = 0; p < wp; p++) z += hp[p] * W[(int64_t)p * w + q];
    t[q] = tanh(z);
    if (w == wp) h[q] = hp[q] + t[q];
    else if (w == 2 * wp) h[q] = hp[q % wp] + t[q];
    else h[q] = t[q];
  }
}

/* Backward of or_dense_fwd: given dh (dE/dh), write dE/dh_prev into dhp and
 * optionally accumulate parameter gradients scaled by gscale.              */
static void or_dense_bwd(const double* hp, int wp, const double* W, const double* t, int w, const double* dh,
                         double* dz, double* dhp, double* gW, double* gb, double gscale) {
  for (int q = 0; q < w; q++) dz[q] = dh[q] * (1.0 - t[q] * t[q]);
  for (int p = 0; p < wp; p++) {
    double acc = 0.0;
    for (int q = 0; q < w; q++) acc += W[(int64_t)p * w + q] * dz[q];
    if (w == wp) acc += dh[p];
    else if (w == 2 * wp) acc += dh[p] + dh[p + wp];
    dhp[p] = acc;
  }
  if (gW) {
    for (int p = 0; p < wp; p++)
      for (int q = 0; q < w; q++) gW[(int64_t)p * w + q] += gscale * hp[p] * dz[q];
    for (int q = 0; q < w; q++) gb[q] += gscale * dz[q];
  }
}

typedef struct {
  double* R;    /* nm x 4 */
  double* dRd;  /* nm x 4 x 3 : dR[k]/dd[alpha] */
  double* d;    /* nm x 3 */
  double* act;  /* nm x (sum emb widths) : h per layer */
  double* tact; /* nm x (sum emb widths) : tanh per layer */
  double* T;    /* m1 x 4 */
  double* D;    /* nd */
  double* fh;   /* fitting h per layer: nfit x maxw */
  double* ft;
  double* gD;
  double* gT;
  double* gG;
  double* nd_;  /* nm x 4 */
  double* tmp1;
  double* tmp2;
  double* tmp3;
} or_scratch;

static int or_maxw(const or_model* m) {
  int w = m->nd;
  for (int l = 0; l < m->nfit; l++) if (m->fit[l] > w) w = m->fit[l];
  for (int l = 0; l < m->nemb; l++) if (m->emb[l] > w) w = m->emb[l];
  return w;
}

static void or_scratch_alloc(const or_model* m, or_scratch* s) {
  int sumw = 0;
  for (int l = 0; l < m->nemb; l++) sumw += m->emb[l];
  int mw = or_maxw(m);
  s->R = (double*)malloc(sizeof(double) * m->nm * 4);
  s->dRd = (double*)malloc(sizeof(double) * m->nm * 12);
  s->d = (double*)malloc(sizeof(double) * m->nm * 3);
  s->act = (double*)malloc(sizeof(double) * m->nm * sumw);
  s->tact = (double*)malloc(sizeof(double) * m->nm * sumw);
  s->T = (double*)malloc(sizeof(double) * m->m1 * 4);
  s->D = (double*)malloc(sizeof(double) * m->nd);
  s->fh = (double*)malloc(sizeof(double) * m->nfit * mw);
  s->ft = (double*)malloc(sizeof(double) * m->nfit * mw);
  s->gD = (double*)malloc(sizeof(double) * m->nd);
  s->gT = (double*)malloc(sizeof(double) * m->m1 * 4);
  s->gG = (double*)malloc(sizeof(double) * m->m1);
  s->nd_ = (double*)malloc(sizeof(double) * m->nm * 4);
  s->tmp1 = (double*)malloc(sizeof(double) * mw);
  s->tmp2 = (double*)malloc(sizeof(double) * mw);
  s->tmp3 = (double*)malloc(sizeof(double) * mw);
}

static void or_scratch_free(or_scratch* s) {
  free(s->R); free(s->dRd); free(s->d); free(s->act); free(s->tact); free(s->T); free(s->D);
  free(s->fh); free(s->ft); free(s->gD); free(s->gT); free(s->gG); free(s->nd_);
  free(s->tmp1); free(s->tmp2); free(s->tmp3);
}

/* ------------------------------------------------------------------------ */
/* DP-compress (the compression of the embedding net cited in the Background
 * section): each embedding net G(x) of one scalar input x = R~[0] is
 * replaced by piecewise fifth-order polynomials in t = x - x_left on a grid
 * of intervals; on each interval the quintic matches G, dG/dx and d2G/dx2 at
 * both ends (Hermite interpolation).  Grid: a fine stride h on [0, X1)
 * (n1 intervals, X1 = n1 h), a coarse stride H = 10 h on [X1, X2) (n2
 * intervals); inputs at or beyond X2 take the value at X2 and are counted.
 * Table layout: [net = ti*ntypes + tj][interval][power p = 0..5][feature]. */

typedef struct {
  double h, H, X1, X2;
  int n1, n2, nint;
} or_grid;

static void or_grid_make(double x1, double x2, double h, or_grid* g) {
  g->h = h;
  g->H = h * 10.0;
  g->n1 = (int)ceil(x1 / h);
  g->X1 = (double)g->n1 * h;
  g->n2 = x2 > g->X1 ? (int)ceil((x2 - g->X1) / g->H) : 0;
  g->X2 = fma((double)g->n2, g->H, g->X1);
  g->nint = g->n1 + g->n2;
}

int or_tab_nint(double x1, double x2, double h) {
  or_grid g;
  if (!(h > 0.0) || !(x1 > 0.0)) return -1;
  or_grid_make(x1, x2, h, &g);
  return g.nint;
}

/* Interval of input x and the offset t in it; *clip set when x >= X2. */
static int or_interval(const or_grid* g, double x, double* t, int* clip) {
  if (x < g->X1) {
    int k = (int)floor(x / g->h);
    if (k >= g->n1) k = g->n1 - 1;
    if (k < 0) k = 0;
    *t = fma(-(double)k, g->h, x);
    return k;
  }
  if (x < g->X2) {
    int m = (int)floor((x - g->X1) / g->H);
    if (m >= g->n2) m = g->n2 - 1;
    *t = fma(-(double)m, g->H, x - g->X1);
    return g->n1 + m;
  }
  *clip = 1;
  *t = g->n2 > 0 ? g->H : g->h;
  return g->nint - 1;
}

/* G, dG/dx and d2G/dx2 of net (ti, tj) at input x, by forward-mode
 * differentiation through the layers of or_dense_fwd: with z = h W + b,
 * z' = h' W, z'' = h'' W and tau = tanh(z): tau' = (1 - tau^2) z',
 * tau'' = (1 - tau^2) (z'' - 2 tau z'^2); the identity skips carry h, h', h''. */
static void or_emb_derivs(const or_model* m, const double* P, int ti, int tj, double x, double* G, double* dG,
                          double* d2G) {
  double hv[OR_MAXL * 256], hd[OR_MAXL * 256], hdd[OR_MAXL * 256];
  double in0 = x, in1 = 1.0, in2 = 0.0;
  const double *pv = &in0, *pd = &in1, *pdd = &in2;
  int wp = 1, off = 0;
  for (int l = 0; l < m->nemb; l++) {
    const int w = m->emb[l];
    const double* W = P + m->emb_w[ti][tj][l];
    const double* b = P + m->emb_b[ti][tj][l];
    for (int q = 0; q < w; q++) {
      double z = b[q], z1 = 0.0, z2 = 0.0;
      for (int p = 0; p < wp; p++) {
        z += pv[p] * W[(int64_t)p * w + q];
        z1 += pd[p] * W[(int64_t)p * w + q];
        z2 += pdd[p] * W[(int64_t)p * w + q];
      }
      const double tt = tanh(z);
      const double g1 = 1.0 - tt * tt;
      double v = tt, v1 = g1 * z1, v2 = g1 * (z2 - 2.0 * tt * z1 * z1);
      if (w == wp) { v += pv[q]; v1 += pd[q]; v2 += pdd[q]; }
      else if (w == 2 * wp) { v += pv[q % wp]; v1 += pd[q % wp]; v2 += pdd[q % wp]; }
      hv[off + q] = v;
      hd[off + q] = v1;
      hdd[off + q] = v2;
    }
    pv = hv + off;
    pd = hd + off;
    pdd = hdd + off;
    wp = w;
    off += w;
  }
  for (int a = 0; a < m->m1; a++) {
    G[a] = pv[a];
    dG[a] = pd[a];
    d2G[a] = pdd[a];
  }
}

/* Quintic on [0, L] from value, first and second derivative at both ends:
 * c0 = y0, c1 = d0, c2 = s0/2, and with A = y1 - y0 - d0 L - s0 L^2/2,
 * B = d1 - d0 - s0 L, C = s1 - s0 the remaining three solve
 * [L^3 L^4 L^5; 3L^2 4L^3 5L^4; 6L 12L^2 20L^3] c = [A B C]. */
static void or_quintic(double L, double y0, double d0, double s0, double y1, double d1, double s1, double* c) {
  const double A = y1 - y0 - d0 * L - 0.5 * s0 * L * L;
  const double B = d1 - d0 - s0 * L;
  const double C = s1 - s0;
  c[0] = y0;
  c[1] = d0;
  c[2] = 0.5 * s0;
  c[3] = (20.0 * A - 8.0 * B * L + C * L * L) / (2.0 * L * L * L);
  c[4] = (-30.0 * A + 14.0 * B * L - 2.0 * C * L * L) / (2.0 * L * L * L * L);
  c[5] = (12.0 * A - 6.0 * B * L + C * L * L) / (2.0 * L * L * L * L * L);
}

/* Builds the table of every net; table has ntypes^2 * nint * 6 * m1 values. */
int or_tab_build(const int32_t* idesc, const double* ddesc, const double* P, double x1, double x2, double h,
                 double* table) {
  or_model m;
  if (or_parse(idesc, ddesc, &m)) return -1;
  if (!(h > 0.0) || !(x1 > 0.0) || m.m1 > 256) return -1;
  or_grid g;
  or_grid_make(x1, x2, h, &g);
  const int nnets = m.ntypes * m.ntypes, m1 = m.m1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int job = 0; job < nnets * g.nint; job++) {
    const int net = job / g.nint, k = job % g.nint;
    const int ti = net / m.ntypes, tj = net % m.ntypes;
    double xl, L;
    if (k < g.n1) { xl = (double)k * g.h; L = g.h; }
    else { xl = fma((double)(k - g.n1), g.H, g.X1); L = g.H; }
    double G0[256], D0[256], S0[256], G1[256], D1[256], S1[256];
    or_emb_derivs(&m, P, ti, tj, xl, G0, D0, S0);
    or_emb_derivs(&m, P, ti, tj, xl + L, G1, D1, S1);
    double* out = table + ((int64_t)net * g.nint + k) * 6 * m1;
    for (int a = 0; a < m1; a++) {
      double c[6];
      or_quintic(L, G0[a], D0[a], S0[a], G1[a], D1[a], S1[a], c);
      for (int q = 0; q < 6; q++) out[(int64_t)q * m1 + a] = c[q];
    }
  }
  return 0;
}

typedef struct {
  const double* table;  /* NULL: exact embedding nets */
  or_grid g;
} or_tab;

/* Debug outputs for one atom (any may be NULL). */
typedef struct {
  double* R;   /* nm x 4 */
  double* T;   /* m1 x 4 */
  double* D;   /* nd */
  double* gD;  /* nd */
  double* gT;  /* m1 x 4 */
  double* nd;  /* nm x 4 */
} or_dbg;

/* Energy E_i of atom i and g_ij = dE_i/dd_ij for each slot (zero for pads).
 * If grad != NULL, accumulates gscale * dE_i/dtheta into grad.            */
static double or_atom(int64_t i, const double* x, const int32_t* type, const double* h, const or_model* m,
                      const double* P, const int32_t* row, or_scratch* S, double* g_rows, double* grad,
                      double gscale, or_dbg* dbg, const or_tab* tab, int64_t* nclip) {
  const int nm = m->nm;
  const int ti = type[i];
  int sumw = 0;
  for (int l = 0; l < m->nemb; l++) sumw += m->emb[l];
  const double inv_nm = 1.0 / (double)nm;

  /* environment matrix R~ = s(r) [1, dx/r, dy/r, dz/r] and dR~/dd */
  for (int q = 0; q < nm; q++) {
    int32_t e = row[q];
    double* R = S->R + 4 * q;
    double* dR = S->dRd + 12 * q;
    double* d = S->d + 3 * q;
    if (e < 0) {
      for (int k = 0; k < 4; k++) R[k] = 0.0;
      for (int k = 0; k < 12; k++) dR[k] = 0.0;
      d[0] = d[1] = d[2] = 0.0;
      continue;
    }
    int64_t j = e / 27;
    int sc = e % 27;
    int sx = sc % 3 - 1, sy = (sc / 3) % 3 - 1, sz = sc / 9 - 1;
    for (int a = 0; a < 3; a++) {
      double sh = (double)sx * h[0 + a] + (double)sy * h[3 + a] + (double)sz * h[6 + a];
      d[a] = (x[3 * j + a] - x[3 * i + a]) + sh;
    }
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double s, ds;
    or_switch(r, m->rs, m->rc, &s, &ds);
    R[0] = s;
    for (int a = 0; a < 3; a++) R[1 + a] = s * d[a] / r;
    for (int a = 0; a < 3; a++) dR[0 * 3 + a] = ds * d[a] / r;
    for (int c = 0; c < 3; c++)
      for (int a = 0; a < 3; a++)
        dR[(1 + c) * 3 + a] = ds * (d[a] / r) * (d[c] / r) + s * ((c == a ? 1.0 : 0.0) / r - d[c] * d[a] / (r * r * r));
    /* normalisation by the environment statistics (mean 0, so padded rows stay 0) */
    for (int k = 0; k < 4; k++) {
      double f = m->inv_std[k == 0 ? 0 : 1];
      R[k] *= f;
      for (int a = 0; a < 3; a++) dR[k * 3 + a] *= f;
    }
  }

  /* embedding nets, G_ij = N_{ti,tj}(s_ij); tabulated: G and dG/dx from
   * the interval's quintic (in the last layer's slots of act and tact) */
  for (int tj = 0; tj < m->ntypes; tj++) {
    for (int q = m->sec[tj]; q < m->sec[tj + 1]; q++) {
      if (row[q] < 0) continue;
      double* act = S->act + (int64_t)q * sumw;
      double* tac = S->tact + (int64_t)q * sumw;
      if (tab->table) {
        double t;
        int clip = 0;
        const int k = or_interval(&tab->g, S->R[4 * q], &t, &clip);
        *nclip += clip;
        const double* c = tab->table + ((int64_t)(ti * m->ntypes + tj) * tab->g.nint + k) * 6 * m->m1;
        const int go = sumw - m->m1;
        for (int a = 0; a < m->m1; a++) {
          const double* ca = c + a;
          const int64_t st = m->m1;
          double v = ca[5 * st];
          for (int p = 4; p >= 0; p--) v = fma(v, t, ca[p * st]);
          double d = 5.0 * ca[5 * st];
          for (int p = 4; p >= 1; p--) d = fma(d, t, (double)p * ca[p * st]);
          act[go + a] = v;
          tac[go + a] = clip ? 0.0 : d;
        }
        continue;
      }
      double in0 = S->R[4 * q];
      const double* hp = &in0;
      int wp = 1, off = 0;
      for (int l = 0; l < m->nemb; l++) {
        or_dense_fwd(hp, wp, P + m->emb_w[ti][tj][l], P + m->emb_b[ti][tj][l], m->emb[l], tac + off, act + off);
        hp = act + off;
        wp = m->emb[l];
        off += m->emb[l];
      }
    }
  }
  const int goff = sumw - m->m1;

  /* T = (1/nm) G^T R~ */
  for (int a = 0; a < m->m1; a++)
    for (int k = 0; k < 4; k++) {
      double acc = 0.0;
      for (int q = 0; q < nm; q++) {
        if (row[q] < 0) continue;
        acc += S->act[(int64_t)q * sumw + goff + a] * S->R[4 * q + k];
      }
      S->T[a * 4 + k] = acc * inv_nm;
    }
  /* D[a, b] = sum_k T[a,k] T[b,k], a < m1, b < m2, flattened a*m2 + b */
  for (int a = 0; a < m->m1; a++)
    for (int b = 0; b < m->m2; b++) {
      double acc = 0.0;
      for (int k = 0; k < 4; k++) acc += S->T[a * 4 + k] * S->T[b * 4 + k];
      S->D[a * m->m2 + b] = acc;
    }

  /* fitting net */
  int mw = or_maxw(m);
  const double* hp = S->D;
  int wp = m->nd;
  for (int l = 0; l < m->nfit; l++) {
    or_dense_fwd(hp, wp, P + m->fit_w[ti][l], P + m->fit_b[ti][l], m->fit[l], S->ft + l * mw, S->fh + l * mw);
    hp = S->fh + l * mw;
    wp = m->fit[l];
  }
  const double* wo = P + m->fit_wo[ti];
  double Ei = P[m->fit_bo[ti]] + P[m->ebias + ti];
  {
    double acc = 0.0;
    for (int p = 0; p < wp; p++) acc += hp[p] * wo[p];
    Ei += acc;
  }

  /* ---- backward (seed dE_i/dE_i = 1) ---- */
  if (grad) {
    for (int p = 0; p < wp; p++) grad[m->fit_wo[ti] + p] += gscale * hp[p];
    grad[m->fit_bo[ti]] += gscale;
    grad[m->ebias + ti] += gscale;
  }
  double* dh = S->tmp1;
  double* dz = S->tmp2;
  double* dhp = S->tmp3;
  for (int p = 0; p < wp; p++) dh[p] = wo[p];
  for (int l = m->nfit - 1; l >= 0; l--) {
    const double* hin = l > 0 ? S->fh + (l - 1) * mw : S->D;
    int win = l > 0 ? m->fit[l - 1] : m->nd;
    double* out = l > 0 ? dhp : S->gD;
    or_dense_bwd(hin, win, P + m->fit_w[ti][l], S->ft + l * mw, m->fit[l], dh, dz, out,
                 grad ? grad + m->fit_w[ti][l] : NULL, grad ? grad + m->fit_b[ti][l] : NULL, gscale);
    if (l > 0) { double* tswap = dh; dh = dhp; dhp = tswap; }
  }
  /* dE/dT[a,k] = sum_b gD[a,b] T[b,k] + [a < m2] sum_a' gD[a',a] T[a',k] */
  for (int a = 0; a < m->m1; a++)
    for (int k = 0; k < 4; k++) {
      double acc = 0.0;
      for (int b = 0; b < m->m2; b++) acc += S->gD[a * m->m2 + b] * S->T[b * 4 + k];
      if (a < m->m2)
        for (int a2 = 0; a2 < m->m1; a2++) acc += S->gD[a2 * m->m2 + a] * S->T[a2 * 4 + k];
      S->gT[a * 4 + k] = acc;
    }

  /* per neighbour row: dE/dG = (1/nm) gT R~^T, direct dE/dR~ = (1/nm) gT^T G,
   * back-propagate through the embedding net to dE/ds, then
   * g_ij[alpha] = sum_k n_ij[k] dR~[k]/dd[alpha] with n = dE/dR~ + dE/ds e_0 */
  for (int tj = 0; tj < m->ntypes; tj++) {
    for (int q = m->sec[tj]; q < m->sec[tj + 1]; q++) {
      double* g = g_rows + 3 * q;
      double* ndq = S->nd_ + 4 * q;
      if (row[q] < 0) {
        g[0] = g[1] = g[2] = 0.0;
        ndq[0] = ndq[1] = ndq[2] = ndq[3] = 0.0;
        continue;
      }
      const double* R = S->R + 4 * q;
      const double* act = S->act + (int64_t)q * sumw;
      const double* tac = S->tact + (int64_t)q * sumw;
      double nd[4];
      for (int k = 0; k < 4; k++) {
        double acc = 0.0;
        for (int a = 0; a < m->m1; a++) acc += S->gT[a * 4 + k] * act[goff + a];
        nd[k] = acc * inv_nm;
      }
      double* dg = S->tmp1;
      double* dz2 = S->tmp2;
      double* dhp2 = S->tmp3;
      for (int a = 0; a < m->m1; a++) {
        double acc = 0.0;
        for (int k = 0; k < 4; k++) acc += S->gT[a * 4 + k] * R[k];
        dg[a] = acc * inv_nm;
      }
      int off = goff;
      double ds = 0.0;
      if (tab->table) {
        /* dE/dx = sum_a dE/dG_a dG_a/dx */
        for (int a = 0; a < m->m1; a++) ds += dg[a] * tac[goff + a];
      }
      for (int l = tab->table ? -1 : m->nemb - 1; l >= 0; l--) {
        int win = l > 0 ? m->emb[l - 1] : 1;
        double in0 = R[0];
        const double* hin = l > 0 ? act + off - win : &in0;
        double* out = l > 0 ? dhp2 : &ds;
        or_dense_bwd(hin, win, P + m->emb_w[ti][tj][l], tac + off, m->emb[l], dg, dz2, out,
                     grad ? grad + m->emb_w[ti][tj][l] : NULL, grad ? grad + m->emb_b[ti][tj][l] : NULL,
                     gscale);
        if (l > 0) { double* tswap = dg; dg = dhp2; dhp2 = tswap; off -= win; }
      }
      nd[0] += ds;
      for (int k = 0; k < 4; k++) ndq[k] = nd[k];
      const double* dR = S->dRd + 12 * q;
      for (int a = 0; a < 3; a++) {
        double acc = 0.0;
        for (int k = 0; k < 4; k++) acc += nd[k] * dR[k * 3 + a];
        g[a] = acc;
      }
    }
  }
  if (dbg) {
    if (dbg->R) memcpy(dbg->R, S->R, sizeof(double) * nm * 4);
    if (dbg->T) memcpy(dbg->T, S->T, sizeof(double) * m->m1 * 4);
    if (dbg->D) memcpy(dbg->D, S->D, sizeof(double) * m->nd);
    if (dbg->gD) memcpy(dbg->gD, S->gD, sizeof(double) * m->nd);
    if (dbg->gT) memcpy(dbg->gT, S->gT, sizeof(double) * m->m1 * 4);
    if (dbg->nd) memcpy(dbg->nd, S->nd_, sizeof(double) * nm * 4);
  }
  return Ei;
}

/* Energy, forces and virial of one frame.
 *   rows[0..nrows) are the centre atoms evaluated (NULL: all n atoms), with
 *   their neighbour rows in nlist [nrows, nm].  Ei[r] receives E_{rows[r]}.
 *   E = sum_r Ei[r] (in row order).  F [n,3] (zeroed here) receives
 *   F_i += g_ij, F_j -= g_ij over the evaluated rows, W[9] (row-major a,b)
 *   receives -sum d_a g_b.  grad (nullable) receives gscale * dE/dtheta.
 *   Debug arrays (nullable): R [nrows,nm,4], T [nrows,m1,4], D [nrows,nd],
 *   gD [nrows,nd], gT [nrows,m1,4], netd [nrows,nm,4].                      */
int or_compute(int64_t n, const double* x, const int32_t* type, const double* h, const int32_t* idesc,
               const double* ddesc, const double* params, const int64_t* rows, int64_t nrows,
               const int32_t* nlist, double* E, double* Ei, double* F, double* W, double* grad, double gscale,
               double* dR, double* dT, double* dD, double* dgD, double* dgT, double* dnd, const double* table,
               double tab_x1, double tab_x2, double tab_h, int64_t* nclip) {
  or_model m;
  if (or_parse(idesc, ddesc, &m)) return -1;
  or_tab tab;
  memset(&tab, 0, sizeof(tab));
  if (table) {
    if (grad || !(tab_h > 0.0) || !(tab_x1 > 0.0)) return -1;  /* the tabulated model has no parameter gradient */
    tab.table = table;
    or_grid_make(tab_x1, tab_x2, tab_h, &tab.g);
  }
  int64_t clipped = 0;
  for (int64_t i = 0; i < n; i++)
    if (type[i] < 0 || type[i] >= m.ntypes) return -1;
  double* g_all = (double*)malloc(sizeof(double) * (size_t)(nrows > 0 ? nrows : 1) * m.nm * 3);
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  double* gbuf = NULL;
  if (grad) gbuf = (double*)calloc((size_t)nthreads * (size_t)m.nparams, sizeof(double));
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    or_scratch S;
    or_scratch_alloc(&m, &S);
#pragma omp for schedule(dynamic, 8)
    for (int64_t r = 0; r < nrows; r++) {
      int64_t i = rows ? rows[r] : r;
      or_dbg dbg = {dR ? dR + r * m.nm * 4 : NULL, dT ? dT + r * m.m1 * 4 : NULL, dD ? dD + r * m.nd : NULL,
                    dgD ? dgD + r * m.nd : NULL, dgT ? dgT + r * m.m1 * 4 : NULL, dnd ? dnd + r * m.nm * 4 : NULL};
      int64_t nc = 0;
      Ei[r] = or_atom(i, x, type, h, &m, params, nlist + r * m.nm, &S, g_all + r * m.nm * 3,
                      grad ? gbuf + (size_t)tid * m.nparams : NULL, gscale, &dbg, &tab, &nc);
      if (nc) {
#pragma omp atomic
        clipped += nc;
      }
    }
    or_scratch_free(&S);
  }
  double e = 0.0;
  for (int64_t r = 0; r < nrows; r++) e += Ei[r];
  *E = e;
  if (F) memset(F, 0, sizeof(double) * 3 * n);
  for (int k = 0; k < 9; k++) W[k] = 0.0;
  for (int64_t r = 0; r < nrows; r++) {
    int64_t i = rows ? rows[r] : r;
    const int32_t* row = nlist + r * m.nm;
    for (int q = 0; q < m.nm; q++) {
      if (row[q] < 0) continue;
      int64_t j = row[q] / 27;
      int sc = row[q] % 27;
      int sx = sc % 3 - 1, sy = (sc / 3) % 3 - 1, sz = sc / 9 - 1;
      const double* g = g_all + (r * m.nm + q) * 3;
      double d[3];
      for (int a = 0; a < 3; a++) {
        double sh = (double)sx * h[0 + a] + (double)sy * h[3 + a] + (double)sz * h[6 + a];
        d[a] = (x[3 * j + a] - x[3 * i + a]) + sh;
      }
      if (F)
        for (int a = 0; a < 3; a++) {
          F[3 * i + a] += g[a];
          F[3 * j + a] -= g[a];
        }
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) W[3 * a + b] -= d[a] * g[b];
    }
  }
  if (grad) {
    for (int64_t p = 0; p < m.nparams; p++) {
      double acc = 0.0;
      for (int t = 0; t < nthreads; t++) acc += gbuf[(size_t)t * m.nparams + p];
      grad[p] += acc;
    }
    free(gbuf);
  }
  free(g_all);
  if (nclip) *nclip = clipped;
  return 0;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
