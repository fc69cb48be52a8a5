/*
 * Serial FP64 oracle for the DPP-PMRF EM optimisation (Lessley et al., LDAV 2018,
 * arXiv:1809.05018).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  The HIP product
 * path shares no code, header, table or helper with it, and never calls it.
 *
 * Everything is plain serial C in double precision, built with
 * -ffp-contract=off and without fast-math, so each expression rounds exactly as
 * written.  Each function names the passage of the paper it follows; where the
 * paper is silent or garbled the reading taken is stated at the function.
 *
 *   or_build_k      maximal cliques (Sec. 3.2.1), k-neighbourhoods (Sec. 3.1; for
 *                   k = 1 the four construction steps of Sec. 3.2.2), in-hood
 *                   adjacency, owner element per vertex (or_build: k = 1)
 *   or_replicate    replication of the neighbourhood array by label (Sec. 3.2.2,
 *                   "Replicate Neighborhoods By Label" and its worked example)
 *   or_gather       gathered per-replica labels and intensities (same example)
 *   or_mstep        parameter update (Sec. 3.2.2, "Update Parameters")
 *   or_em_step      one EM iteration: energies, per-vertex minimum, neighbourhood
 *                   sums, label update under a scatter rule, parameter update
 *                   (Alg. 2, EM loop)
 *   or_hood_converged  convergence test over the last W sums (Sec. 3.2.2,
 *                   "MAP Convergence Check" / "EM Convergence Check")
 *   or_em_run       the fixed-count EM loop with convergence bookkeeping
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long long i64;

typedef struct {
  int n;
  int *row_ptr, *col_idx;
  /* maximal cliques C_0..C_{H-1}: each ascending, list in lexicographic order */
  int H;
  i64 *clq_ptr;
  int *clq_vid;
  /* k-neighbourhoods: hood_h = sorted(C_h u {u within k edges of C_h}); M elements in total */
  i64 *hood_ptr;
  int *hood_vid;
  i64 M;
  /* in-hood adjacency of element e=(h,j): positions j' with hood_h[j'] in N(v) */
  i64 *adj_ptr;
  int *adj_loc;
  i64 A;
  /* owner[v]: element index of v inside the first clique (lowest h) holding v */
  i64 *owner;
  int max_hood;
} or_graph;

/* ---------------------------------------------------------------- helpers */

static int is_neighbor(const or_graph *g, int v, int u) {
  int lo = g->row_ptr[v], hi = g->row_ptr[v + 1] - 1;
  while (lo <= hi) {
    int mid = lo + (hi - lo) / 2;
    int c = g->col_idx[mid];
    if (c == u) return 1;
    if (c < u) lo = mid + 1; else hi = mid - 1;
  }
  return 0;
}

typedef struct { int *a; i64 n, cap; } ivec;

static void iv_push(ivec *v, int x) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 64;
    v->a = (int *)realloc(v->a, (size_t)v->cap * sizeof(int));
  }
  v->a[v->n++] = x;
}

typedef struct { i64 *a; i64 n, cap; } lvec;

static void lv_push(lvec *v, i64 x) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 64;
    v->a = (i64 *)realloc(v->a, (size_t)v->cap * sizeof(i64));
  }
  v->a[v->n++] = x;
}

static int cmp_int(const void *x, const void *y) {
  int a = *(const int *)x, b = *(const int *)y;
  return (a > b) - (a < b);
}

/* ------------------------------------------- maximal clique enumeration */
/*
 * Plain Bron-Kerbosch without pivoting: R grows by one candidate at a time,
 * candidates already explored move to the excluded set X, and R is reported
 * when nothing can extend it (P and X empty).  The outer loop starts one search
 * per vertex v with candidates = later neighbours and excluded = earlier ones,
 * which is exactly the first level of the textbook recursion in vertex order.
 * An isolated vertex is the clique {v}.  A branch stops early when some
 * excluded vertex is adjacent to every candidate: every clique the branch could
 * report would then extend by that vertex, so none of them is maximal.
 */

typedef struct { ivec members; lvec ptr; } clique_list;

static void bk(const or_graph *g, int *R, int r, const int *P, int np, const int *X, int nx,
               clique_list *out) {
  for (int i = 0; i < nx; ++i) {
    int all = 1;
    for (int k = 0; k < np && all; ++k) all = is_neighbor(g, X[i], P[k]);
    if (all) return;
  }
  if (np == 0 && nx == 0) {
    if (out->ptr.n == 0) lv_push(&out->ptr, 0);
    int *tmp = (int *)malloc((size_t)r * sizeof(int));
    memcpy(tmp, R, (size_t)r * sizeof(int));
    qsort(tmp, (size_t)r, sizeof(int), cmp_int);
    for (int i = 0; i < r; ++i) iv_push(&out->members, tmp[i]);
    lv_push(&out->ptr, out->members.n);
    free(tmp);
    return;
  }
  int *Pl = (int *)malloc((size_t)(np + 1) * sizeof(int));
  int *Xl = (int *)malloc((size_t)(nx + np + 1) * sizeof(int));
  memcpy(Pl, P, (size_t)np * sizeof(int));
  memcpy(Xl, X, (size_t)nx * sizeof(int));
  int pn = np, xn = nx;
  int *P2 = (int *)malloc((size_t)(np + 1) * sizeof(int));
  int *X2 = (int *)malloc((size_t)(nx + np + 1) * sizeof(int));
  while (pn > 0) {
    int u = Pl[0];
    int p2 = 0, x2 = 0;
    for (int i = 1; i < pn; ++i) if (is_neighbor(g, u, Pl[i])) P2[p2++] = Pl[i];
    for (int i = 0; i < xn; ++i) if (is_neighbor(g, u, Xl[i])) X2[x2++] = Xl[i];
    R[r] = u;
    bk(g, R, r + 1, P2, p2, X2, x2, out);
    /* move u from P to X */
    memmove(Pl, Pl + 1, (size_t)(pn - 1) * sizeof(int));
    pn--;
    Xl[xn++] = u;
  }
  free(Pl); free(Xl); free(P2); free(X2);
}

static const i64 *g_cmp_ptr;
static const int *g_cmp_vid;

static int cmp_clique(const void *x, const void *y) {
  i64 a = *(const i64 *)x, b = *(const i64 *)y;
  i64 la = g_cmp_ptr[a + 1] - g_cmp_ptr[a], lb = g_cmp_ptr[b + 1] - g_cmp_ptr[b];
  const int *pa = g_cmp_vid + g_cmp_ptr[a], *pb = g_cmp_vid + g_cmp_ptr[b];
  i64 m = la < lb ? la : lb;
  for (i64 i = 0; i < m; ++i) {
    if (pa[i] != pb[i]) return pa[i] < pb[i] ? -1 : 1;
  }
  return (la > lb) - (la < lb);
}

/* ------------------------------------------------------------------ build */

void or_free(or_graph *g);

/* Returns NULL if the CSR is not a simple undirected graph with sorted rows,
   or k < 1. */
or_graph *or_build_k(int n, const int *row_ptr, const int *col_idx, int k) {
  if (n < 0 || !row_ptr || k < 1) return NULL;
  if (row_ptr[0] != 0) return NULL;
  for (int v = 0; v < n; ++v) {
    if (row_ptr[v + 1] < row_ptr[v]) return NULL;
    for (int k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
      int u = col_idx[k];
      if (u < 0 || u >= n || u == v) return NULL;
      if (k > row_ptr[v] && col_idx[k - 1] >= u) return NULL;
    }
  }
  or_graph *g = (or_graph *)calloc(1, sizeof(or_graph));
  g->n = n;
  g->row_ptr = (int *)malloc((size_t)(n + 1) * sizeof(int));
  memcpy(g->row_ptr, row_ptr, (size_t)(n + 1) * sizeof(int));
  int nnz = row_ptr[n];
  g->col_idx = (int *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int));
  if (nnz) memcpy(g->col_idx, col_idx, (size_t)nnz * sizeof(int));
  for (int v = 0; v < n; ++v)
    for (int k = row_ptr[v]; k < row_ptr[v + 1]; ++k)
      if (!is_neighbor(g, col_idx[k], v)) { or_free(g); return NULL; }

  /* B1: maximal cliques */
  clique_list cl = {{0}, {0}};
  int *R = (int *)malloc((size_t)(n + 1) * sizeof(int));
  int maxdeg = 0;
  for (int v = 0; v < n; ++v) {
    int d = row_ptr[v + 1] - row_ptr[v];
    if (d > maxdeg) maxdeg = d;
  }
  int *P = (int *)malloc((size_t)(maxdeg + 1) * sizeof(int));
  int *X = (int *)malloc((size_t)(maxdeg + 1) * sizeof(int));
  for (int v = 0; v < n; ++v) {
    int np = 0, nx = 0;
    for (int k = row_ptr[v]; k < row_ptr[v + 1]; ++k) {
      int u = col_idx[k];
      if (u > v) P[np++] = u; else X[nx++] = u;
    }
    R[0] = v;
    bk(g, R, 1, P, np, X, nx, &cl);
  }
  free(R); free(P); free(X);
  i64 H = cl.ptr.n > 0 ? cl.ptr.n - 1 : 0;
  i64 *order = (i64 *)malloc((size_t)(H > 0 ? H : 1) * sizeof(i64));
  for (i64 h = 0; h < H; ++h) order[h] = h;
  g_cmp_ptr = cl.ptr.a; g_cmp_vid = cl.members.a;
  qsort(order, (size_t)H, sizeof(i64), cmp_clique);
  g->H = (int)H;
  g->clq_ptr = (i64 *)malloc((size_t)(H + 1) * sizeof(i64));
  g->clq_vid = (int *)malloc((size_t)(cl.members.n > 0 ? cl.members.n : 1) * sizeof(int));
  g->clq_ptr[0] = 0;
  for (i64 h = 0; h < H; ++h) {
    i64 src = order[h];
    i64 len = cl.ptr.a[src + 1] - cl.ptr.a[src];
    memcpy(g->clq_vid + g->clq_ptr[h], cl.members.a + cl.ptr.a[src], (size_t)len * sizeof(int));
    g->clq_ptr[h + 1] = g->clq_ptr[h] + len;
  }
  free(order); free(cl.members.a); free(cl.ptr.a);

  /* B2: hood_h = the clique's members and every vertex within k edges of one
     of them (Sec. 3.1), ascending: a breadth-first search of depth k from the
     members, each vertex taken once (mark[u] = h + 1 once u is in hood h) */
  ivec hv = {0};
  ivec front = {0};
  int *mark = (int *)calloc((size_t)(n > 0 ? n : 1), sizeof(int));
  g->hood_ptr = (i64 *)malloc((size_t)(H + 1) * sizeof(i64));
  g->hood_ptr[0] = 0;
  g->max_hood = 0;
  for (i64 h = 0; h < H; ++h) {
    i64 start = hv.n;
    front.n = 0;
    for (i64 q = g->clq_ptr[h]; q < g->clq_ptr[h + 1]; ++q) {
      int c = g->clq_vid[q];
      mark[c] = (int)h + 1;
      iv_push(&hv, c);
      iv_push(&front, c);
    }
    i64 fb = 0;
    for (int depth = 1; depth <= k; ++depth) {
      i64 fe = front.n;
      for (i64 f = fb; f < fe; ++f) {
        int u = front.a[f];
        for (int q = row_ptr[u]; q < row_ptr[u + 1]; ++q) {
          int w = col_idx[q];
          if (mark[w] == (int)h + 1) continue;
          mark[w] = (int)h + 1;
          iv_push(&hv, w);
          iv_push(&front, w);
        }
      }
      fb = fe;
    }
    qsort(hv.a + start, (size_t)(hv.n - start), sizeof(int), cmp_int);
    g->hood_ptr[h + 1] = hv.n;
    if (hv.n - start > g->max_hood) g->max_hood = (int)(hv.n - start);
  }
  free(mark);
  free(front.a);
  g->M = hv.n;
  g->hood_vid = hv.a ? hv.a : (int *)malloc(sizeof(int));

  /* B3: in-hood neighbours of each element, by direct adjacency lookup */
  ivec al = {0};
  g->adj_ptr = (i64 *)malloc((size_t)(g->M + 1) * sizeof(i64));
  g->adj_ptr[0] = 0;
  for (i64 h = 0; h < H; ++h) {
    i64 o = g->hood_ptr[h], s = g->hood_ptr[h + 1] - o;
    for (i64 j = 0; j < s; ++j) {
      int v = g->hood_vid[o + j];
      for (i64 jj = 0; jj < s; ++jj)
        if (is_neighbor(g, v, g->hood_vid[o + jj])) iv_push(&al, (int)jj);
      g->adj_ptr[o + j + 1] = al.n;
    }
  }
  g->A = al.n;
  g->adj_loc = al.a ? al.a : (int *)malloc(sizeof(int));

  /* B4: owner element of each vertex = its place in the lowest clique holding it */
  g->owner = (i64 *)malloc((size_t)(n > 0 ? n : 1) * sizeof(i64));
  for (int v = 0; v < n; ++v) g->owner[v] = -1;
  for (i64 h = 0; h < H; ++h) {
    for (i64 k = g->clq_ptr[h]; k < g->clq_ptr[h + 1]; ++k) {
      int v = g->clq_vid[k];
      if (g->owner[v] >= 0) continue;
      for (i64 e = g->hood_ptr[h]; e < g->hood_ptr[h + 1]; ++e)
        if (g->hood_vid[e] == v) { g->owner[v] = e; break; }
    }
  }
  return g;
}

or_graph *or_build(int n, const int *row_ptr, const int *col_idx) { return or_build_k(n, row_ptr, col_idx, 1); }

void or_free(or_graph *g) {
  if (!g) return;
  free(g->row_ptr); free(g->col_idx); free(g->clq_ptr); free(g->clq_vid);
  free(g->hood_ptr); free(g->hood_vid); free(g->adj_ptr); free(g->adj_loc); free(g->owner);
  free(g);
}

/* info: n, H, M, A, max_hood, clique members */
void or_info(const or_graph *g, i64 *out) {
  out[0] = g->n; out[1] = g->H; out[2] = g->M; out[3] = g->A; out[4] = g->max_hood;
  out[5] = g->H ? g->clq_ptr[g->H] : 0;
}

void or_get_cliques(const or_graph *g, i64 *ptr, int *vid) {
  memcpy(ptr, g->clq_ptr, (size_t)(g->H + 1) * sizeof(i64));
  if (g->H) memcpy(vid, g->clq_vid, (size_t)g->clq_ptr[g->H] * sizeof(int));
}

void or_get_hoods(const or_graph *g, i64 *ptr, int *vid) {
  memcpy(ptr, g->hood_ptr, (size_t)(g->H + 1) * sizeof(i64));
  if (g->M) memcpy(vid, g->hood_vid, (size_t)g->M * sizeof(int));
}

void or_get_adjacency(const or_graph *g, i64 *adj_ptr, int *adj_loc) {
  memcpy(adj_ptr, g->adj_ptr, (size_t)(g->M + 1) * sizeof(i64));
  if (g->A) memcpy(adj_loc, g->adj_loc, (size_t)g->A * sizeof(int));
}

void or_get_owner(const or_graph *g, i64 *owner) {
  if (g->n) memcpy(owner, g->owner, (size_t)g->n * sizeof(i64));
}

/* ------------------------------------------------------- replicate, gather */
/*
 * Sec. 3.2.2 "Replicate Neighborhoods By Label": each neighbourhood is copied
 * once per label; within the copy for label l the members keep their order.
 * testLabel = l of the copy, oldIndex = index of the member in the flat
 * neighbourhood array, hoodId = neighbourhood id.  Output length L * M.
 */
void or_replicate(int H, const i64 *hood_ptr, int L, int *test_label, i64 *old_index, int *hood_id) {
  i64 k = 0;
  for (int h = 0; h < H; ++h)
    for (int l = 0; l < L; ++l)
      for (i64 e = hood_ptr[h]; e < hood_ptr[h + 1]; ++e) {
        test_label[k] = l;
        old_index[k] = e;
        hood_id[k] = h;
        ++k;
      }
}

/* Sec. 3.2.2 "Compute Energy Function": per replica, gather the current label
 * and intensity of the vertex through oldIndex into the neighbourhood array. */
void or_gather(i64 K, const i64 *old_index, const int *hood_vid, const int *x, const double *y,
               int *vert_label, double *vert_mu) {
  for (i64 k = 0; k < K; ++k) {
    int v = hood_vid[old_index[k]];
    vert_label[k] = x[v];
    vert_mu[k] = y[v];
  }
}

/* ------------------------------------------------------------------ M-step */
/*
 * Sec. 3.2.2 "Update Parameters" (text partly garbled).  Reading taken: hard
 * assignment over vertices, each vertex once, using the updated labels;
 * mu_l is the mean of y over vertices labelled l, sigma_l the population
 * standard deviation about that mean (two passes), floored at sigma_min.
 * A label with no vertices keeps its previous mu and sigma.
 */
int or_mstep(int n, const double *y, int L, const int *x, const double *mu_in, const double *sigma_in,
             double sigma_min, double *mu_out, double *sigma_out) {
  for (int l = 0; l < L; ++l) {
    i64 cnt = 0;
    double sum = 0.0;
    for (int v = 0; v < n; ++v)
      if (x[v] == l) { cnt++; sum = sum + y[v]; }
    if (cnt == 0) { mu_out[l] = mu_in[l]; sigma_out[l] = sigma_in[l]; continue; }
    double mu = sum / (double)cnt;
    double ss = 0.0;
    for (int v = 0; v < n; ++v)
      if (x[v] == l) { double d = y[v] - mu; ss = ss + d * d; }
    double sigma = sqrt(ss / (double)cnt);
    if (sigma < sigma_min) sigma = sigma_min;
    mu_out[l] = mu;
    sigma_out[l] = sigma;
  }
  return 0;
}

/* ---------------------------------------------------------------- E-step */
/*
 * One EM iteration (Alg. 2 loop body, Sec. 3.2.2 steps 2-4), from state
 * (x_in, mu_in, sigma_in):
 *
 *  energy of element (h,j) = vertex v under label l (MAP criterion of Sec. 2.1:
 *  likelihood energy plus prior energy; the concrete forms are a reading):
 *     data(v,l) = (y_v - mu_l)(y_v - mu_l) / (2 sigma_l sigma_l) + ln sigma_l
 *                 (Gaussian negative log-likelihood without the constant,
 *                 evaluated per element in exactly this order)
 *     E(h,j,l)  = data(v,l) + beta * #{in-hood neighbours u of v : x_u != l}
 *                 (Potts prior restricted to the neighbourhood)
 *  m(h,j) = min over l of E, a(h,j) = lowest l attaining it,
 *  gap(h,j) = second smallest E - m  ("Compute Minimum Vertex and Label Energies")
 *  S_h = sum over j ascending of m(h,j); T = sum over h ascending of S_h
 *                                      ("Compute Neighborhood Energy Sums")
 *  x_out[v] = a(e_v)                   ("Update Output Labels": every element
 *                                       scatters its argmin to its vertex; the
 *                                       rule picks the element e_v whose write
 *                                       stands, a reading of the paper's
 *                                       write conflicts)
 *     rule 0 (owner): e_v = owner(v), v's element in the first clique holding v
 *     rule 1 (last):  e_v = the last element holding v in the hood-major array
 *                     (the outcome of a serial Scatter)
 *     rule 2 (min):   e_v = the element holding v with the smallest m, the
 *                     first such element on ties
 *  near_ties = #{v : gap(e_v) < tie_eps, or (rule 2) another element e of v
 *               has m(e) - m(e_v) < tie_eps and a(e) != a(e_v)}
 *  (mu_out, sigma_out) = or_mstep(x_out) ("Update Parameters")
 *
 * m, a, gap may be NULL; otherwise they receive the per-element values.
 */
int or_em_step(const or_graph *g, const double *y, int L, double beta, int rule, const int *x_in,
               const double *mu_in, const double *sigma_in, double sigma_min, double tie_eps,
               int *x_out, double *mu_out, double *sigma_out, double *S, double *T, i64 *near_ties,
               double *m_out, int *a_out, double *gap_out) {
  if (L < 2 || L > 16 || rule < 0 || rule > 2) return -1;
  double E[16];
  double *gap_elem = (double *)malloc((size_t)(g->M > 0 ? g->M : 1) * sizeof(double));
  double *m_elem = (double *)malloc((size_t)(g->M > 0 ? g->M : 1) * sizeof(double));
  int *a_elem = (int *)malloc((size_t)(g->M > 0 ? g->M : 1) * sizeof(int));
  double total = 0.0;
  for (int h = 0; h < g->H; ++h) {
    double sh = 0.0;
    for (i64 e = g->hood_ptr[h]; e < g->hood_ptr[h + 1]; ++e) {
      int v = g->hood_vid[e];
      for (int l = 0; l < L; ++l) {
        int c = 0;
        for (i64 k = g->adj_ptr[e]; k < g->adj_ptr[e + 1]; ++k) {
          int u = g->hood_vid[g->hood_ptr[h] + g->adj_loc[k]];
          if (x_in[u] != l) c++;
        }
        double d = y[v] - mu_in[l];
        double data = (d * d) / (2.0 * sigma_in[l] * sigma_in[l]) + log(sigma_in[l]);
        E[l] = data + beta * (double)c;
      }
      double m = E[0];
      int a = 0;
      for (int l = 1; l < L; ++l)
        if (E[l] < m) { m = E[l]; a = l; }
      double second = INFINITY;
      for (int l = 0; l < L; ++l)
        if (l != a && E[l] < second) second = E[l];
      a_elem[e] = a;
      m_elem[e] = m;
      gap_elem[e] = second - m;
      if (m_out) m_out[e] = m;
      if (a_out) a_out[e] = a;
      if (gap_out) gap_out[e] = second - m;
      sh = sh + m;
    }
    S[h] = sh;
    total = total + sh;
  }
  *T = total;
  /* the element whose write stands, per vertex */
  i64 *pick = (i64 *)malloc((size_t)(g->n > 0 ? g->n : 1) * sizeof(i64));
  for (int v = 0; v < g->n; ++v) pick[v] = rule == 0 ? g->owner[v] : -1;
  if (rule == 1)
    for (i64 e = 0; e < g->M; ++e) pick[g->hood_vid[e]] = e;
  if (rule == 2)
    for (i64 e = 0; e < g->M; ++e) {
      int v = g->hood_vid[e];
      if (pick[v] < 0 || m_elem[e] < m_elem[pick[v]]) pick[v] = e;
    }
  char *tie = (char *)calloc((size_t)(g->n > 0 ? g->n : 1), 1);
  for (int v = 0; v < g->n; ++v) {
    x_out[v] = a_elem[pick[v]];
    if (gap_elem[pick[v]] < tie_eps) tie[v] = 1;
  }
  if (rule == 2)
    for (i64 e = 0; e < g->M; ++e) {
      int v = g->hood_vid[e];
      i64 c = pick[v];
      if (e != c && m_elem[e] - m_elem[c] < tie_eps && a_elem[e] != a_elem[c]) tie[v] = 1;
    }
  i64 ties = 0;
  for (int v = 0; v < g->n; ++v) ties += tie[v];
  *near_ties = ties;
  free(tie);
  free(pick);
  free(gap_elem);
  free(m_elem);
  free(a_elem);
  return or_mstep(g->n, y, L, x_out, mu_in, sigma_in, sigma_min, mu_out, sigma_out);
}

/* -------------------------------------------------------------- convergence */
/*
 * Sec. 3.2.2 "MAP Convergence Check": a sum is converged at iteration t when its
 * change against each of the previous W iterations is below tol (absolute).
 * hist holds W+1 values, oldest first, newest (iteration t) last.  Fewer than
 * W earlier values (t < W) never count as converged.
 */
int or_hood_converged(int W, double tol, const double *hist) {
  double now = hist[W];
  for (int w = 1; w <= W; ++w)
    if (!(fabs(now - hist[W - w]) < tol)) return 0;
  return 1;
}

/*
 * The EM loop (Alg. 2) under scatter rule `rule` (or_em_step): a fixed number of iterations T (Sec. 3.2.2, last
 * paragraph), each one or_em_step.  Per iteration it records the energy total
 * T_t (computed with the incoming state), the near-tie count and the number of
 * neighbourhoods not yet converged.  summary = {iterations run, first iteration
 * at which every neighbourhood sum had converged (or -1), first iteration at
 * which the total had converged (or -1), total near ties}.  With early_exit the
 * loop stops after the iteration at which every neighbourhood converged.  With
 * init_from_labels the starting parameters are or_mstep of the starting labels.
 */
int or_em_run(const or_graph *g, const double *y, int L, double beta, int rule, int iters, int W, double tol,
              int early_exit, double sigma_min, double tie_eps, int init_from_labels, int *x,
              double *mu, double *sigma, double *trace, double *S_last, i64 *near_ties,
              i64 *nonconv, i64 *summary) {
  if (L < 2 || L > 16 || iters < 0 || W < 1 || rule < 0 || rule > 2) return -1;
  int n = g->n, H = g->H;
  if (init_from_labels) {
    double m2[16], s2[16];
    or_mstep(n, y, L, x, mu, sigma, sigma_min, m2, s2);
    memcpy(mu, m2, (size_t)L * sizeof(double));
    memcpy(sigma, s2, (size_t)L * sizeof(double));
  }
  double *hist = (double *)malloc((size_t)(W + 1) * (size_t)(H > 0 ? H : 1) * sizeof(double));
  double *Thist = (double *)malloc((size_t)(iters > 0 ? iters : 1) * sizeof(double));
  double *S = (double *)malloc((size_t)(H > 0 ? H : 1) * sizeof(double));
  int *xn = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
  double *hw = (double *)malloc((size_t)(W + 1) * sizeof(double));
  double mu2[16], s2[16];
  summary[0] = 0; summary[1] = -1; summary[2] = -1; summary[3] = 0;
  for (int t = 0; t < iters; ++t) {
    double Tt;
    i64 ties;
    or_em_step(g, y, L, beta, rule, x, mu, sigma, sigma_min, tie_eps, xn, mu2, s2, S, &Tt, &ties,
               NULL, NULL, NULL);
    trace[t] = Tt;
    Thist[t] = Tt;
    near_ties[t] = ties;
    summary[3] += ties;
    /* history slot of iteration t is t mod (W+1) */
    int slot = t % (W + 1);
    for (int h = 0; h < H; ++h) hist[(size_t)slot * H + h] = S[h];
    i64 nc = 0;
    for (int h = 0; h < H; ++h) {
      int ok = 0;
      if (t >= W) {
        for (int k = 0; k <= W; ++k) hw[k] = hist[(size_t)((t - W + k) % (W + 1)) * H + h];
        ok = or_hood_converged(W, tol, hw);
      }
      if (!ok) nc++;
    }
    nonconv[t] = nc;
    if (nc == 0 && t >= W && summary[1] < 0) summary[1] = t;
    if (t >= W && summary[2] < 0) {
      for (int k = 0; k <= W; ++k) hw[k] = Thist[t - W + k];
      if (or_hood_converged(W, tol, hw)) summary[2] = t;
    }
    memcpy(x, xn, (size_t)n * sizeof(int));
    memcpy(mu, mu2, (size_t)L * sizeof(double));
    memcpy(sigma, s2, (size_t)L * sizeof(double));
    summary[0] = t + 1;
    if (S_last) memcpy(S_last, S, (size_t)H * sizeof(double));
    if (early_exit && nc == 0 && t >= W) break;
  }
  free(hist); free(Thist); free(S); free(xn); free(hw);
  return 0;
}
