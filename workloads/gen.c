/*
 * Seeded input preparation for the combined-kernel workloads: octree build,
 * bucket lists from a Barnes-Hut walk, and Lennard-Jones cell-pair tasks.
 *
 * This is input generation only.  It builds the work requests (a bucket of
 * target particles with its interaction lists, or a pair of cells) that the
 * runtime combines, the way the application side of the paper produces them
 * on the host (Sec. 4.1: buckets sharing one set of interaction lists; the tree
 * walk ran on the CPU cores, Sec. 4.6; Sec. 4.2: compute objects per pair of
 * patches).  It evaluates no forces.
 *
 * Node multipole records (mass, centre of mass, raw second moment) are tree
 * data written here in FP64 and rounded to FP32 once; both the force path and
 * the checker consume the rounded records.
 *
 * Conventions (stated because the paper gives none):
 *  - root cube: centred on the bounding box of the FP32 positions, side =
 *    max extent * (1 + 2^-20) (side 1 when the extent is 0);
 *  - octant index = (x >= cx) | (y >= cy) << 1 | (z >= cz) << 2; a node is
 *    split while it holds more than `bucket` particles and depth < WL_MAXDEPTH;
 *    empty octants get no node; children are visited in ascending octant index;
 *  - ids are relabelled in depth-first leaf order, stable in input order, so
 *    every node covers one contiguous id range; buckets are the leaves in that
 *    order;
 *  - a bucket B accepts node N iff theta > 0, N's id range is disjoint from
 *    B's, and side(N) < theta * dist(com(N), box(B)) strictly, where box(B) is
 *    the tight bounding box of B's particles; otherwise a leaf goes to the
 *    direct list as one id range and an internal node is opened.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define WL_MAXDEPTH 48

typedef struct {
  int32_t first, count;      /* id range in relabelled order */
  int32_t child0, nchild;    /* children: child[child0 .. child0+nchild) in the tree's child list */
  int32_t depth, leaf;
  double cx, cy, cz, side;   /* geometric cube */
  double M, com[3], S[6];    /* moments: S = sum m (x-com)(x-com)^T, order xx yy zz xy xz yz */
} wl_node;

typedef struct {
  int64_t n;
  int32_t bucket;
  int32_t nnodes, cap;
  wl_node* nodes;
  int32_t* child;            /* child index lists, child[node.child0 + k] */
  int32_t nchildren, cchild;
  int32_t* perm;             /* perm[new id] = input index */
  float* rec;                /* relabelled records (x, y, z, m), 4 floats each */
} wl_tree;

static int32_t push_node(wl_tree* t) {
  if (t->nnodes == t->cap) {
    t->cap = t->cap ? 2 * t->cap : 1024;
    t->nodes = (wl_node*)realloc(t->nodes, sizeof(wl_node) * (size_t)t->cap);
  }
  memset(&t->nodes[t->nnodes], 0, sizeof(wl_node));
  return t->nnodes++;
}

static int32_t push_children(wl_tree* t, int32_t k) {
  if (t->nchildren + k > t->cchild) {
    while (t->nchildren + k > t->cchild) t->cchild = t->cchild ? 2 * t->cchild : 1024;
    t->child = (int32_t*)realloc(t->child, sizeof(int32_t) * (size_t)t->cchild);
  }
  int32_t at = t->nchildren;
  t->nchildren += k;
  return at;
}

/* Recursive build over the index range idx[first, first+count) (input indices). */
static int32_t build_rec(wl_tree* t, const float* in, int32_t* idx, int32_t* tmp, int32_t first, int32_t count,
                         double cx, double cy, double cz, double side, int32_t depth) {
  int32_t me = push_node(t);
  wl_node* nd = &t->nodes[me];
  nd->first = first; nd->count = count; nd->depth = depth;
  nd->cx = cx; nd->cy = cy; nd->cz = cz; nd->side = side;
  if (count <= t->bucket || depth >= WL_MAXDEPTH) {
    nd->leaf = 1;
    return me;
  }
  /* stable counting sort of the range into octants */
  int32_t cnt[8] = {0}, off[8];
  for (int32_t k = 0; k < count; ++k) {
    const float* r = in + 4 * (size_t)idx[first + k];
    int o = ((double)r[0] >= cx) | (((double)r[1] >= cy) << 1) | (((double)r[2] >= cz) << 2);
    cnt[o]++;
  }
  off[0] = 0;
  for (int o = 1; o < 8; ++o) off[o] = off[o - 1] + cnt[o - 1];
  int32_t pos[8];
  memcpy(pos, off, sizeof pos);
  for (int32_t k = 0; k < count; ++k) {
    const float* r = in + 4 * (size_t)idx[first + k];
    int o = ((double)r[0] >= cx) | (((double)r[1] >= cy) << 1) | (((double)r[2] >= cz) << 2);
    tmp[pos[o]++] = idx[first + k];
  }
  memcpy(idx + first, tmp, sizeof(int32_t) * (size_t)count);
  int nch = 0;
  for (int o = 0; o < 8; ++o) nch += cnt[o] > 0;
  int32_t c0 = push_children(t, nch);
  t->nodes[me].child0 = c0;
  t->nodes[me].nchild = nch;
  int k = 0;
  double h = side * 0.25;
  for (int o = 0; o < 8; ++o) {
    if (!cnt[o]) continue;
    double ncx = cx + ((o & 1) ? h : -h);
    double ncy = cy + ((o & 2) ? h : -h);
    double ncz = cz + ((o & 4) ? h : -h);
    int32_t c = build_rec(t, in, idx, tmp, first + off[o], cnt[o], ncx, ncy, ncz, side * 0.5, depth + 1);
    t->child[c0 + k++] = c;
  }
  return me;
}

/* Build the tree over n records (x, y, z, m) in input order. */
wl_tree* wl_tree_build(int64_t n, const float* in, int32_t bucket) {
  if (n <= 0 || n > 0x7fffffff || bucket < 1) return NULL;
  wl_tree* t = (wl_tree*)calloc(1, sizeof(wl_tree));
  t->n = n;
  t->bucket = bucket;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      double v = in[4 * i + d];
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  double ext = 0;
  for (int d = 0; d < 3; ++d) ext = fmax(ext, hi[d] - lo[d]);
  double side = ext > 0 ? ext * (1.0 + ldexp(1.0, -20)) : 1.0;
  int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int64_t i = 0; i < n; ++i) idx[i] = (int32_t)i;
  build_rec(t, in, idx, tmp, 0, (int32_t)n, 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2]), side, 0);
  free(tmp);
  t->perm = idx;
  t->rec = (float*)malloc(sizeof(float) * 4 * (size_t)n);
  for (int64_t i = 0; i < n; ++i) memcpy(t->rec + 4 * i, in + 4 * (size_t)idx[i], 4 * sizeof(float));
  /* moments in FP64 from the FP32 member records */
  for (int32_t k = 0; k < t->nnodes; ++k) {
    wl_node* nd = &t->nodes[k];
    double M = 0, cx = 0, cy = 0, cz = 0;
    for (int32_t i = nd->first; i < nd->first + nd->count; ++i) {
      const float* r = t->rec + 4 * (size_t)i;
      M += r[3];
      cx += (double)r[3] * r[0];
      cy += (double)r[3] * r[1];
      cz += (double)r[3] * r[2];
    }
    nd->M = M;
    nd->com[0] = cx / M; nd->com[1] = cy / M; nd->com[2] = cz / M;
    double S[6] = {0};
    for (int32_t i = nd->first; i < nd->first + nd->count; ++i) {
      const float* r = t->rec + 4 * (size_t)i;
      double m = r[3], dx = r[0] - nd->com[0], dy = r[1] - nd->com[1], dz = r[2] - nd->com[2];
      S[0] += m * dx * dx; S[1] += m * dy * dy; S[2] += m * dz * dz;
      S[3] += m * dx * dy; S[4] += m * dx * dz; S[5] += m * dy * dz;
    }
    memcpy(nd->S, S, sizeof S);
  }
  return t;
}

void wl_tree_free(wl_tree* t) {
  if (!t) return;
  free(t->nodes); free(t->child); free(t->perm); free(t->rec); free(t);
}

int32_t wl_tree_nnodes(const wl_tree* t) { return t->nnodes; }

int32_t wl_tree_nleaves(const wl_tree* t) {
  int32_t c = 0;
  for (int32_t k = 0; k < t->nnodes; ++k) c += t->nodes[k].leaf;
  return c;
}

/* perm[n]; rec[4n]; node_rec[12*nnodes] = (com xyz, M, Sxx Syy Szz Sxy, Sxz Syz T, 0) as FP32;
 * node_range[2*nnodes] = (first, count); node_geom[4*nnodes] = (cx, cy, cz, side) FP64;
 * node_depth[nnodes]; node_parent[nnodes] (-1 for the root). */
void wl_tree_export(const wl_tree* t, int32_t* perm, float* rec, float* node_rec, int32_t* node_range,
                    double* node_geom, int32_t* node_depth, int32_t* node_parent, double* node_mom64) {
  if (perm) memcpy(perm, t->perm, sizeof(int32_t) * (size_t)t->n);
  if (rec) memcpy(rec, t->rec, sizeof(float) * 4 * (size_t)t->n);
  if (node_parent) {
    for (int32_t k = 0; k < t->nnodes; ++k) node_parent[k] = -1;
    for (int32_t k = 0; k < t->nnodes; ++k)
      for (int32_t c = 0; c < t->nodes[k].nchild; ++c) node_parent[t->child[t->nodes[k].child0 + c]] = k;
  }
  for (int32_t k = 0; k < t->nnodes; ++k) {
    const wl_node* nd = &t->nodes[k];
    if (node_rec) {
      float* o = node_rec + 12 * (size_t)k;
      o[0] = (float)nd->com[0]; o[1] = (float)nd->com[1]; o[2] = (float)nd->com[2]; o[3] = (float)nd->M;
      o[4] = (float)nd->S[0]; o[5] = (float)nd->S[1]; o[6] = (float)nd->S[2]; o[7] = (float)nd->S[3];
      o[8] = (float)nd->S[4]; o[9] = (float)nd->S[5]; o[10] = (float)(nd->S[0] + nd->S[1] + nd->S[2]); o[11] = 0.0f;
    }
    if (node_range) { node_range[2 * k] = nd->first; node_range[2 * k + 1] = nd->count; }
    if (node_geom) {
      node_geom[4 * k] = nd->cx; node_geom[4 * k + 1] = nd->cy; node_geom[4 * k + 2] = nd->cz; node_geom[4 * k + 3] = nd->side;
    }
    if (node_depth) node_depth[k] = nd->depth;
    if (node_mom64) {
      double* o = node_mom64 + 10 * (size_t)k;
      o[0] = nd->com[0]; o[1] = nd->com[1]; o[2] = nd->com[2]; o[3] = nd->M;
      memcpy(o + 4, nd->S, sizeof nd->S);
    }
  }
}

/* ---- Barnes-Hut walk: per bucket (leaf), node list and direct id ranges ---- */

typedef struct { int32_t* v; int64_t n, cap; } ivec;
static void iv_push(ivec* a, int32_t x) {
  if (a->n == a->cap) { a->cap = a->cap ? 2 * a->cap : 256; a->v = (int32_t*)realloc(a->v, sizeof(int32_t) * (size_t)a->cap); }
  a->v[a->n++] = x;
}

static double box_dist(const double* c, const double* lo, const double* hi) {
  double s = 0;
  for (int d = 0; d < 3; ++d) {
    double e = 0;
    if (c[d] < lo[d]) e = lo[d] - c[d];
    else if (c[d] > hi[d]) e = c[d] - hi[d];
    s += e * e;
  }
  return sqrt(s);
}

static void walk_bucket(const wl_tree* t, int32_t bk, double theta, ivec* nodes, ivec* ranges, int32_t* stack) {
  const wl_node* B = &t->nodes[bk];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t i = B->first; i < B->first + B->count; ++i)
    for (int d = 0; d < 3; ++d) {
      double v = t->rec[4 * (size_t)i + d];
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  int32_t sp = 0;
  stack[sp++] = 0;
  while (sp) {
    int32_t k = stack[--sp];
    const wl_node* N = &t->nodes[k];
    int disjoint = (N->first + N->count <= B->first) || (B->first + B->count <= N->first);
    if (theta > 0 && disjoint && N->side < theta * box_dist(N->com, lo, hi)) {
      iv_push(nodes, k);
    } else if (N->leaf) {
      iv_push(ranges, N->first);
      iv_push(ranges, N->count);
    } else {
      for (int32_t c = N->nchild - 1; c >= 0; --c) stack[sp++] = t->child[N->child0 + c];
    }
  }
}

typedef struct {
  int32_t nb;
  int32_t* leaf;       /* bucket -> leaf node */
  int32_t* nfirst;     /* CSR over node refs, nb+1 */
  int32_t* rfirst;     /* CSR over ranges, nb+1 */
  int32_t* node_idx;
  int32_t* ranges;     /* (begin, count) pairs */
} wl_lists;

wl_lists* wl_walk(const wl_tree* t, double theta) {
  wl_lists* L = (wl_lists*)calloc(1, sizeof(wl_lists));
  int32_t nb = wl_tree_nleaves(t);
  L->nb = nb;
  L->leaf = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
  int32_t b = 0;
  for (int32_t k = 0; k < t->nnodes; ++k)
    if (t->nodes[k].leaf) L->leaf[b++] = k;
  ivec* pn = (ivec*)calloc((size_t)nb, sizeof(ivec));
  ivec* pr = (ivec*)calloc((size_t)nb, sizeof(ivec));
  int32_t maxstack = 8 * (WL_MAXDEPTH + 2);
#pragma omp parallel
  {
    int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)maxstack);
#pragma omp for schedule(dynamic, 64)
    for (int32_t i = 0; i < nb; ++i) walk_bucket(t, L->leaf[i], theta, &pn[i], &pr[i], stack);
    free(stack);
  }
  L->nfirst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb + 1));
  L->rfirst = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nb + 1));
  int64_t tn = 0, tr = 0;
  for (int32_t i = 0; i < nb; ++i) {
    L->nfirst[i] = (int32_t)tn; L->rfirst[i] = (int32_t)tr;
    tn += pn[i].n; tr += pr[i].n / 2;
  }
  L->nfirst[nb] = (int32_t)tn; L->rfirst[nb] = (int32_t)tr;
  L->node_idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(tn ? tn : 1));
  L->ranges = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(tr ? tr : 1));
  for (int32_t i = 0; i < nb; ++i) {
    if (pn[i].n) memcpy(L->node_idx + L->nfirst[i], pn[i].v, sizeof(int32_t) * (size_t)pn[i].n);
    if (pr[i].n) memcpy(L->ranges + 2 * (size_t)L->rfirst[i], pr[i].v, sizeof(int32_t) * (size_t)pr[i].n);
    free(pn[i].v); free(pr[i].v);
  }
  free(pn); free(pr);
  return L;
}

void wl_lists_sizes(const wl_lists* L, int32_t* nb, int32_t* n_node_refs, int32_t* n_ranges) {
  *nb = L->nb; *n_node_refs = L->nfirst[L->nb]; *n_ranges = L->rfirst[L->nb];
}

void wl_lists_export(const wl_lists* L, int32_t* leaf, int32_t* nfirst, int32_t* rfirst, int32_t* node_idx, int32_t* ranges) {
  memcpy(leaf, L->leaf, sizeof(int32_t) * (size_t)L->nb);
  memcpy(nfirst, L->nfirst, sizeof(int32_t) * (size_t)(L->nb + 1));
  memcpy(rfirst, L->rfirst, sizeof(int32_t) * (size_t)(L->nb + 1));
  memcpy(node_idx, L->node_idx, sizeof(int32_t) * (size_t)L->nfirst[L->nb]);
  memcpy(ranges, L->ranges, sizeof(int32_t) * 2 * (size_t)L->rfirst[L->nb]);
}

void wl_lists_free(wl_lists* L) {
  if (!L) return;
  free(L->leaf); free(L->nfirst); free(L->rfirst); free(L->node_idx); free(L->ranges); free(L);
}

/* ---- Lennard-Jones cells: periodic box [0,L)^3, cells of side >= r_cut ----
 * Positions must already be wrapped into [0, L).  cell = floor(x * n / L)
 * clamped to [0, n-1]; linear id = cx + nx * (cy + ny * cz); atoms are stably
 * sorted by linear id.  Tasks per cell c in ascending order: the self task,
 * then the 13 half-shell neighbours with (dz, dy, dx) lexicographically
 * positive, enumerated dz = 0..1, dy = -1..1, dx = -1..1.  A neighbour index
 * that wraps gets the image shift +-L in that dimension: the j atom's image is
 * at x_j + shift. */
int32_t wl_cells_dims(const double* L, double rcut, int32_t* ncell) {
  for (int d = 0; d < 3; ++d) {
    ncell[d] = (int32_t)floor(L[d] / rcut);
    if (ncell[d] < 3) return -1;
  }
  return 0;
}

/* perm[n]: sorted order (perm[new] = old); cell_start[ncells+1]. */
void wl_cells_sort(int64_t n, const float* xyz4, const double* L, const int32_t* ncell, int32_t* perm, int32_t* cell_start) {
  int64_t nc = (int64_t)ncell[0] * ncell[1] * ncell[2];
  int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  memset(cell_start, 0, sizeof(int32_t) * (size_t)(nc + 1));
  for (int64_t i = 0; i < n; ++i) {
    int32_t c3[3];
    for (int d = 0; d < 3; ++d) {
      int32_t c = (int32_t)floor((double)xyz4[4 * i + d] * ncell[d] / L[d]);
      if (c < 0) c = 0;
      if (c >= ncell[d]) c = ncell[d] - 1;
      c3[d] = c;
    }
    cell[i] = c3[0] + ncell[0] * (c3[1] + ncell[1] * c3[2]);
    cell_start[cell[i] + 1]++;
  }
  for (int64_t c = 0; c < nc; ++c) cell_start[c + 1] += cell_start[c];
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)nc);
  memcpy(fill, cell_start, sizeof(int32_t) * (size_t)nc);
  for (int64_t i = 0; i < n; ++i) perm[fill[cell[i]]++] = (int32_t)i;
  free(fill); free(cell);
}

/* 14 tasks per cell: (i_begin, i_count, j_begin, j_count, self) int32 x5 and shift float x3. */
void wl_cells_tasks(const double* L, const int32_t* ncell, const int32_t* cell_start, int32_t* itask, float* shift) {
  static const int off[13][3] = {
      /* dz = 0 */ {1, 0, 0}, {-1, 1, 0}, {0, 1, 0}, {1, 1, 0},
      /* dz = 1 */ {-1, -1, 1}, {0, -1, 1}, {1, -1, 1}, {-1, 0, 1}, {0, 0, 1}, {1, 0, 1}, {-1, 1, 1}, {0, 1, 1}, {1, 1, 1}};
  int64_t t = 0;
  for (int32_t cz = 0; cz < ncell[2]; ++cz)
    for (int32_t cy = 0; cy < ncell[1]; ++cy)
      for (int32_t cx = 0; cx < ncell[0]; ++cx) {
        int32_t c = cx + ncell[0] * (cy + ncell[1] * cz);
        int32_t* o = itask + 5 * t;
        o[0] = cell_start[c]; o[1] = cell_start[c + 1] - cell_start[c];
        o[2] = cell_start[c]; o[3] = o[1]; o[4] = 1;
        shift[3 * t] = shift[3 * t + 1] = shift[3 * t + 2] = 0.0f;
        ++t;
        for (int k = 0; k < 13; ++k) {
          int32_t q[3] = {cx + off[k][0], cy + off[k][1], cz + off[k][2]};
          float s[3] = {0, 0, 0};
          for (int d = 0; d < 3; ++d) {
            if (q[d] < 0) { q[d] += ncell[d]; s[d] = (float)(-L[d]); }
            else if (q[d] >= ncell[d]) { q[d] -= ncell[d]; s[d] = (float)L[d]; }
          }
          int32_t cj = q[0] + ncell[0] * (q[1] + ncell[1] * q[2]);
          o = itask + 5 * t;
          o[0] = cell_start[c]; o[1] = cell_start[c + 1] - cell_start[c];
          o[2] = cell_start[cj]; o[3] = cell_start[cj + 1] - cell_start[cj]; o[4] = 0;
          shift[3 * t] = s[0]; shift[3 * t + 1] = s[1]; shift[3 * t + 2] = s[2];
          ++t;
        }
      }
}
