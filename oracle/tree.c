/*
 * Oracle (test infrastructure only): the cluster tree of Section 6 and the
 * target batches of the shared-list walk.
 *
 * Tree rules (Section 6, with the readings listed in the design notes):
 *  - every cluster's box is the smallest axis-aligned box holding its own
 *    particles (the paper states this for the root and says the children are
 *    bisected the same way);
 *  - a cluster with more than leaf_max particles is split; a cluster whose
 *    longest side l_max is zero, or whose split would leave all particles in
 *    one child, stays a leaf;
 *  - an axis is bisected when its side is greater than l_max/sqrt(2), l_max
 *    being the cluster's own longest side, so the cluster gets 8, 4 or 2
 *    children;
 *  - the bisection point is the box midpoint 0.5*(lo+hi); a coordinate below
 *    it goes to the low half, otherwise to the high half;
 *  - the child code is bx + 2 by + 4 bz over the bisected axes, children are
 *    kept in increasing code order, empty children are dropped, and the
 *    particle order inside a cluster is a stable partition of its parent's;
 *  - the cluster center is the box midpoint and its radius r is half the box
 *    diagonal (Fig. 1 shows y_c and r without defining them);
 *  - nodes are numbered breadth first.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

struct orc_tree {
  int64_t n, nn, cap;
  int64_t* perm;
  double* box;
  double* center;
  double* radius;
  int32_t* child_first;
  int32_t* child_count;
  int32_t* level;
  int32_t* parent;
  int64_t* pbegin;
  int64_t* pend;
  int32_t depth;
};

static void grow(orc_tree* t) {
  int64_t c = t->cap ? 2 * t->cap : 64;
  t->box = realloc(t->box, sizeof(double) * 6 * c);
  t->center = realloc(t->center, sizeof(double) * 3 * c);
  t->radius = realloc(t->radius, sizeof(double) * c);
  t->child_first = realloc(t->child_first, sizeof(int32_t) * c);
  t->child_count = realloc(t->child_count, sizeof(int32_t) * c);
  t->level = realloc(t->level, sizeof(int32_t) * c);
  t->parent = realloc(t->parent, sizeof(int32_t) * c);
  t->pbegin = realloc(t->pbegin, sizeof(int64_t) * c);
  t->pend = realloc(t->pend, sizeof(int64_t) * c);
  t->cap = c;
}

static int64_t add_node(orc_tree* t, int64_t b, int64_t e, int32_t lev,
                        int32_t par) {
  if (t->nn == t->cap) grow(t);
  int64_t q = t->nn++;
  t->pbegin[q] = b;
  t->pend[q] = e;
  t->level[q] = lev;
  t->parent[q] = par;
  t->child_first[q] = -1;
  t->child_count[q] = 0;
  if (lev > t->depth) t->depth = lev;
  return q;
}

orc_tree* orc_tree_new(const double* x, const double* y, const double* z,
                       int64_t n, int64_t leaf_max) {
  orc_tree* t = calloc(1, sizeof(orc_tree));
  const double* xyz[3] = {x, y, z};
  t->n = n;
  t->perm = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) t->perm[i] = i;
  if (n == 0) return t;
  int64_t* tmp = malloc(sizeof(int64_t) * n);
  unsigned char* code = malloc(n);
  add_node(t, 0, n, 0, -1);
  for (int64_t q = 0; q < t->nn; ++q) {           /* breadth-first sweep */
    int64_t b = t->pbegin[q], e = t->pend[q];
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {                 /* tight box */
      lo[a] = hi[a] = xyz[a][t->perm[b]];
      for (int64_t i = b + 1; i < e; ++i) {
        double v = xyz[a][t->perm[i]];
        if (v < lo[a]) lo[a] = v;
        if (v > hi[a]) hi[a] = v;
      }
    }
    double h[3];
    for (int a = 0; a < 3; ++a) {
      t->box[6 * q + a] = lo[a];
      t->box[6 * q + 3 + a] = hi[a];
      t->center[3 * q + a] = 0.5 * (lo[a] + hi[a]);
      h[a] = 0.5 * (hi[a] - lo[a]);
    }
    t->radius[q] = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);

    double side[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    double lmax = side[0];
    if (side[1] > lmax) lmax = side[1];
    if (side[2] > lmax) lmax = side[2];
    if (e - b <= leaf_max || lmax == 0.0) continue;   /* leaf */

    double thresh = lmax * M_SQRT1_2;
    int split[3];
    double mid[3];
    for (int a = 0; a < 3; ++a) {
      split[a] = side[a] > thresh;
      mid[a] = 0.5 * (lo[a] + hi[a]);
    }
    int64_t cnt[8] = {0};
    for (int64_t i = b; i < e; ++i) {
      int c = 0;
      for (int a = 0; a < 3; ++a)
        if (split[a] && xyz[a][t->perm[i]] >= mid[a]) c |= 1 << a;
      code[i] = (unsigned char)c;
      cnt[c]++;
    }
    int nonempty = 0;
    for (int c = 0; c < 8; ++c) nonempty += cnt[c] > 0;
    if (nonempty < 2) continue;   /* the split separated nothing: leaf */

    int64_t start[8], pos = b;
    for (int c = 0; c < 8; ++c) { start[c] = pos; pos += cnt[c]; }
    int64_t fill[8];
    memcpy(fill, start, sizeof fill);
    for (int64_t i = b; i < e; ++i) tmp[fill[code[i]]++] = t->perm[i];
    memcpy(t->perm + b, tmp + b, sizeof(int64_t) * (e - b));

    int32_t first = -1, count = 0;
    for (int c = 0; c < 8; ++c) {
      if (!cnt[c]) continue;
      int64_t k = add_node(t, start[c], start[c] + cnt[c], t->level[q] + 1,
                           (int32_t)q);
      if (first < 0) first = (int32_t)k;
      count++;
    }
    t->child_first[q] = first;
    t->child_count[q] = count;
  }
  free(tmp);
  free(code);
  return t;
}

void orc_tree_free(orc_tree* t) {
  if (!t) return;
  free(t->perm); free(t->box); free(t->center); free(t->radius);
  free(t->child_first); free(t->child_count); free(t->level);
  free(t->parent); free(t->pbegin); free(t->pend);
  free(t);
}

int64_t orc_tree_nnodes(const orc_tree* t) { return t->nn; }
int32_t orc_tree_depth(const orc_tree* t) { return t->depth; }
int64_t orc_tree_npoints(const orc_tree* t) { return t->n; }

void orc_tree_export(const orc_tree* t, int64_t* perm, double* box,
                     double* center, double* radius, int32_t* child_first,
                     int32_t* child_count, int64_t* pbegin, int64_t* pend,
                     int32_t* level, int32_t* parent) {
  int64_t nn = t->nn;
  if (perm && t->n) memcpy(perm, t->perm, sizeof(int64_t) * t->n);
  if (nn == 0) return;   /* an empty set has no nodes (and no arrays) */
  if (box) memcpy(box, t->box, sizeof(double) * 6 * nn);
  if (center) memcpy(center, t->center, sizeof(double) * 3 * nn);
  if (radius) memcpy(radius, t->radius, sizeof(double) * nn);
  if (child_first) memcpy(child_first, t->child_first, sizeof(int32_t) * nn);
  if (child_count) memcpy(child_count, t->child_count, sizeof(int32_t) * nn);
  if (pbegin) memcpy(pbegin, t->pbegin, sizeof(int64_t) * nn);
  if (pend) memcpy(pend, t->pend, sizeof(int64_t) * nn);
  if (level) memcpy(level, t->level, sizeof(int32_t) * nn);
  if (parent) memcpy(parent, t->parent, sizeof(int32_t) * nn);
}

/* Target batches: the targets are ordered by a tree with leaf size
 * order_leaf.  Group nodes are the nodes of that tree holding at most
 * group_max targets whose parent holds more, together with leaves that are
 * larger (degenerate leaves); their target ranges tile the order.  Each group,
 * in order, is cut into consecutive chunks of batch_size targets, so no batch
 * spans two groups.  Each batch gets the tight box of its own targets, its
 * midpoint as center and half its diagonal as radius, by the same formulas as
 * a cluster.  With output arrays NULL only the batch count is returned; bptr
 * needs nb + 1 entries, bcenter 3 nb, bradius nb. */
static void collect_groups(const orc_tree* t, int64_t q, int64_t group_max,
                           int64_t* gb, int64_t* ge, int64_t* ng) {
  if (t->pend[q] - t->pbegin[q] <= group_max || t->child_count[q] == 0) {
    gb[*ng] = t->pbegin[q];
    ge[*ng] = t->pend[q];
    (*ng)++;
    return;
  }
  for (int32_t c = 0; c < t->child_count[q]; ++c)
    collect_groups(t, t->child_first[q] + c, group_max, gb, ge, ng);
}

/* Balanced k-d batches (order_leaf = 0).  A set of c targets with c <=
 * batch_size is one batch.  A larger set is cut in two along the longest
 * side of its tight box (the first of equal sides), the first part taking
 * the batch_size * floor(nb / 2) targets with the smallest coordinates on
 * that axis, nb = ceil(c / batch_size) (ties ordered by target index), so
 * every batch is full except at most one.  Parts are emitted first part
 * first; inside a batch the targets are in increasing index. */
static int64_t kd_less(const double* key, int64_t i, int64_t j) {
  return key[i] < key[j] || (key[i] == key[j] && i < j);
}

/* Reorders idx[0..c) so that its first k entries are the k smallest by
 * (key, index) (quickselect; the set is unique because the order is total). */
static void kd_select(int64_t* idx, int64_t c, int64_t k, const double* key) {
  int64_t lo = 0, hi = c - 1;
  while (lo < hi) {
    const int64_t pv = idx[lo + (hi - lo) / 2];
    int64_t i = lo, j = hi;
    while (i <= j) {
      while (kd_less(key, idx[i], pv)) ++i;
      while (kd_less(key, pv, idx[j])) --j;
      if (i <= j) {
        const int64_t tmp = idx[i];
        idx[i] = idx[j];
        idx[j] = tmp;
        ++i;
        --j;
      }
    }
    if (k - 1 <= j) hi = j;
    else if (k - 1 >= i) lo = i;
    else return;
  }
}

static int cmp_i64(const void* a, const void* b) {
  const int64_t u = *(const int64_t*)a, v = *(const int64_t*)b;
  return (u > v) - (u < v);
}

static void kd_split(int64_t* idx, int64_t c, int64_t bs, const double* xyz[3],
                     int64_t base, int64_t* bptr, int64_t* nb) {
  if (c <= bs) {
    qsort(idx, (size_t)c, sizeof(int64_t), cmp_i64);
    if (bptr) bptr[*nb] = base;
    (*nb)++;
    return;
  }
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = hi[a] = xyz[a][idx[0]];
    for (int64_t i = 1; i < c; ++i) {
      const double v = xyz[a][idx[i]];
      if (v < lo[a]) lo[a] = v;
      if (v > hi[a]) hi[a] = v;
    }
  }
  int ax = 0;
  for (int a = 1; a < 3; ++a)
    if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
  const int64_t nbc = (c + bs - 1) / bs;
  const int64_t left = bs * (nbc / 2);
  kd_select(idx, c, left, xyz[ax]);
  kd_split(idx, left, bs, xyz, base, bptr, nb);
  kd_split(idx + left, c - left, bs, xyz, base + left, bptr, nb);
}

int64_t orc_batches(const double* tx, const double* ty, const double* tz,
                    int64_t m, int64_t batch_size, int64_t order_leaf,
                    int64_t group_max, int64_t* tperm, int64_t* bptr,
                    double* bcenter, double* bradius) {
  if (m == 0) {
    if (bptr) bptr[0] = 0;
    return 0;
  }
  if (order_leaf == 0) {
    const double* xyz[3] = {tx, ty, tz};
    if (!bptr) return (m + batch_size - 1) / batch_size;
    for (int64_t i = 0; i < m; ++i) tperm[i] = i;
    int64_t nb = 0;
    kd_split(tperm, m, batch_size, xyz, 0, bptr, &nb);
    bptr[nb] = m;
    for (int64_t b = 0; b < nb; ++b) {
      double h[3];
      for (int a = 0; a < 3; ++a) {
        double lo = xyz[a][tperm[bptr[b]]], hi = lo;
        for (int64_t i = bptr[b] + 1; i < bptr[b + 1]; ++i) {
          const double v = xyz[a][tperm[i]];
          if (v < lo) lo = v;
          if (v > hi) hi = v;
        }
        bcenter[3 * b + a] = 0.5 * (lo + hi);
        h[a] = 0.5 * (hi - lo);
      }
      bradius[b] = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    }
    return nb;
  }
  orc_tree* t = orc_tree_new(tx, ty, tz, m, order_leaf);
  const double* xyz[3] = {tx, ty, tz};
  int64_t* gb = malloc(sizeof(int64_t) * t->nn);
  int64_t* ge = malloc(sizeof(int64_t) * t->nn);
  int64_t ng = 0;
  collect_groups(t, 0, group_max, gb, ge, &ng);
  int64_t nb = 0;
  for (int64_t g = 0; g < ng; ++g)
    for (int64_t s = gb[g]; s < ge[g]; s += batch_size) {
      int64_t e = s + batch_size;
      if (e > ge[g]) e = ge[g];
      if (bptr) {
        bptr[nb] = s;
        double h[3];
        for (int a = 0; a < 3; ++a) {
          double lo = xyz[a][t->perm[s]], hi = lo;
          for (int64_t i = s + 1; i < e; ++i) {
            double v = xyz[a][t->perm[i]];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
          }
          bcenter[3 * nb + a] = 0.5 * (lo + hi);
          h[a] = 0.5 * (hi - lo);
        }
        bradius[nb] = sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
      }
      nb++;
    }
  if (bptr) {
    bptr[nb] = m;
    memcpy(tperm, t->perm, sizeof(int64_t) * m);
  }
  free(gb);
  free(ge);
  orc_tree_free(t);
  return nb;
}
