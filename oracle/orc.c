/*
 * orc.c -- plain, slow, FP64 CPU oracle for the adaptive multi-NeRF rendering path.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load this library.  It shares no code, header, table or helper with
 * the HIP library; both consume the same seeded float32 inputs.
 *
 * What it computes, and where the paper defines it:
 *   - quantised guidance grid and density-median KD tree .......... Section 3.4
 *     (BuildKDTree: sort, median of the cumulative density, split, recurse);
 *     the distillation-based TestLeaf is replaced by max_leaves / max_depth.
 *   - ray / KD-tree traversal producing leaf intervals ........... Section 3.5, Algorithm 1
 *     (Traverse), taken near-side first so intervals come out front to back.
 *   - equal sample count per leaf interval ........................ Section 3.5, Algorithm 1
 *     (Sampling) and the figure on normalised intervals.
 *   - per-leaf MLP F_theta_i(x, d) -> (c, sigma) .................. Section 3.1, with
 *     frequency positional encoding (Section 3.2 figure caption).
 *   - front-to-back volume rendering with early ray termination ... Section 3.1 (defers to
 *     the NeRF quadrature), Section 4.1 (early termination).
 *   - analytic gradient of that quadrature and of the MLPs, and Adam (training step;
 *     not in the paper, so it follows the standard definitions).
 *   - regular subdivision (middle planes, breadth first) for the ablation against it
 *     ............................................................... Section 4.2, table
 *   - hierarchical sampling: HCheck stops the descent at inner nodes, whose own MLPs
 *     take their segments ........................................... Section 3.5, Algorithm 1
 *   - occupancy grid and empty-space skipping ..................... Section 4.1
 *   - the learned proposal (not in the paper): features, network, slot selection,
 *     targets and loss, following the stated reading step by step.
 *   - float8 activations (not in the paper; the large workload's float8 matrix-core
 *     path): the input features rounded to bfloat16 and every hidden activation rounded to
 *     the nearest e4m3 value times a power-of-two scale 2^k per leaf and layer, saturating
 *     at 256 * 2^k; and the calibration maxima
 *     those scales come from (the largest ReLU output per leaf and hidden layer over the
 *     samples of a render).
 *
 * Everything is double precision; float inputs are promoted exactly.  No blocking,
 * sorting, batching or fusion: every ray is processed on its own, sample by sample.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NODE_COLS 12
#define IN_DIM 30
#define OUT_DIM 4
#define MAX_HIDDEN 256
#define MAX_LAYERS 16

/* ------------------------------------------------------------------------- */
/* Guidance grid quantisation                                                 */
/* ------------------------------------------------------------------------- */
/* q = floor(g / g_max * 2^24 + 1/2); negative densities count as 0.  Integer masses make
 * the median splits exact, so any two implementations build the same tree. */
static void quantise(const float* g, int64_t ncell, uint32_t* q) {
  double gmax = 0.0;
  for (int64_t i = 0; i < ncell; ++i)
    if ((double)g[i] > gmax) gmax = (double)g[i];
  for (int64_t i = 0; i < ncell; ++i) {
    double v = (double)g[i];
    if (!(gmax > 0.0) || !(v > 0.0)) { q[i] = 0u; continue; }
    q[i] = (uint32_t)floor(ldexp(v / gmax, 24) + 0.5);
  }
}

/* ------------------------------------------------------------------------- */
/* KD tree construction (Section 3.4)                                         */
/* ------------------------------------------------------------------------- */
typedef struct {
  int lo[3], hi[3];
  uint32_t code;      /* binary node code: root 1, left child 2c, right child 2c+1 */
  int depth;
  int axis, plane;    /* split (inner nodes); plane is a cell index */
  int child[2];
  int slot;           /* leaf rank in left-first depth-first order */
  int nslot;          /* rank among all nodes in left-first depth-first preorder */
  uint64_t mass;
  int leaf;
} onode;

static uint64_t mass_of_slab(const uint32_t* q, int n, const int lo[3], const int hi[3],
                             int axis, int c) {
  int a0 = lo[0], a1 = hi[0], b0 = lo[1], b1 = hi[1], e0 = lo[2], e1 = hi[2];
  if (axis == 0) { a0 = c; a1 = c + 1; }
  if (axis == 1) { b0 = c; b1 = c + 1; }
  if (axis == 2) { e0 = c; e1 = c + 1; }
  uint64_t s = 0;
  for (int k = e0; k < e1; ++k)
    for (int j = b0; j < b1; ++j)
      for (int i = a0; i < a1; ++i) s += q[(int64_t)i + (int64_t)n * ((int64_t)j + (int64_t)n * k)];
  return s;
}

static int longest_axis(const onode* nd) {
  int a = 0;
  for (int ax = 1; ax < 3; ++ax)
    if (nd->hi[ax] - nd->lo[ax] > nd->hi[a] - nd->lo[a]) a = ax;
  return a;
}

static int splittable(const onode* nd, int max_depth) {
  int a = longest_axis(nd);
  return nd->depth < max_depth && nd->hi[a] - nd->lo[a] >= 2;
}

static int slot_counter, nslot_counter;
static void assign_slots(onode* nodes, int i) {
  nodes[i].nslot = nslot_counter++;   /* preorder: the node before its subtrees */
  if (nodes[i].leaf) { nodes[i].slot = slot_counter++; return; }
  assign_slots(nodes, nodes[i].child[0]);
  assign_slots(nodes, nodes[i].child[1]);
}

static const onode* sort_base;
static int cmp_code(const void* a, const void* b) {
  uint32_t ca = sort_base[*(const int*)a].code, cb = sort_base[*(const int*)b].code;
  return ca < cb ? -1 : (ca > cb ? 1 : 0);
}

/* Splits leaf `best` on its longest axis: at the weighted median plane (split = 0: the
 * smallest plane whose lower side holds at least half of the node's mass, the last plane
 * if none does, the middle plane for a massless node) or at the middle plane (split = 1).
 * The children are appended at nodes[*nn] and nodes[*nn + 1]. */
static void split_leaf(onode* nodes, int* nn, int best, const uint32_t* q, int n, int split, uint64_t* slab) {
  onode* p = &nodes[best];
  int a = longest_axis(p);
  int lo = p->lo[a], hi = p->hi[a];
  for (int c = lo; c < hi; ++c) slab[c - lo] = mass_of_slab(q, n, p->lo, p->hi, a, c);
  int plane;
  if (split == 1 || p->mass == 0) {
    plane = (lo + hi) / 2;
  } else {
    /* weighted median: smallest plane whose lower side holds at least half the mass */
    plane = hi - 1;
    uint64_t acc = 0;
    for (int c = lo + 1; c <= hi - 1; ++c) {
      acc += slab[c - 1 - lo];
      if (2 * acc >= p->mass) { plane = c; break; }
    }
  }
  uint64_t left_mass = 0;
  for (int c = lo; c < plane; ++c) left_mass += slab[c - lo];
  for (int side = 0; side < 2; ++side) {
    onode* ch = &nodes[*nn];
    *ch = *p;
    ch->code = 2u * p->code + (uint32_t)side;
    ch->depth = p->depth + 1;
    ch->leaf = 1; ch->axis = -1; ch->plane = -1; ch->child[0] = ch->child[1] = -1;
    if (side == 0) { ch->hi[a] = plane; ch->mass = left_mass; }
    else { ch->lo[a] = plane; ch->mass = p->mass - left_mass; }
    p->child[side] = *nn;
    ++*nn;
  }
  p->leaf = 0; p->axis = a; p->plane = plane;
}

/* Slots, then the rows (sorted by code) and masses of the first nn nodes. */
static void export_rows(onode* nodes, int nn, int32_t* rows, uint64_t* mass_out) {
  slot_counter = 0;
  nslot_counter = 0;
  for (int i = 0; i < nn; ++i) nodes[i].slot = -1;
  assign_slots(nodes, 0);
  int* order = (int*)malloc(sizeof(int) * nn);
  for (int i = 0; i < nn; ++i) order[i] = i;
  sort_base = nodes;
  qsort(order, nn, sizeof(int), cmp_code);
  for (int k = 0; k < nn; ++k) {
    const onode* nd = &nodes[order[k]];
    int32_t* row = rows + (int64_t)k * NODE_COLS;
    row[0] = (int32_t)nd->code; row[1] = nd->depth;
    for (int a = 0; a < 3; ++a) { row[2 + a] = nd->lo[a]; row[5 + a] = nd->hi[a]; }
    row[8] = nd->leaf ? -1 : nd->axis;
    row[9] = nd->leaf ? -1 : nd->plane;
    row[10] = nd->leaf ? nd->slot : -1;
    row[11] = nd->nslot;
    if (mass_out) mass_out[k] = nd->mass;
  }
  free(order);
}

static void init_root(onode* r, int n, const uint32_t* q, int64_t ncell) {
  for (int a = 0; a < 3; ++a) { r->lo[a] = 0; r->hi[a] = n; }
  r->code = 1; r->depth = 0; r->leaf = 1; r->axis = -1; r->plane = -1;
  r->child[0] = r->child[1] = -1;
  r->mass = 0;
  for (int64_t i = 0; i < ncell; ++i) r->mass += q[i];
}

/* Builds the tree and exports it as rows of 12 int32, sorted by node code:
 *   code, depth, lo[3], hi[3], axis (-1 leaf), plane (-1 leaf), slot (-1 inner), node slot
 * (preorder rank among all nodes: the MLP index of a node under hierarchical sampling)
 * plus the integer mass of each node.  Returns 0, or -1 on bad arguments / capacity. */
int orc_build_tree(const float* grid, int n, int max_depth, int max_leaves, int split, int cap,
                   int32_t* rows, uint64_t* mass_out, int* n_nodes_out, int* n_leaves_out) {
  if (!grid || n < 1 || max_depth < 0 || max_depth > 30 || max_leaves < 1 || !rows) return -1;
  if (split != 0 && split != 1) return -1;
  int64_t ncell = (int64_t)n * n * n;
  uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * ncell);
  if (!q) return -1;
  quantise(grid, ncell, q);
  int maxn = 2 * max_leaves;
  onode* nodes = (onode*)calloc(maxn, sizeof(onode));
  uint64_t* slab = (uint64_t*)malloc(sizeof(uint64_t) * n);
  int nn = 1, nleaves = 1;
  init_root(&nodes[0], n, q, ncell);

  while (nleaves < max_leaves) {
    /* median split (split = 0): best-first, the splittable leaf of largest mass; middle
       split (split = 1): breadth-first, the splittable leaf of smallest depth; ties to the
       smallest code */
    int best = -1;
    for (int i = 0; i < nn; ++i) {
      if (!nodes[i].leaf || !splittable(&nodes[i], max_depth)) continue;
      int better;
      if (best < 0) better = 1;
      else if (split == 0) better = nodes[i].mass > nodes[best].mass ||
                                    (nodes[i].mass == nodes[best].mass && nodes[i].code < nodes[best].code);
      else better = nodes[i].depth < nodes[best].depth ||
                    (nodes[i].depth == nodes[best].depth && nodes[i].code < nodes[best].code);
      if (better) best = i;
    }
    if (best < 0) break;
    split_leaf(nodes, &nn, best, q, n, split, slab);
    ++nleaves;
  }
  free(slab);
  free(q);
  if (nn > cap) { free(nodes); return -1; }
  export_rows(nodes, nn, rows, mass_out);
  free(nodes);
  *n_nodes_out = nn;
  *n_leaves_out = nleaves;
  return 0;
}

/* The tree whose inner nodes are exactly the given node codes (each split at the density
 * median as above): the codes are taken in increasing order, and each must name a leaf of
 * the tree built so far (so a node's parent comes first) whose longest side is at least 2
 * cells.  This is how BuildKDTree's recursion is driven by an outside stopping rule
 * (Section 3.4, TestLeaf).  Rows and masses as orc_build_tree.  Returns 0, or -1 on bad
 * arguments, a code that is not a splittable leaf, or capacity. */
int orc_build_tree_codes(const float* grid, int n, int n_split, const uint32_t* codes, int cap,
                         int32_t* rows, uint64_t* mass_out, int* n_nodes_out, int* n_leaves_out) {
  if (!grid || n < 1 || n_split < 0 || (n_split > 0 && !codes) || !rows) return -1;
  int nn_need = 2 * n_split + 1;
  if (nn_need > cap) return -1;
  int64_t ncell = (int64_t)n * n * n;
  uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * ncell);
  onode* nodes = (onode*)calloc(nn_need, sizeof(onode));
  uint64_t* slab = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint32_t* sorted = (uint32_t*)malloc(sizeof(uint32_t) * (n_split > 0 ? n_split : 1));
  if (!q || !nodes || !slab || !sorted) { free(q); free(nodes); free(slab); free(sorted); return -1; }
  quantise(grid, ncell, q);
  for (int i = 0; i < n_split; ++i) sorted[i] = codes[i];
  /* insertion sort: the lists are short */
  for (int i = 1; i < n_split; ++i)
    for (int j = i; j > 0 && sorted[j - 1] > sorted[j]; --j) { uint32_t t = sorted[j]; sorted[j] = sorted[j - 1]; sorted[j - 1] = t; }
  int nn = 1, rc = 0;
  init_root(&nodes[0], n, q, ncell);
  for (int s = 0; s < n_split && rc == 0; ++s) {
    int at = -1;
    for (int i = 0; i < nn; ++i)
      if (nodes[i].code == sorted[s]) at = i;
    if (at < 0 || !nodes[at].leaf || !splittable(&nodes[at], 30)) { rc = -1; break; }
    split_leaf(nodes, &nn, at, q, n, 0, slab);
  }
  free(slab);
  free(q);
  free(sorted);
  if (rc == 0) {
    export_rows(nodes, nn, rows, mass_out);
    *n_nodes_out = nn;
    *n_leaves_out = n_split + 1;
  }
  free(nodes);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Occupancy grid (Section 4.1: the density grid also detects empty space)    */
/* ------------------------------------------------------------------------- */
/* Cell (i,j,k) of the G^3 grid, G = n / block, covers guidance cells [b i, b i + b) x ...;
   it is occupied iff its largest quantised density reaches q_thr = max(1, floor(thresh 2^24
   + 1/2)).  out: uint8[G^3], cell (i,j,k) at i + G (j + G k).  Returns G or -1. */
int orc_occupancy(const float* grid, int n, int block, double thresh, uint8_t* out) {
  if (!grid || !out || n < 1 || block < 1 || n % block != 0 || !(thresh >= 0.0 && thresh <= 1.0)) return -1;
  int64_t ncell = (int64_t)n * n * n;
  uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * ncell);
  if (!q) return -1;
  quantise(grid, ncell, q);
  double t = floor(ldexp(thresh, 24) + 0.5);
  uint32_t q_thr = t < 1.0 ? 1u : (uint32_t)t;
  int G = n / block;
  for (int k = 0; k < G; ++k)
    for (int j = 0; j < G; ++j)
      for (int i = 0; i < G; ++i) {
        uint32_t mx = 0;
        for (int c = 0; c < block; ++c)
          for (int b = 0; b < block; ++b)
            for (int a = 0; a < block; ++a) {
              uint32_t v = q[(int64_t)(block * i + a) + (int64_t)n * ((int64_t)(block * j + b) + (int64_t)n * (block * k + c))];
              if (v > mx) mx = v;
            }
        out[(int64_t)i + (int64_t)G * ((int64_t)j + (int64_t)G * k)] = mx >= q_thr;
      }
  free(q);
  return G;
}

/* ------------------------------------------------------------------------- */
/* Tree view over an exported node table                                      */
/* ------------------------------------------------------------------------- */
typedef struct {
  int nn, n_leaves, grid_n;
  const int32_t* rows;
  int* left;
  int* right;
  int root;
  float footprint;    /* hierarchical sampling (HCheck) when > 0 */
  float* t_stop;      /* per node: longest side / footprint, in float32 */
} otree;

static int find_code(const int32_t* rows, int nn, uint32_t code) {
  int lo = 0, hi = nn - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    uint32_t c = (uint32_t)rows[(int64_t)mid * NODE_COLS];
    if (c == code) return mid;
    if (c < code) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

/* Hierarchical sampling (Section 3.5, HCheck), read as a level-of-detail test: a node whose
   longest side s is small next to the spacing of samples at the distance where the ray
   enters it is not refined.  With the caller's footprint f (sample spacing per unit
   distance), the descent continues into the children iff the entry parameter t satisfies
   t <= s / f; both sides of the test in float32 (the quotient rounded once). */
static int otree_init_hcheck(otree* T, const int32_t* rows, int nn, int grid_n, float footprint);

static int otree_init(otree* T, const int32_t* rows, int nn, int grid_n) {
  return otree_init_hcheck(T, rows, nn, grid_n, 0.0f);
}

static int otree_init_hcheck(otree* T, const int32_t* rows, int nn, int grid_n, float footprint) {
  T->nn = nn; T->rows = rows; T->grid_n = grid_n; T->n_leaves = 0;
  T->footprint = footprint;
  T->left = (int*)malloc(sizeof(int) * nn);
  T->right = (int*)malloc(sizeof(int) * nn);
  T->t_stop = (float*)malloc(sizeof(float) * nn);
  T->root = find_code(rows, nn, 1u);
  if (T->root < 0) return -1;
  for (int i = 0; i < nn; ++i) {
    const int32_t* r = rows + (int64_t)i * NODE_COLS;
    int ext = 0;
    for (int a = 0; a < 3; ++a) if (r[5 + a] - r[2 + a] > ext) ext = r[5 + a] - r[2 + a];
    float side = (float)ext / (float)grid_n;
    T->t_stop[i] = footprint > 0.0f ? side / footprint : INFINITY;
    if (r[8] < 0) { T->left[i] = T->right[i] = -1; T->n_leaves++; continue; }
    T->left[i] = find_code(rows, nn, 2u * (uint32_t)r[0]);
    T->right[i] = find_code(rows, nn, 2u * (uint32_t)r[0] + 1u);
    if (T->left[i] < 0 || T->right[i] < 0) return -1;
  }
  return 0;
}

static void otree_free(otree* T) { free(T->left); free(T->right); free(T->t_stop); }

/* ------------------------------------------------------------------------- */
/* Traversal (Algorithm 1, Traverse)                                          */
/* ------------------------------------------------------------------------- */
typedef struct { double t0, t1; int slot; } oiv;

typedef struct { oiv* iv; int m, cap; } ivlist;

static void descend(const otree* T, int node, const double o[3], const double d[3],
                    double t0, double t1, ivlist* L, int hcheck) {
  const int32_t* r = T->rows + (int64_t)node * NODE_COLS;
  /* a leaf, or an inner node where HCheck stops the descent: the node takes the segment
     (keyed by its leaf slot, or by its preorder node slot under hierarchical sampling) */
  if (r[8] < 0 || (hcheck && (float)t0 > T->t_stop[node])) {
    int slot = hcheck ? r[11] : r[10];
    if (t1 > t0 && L->m < L->cap) { L->iv[L->m].t0 = t0; L->iv[L->m].t1 = t1; L->iv[L->m].slot = slot; }
    if (t1 > t0) L->m++;
    return;
  }
  int a = r[8];
  double s = (double)r[9] / (double)T->grid_n;
  if (d[a] == 0.0) {
    /* parallel to the plane: the whole segment lies on o's side (a point on the plane
       belongs to the upper cell, matching half-open cells [lo, hi)) */
    descend(T, o[a] >= s ? T->right[node] : T->left[node], o, d, t0, t1, L, hcheck);
    return;
  }
  double ts = (s - o[a]) / d[a];
  int before = d[a] > 0.0 ? T->left[node] : T->right[node];
  int after = d[a] > 0.0 ? T->right[node] : T->left[node];
  if (ts >= t1) descend(T, before, o, d, t0, t1, L, hcheck);
  else if (ts <= t0) descend(T, after, o, d, t0, t1, L, hcheck);
  else { descend(T, before, o, d, t0, ts, L, hcheck); descend(T, after, o, d, ts, t1, L, hcheck); }
}

/* Root box [0,1]^3 slab test, then front-to-back descent; returns the interval count.
   hcheck: stop the descent by HCheck (the tree's footprint must be > 0). */
static int trace_ray_mode(const otree* T, const double o[3], const double d[3], ivlist* L, int hcheck) {
  L->m = 0;
  double tin = 0.0, tout = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (o[a] < 0.0 || o[a] > 1.0) return 0;
      continue;
    }
    double ta = (0.0 - o[a]) / d[a], tb = (1.0 - o[a]) / d[a];
    if (ta > tb) { double t = ta; ta = tb; tb = t; }
    if (ta > tin) tin = ta;
    if (tb < tout) tout = tb;
  }
  if (!(tin < tout)) return 0;
  descend(T, T->root, o, d, tin, tout, L, hcheck);
  return L->m;
}

/* The intervals a render samples: HCheck's when the tree has a footprint, else the leaves'. */
static int trace_ray(const otree* T, const double o[3], const double d[3], ivlist* L) {
  return trace_ray_mode(T, o, d, L, T->footprint > 0.0f);
}

/* The ray's leaf-interval count, which sets the samples per interval in either mode. */
static int leaf_count(const otree* T, const double o[3], const double d[3]) {
  ivlist L = {NULL, 0, 0};
  return trace_ray_mode(T, o, d, &L, 0);
}

static void load_ray(const float* o, const float* d, int64_t R, int64_t r, double oo[3], double dd[3]) {
  for (int a = 0; a < 3; ++a) { oo[a] = (double)o[a * R + r]; dd[a] = (double)d[a * R + r]; }
}

int orc_trace_rays(const int32_t* rows, int nn, int grid_n, const float* o, const float* d,
                   int64_t R, const int64_t* ray_idx, int64_t n_sel, int cap,
                   double* t0, double* t1, int32_t* slot, int32_t* m_out, float footprint) {
  otree T;
  if (otree_init_hcheck(&T, rows, nn, grid_n, footprint)) { otree_free(&T); return -1; }
  oiv* buf = (oiv*)malloc(sizeof(oiv) * (T.n_leaves + 1));
  for (int64_t s = 0; s < n_sel; ++s) {
    int64_t r = ray_idx ? ray_idx[s] : s;
    double oo[3], dd[3];
    load_ray(o, d, R, r, oo, dd);
    ivlist L = {buf, 0, T.n_leaves + 1};
    int m = trace_ray(&T, oo, dd, &L);
    m_out[s] = m;
    for (int k = 0; k < m && k < cap; ++k) {
      t0[s * cap + k] = buf[k].t0; t1[s * cap + k] = buf[k].t1; slot[s * cap + k] = buf[k].slot;
    }
  }
  free(buf);
  otree_free(&T);
  return 0;
}

/* A ray is robust when every interval is at least min_len long and its leaf sequence is
   unchanged when o moves by +-eps along each axis.  Node ids are compared only there. */
int orc_robust(const int32_t* rows, int nn, int grid_n, const float* o, const float* d,
               int64_t R, const int64_t* ray_idx, int64_t n_sel, double min_len, double eps,
               int32_t* robust, float footprint) {
  otree T;
  if (otree_init_hcheck(&T, rows, nn, grid_n, footprint)) { otree_free(&T); return -1; }
  int cap = T.n_leaves + 1;
  oiv* a = (oiv*)malloc(sizeof(oiv) * cap);
  oiv* b = (oiv*)malloc(sizeof(oiv) * cap);
  for (int64_t s = 0; s < n_sel; ++s) {
    int64_t r = ray_idx ? ray_idx[s] : s;
    double oo[3], dd[3];
    load_ray(o, d, R, r, oo, dd);
    ivlist La = {a, 0, cap};
    int m = trace_ray(&T, oo, dd, &La);
    int ok = 1;
    for (int k = 0; k < m; ++k) if (a[k].t1 - a[k].t0 < min_len) ok = 0;
    for (int ax = 0; ax < 3 && ok; ++ax)
      for (int sg = -1; sg <= 1 && ok; sg += 2) {
        double op[3] = {oo[0], oo[1], oo[2]};
        op[ax] += sg * eps;
        ivlist Lb = {b, 0, cap};
        int mb = trace_ray(&T, op, dd, &Lb);
        if (mb != m) { ok = 0; break; }
        for (int k = 0; k < m; ++k) if (a[k].slot != b[k].slot) ok = 0;
      }
    robust[s] = ok;
  }
  free(a); free(b);
  otree_free(&T);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Sampling (Algorithm 1, Sampling)                                           */
/* ------------------------------------------------------------------------- */
/* splitmix64 (Steele, Lea, Flood 2014; constants as published by Vigna). */
static uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Offset u in [0,1) of the stratified samples of interval k of ray r: 1/2 (the centred
   one-dimensional lattice) unless jittered, then a counter-based hash of (seed, r, k). */
static double stratum_offset(int jitter, uint64_t seed, int64_t r, int k) {
  if (!jitter) return 0.5;
  uint64_t h = splitmix64(seed ^ ((uint64_t)r * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)k * 0xD1B54A32D192ED03ull));
  return (double)(h >> 40) * (1.0 / 16777216.0);
}

/* Equal count per interval: n = max(1, floor(S_max/m)) for a ray crossing m leaves; when
   m > S_max only the first S_max intervals receive one sample each.  Under hierarchical
   sampling the ray has m' <= m intervals and each still gets the leaf share n (a node
   that stops the descent is sampled like one leaf interval). */
static int samples_per_interval(int m, int s_max) { return m <= s_max ? s_max / m : 1; }

typedef struct { int slot; double t, delta; } osample;

/* m: the ray's intervals in iv; m_leaf: its leaf-interval count (m_leaf = m without
   hierarchical sampling). */
static int make_samples(const oiv* iv, int m, int m_leaf, int s_max, int jitter, uint64_t seed, int64_t r,
                        osample* out) {
  if (m == 0) return 0;
  int n = samples_per_interval(m_leaf, s_max);
  int meff = m <= s_max ? m : s_max;
  int c = 0;
  for (int k = 0; k < meff; ++k) {
    double len = iv[k].t1 - iv[k].t0;
    double u = stratum_offset(jitter, seed, r, k);
    for (int j = 0; j < n; ++j) {
      out[c].slot = iv[k].slot;
      out[c].t = iv[k].t0 + ((double)j + u) / (double)n * len;
      out[c].delta = len / (double)n;
      ++c;
    }
  }
  return c;
}

/* ------------------------------------------------------------------------- */
/* Per-leaf MLP (Section 3.1)                                                 */
/* ------------------------------------------------------------------------- */
typedef struct { int n_lin; int din[MAX_LAYERS], dout[MAX_LAYERS]; int off_w[MAX_LAYERS], off_b[MAX_LAYERS]; int P; } olayout;

static int make_layout(int n_hidden, int hidden, olayout* L) {
  if (n_hidden < 1 || n_hidden + 1 > MAX_LAYERS || hidden < 1 || hidden > MAX_HIDDEN) return -1;
  L->n_lin = n_hidden + 1;
  int off = 0;
  for (int l = 0; l < L->n_lin; ++l) {
    L->din[l] = l == 0 ? IN_DIM : hidden;
    L->dout[l] = l == L->n_lin - 1 ? OUT_DIM : hidden;
    L->off_w[l] = off; off += L->din[l] * L->dout[l];
    L->off_b[l] = off; off += L->dout[l];
  }
  L->P = off;
  return 0;
}

/* gamma(p) for p = 2x - 1: [p, sin(2^k pi p), cos(2^k pi p) for k = 0..3], then d. */
static void features(const double x[3], const double dir[3], double u[IN_DIM]) {
  double p[3];
  for (int a = 0; a < 3; ++a) p[a] = 2.0 * x[a] - 1.0;
  for (int a = 0; a < 3; ++a) u[a] = p[a];
  for (int k = 0; k < 4; ++k) {
    double f = ldexp(M_PI, k);
    for (int a = 0; a < 3; ++a) {
      u[3 + 6 * k + a] = sin(f * p[a]);
      u[3 + 6 * k + 3 + a] = cos(f * p[a]);
    }
  }
  for (int a = 0; a < 3; ++a) u[27 + a] = dir[a];
}

static double softplus(double z) { return (z > 0 ? z : 0.0) + log1p(exp(-fabs(z))); }
static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

/* Nearest OCP e4m3 value of x in [0, 448] (3 mantissa bits; normal values from 2^-6,
   subnormal steps of 2^-9; largest finite value 448), ties to even; x >= 448 gives 448. */
static double e4m3_round(double x) {
  if (x >= 448.0) return 448.0;
  if (x < ldexp(1.0, -6)) return ldexp(nearbyint(ldexp(x, 9)), -9);
  int e;
  frexp(x, &e);                      /* x in [2^(e-1), 2^e): the step is 2^(e-4) */
  return ldexp(nearbyint(ldexp(x, 4 - e)), e - 4);
}

double orc_e4m3_round(double x) { return e4m3_round(x); }

/* Nearest bfloat16 value of x (8 significant bits), ties to even. */
static double bf16_round(double x) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  frexp(x, &e);                      /* |x| in [2^(e-1), 2^e): the step is 2^(e-8) */
  return ldexp(nearbyint(ldexp(x, 8 - e)), e - 8);
}

double orc_bf16_round(double x) { return bf16_round(x); }

/* A ReLU output a >= 0 held as float8 with scale 2^k, saturating at 256 * 2^k (the largest
   power of two e4m3 holds): 2^k * e4m3(min(a / 2^k, 256)). */
static double act_round(double a, int k) {
  const double x = ldexp(a, -k);
  return ldexp(e4m3_round(x < 256.0 ? x : 256.0), k);
}

/* Forward of one leaf MLP.  acts (optional) receives the input features followed by the
   pre-activation of every layer (widths din[0], dout[0], ..., dout[last]).  aexp (optional,
   one exponent per hidden layer): the float8 model -- the input features are rounded to
   bfloat16 (the first layer's operands), and each hidden layer's ReLU outputs are rounded by
   act_round with that layer's exponent before the next layer reads them. */
static void mlp_forward(const olayout* L, const double* P, const double u[IN_DIM], double out[OUT_DIM],
                        double* acts, const int32_t* aexp) {
  double a[MAX_HIDDEN], z[MAX_HIDDEN];
  int w = IN_DIM;
  for (int i = 0; i < IN_DIM; ++i) a[i] = aexp ? bf16_round(u[i]) : u[i];
  double* rec = acts;
  if (rec) { memcpy(rec, u, sizeof(double) * IN_DIM); rec += IN_DIM; }
  for (int l = 0; l < L->n_lin; ++l) {
    const double* W = P + L->off_w[l];
    const double* b = P + L->off_b[l];
    for (int o = 0; o < L->dout[l]; ++o) {
      double s = b[o];
      for (int i = 0; i < w; ++i) s += W[o * w + i] * a[i];
      z[o] = s;
    }
    if (rec) { memcpy(rec, z, sizeof(double) * L->dout[l]); rec += L->dout[l]; }
    w = L->dout[l];
    if (l < L->n_lin - 1)
      for (int o = 0; o < w; ++o) {
        a[o] = z[o] > 0.0 ? z[o] : 0.0;
        if (aexp) a[o] = act_round(a[o], aexp[l]);
      }
  }
  out[0] = softplus(z[0]);
  for (int c = 1; c < OUT_DIM; ++c) out[c] = sigmoid(z[c]);
}

static int mlp_eval(const float* params_leaf, int n_hidden, int hidden, const double* x,
                    const double* dir, int64_t n, double* out, double* feat, const int32_t* aexp) {
  olayout L;
  if (make_layout(n_hidden, hidden, &L)) return -1;
  double* P = (double*)malloc(sizeof(double) * L.P);
  for (int i = 0; i < L.P; ++i) P[i] = (double)params_leaf[i];
  for (int64_t s = 0; s < n; ++s) {
    double u[IN_DIM];
    features(x + 3 * s, dir + 3 * s, u);
    if (feat) memcpy(feat + IN_DIM * s, u, sizeof(u));
    mlp_forward(&L, P, u, out + OUT_DIM * s, NULL, aexp);
  }
  free(P);
  return 0;
}

int orc_mlp_eval(const float* params_leaf, int n_hidden, int hidden, const double* x,
                 const double* dir, int64_t n, double* out, double* feat) {
  return mlp_eval(params_leaf, n_hidden, hidden, x, dir, n, out, feat, NULL);
}

/* As orc_mlp_eval, with float8 hidden activations: act_exp[n_hidden] (the leaf's exponents). */
int orc_mlp_eval_q8(const float* params_leaf, int n_hidden, int hidden, const double* x,
                    const double* dir, int64_t n, const int32_t* act_exp, double* out) {
  if (!act_exp) return -1;
  return mlp_eval(params_leaf, n_hidden, hidden, x, dir, n, out, NULL, act_exp);
}

/* ------------------------------------------------------------------------- */
/* Volume rendering (Section 3.1 -> NeRF quadrature) with early termination   */
/* ------------------------------------------------------------------------- */
#define FLAG_ERT_AMBIGUOUS 1
#define FLAG_ERT_FIRED 2
#define FLAG_CLIPPED 4
#define FLAG_OCC_AMBIGUOUS 8

typedef struct {
  const otree* T;
  const olayout* L;
  const double* P;      /* [n_leaves][P] */
  const float *o, *d;
  int64_t R;
  int s_max;
  double eps;
  int jitter;
  uint64_t seed;
  const uint8_t* occ;   /* empty-space skipping: G^3 occupancy cells, or NULL */
  int occ_g;
  const int32_t* aexp;  /* float8 activations: [n_leaves][n_hidden] exponents, or NULL */
} octx;

/* Per-ray result plus optional per-sample record. */
typedef struct {
  double rgb[3], depth, opac;
  int n_samples, n_used, flags, m;
} oray;

/* Occupancy of the cell holding x: floor(x G) per axis, clamped to [0, G-1]. */
static int occ_at(const octx* C, const double x[3]) {
  int c[3];
  for (int a = 0; a < 3; ++a) {
    double f = floor(x[a] * (double)C->occ_g);
    c[a] = f < 0.0 ? 0 : (f > (double)(C->occ_g - 1) ? C->occ_g - 1 : (int)f);
  }
  return C->occ[(int64_t)c[0] + (int64_t)C->occ_g * ((int64_t)c[1] + (int64_t)C->occ_g * c[2])] != 0;
}

/* A sample whose occupancy changes when it moves by 2e-6 along an axis: a float32 position
   may land on the other side of the cell boundary. */
static int occ_ambiguous(const octx* C, const double x[3]) {
  int v = occ_at(C, x);
  for (int a = 0; a < 3; ++a)
    for (int sg = -1; sg <= 1; sg += 2) {
      double y[3] = {x[0], x[1], x[2]};
      y[a] += sg * 2e-6;
      if (occ_at(C, y) != v) return 1;
    }
  return 0;
}

static void render_ray(const octx* C, int64_t r, oiv* ivbuf, osample* sbuf, oray* res,
                       double* s_sigma, double* s_rgb, double* s_w) {
  double oo[3], dd[3];
  load_ray(C->o, C->d, C->R, r, oo, dd);
  ivlist L = {ivbuf, 0, C->T->n_leaves + 1};
  int m = trace_ray(C->T, oo, dd, &L);
  int m_leaf = C->T->footprint > 0.0f ? leaf_count(C->T, oo, dd) : m;
  int ns = make_samples(ivbuf, m, m_leaf, C->s_max, C->jitter, C->seed, r, sbuf);
  memset(res, 0, sizeof(*res));
  res->m = m;
  res->n_samples = ns;
  if (m > C->s_max) res->flags |= FLAG_CLIPPED;
  if (C->occ) {
    /* empty-space skipping: a sample in an empty cell is dropped (density 0); the count
       reported is that of the kept samples */
    int kept = 0;
    for (int j = 0; j < ns; ++j) {
      double x[3];
      for (int a = 0; a < 3; ++a) x[a] = oo[a] + sbuf[j].t * dd[a];
      kept += occ_at(C, x);
      if (occ_ambiguous(C, x)) res->flags |= FLAG_OCC_AMBIGUOUS;
    }
    res->n_samples = kept;
  }
  double S = 0.0;
  int used = 0;
  for (int j = 0; j < ns; ++j) {
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = oo[a] + sbuf[j].t * dd[a];
    if (C->occ && !occ_at(C, x)) {
      if (s_sigma) s_sigma[j] = 0.0;
      if (s_rgb) for (int c = 0; c < 3; ++c) s_rgb[3 * j + c] = 0.0;
      if (s_w) s_w[j] = 0.0;
      used = j + 1;
      continue;
    }
    double u[IN_DIM], out[OUT_DIM];
    features(x, dd, u);
    mlp_forward(C->L, C->P + (int64_t)sbuf[j].slot * C->L->P, u, out, NULL,
                C->aexp ? C->aexp + (int64_t)sbuf[j].slot * (C->L->n_lin - 1) : NULL);
    double tau = out[0] * sbuf[j].delta;
    double T = exp(-S);
    double alpha = -expm1(-tau);
    double w = T * alpha;
    for (int c = 0; c < 3; ++c) res->rgb[c] += w * out[1 + c];
    res->depth += w * sbuf[j].t;
    res->opac += w;
    if (s_sigma) s_sigma[j] = out[0];
    if (s_rgb) for (int c = 0; c < 3; ++c) s_rgb[3 * j + c] = out[1 + c];
    if (s_w) s_w[j] = w;
    S += tau;
    used = j + 1;
    if (C->eps > 0.0) {
      double Tn = exp(-S);
      if (fabs(Tn - C->eps) <= 1e-4 * C->eps) res->flags |= FLAG_ERT_AMBIGUOUS;
      if (Tn < C->eps) { res->flags |= FLAG_ERT_FIRED; break; }
    }
  }
  /* samples after the stop are not evaluated: record them as zero */
  for (int j = used; j < ns; ++j) {
    if (s_w) s_w[j] = 0.0;
    if (s_sigma) s_sigma[j] = 0.0;
    if (s_rgb) for (int c = 0; c < 3; ++c) s_rgb[3 * j + c] = 0.0;
  }
  res->n_used = used;
}

/* n_leaves: parameter sets in params, one per leaf (one per node under hierarchical
   sampling, footprint > 0). */
static int make_ctx(octx* C, otree* T, olayout* L, double** P, const int32_t* rows, int nn, int grid_n,
                    const float* params, int n_leaves, int n_hidden, int hidden, float footprint) {
  if (otree_init_hcheck(T, rows, nn, grid_n, footprint)) return -1;
  if (make_layout(n_hidden, hidden, L)) return -1;
  if ((footprint > 0.0f ? T->nn : T->n_leaves) != n_leaves) return -1;
  *P = (double*)malloc(sizeof(double) * (int64_t)n_leaves * L->P);
  for (int64_t i = 0; i < (int64_t)n_leaves * L->P; ++i) (*P)[i] = (double)params[i];
  C->T = T; C->L = L; C->P = *P;
  C->occ = NULL; C->occ_g = 0;
  C->aexp = NULL;
  return 0;
}

/* Renders the selected rays (all rays when ray_idx is NULL); aexp: see octx. */
static int render_impl(const int32_t* rows, int nn, int grid_n, const float* params, int n_leaves,
                       int n_hidden, int hidden, const float* o, const float* d, int64_t R,
                       const int64_t* ray_idx, int64_t n_sel, int s_max, double eps, int jitter,
                       uint64_t seed, double* rgb, double* depth, double* opac, int32_t* n_samples,
                       int32_t* flags, int n_threads, float footprint, const uint8_t* occ, int occ_g,
                       const int32_t* aexp) {
  if (s_max < 1 || (occ && occ_g < 1)) return -1;
  otree T; olayout L; double* P = NULL; octx C;
  if (make_ctx(&C, &T, &L, &P, rows, nn, grid_n, params, n_leaves, n_hidden, hidden, footprint)) {
    free(P); otree_free(&T); return -1;
  }
  C.o = o; C.d = d; C.R = R; C.s_max = s_max; C.eps = eps; C.jitter = jitter; C.seed = seed;
  C.occ = occ; C.occ_g = occ_g;
  C.aexp = aexp;
  int cap_iv = T.n_leaves + 1;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
  {
    oiv* ivbuf = (oiv*)malloc(sizeof(oiv) * cap_iv);
    osample* sbuf = (osample*)malloc(sizeof(osample) * (s_max + 1));
#pragma omp for schedule(dynamic, 64)
    for (int64_t s = 0; s < n_sel; ++s) {
      int64_t r = ray_idx ? ray_idx[s] : s;
      oray res;
      render_ray(&C, r, ivbuf, sbuf, &res, NULL, NULL, NULL);
      for (int c = 0; c < 3; ++c) rgb[3 * s + c] = res.rgb[c];
      depth[s] = res.depth;
      opac[s] = res.opac;
      if (n_samples) n_samples[s] = res.n_samples;
      if (flags) flags[s] = res.flags;
    }
    free(ivbuf);
    free(sbuf);
  }
  free(P);
  otree_free(&T);
  return 0;
}

int orc_render(const int32_t* rows, int nn, int grid_n, const float* params, int n_leaves,
               int n_hidden, int hidden, const float* o, const float* d, int64_t R,
               const int64_t* ray_idx, int64_t n_sel, int s_max, double eps, int jitter,
               uint64_t seed, double* rgb, double* depth, double* opac, int32_t* n_samples,
               int32_t* flags, int n_threads, float footprint, const uint8_t* occ, int occ_g) {
  return render_impl(rows, nn, grid_n, params, n_leaves, n_hidden, hidden, o, d, R, ray_idx, n_sel, s_max,
                     eps, jitter, seed, rgb, depth, opac, n_samples, flags, n_threads, footprint, occ, occ_g,
                     NULL);
}

/* Leaf samples only (no hierarchical sampling, no skipping), float8 hidden activations with
   the exponents act_exp[n_leaves][n_hidden]. */
int orc_render_q8(const int32_t* rows, int nn, int grid_n, const float* params, int n_leaves,
                  int n_hidden, int hidden, const float* o, const float* d, int64_t R,
                  const int64_t* ray_idx, int64_t n_sel, int s_max, double eps, const int32_t* act_exp,
                  double* rgb, double* depth, double* opac, int n_threads) {
  if (!act_exp) return -1;
  return render_impl(rows, nn, grid_n, params, n_leaves, n_hidden, hidden, o, d, R, ray_idx, n_sel, s_max,
                     eps, 0, 0, rgb, depth, opac, NULL, NULL, n_threads, 0.0f, NULL, 0, act_exp);
}

/* Calibration maxima: out[n_leaves][n_hidden] = the largest ReLU output of each hidden layer
   of each leaf over every sample placed on the selected rays (all of a ray's samples, with
   no early termination; float64 weights as given), 0 where a leaf has no sample. */
int orc_act_max(const int32_t* rows, int nn, int grid_n, const float* params, int n_leaves,
                int n_hidden, int hidden, const float* o, const float* d, int64_t R,
                const int64_t* ray_idx, int64_t n_sel, int s_max, double* out, int n_threads) {
  if (s_max < 1) return -1;
  otree T; olayout L; double* P = NULL; octx C;
  if (make_ctx(&C, &T, &L, &P, rows, nn, grid_n, params, n_leaves, n_hidden, hidden, 0.0f)) {
    free(P); otree_free(&T); return -1;
  }
  const int nt = n_threads > 0 ? n_threads : 1;
  const int64_t nmax = (int64_t)n_leaves * n_hidden;
  double* part = (double*)calloc((size_t)(nt * nmax), sizeof(double));
  int act_w = IN_DIM;
  for (int l = 0; l < L.n_lin; ++l) act_w += L.dout[l];
#pragma omp parallel num_threads(nt)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* mx = part + (int64_t)tid * nmax;
    oiv* ivbuf = (oiv*)malloc(sizeof(oiv) * (T.n_leaves + 1));
    osample* sbuf = (osample*)malloc(sizeof(osample) * (s_max + 1));
    double* acts = (double*)malloc(sizeof(double) * act_w);
#pragma omp for schedule(dynamic, 64)
    for (int64_t s = 0; s < n_sel; ++s) {
      int64_t r = ray_idx ? ray_idx[s] : s;
      double oo[3], dd[3];
      load_ray(o, d, R, r, oo, dd);
      ivlist IL = {ivbuf, 0, T.n_leaves + 1};
      int m = trace_ray(&T, oo, dd, &IL);
      int ns = make_samples(ivbuf, m, m, s_max, 0, 0, r, sbuf);
      for (int j = 0; j < ns; ++j) {
        double x[3], u[IN_DIM], res[OUT_DIM];
        for (int a = 0; a < 3; ++a) x[a] = oo[a] + sbuf[j].t * dd[a];
        features(x, dd, u);
        mlp_forward(&L, P + (int64_t)sbuf[j].slot * L.P, u, res, acts, NULL);
        const double* z = acts + IN_DIM;
        for (int l = 0; l < n_hidden; ++l) {
          double* cell = mx + (int64_t)sbuf[j].slot * n_hidden + l;
          for (int k = 0; k < L.dout[l]; ++k)
            if (z[k] > *cell) *cell = z[k];
          z += L.dout[l];
        }
      }
    }
    free(ivbuf); free(sbuf); free(acts);
  }
  for (int64_t i = 0; i < nmax; ++i) {
    double v = 0.0;
    for (int t = 0; t < nt; ++t) if (part[(int64_t)t * nmax + i] > v) v = part[(int64_t)t * nmax + i];
    out[i] = v;
  }
  free(part);
  free(P);
  otree_free(&T);
  return 0;
}

/* Per-sample record of one ray, front to back: leaf slot, t, delta, sigma, rgb, weight.
   Returns the number of samples (<= cap) or -1. */
int orc_ray_samples(const int32_t* rows, int nn, int grid_n, const float* params, int n_leaves,
                    int n_hidden, int hidden, const float* o, const float* d, int64_t R,
                    int64_t r, int s_max, double eps, int jitter, uint64_t seed, int cap,
                    int32_t* slot, double* t, double* delta, double* sigma, double* rgb3,
                    double* w, double* ray_out /* rgb3, depth, opac, flags, n_used */, float footprint) {
  otree T; olayout L; double* P = NULL; octx C;
  if (make_ctx(&C, &T, &L, &P, rows, nn, grid_n, params, n_leaves, n_hidden, hidden, footprint)) {
    free(P); otree_free(&T); return -1;
  }
  C.o = o; C.d = d; C.R = R; C.s_max = s_max; C.eps = eps; C.jitter = jitter; C.seed = seed;
  C.occ = NULL; C.occ_g = 0;
  oiv* ivbuf = (oiv*)malloc(sizeof(oiv) * (T.n_leaves + 1));
  osample* sbuf = (osample*)malloc(sizeof(osample) * (s_max + 1));
  double* sg = (double*)malloc(sizeof(double) * (s_max + 1));
  double* sc = (double*)malloc(sizeof(double) * 3 * (s_max + 1));
  double* sw = (double*)malloc(sizeof(double) * (s_max + 1));
  oray res;
  render_ray(&C, r, ivbuf, sbuf, &res, sg, sc, sw);
  int ns = res.n_samples;
  if (ns > cap) ns = -1;
  for (int j = 0; j < ns; ++j) {
    slot[j] = sbuf[j].slot; t[j] = sbuf[j].t; delta[j] = sbuf[j].delta;
    sigma[j] = sg[j]; w[j] = sw[j];
    for (int c = 0; c < 3; ++c) rgb3[3 * j + c] = sc[3 * j + c];
  }
  if (ray_out) {
    for (int c = 0; c < 3; ++c) ray_out[c] = res.rgb[c];
    ray_out[3] = res.depth; ray_out[4] = res.opac; ray_out[5] = res.flags; ray_out[6] = res.n_used;
  }
  free(ivbuf); free(sbuf); free(sg); free(sc); free(sw); free(P);
  otree_free(&T);
  return ns;
}

/* ------------------------------------------------------------------------- */
/* Gradient of the rendered outputs w.r.t. all leaf parameters                */
/* ------------------------------------------------------------------------- */
/* Given g = dL/d(rgb, depth, opacity) per ray, accumulates dL/dtheta into grad[L][P].
   Along a ray with samples j <= J kept by early termination:
     dC/dc_j = w_j,   dC/dtau_j = T_{j+1} c_j - (C - sum_{i<=j} w_i c_i)
   (the same form for depth with c_j -> t_j and for opacity with c_j -> 1), then
   dtau_j/dsigma_j = delta_j, softplus' = logistic, logistic' = c(1-c), and the chain
   rule through the linear layers and ReLUs. */
int orc_render_grad(const int32_t* rows, int nn, int grid_n, const float* params, int n_leaves,
                    int n_hidden, int hidden, const float* o, const float* d, int64_t R,
                    const int64_t* ray_idx, int64_t n_sel, int s_max, double eps, int jitter,
                    uint64_t seed, const double* g_rgb, const double* g_depth,
                    const double* g_opac, double* grad, float footprint) {
  otree T; olayout L; double* P = NULL; octx C;
  if (make_ctx(&C, &T, &L, &P, rows, nn, grid_n, params, n_leaves, n_hidden, hidden, footprint)) {
    free(P); otree_free(&T); return -1;
  }
  C.o = o; C.d = d; C.R = R; C.s_max = s_max; C.eps = eps; C.jitter = jitter; C.seed = seed;
  int act_w = IN_DIM;
  for (int l = 0; l < L.n_lin; ++l) act_w += L.dout[l];
  int cap = s_max + 1;
  oiv* ivbuf = (oiv*)malloc(sizeof(oiv) * (T.n_leaves + 1));
  osample* sbuf = (osample*)malloc(sizeof(osample) * cap);
  double* acts = (double*)malloc(sizeof(double) * (int64_t)act_w * cap);
  double* outs = (double*)malloc(sizeof(double) * OUT_DIM * cap);
  double* Tj = (double*)malloc(sizeof(double) * (cap + 1));
  double* wj = (double*)malloc(sizeof(double) * cap);
  for (int64_t s = 0; s < n_sel; ++s) {
    int64_t r = ray_idx ? ray_idx[s] : s;
    double oo[3], dd[3];
    load_ray(o, d, R, r, oo, dd);
    ivlist IL = {ivbuf, 0, T.n_leaves + 1};
    int m = trace_ray(&T, oo, dd, &IL);
    int m_leaf = T.footprint > 0.0f ? leaf_count(&T, oo, dd) : m;
    int ns = make_samples(ivbuf, m, m_leaf, s_max, jitter, seed, r, sbuf);
    /* forward, keeping activations */
    double S = 0.0, Cc[3] = {0, 0, 0}, D = 0.0, A = 0.0;
    int J = ns;
    Tj[0] = 1.0;
    for (int j = 0; j < ns; ++j) {
      double x[3], u[IN_DIM];
      for (int a = 0; a < 3; ++a) x[a] = oo[a] + sbuf[j].t * dd[a];
      features(x, dd, u);
      mlp_forward(&L, P + (int64_t)sbuf[j].slot * L.P, u, outs + OUT_DIM * j, acts + (int64_t)act_w * j, NULL);
      double tau = outs[OUT_DIM * j] * sbuf[j].delta;
      double Tcur = exp(-S);
      double w = Tcur * (-expm1(-tau));
      wj[j] = w;
      for (int c = 0; c < 3; ++c) Cc[c] += w * outs[OUT_DIM * j + 1 + c];
      D += w * sbuf[j].t;
      A += w;
      S += tau;
      Tj[j + 1] = exp(-S);
      if (eps > 0.0 && Tj[j + 1] < eps) { J = j + 1; break; }
    }
    const double* gc = g_rgb + 3 * s;
    double gd = g_depth ? g_depth[s] : 0.0, ga = g_opac ? g_opac[s] : 0.0;
    double Cp[3] = {0, 0, 0}, Dp = 0.0, Ap = 0.0;
    for (int j = 0; j < J; ++j) {
      const double* out = outs + OUT_DIM * j;
      for (int c = 0; c < 3; ++c) Cp[c] += wj[j] * out[1 + c];
      Dp += wj[j] * sbuf[j].t;
      Ap += wj[j];
      double dtau = 0.0;
      for (int c = 0; c < 3; ++c) dtau += gc[c] * (Tj[j + 1] * out[1 + c] - (Cc[c] - Cp[c]));
      dtau += gd * (Tj[j + 1] * sbuf[j].t - (D - Dp));
      dtau += ga * (Tj[j + 1] - (A - Ap));
      double dsig = dtau * sbuf[j].delta;
      /* output pre-activations */
      const double* act = acts + (int64_t)act_w * j;
      int zoff = act_w - OUT_DIM;
      double dz[MAX_HIDDEN], dh[MAX_HIDDEN];
      dz[0] = dsig * sigmoid(act[zoff + 0]);
      for (int c = 0; c < 3; ++c) dz[1 + c] = gc[c] * wj[j] * out[1 + c] * (1.0 - out[1 + c]);
      double* G = grad + (int64_t)sbuf[j].slot * L.P;
      const double* Pl = P + (int64_t)sbuf[j].slot * L.P;
      for (int l = L.n_lin - 1; l >= 0; --l) {
        int din = L.din[l], dout = L.dout[l];
        /* input of layer l: features for l == 0, else ReLU of layer l-1's pre-activation */
        int in_off = IN_DIM;
        for (int k = 0; k < l - 1; ++k) in_off += L.dout[k];
        const double* zin = l == 0 ? act : act + in_off;
        double xin[MAX_HIDDEN];
        for (int i = 0; i < din; ++i) xin[i] = l == 0 ? zin[i] : (zin[i] > 0.0 ? zin[i] : 0.0);
        const double* W = Pl + L.off_w[l];
        for (int oi = 0; oi < dout; ++oi) {
          G[L.off_b[l] + oi] += dz[oi];
          for (int i = 0; i < din; ++i) G[L.off_w[l] + oi * din + i] += dz[oi] * xin[i];
        }
        if (l == 0) break;
        for (int i = 0; i < din; ++i) {
          double acc = 0.0;
          for (int oi = 0; oi < dout; ++oi) acc += W[oi * din + i] * dz[oi];
          dh[i] = zin[i] > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < din; ++i) dz[i] = dh[i];
      }
    }
  }
  free(ivbuf); free(sbuf); free(acts); free(outs); free(Tj); free(wj); free(P);
  otree_free(&T);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Compositing of one ray from its samples' MLP outputs, and its gradient      */
/* ------------------------------------------------------------------------- */
/* The quadrature of Section 3.1 (the NeRF volume-rendering sum) over one ray, given per
   sample the output pre-activations z = (sigma^, r^, g^, b^), the position t and the
   segment length delta: sigma = softplus(sigma^), c = logistic(r^, g^, b^),
   tau_j = sigma_j delta_j, T_j = exp(-sum_{i<j} tau_i), w_j = T_j (1 - exp(-tau_j));
   rgb = sum w_j c_j, depth = sum w_j t_j, opacity = sum w_j, stopping after the first j
   with T_{j+1} < eps (Section 4.1 early termination; eps = 0: never).
   out[5] = (rgb, depth, opacity); w (optional) receives every sample's weight (0 after
   the stop).  Returns the number of samples composited (stop index + 1, or ns). */
int orc_composite(int ns, const double* z, const double* t, const double* delta, double eps, double* out,
                  double* w) {
  double S = 0.0;
  int used = 0;
  for (int c = 0; c < 5; ++c) out[c] = 0.0;
  if (w) for (int j = 0; j < ns; ++j) w[j] = 0.0;
  for (int j = 0; j < ns; ++j) {
    double sigma = softplus(z[4 * j]);
    double tau = sigma * delta[j];
    double wj = exp(-S) * (-expm1(-tau));
    for (int c = 0; c < 3; ++c) out[c] += wj * sigmoid(z[4 * j + 1 + c]);
    out[3] += wj * t[j];
    out[4] += wj;
    if (w) w[j] = wj;
    S += tau;
    used = j + 1;
    if (eps > 0.0 && exp(-S) < eps) break;
  }
  return used;
}

/* Gradient of L = g . (rgb, depth, opacity) of orc_composite with respect to every z:
   dz[ns][4].  With J samples composited, for j < J
     dL/dc_j = g_rgb w_j,
     dL/dtau_j = sum_c g_c (T_{j+1} c_j - sum_{J > i > j} w_i c_i)
               + g_depth (T_{j+1} t_j - sum_{J > i > j} w_i t_i) + g_opac (T_{j+1} - sum_{J > i > j} w_i)
   (moving tau_j scales the transmittance of every later sample by e^{-d tau_j} and the
   weight of sample j by its derivative), then dsigma^ = dtau delta logistic(sigma^) and
   dc^ = dc c (1 - c).  The stop index is held fixed (the loss is the truncated sum).
   Samples at or after J get 0.  Returns J. */
int orc_composite_grad(int ns, const double* z, const double* t, const double* delta, double eps,
                       const double g[5], double* dz) {
  double* w = (double*)malloc(sizeof(double) * (ns > 0 ? ns : 1));
  double* Tn = (double*)malloc(sizeof(double) * (ns > 0 ? ns : 1));
  double out[5];
  int J = orc_composite(ns, z, t, delta, eps, out, w);
  double S = 0.0;
  for (int j = 0; j < J; ++j) {
    S += softplus(z[4 * j]) * delta[j];
    Tn[j] = exp(-S);
  }
  /* suffix sums over i > j of w_i c_i, w_i t_i, w_i */
  double suf[5] = {0, 0, 0, 0, 0};
  for (int j = ns - 1; j >= 0; --j) {
    double* d = dz + 4 * j;
    if (j >= J) { d[0] = d[1] = d[2] = d[3] = 0.0; continue; }
    double c[3];
    for (int k = 0; k < 3; ++k) c[k] = sigmoid(z[4 * j + 1 + k]);
    double dtau = 0.0;
    for (int k = 0; k < 3; ++k) dtau += g[k] * (Tn[j] * c[k] - suf[k]);
    dtau += g[3] * (Tn[j] * t[j] - suf[3]);
    dtau += g[4] * (Tn[j] - suf[4]);
    d[0] = dtau * delta[j] * sigmoid(z[4 * j]);
    for (int k = 0; k < 3; ++k) d[1 + k] = g[k] * w[j] * c[k] * (1.0 - c[k]);
    for (int k = 0; k < 3; ++k) suf[k] += w[j] * c[k];
    suf[3] += w[j] * t[j];
    suf[4] += w[j];
  }
  free(w);
  free(Tn);
  return J;
}

/* ------------------------------------------------------------------------- */
/* Adam (Kingma & Ba 2015) with bias correction                               */
/* ------------------------------------------------------------------------- */
void orc_adam(double* p, double* m, double* v, const double* g, int64_t n, int step, double lr,
              double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    double mh = m[i] / c1, vh = v[i] / c2;
    p[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* Exposed for the published-vector check of the counter-based generator. */
uint64_t orc_splitmix64(uint64_t x) { return splitmix64(x); }
double orc_stratum_offset(int jitter, uint64_t seed, int64_t r, int k) {
  return stratum_offset(jitter, seed, r, k);
}

/* ------------------------------------------------------------------------- */
/* Learned proposal (not in the paper; it only cites sample-predicting        */
/* networks as prior art).  Per (ray, leaf interval): 43 features ->          */
/* 64 -> 64 (ReLU) -> 32 bin optical thicknesses tau^ = softplus(.), bins     */
/* uniform over the interval.  Compositing the bins front to back along the   */
/* ray gives the predicted weight histogram over the ray's leaf intervals.    */
/* ------------------------------------------------------------------------- */
#define PROP_IN 43
#define PROP_H 64
#define PROP_BINS 32
#define PROP_P (PROP_H * PROP_IN + PROP_H + PROP_H * PROP_H + PROP_H + PROP_BINS * PROP_H + PROP_BINS)

/* [q, d, sin/cos(2^k pi q) k=0,1, sin/cos(2^k pi d) k=0,1, k/S_max, 2*centre-1, size,
    2*entry-1, 2*exit-1] with q = (o - 1/2)/2; sin block before cos block per k. */
static void prop_features(const double o[3], const double d[3], double t0, double t1, int k, int s_max,
                          const int32_t* row, int grid_n, double f[PROP_IN]) {
  double q[3];
  int c = 0;
  for (int a = 0; a < 3; ++a) q[a] = (o[a] - 0.5) * 0.5;
  for (int a = 0; a < 3; ++a) f[c++] = q[a];
  for (int a = 0; a < 3; ++a) f[c++] = d[a];
  for (int src = 0; src < 2; ++src) {
    const double* v = src == 0 ? q : d;
    for (int kk = 0; kk < 2; ++kk) {
      double fr = ldexp(M_PI, kk);
      for (int a = 0; a < 3; ++a) f[c++] = sin(fr * v[a]);
      for (int a = 0; a < 3; ++a) f[c++] = cos(fr * v[a]);
    }
  }
  f[c++] = (double)k / (double)s_max;
  for (int a = 0; a < 3; ++a) f[c++] = (double)(row[2 + a] + row[5 + a]) / (double)grid_n - 1.0;
  for (int a = 0; a < 3; ++a) f[c++] = (double)(row[5 + a] - row[2 + a]) / (double)grid_n;
  for (int a = 0; a < 3; ++a) f[c++] = 2.0 * (o[a] + t0 * d[a]) - 1.0;
  for (int a = 0; a < 3; ++a) f[c++] = 2.0 * (o[a] + t1 * d[a]) - 1.0;
}

/* acts (optional): z0[64], z1[64], zo[32] pre-activations. */
static void prop_forward(const double* P, const double f[PROP_IN], double tau[PROP_BINS], double* acts) {
  const double* W0 = P;
  const double* b0 = W0 + PROP_H * PROP_IN;
  const double* W1 = b0 + PROP_H;
  const double* b1 = W1 + PROP_H * PROP_H;
  const double* W2 = b1 + PROP_H;
  const double* b2 = W2 + PROP_BINS * PROP_H;
  double z0[PROP_H], h0[PROP_H], z1[PROP_H], h1[PROP_H], zo[PROP_BINS];
  for (int o = 0; o < PROP_H; ++o) {
    double s = b0[o];
    for (int i = 0; i < PROP_IN; ++i) s += W0[o * PROP_IN + i] * f[i];
    z0[o] = s;
    h0[o] = s > 0.0 ? s : 0.0;
  }
  for (int o = 0; o < PROP_H; ++o) {
    double s = b1[o];
    for (int i = 0; i < PROP_H; ++i) s += W1[o * PROP_H + i] * h0[i];
    z1[o] = s;
    h1[o] = s > 0.0 ? s : 0.0;
  }
  for (int o = 0; o < PROP_BINS; ++o) {
    double s = b2[o];
    for (int i = 0; i < PROP_H; ++i) s += W2[o * PROP_H + i] * h1[i];
    zo[o] = s;
    tau[o] = softplus(s);
  }
  if (acts) {
    memcpy(acts, z0, sizeof(z0));
    memcpy(acts + PROP_H, z1, sizeof(z1));
    memcpy(acts + 2 * PROP_H, zo, sizeof(zo));
  }
}

/* Length of [a0, a1) intersected with [b0, b1). */
static double overlap(double a0, double a1, double b0, double b1) {
  double lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
  return hi > lo ? hi - lo : 0.0;
}

typedef struct {
  int n_sel;          /* selected plain slots (-1: fallback to all plain slots) */
  int n_plain;        /* plain slots of the ray */
  double mass;        /* predicted mass M^ = 1 - T^_end */
} oplan;

/* Slot indices ordered by decreasing p, equal p in increasing index (stable insertion). */
static void order_desc(const double* p, int n, int* order) {
  for (int j = 0; j < n; ++j) {
    int q = j;
    while (q > 0 && p[order[q - 1]] < p[j]) { order[q] = order[q - 1]; --q; }
    order[q] = j;
  }
}

/* Plan of one ray: predicted slot masses p_j of the plain slots, then the fewest slots of
   largest p (ties: earlier slot) whose sum reaches mass_thresh * M^, if M^ >= mass_thresh and
   that set has at most cap slots; otherwise fallback.  sel[] receives the chosen plain slot
   indices in increasing order. */
/* tau_in: when not NULL, the bins' optical thicknesses of the ray's intervals ([meff][32])
   are taken from it instead of the network (for pins with known thicknesses). */
static void plan_ray(const otree* T, const double* PP, const double o[3], const double d[3], const oiv* iv,
                     int m, int s_max, double mass_thresh, int cap, oplan* pl, int* sel, double* p_out,
                     const double* tau_in) {
  pl->n_sel = -1;
  pl->mass = 0.0;
  pl->n_plain = 0;
  if (m == 0) { pl->n_sel = 0; return; }
  int n = samples_per_interval(m, s_max);
  int meff = m <= s_max ? m : s_max;
  pl->n_plain = n * meff;
  double S = 0.0;
  double* p = p_out;
  for (int j = 0; j < pl->n_plain; ++j) p[j] = 0.0;
  for (int k = 0; k < meff; ++k) {
    int node = -1;
    for (int i = 0; i < T->nn; ++i) if (T->rows[(int64_t)i * NODE_COLS + 10] == iv[k].slot) { node = i; break; }
    double f[PROP_IN], tau[PROP_BINS];
    if (tau_in) {
      for (int b = 0; b < PROP_BINS; ++b) tau[b] = tau_in[k * PROP_BINS + b];
    } else {
      prop_features(o, d, iv[k].t0, iv[k].t1, k, s_max, T->rows + (int64_t)node * NODE_COLS, T->grid_n, f);
      prop_forward(PP, f, tau, NULL);
    }
    for (int b = 0; b < PROP_BINS; ++b) {
      double w = exp(-S) * (-expm1(-tau[b]));
      S += tau[b];
      /* spread the bin's weight over the plain slots it overlaps: in units of 1/(32 n) of
         the interval, slot j is [32 j, 32 (j+1)) and bin b is [b n, (b+1) n), so the covered
         fraction of the bin is an integer over n (slots inside one bin get exactly equal
         weights, which the selection must see as ties) */
      for (int j = 0; j < n; ++j) {
        int lo = PROP_BINS * j > b * n ? PROP_BINS * j : b * n;
        int hi = PROP_BINS * (j + 1) < (b + 1) * n ? PROP_BINS * (j + 1) : (b + 1) * n;
        if (hi > lo) p[k * n + j] += w * ((double)(hi - lo) / n);
      }
    }
  }
  pl->mass = -expm1(-S);
  if (pl->mass < mass_thresh) return;
  int* order = (int*)malloc(sizeof(int) * pl->n_plain);
  order_desc(p, pl->n_plain, order);
  double target = mass_thresh * pl->mass, acc = 0.0;
  int cnt = 0;
  while (cnt < pl->n_plain && acc < target) acc += p[order[cnt++]];
  if (cnt <= cap && acc >= target) {
    pl->n_sel = cnt;
    /* increasing slot order */
    char* mark = (char*)calloc(pl->n_plain, 1);
    for (int i = 0; i < cnt; ++i) mark[order[i]] = 1;
    int c = 0;
    for (int j = 0; j < pl->n_plain; ++j) if (mark[j]) sel[c++] = j;
    free(mark);
  }
  free(order);
}

/* Renders rays with the proposal: per ray the plan's slots (plain positions and segment
   lengths, centred strata) are composited front to back and the other slots are skipped;
   fallback rays use every plain slot.  Also returns the plan (n_sel per ray, -1 =
   fallback; sel[ray][cap] slot lists) and the predicted mass. */
int orc_render_proposal(const int32_t* rows, int nn, int grid_n, const float* params, int n_leaves, int n_hidden,
                        int hidden, const float* prop_params, const float* o, const float* d, int64_t R,
                        const int64_t* ray_idx, int64_t n_sel, int s_max, double eps, double mass_thresh, int cap,
                        double* rgb, double* depth, double* opac, int32_t* n_samples, int32_t* plan_n,
                        int32_t* plan_sel, double* mass, int n_threads, const double* tau_in) {
  /* tau_in (given bin thicknesses instead of the network's) serves a single ray */
  if (s_max < 1 || cap < 1 || (tau_in && n_sel != 1)) return -1;
  otree T; olayout L; double* P = NULL; octx C;
  if (make_ctx(&C, &T, &L, &P, rows, nn, grid_n, params, n_leaves, n_hidden, hidden, 0.0f)) {
    free(P); otree_free(&T); return -1;
  }
  double* PP = (double*)malloc(sizeof(double) * PROP_P);
  for (int i = 0; i < PROP_P; ++i) PP[i] = (double)prop_params[i];
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
  {
    oiv* ivbuf = (oiv*)malloc(sizeof(oiv) * (T.n_leaves + 1));
    osample* sbuf = (osample*)malloc(sizeof(osample) * (s_max + 1));
    double* p = (double*)malloc(sizeof(double) * (s_max + 1));
    int* sel = (int*)malloc(sizeof(int) * (s_max + 1));
#pragma omp for schedule(dynamic, 16)
    for (int64_t s = 0; s < n_sel; ++s) {
      int64_t r = ray_idx ? ray_idx[s] : s;
      double oo[3], dd[3];
      load_ray(o, d, R, r, oo, dd);
      ivlist IL = {ivbuf, 0, T.n_leaves + 1};
      int m = trace_ray(&T, oo, dd, &IL);
      int ns = make_samples(ivbuf, m, m, s_max, 0, 0, r, sbuf);
      oplan pl;
      plan_ray(&T, PP, oo, dd, ivbuf, m, s_max, mass_thresh, cap, &pl, sel, p, tau_in);
      int use = pl.n_sel < 0 ? ns : pl.n_sel;
      double Sacc = 0.0, cr[3] = {0, 0, 0}, dep = 0.0, op = 0.0;
      for (int q = 0; q < use; ++q) {
        int j = pl.n_sel < 0 ? q : sel[q];
        double x[3], u[IN_DIM], out[OUT_DIM];
        for (int a = 0; a < 3; ++a) x[a] = oo[a] + sbuf[j].t * dd[a];
        features(x, dd, u);
        mlp_forward(&L, P + (int64_t)sbuf[j].slot * L.P, u, out, NULL, NULL);
        double tau = out[0] * sbuf[j].delta;
        double w = exp(-Sacc) * (-expm1(-tau));
        for (int c = 0; c < 3; ++c) cr[c] += w * out[1 + c];
        dep += w * sbuf[j].t;
        op += w;
        Sacc += tau;
        if (eps > 0.0 && exp(-Sacc) < eps) break;
      }
      for (int c = 0; c < 3; ++c) rgb[3 * s + c] = cr[c];
      depth[s] = dep;
      opac[s] = op;
      if (n_samples) n_samples[s] = use;
      if (plan_n) plan_n[s] = pl.n_sel;
      if (plan_sel) for (int q = 0; q < cap; ++q) plan_sel[s * cap + q] = (pl.n_sel >= 0 && q < pl.n_sel) ? sel[q] : -1;
      if (mass) mass[s] = pl.mass;
    }
    free(ivbuf); free(sbuf); free(p); free(sel);
  }
  free(PP); free(P);
  otree_free(&T);
  return 0;
}

/* Proposal features and predicted bin thicknesses of every interval of the given rays
   (front to back, ray by ray): feat[N][43], tau[N][32]; returns N. */
int64_t orc_prop_eval(const int32_t* rows, int nn, int grid_n, const float* prop_params, const float* o,
                      const float* d, int64_t R, const int64_t* ray_idx, int64_t n_sel, int s_max, int64_t cap,
                      double* feat, double* tau) {
  otree T;
  if (otree_init(&T, rows, nn, grid_n)) { otree_free(&T); return -1; }
  double* PP = (double*)malloc(sizeof(double) * PROP_P);
  for (int i = 0; i < PROP_P; ++i) PP[i] = (double)prop_params[i];
  oiv* ivbuf = (oiv*)malloc(sizeof(oiv) * (T.n_leaves + 1));
  int64_t c = 0;
  for (int64_t s = 0; s < n_sel; ++s) {
    int64_t r = ray_idx ? ray_idx[s] : s;
    double oo[3], dd[3];
    load_ray(o, d, R, r, oo, dd);
    ivlist IL = {ivbuf, 0, T.n_leaves + 1};
    int m = trace_ray(&T, oo, dd, &IL);
    int meff = m <= s_max ? m : s_max;
    for (int k = 0; k < meff; ++k, ++c) {
      if (c >= cap) continue;
      int node = -1;
      for (int i = 0; i < T.nn; ++i) if (T.rows[(int64_t)i * NODE_COLS + 10] == ivbuf[k].slot) { node = i; break; }
      double f[PROP_IN], tt[PROP_BINS];
      prop_features(oo, dd, ivbuf[k].t0, ivbuf[k].t1, k, s_max, T.rows + (int64_t)node * NODE_COLS, grid_n, f);
      prop_forward(PP, f, tt, NULL);
      if (feat) memcpy(feat + c * PROP_IN, f, sizeof(f));
      if (tau) memcpy(tau + c * PROP_BINS, tt, sizeof(tt));
    }
  }
  free(ivbuf); free(PP);
  otree_free(&T);
  return c;
}

/* Training targets of the proposal from the plain render: per interval and bin b, the
   plain quadrature's optical thickness over the bin, tau_b = sum_j sigma_j |slot_j n bin_b|
   (lengths in t), as the bin opacity alpha_b = 1 - exp(-tau_b).  Every plain sample counts
   (targets describe the field, not one ray's early termination).  Returns the count. */
int64_t orc_prop_targets(const int32_t* rows, int nn, int grid_n, const float* params, int n_leaves, int n_hidden,
                         int hidden, const float* o, const float* d, int64_t R, const int64_t* ray_idx,
                         int64_t n_sel, int s_max, int64_t cap, double* alpha) {
  otree T; olayout L; double* P = NULL; octx C;
  if (make_ctx(&C, &T, &L, &P, rows, nn, grid_n, params, n_leaves, n_hidden, hidden, 0.0f)) {
    free(P); otree_free(&T); return -1;
  }
  oiv* ivbuf = (oiv*)malloc(sizeof(oiv) * (T.n_leaves + 1));
  osample* sbuf = (osample*)malloc(sizeof(osample) * (s_max + 1));
  int64_t c = 0;
  for (int64_t s = 0; s < n_sel; ++s) {
    int64_t r = ray_idx ? ray_idx[s] : s;
    double oo[3], dd[3];
    load_ray(o, d, R, r, oo, dd);
    ivlist IL = {ivbuf, 0, T.n_leaves + 1};
    int m = trace_ray(&T, oo, dd, &IL);
    make_samples(ivbuf, m, m, s_max, 0, 0, r, sbuf);
    int n = m == 0 ? 0 : samples_per_interval(m, s_max);
    int meff = m <= s_max ? m : s_max;
    for (int k = 0; k < meff; ++k, ++c) {
      double len = ivbuf[k].t1 - ivbuf[k].t0;
      double tb[PROP_BINS];
      for (int b = 0; b < PROP_BINS; ++b) tb[b] = 0.0;
      for (int j = 0; j < n; ++j) {
        const osample* sm = &sbuf[k * n + j];
        double x[3], u[IN_DIM], out[OUT_DIM];
        for (int a = 0; a < 3; ++a) x[a] = oo[a] + sm->t * dd[a];
        features(x, dd, u);
        mlp_forward(&L, P + (int64_t)sm->slot * L.P, u, out, NULL, NULL);
        for (int b = 0; b < PROP_BINS; ++b)
          tb[b] += out[0] * len * overlap((double)j / n, (double)(j + 1) / n, (double)b / PROP_BINS,
                                          (double)(b + 1) / PROP_BINS);
      }
      if (c < cap) for (int b = 0; b < PROP_BINS; ++b) alpha[c * PROP_BINS + b] = -expm1(-tb[b]);
    }
  }
  free(ivbuf); free(sbuf); free(P);
  otree_free(&T);
  return c;
}

/* Loss L = mean over items and bins of (alpha^ - alpha)^2 with alpha^ = 1 - exp(-tau^), and
   its gradient w.r.t. the proposal parameters (analytic, float64).  Returns L. */
double orc_prop_loss_grad(const float* prop_params, const double* feat, const double* alpha, int64_t N,
                          double* grad) {
  double* PP = (double*)malloc(sizeof(double) * PROP_P);
  for (int i = 0; i < PROP_P; ++i) PP[i] = (double)prop_params[i];
  const double* W1 = PP + PROP_H * PROP_IN + PROP_H;
  const double* W2 = W1 + PROP_H * PROP_H + PROP_H;
  double* G0 = grad;
  double* gb0 = G0 + PROP_H * PROP_IN;
  double* G1 = gb0 + PROP_H;
  double* gb1 = G1 + PROP_H * PROP_H;
  double* G2 = gb1 + PROP_H;
  double* gb2 = G2 + PROP_BINS * PROP_H;
  double loss = 0.0;
  const double scale = 1.0 / ((double)N * PROP_BINS);
  for (int64_t s = 0; s < N; ++s) {
    const double* f = feat + s * PROP_IN;
    double tau[PROP_BINS], acts[2 * PROP_H + PROP_BINS];
    prop_forward(PP, f, tau, acts);
    const double* z0 = acts;
    const double* z1 = acts + PROP_H;
    const double* zo = acts + 2 * PROP_H;
    double dzo[PROP_BINS], dh1[PROP_H], dz1[PROP_H], dh0[PROP_H], dz0[PROP_H];
    for (int b = 0; b < PROP_BINS; ++b) {
      double ah = -expm1(-tau[b]);
      double e = ah - alpha[s * PROP_BINS + b];
      loss += e * e * scale;
      /* d/dtau (1 - e^-tau) = e^-tau; d tau/d zo = logistic(zo) */
      dzo[b] = 2.0 * e * scale * exp(-tau[b]) * sigmoid(zo[b]);
    }
    for (int b = 0; b < PROP_BINS; ++b) {
      gb2[b] += dzo[b];
      for (int i = 0; i < PROP_H; ++i) G2[b * PROP_H + i] += dzo[b] * (z1[i] > 0.0 ? z1[i] : 0.0);
    }
    for (int i = 0; i < PROP_H; ++i) {
      double acc = 0.0;
      for (int b = 0; b < PROP_BINS; ++b) acc += W2[b * PROP_H + i] * dzo[b];
      dh1[i] = acc;
      dz1[i] = z1[i] > 0.0 ? acc : 0.0;
    }
    for (int o = 0; o < PROP_H; ++o) {
      gb1[o] += dz1[o];
      for (int i = 0; i < PROP_H; ++i) G1[o * PROP_H + i] += dz1[o] * (z0[i] > 0.0 ? z0[i] : 0.0);
    }
    for (int i = 0; i < PROP_H; ++i) {
      double acc = 0.0;
      for (int o = 0; o < PROP_H; ++o) acc += W1[o * PROP_H + i] * dz1[o];
      dh0[i] = acc;
      dz0[i] = z0[i] > 0.0 ? acc : 0.0;
    }
    for (int o = 0; o < PROP_H; ++o) {
      gb0[o] += dz0[o];
      for (int i = 0; i < PROP_IN; ++i) G0[o * PROP_IN + i] += dz0[o] * f[i];
    }
    (void)dh1; (void)dh0;
  }
  free(PP);
  return loss;
}

int orc_prop_param_count(void) { return PROP_P; }
