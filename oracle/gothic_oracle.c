/*
 * Oracle for the block-step Barnes-Hut tree gravity of Miki & Umemura,
 * "GOTHIC: Gravitational oct-tree code accelerated by hierarchical time step
 * controlling" (arXiv:1610.07279).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, float64 CPU
 * implementation used by the tests, the smoke check and the CPU baseline of
 * the benchmark to check the HIP library.  The product path never calls it,
 * and it shares no code, header or table with the HIP sources.
 *
 * Every function restates one step of the paper in the paper's order:
 *   keys            Section 2.1 + Appendix A (Morton: the 63-bit interleave;
 *                   Peano-Hilbert: the level-by-level rotation/inversion)
 *   sort            Section 2.1 (stable radix sort of (key, index) pairs)
 *   tree            Section 2.1 (breadth-first octree from the sorted keys)
 *   moments         Section 2.1 (pseudo j-particles: mass, centre of mass,
 *                   enclosing radius) + a quadrupole extension (second moments)
 *   groups          Section 2.3 (pseudo i-particles, geometric-centre ball of
 *                   Appendix B)
 *   walk            Sections 2.2-2.3 (opening-angle MAC of Barnes & Hut, or the
 *                   acceleration MAC of Springel, or the multipole MAC of
 *                   Warren & Salmon, with the lambda-distance of the pseudo
 *                   i-particle)
 *   direct          Section 1, the softened direct sum
 *   time levels and RK2 / leap-frog integration, Section 2.7
 * Readings where the paper is silent are stated at each function.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see build.py).
 * FP contraction stays off so every double operation is one IEEE rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NLEV 21 /* bits per axis; 3*21 = 63-bit keys (Appendix A) */

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------------- */
/* Direct sum (Section 1): a_i = sum_{j != i} m_j (r_j - r_i)/(|r_j-r_i|^2+eps^2)^{3/2}
 * and phi_i = -sum_{j != i} m_j / (|r_j-r_i|^2+eps^2)^{1/2}, G = 1.
 * The potential sign is a reading (the paper only says phi is computed).
 * idx[k] selects the i-particles; out[k*4 + {0,1,2,3}] = ax, ay, az, phi.   */
void orc_direct(int64_t n, const float *xyzm, double eps, int64_t ni,
                const int64_t *idx, double *out) {
  const double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < ni; ++k) {
    const int64_t i = idx[k];
    const double xi = xyzm[4 * i], yi = xyzm[4 * i + 1], zi = xyzm[4 * i + 2];
    double ax = 0, ay = 0, az = 0, ph = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = (double)xyzm[4 * j] - xi;
      const double dy = (double)xyzm[4 * j + 1] - yi;
      const double dz = (double)xyzm[4 * j + 2] - zi;
      const double m = xyzm[4 * j + 3];
      const double r2 = dx * dx + dy * dy + dz * dz + e2;
      const double r = sqrt(r2);
      const double inv3 = 1.0 / (r2 * r);
      ax += m * dx * inv3;
      ay += m * dy * inv3;
      az += m * dz * inv3;
      ph -= m / r;
    }
    out[4 * k] = ax;
    out[4 * k + 1] = ay;
    out[4 * k + 2] = az;
    out[4 * k + 3] = ph;
  }
}

/* ---------------------------------------------------------------------- */
/* Keys (Appendix A).  Morton: bit b of (x, y, z) goes to key bit 3b+2, 3b+1, 3b. */
uint64_t orc_morton(uint64_t x, uint64_t y, uint64_t z) {
  uint64_t key = 0;
  for (int b = 0; b < NLEV; ++b) {
    key |= ((x >> b) & 1u) << (3 * b + 2);
    key |= ((y >> b) & 1u) << (3 * b + 1);
    key |= ((z >> b) & 1u) << (3 * b);
  }
  return key;
}

/* Peano-Hilbert curve of Appendix A.  Level by level, from the coarsest: the
 * octant bits (a0, a1, a2) of the point in the current frame give the key
 * digit as the inverse Gray code of a0 a1 a2; then the frame is inverted
 * along some axes and its axes are permuted, depending on the octant.
 *
 * The frame is tracked as perm[] / flip[]: frame axis a reads original axis
 * perm[a], complemented when flip[a] is set.  Per octant o = 4 a0 + 2 a1 + a2:
 *   INV[o]  bit mask (4: axis 0, 2: axis 1, 1: axis 2) of axes inverted,
 *   ROT[o]  0 = keep, 1 = cycle (new 0,1,2 <- old 1,2,0), 2 = exchange 0 and 2.
 * These two tables were worked out by hand from the encoder printed in
 * Appendix A (inversion first, then the permutation).                        */
static const int PH_INV[8] = {0, 0, 3, 0, 5, 6, 3, 6};
static const int PH_ROT[8] = {2, 1, 0, 1, 2, 1, 0, 1};

static int inv_gray3(int g) { /* g = a0 a1 a2 (a0 most significant) */
  int d = g;
  d ^= d >> 1;
  d ^= d >> 2;
  return d & 7;
}

static void ph_update_frame(int o, int perm[3], int flip[3]) {
  int inv = PH_INV[o];
  int f[3] = {flip[0] ^ ((inv >> 2) & 1), flip[1] ^ ((inv >> 1) & 1), flip[2] ^ (inv & 1)};
  int p[3] = {perm[0], perm[1], perm[2]};
  if (PH_ROT[o] == 1) {
    perm[0] = p[1]; perm[1] = p[2]; perm[2] = p[0];
    flip[0] = f[1]; flip[1] = f[2]; flip[2] = f[0];
  } else if (PH_ROT[o] == 2) {
    perm[0] = p[2]; perm[1] = p[1]; perm[2] = p[0];
    flip[0] = f[2]; flip[1] = f[1]; flip[2] = f[0];
  } else {
    flip[0] = f[0]; flip[1] = f[1]; flip[2] = f[2];
  }
}

uint64_t orc_ph_encode(int nlev, uint64_t x, uint64_t y, uint64_t z) {
  const uint64_t c[3] = {x, y, z};
  int perm[3] = {0, 1, 2}, flip[3] = {0, 0, 0};
  uint64_t key = 0;
  for (int lev = nlev - 1; lev >= 0; --lev) {
    int a[3];
    for (int ax = 0; ax < 3; ++ax) a[ax] = (int)((c[perm[ax]] >> lev) & 1u) ^ flip[ax];
    const int o = (a[0] << 2) | (a[1] << 1) | a[2];
    key |= (uint64_t)inv_gray3(o) << (3 * lev);
    ph_update_frame(o, perm, flip);
  }
  return key;
}

void orc_ph_decode(int nlev, uint64_t key, uint64_t *x, uint64_t *y, uint64_t *z) {
  uint64_t c[3] = {0, 0, 0};
  int perm[3] = {0, 1, 2}, flip[3] = {0, 0, 0};
  for (int lev = nlev - 1; lev >= 0; --lev) {
    const int d = (int)((key >> (3 * lev)) & 7u);
    const int o = d ^ (d >> 1); /* Gray code of the digit = octant in frame */
    const int a[3] = {(o >> 2) & 1, (o >> 1) & 1, o & 1};
    for (int ax = 0; ax < 3; ++ax) c[perm[ax]] |= (uint64_t)(a[ax] ^ flip[ax]) << lev;
    ph_update_frame(o, perm, flip);
  }
  *x = c[0]; *y = c[1]; *z = c[2];
}

/* Bounding cube and quantisation (a reading; the paper does not say how the
 * positions are mapped to integers).  The cube origin is the bounding-box
 * minimum, its side L the smallest power of two >= the largest extent (1 if
 * the extent is 0), and q = min(floor((x - x_min) * 2^21 / L), 2^21 - 1) per
 * axis, all in float64.  cube[] = x_min, y_min, z_min, L.                     */
void orc_cube(int64_t n, const float *xyzm, double cube[4]) {
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      const double v = xyzm[4 * i + a];
      if (i == 0 || v < lo[a]) lo[a] = v;
      if (i == 0 || v > hi[a]) hi[a] = v;
    }
  double ext = 0;
  for (int a = 0; a < 3; ++a)
    if (hi[a] - lo[a] > ext) ext = hi[a] - lo[a];
  double L = 1.0;
  if (ext > 0) {
    int e;
    const double f = frexp(ext, &e); /* ext = f 2^e, f in [0.5, 1) */
    L = (f == 0.5) ? ext : ldexp(1.0, e);
  }
  cube[0] = lo[0]; cube[1] = lo[1]; cube[2] = lo[2]; cube[3] = L;
}

void orc_keys(int64_t n, const float *xyzm, int key_kind, const double cube[4],
              uint64_t *keys) {
  const double scale = ldexp(1.0, NLEV) / cube[3];
  const uint64_t qmax = ((uint64_t)1 << NLEV) - 1;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
      const double t = floor(((double)xyzm[4 * i + a] - cube[a]) * scale);
      q[a] = (uint64_t)t > qmax ? qmax : (uint64_t)t;
    }
    keys[i] = key_kind == 1 ? orc_ph_encode(NLEV, q[0], q[1], q[2])
                            : orc_morton(q[0], q[1], q[2]);
  }
}

/* ---------------------------------------------------------------------- */
/* Sort (Section 2.1): a stable sort of the particles by key, so equal keys
 * keep ascending original index; i.e. lexicographic (key, index) order.     */
typedef struct { uint64_t key; uint32_t idx; } kv_t;
static int kv_cmp(const void *a, const void *b) {
  const kv_t *p = (const kv_t *)a, *q = (const kv_t *)b;
  if (p->key != q->key) return p->key < q->key ? -1 : 1;
  return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

void orc_sort(int64_t n, const uint64_t *keys, uint64_t *keys_sorted, uint32_t *perm) {
  kv_t *t = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) { t[i].key = keys[i]; t[i].idx = (uint32_t)i; }
  qsort(t, (size_t)n, sizeof(kv_t), kv_cmp);
  for (int64_t i = 0; i < n; ++i) { keys_sorted[i] = t[i].key; perm[i] = t[i].idx; }
  free(t);
}

/* ---------------------------------------------------------------------- */
/* Tree (Section 2.1): a cell at level l is a run of sorted keys sharing their
 * top 3l bits; splitting it into eight sub-cubes is cutting its key run at the
 * next 3-bit digit.  Built breadth first: the root (all particles, level 0) is
 * node 0; a node with more than n_leaf particles below level 21 gets one child
 * per non-empty digit, in increasing digit order, appended in the order the
 * parents are visited.  Leaves have n_child = 0 and child_first = 0.
 * Returns the node count, or -1 if max_nodes is too small.                  */
int64_t orc_build(int64_t n, const uint64_t *ks, int n_leaf, int64_t max_nodes,
                  uint32_t *first, uint32_t *count, uint32_t *child_first,
                  uint8_t *n_child, uint8_t *level) {
  if (n <= 0) return 0;
  if (max_nodes < 1) return -1;
  int64_t nn = 1;
  first[0] = 0; count[0] = (uint32_t)n; level[0] = 0;
  for (int64_t k = 0; k < nn; ++k) {
    child_first[k] = 0; n_child[k] = 0;
    const int l = level[k];
    if (count[k] <= (uint32_t)n_leaf || l >= NLEV) continue;
    const int shift = 3 * (NLEV - 1 - l); /* digit of level l+1 */
    child_first[k] = (uint32_t)nn;
    uint32_t s = first[k];
    const uint32_t e = first[k] + count[k];
    while (s < e) {
      const uint64_t d = (ks[s] >> shift) & 7u;
      uint32_t t = s;
      while (t < e && ((ks[t] >> shift) & 7u) == d) ++t;
      if (nn >= max_nodes) return -1;
      first[nn] = s; count[nn] = t - s; level[nn] = (uint8_t)(l + 1);
      ++nn; ++n_child[k];
      s = t;
    }
  }
  return nn;
}

/* ---------------------------------------------------------------------- */
/* Pseudo j-particles (Section 2.1), straight from the member particles of
 * each node: mass M = sum m, centre of mass r_J = sum m r / M, radius
 * b_J = max |r - r_J| over the members (the smallest sphere about r_J that
 * holds them), and the second moments S_ab = sum m (r-r_J)_a (r-r_J)_b used
 * by the quadrupole extension.  A node of zero mass gets r_J = its first
 * member, b_J = 0, S = 0.  pos_sorted: float64 [n][4] in key order.
 * com[4k..] = x, y, z, M; S[6k..] = xx, yy, zz, xy, xz, yz.                   */
void orc_moments(int64_t nn, const uint32_t *first, const uint32_t *count,
                 const double *ps, double *com, double *b, double *S) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < nn; ++k) {
    const uint32_t s = first[k], e = first[k] + count[k];
    double M = 0, cx = 0, cy = 0, cz = 0;
    for (uint32_t j = s; j < e; ++j) {
      const double m = ps[4 * j + 3];
      M += m;
      cx += m * ps[4 * j];
      cy += m * ps[4 * j + 1];
      cz += m * ps[4 * j + 2];
    }
    double *Sk = S + 6 * k;
    for (int a = 0; a < 6; ++a) Sk[a] = 0;
    if (M > 0) {
      cx /= M; cy /= M; cz /= M;
    } else {
      cx = ps[4 * s]; cy = ps[4 * s + 1]; cz = ps[4 * s + 2];
    }
    double bmax = 0;
    for (uint32_t j = s; j < e; ++j) {
      const double dx = ps[4 * j] - cx, dy = ps[4 * j + 1] - cy, dz = ps[4 * j + 2] - cz;
      const double m = ps[4 * j + 3];
      if (M > 0) {
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        if (d > bmax) bmax = d;
      }
      Sk[0] += m * dx * dx; Sk[1] += m * dy * dy; Sk[2] += m * dz * dz;
      Sk[3] += m * dx * dy; Sk[4] += m * dx * dz; Sk[5] += m * dy * dz;
    }
    com[4 * k] = cx; com[4 * k + 1] = cy; com[4 * k + 2] = cz; com[4 * k + 3] = M;
    b[k] = bmax;
  }
}

/* ---------------------------------------------------------------------- */
/* Enclosing balls of a group (pseudo i-particles, Appendix B).  Each kind
 * picks a centre; the radius is then the largest member distance from it.
 *   0 GEO  centre of the bounding box
 *   1 SEB  smallest enclosing ball (unique): Welzl's recursion
 *   2 EBS  Ritter's bounding sphere: diameter of two far points (the one
 *          farthest from the first member, and the one farthest from that),
 *          grown in member order to take in every member outside it
 *   3 COM  centre of mass
 *   4 CMP  the smaller of GEO and COM (COM only if its radius is smaller by
 *          more than a relative 1e-5, so the choice is robust to rounding)  */
typedef struct { double c[3]; double r2; } OBall;

static double dist2(const double *a, const double *b) {
  const double x = a[0] - b[0], y = a[1] - b[1], z = a[2] - b[2];
  return x * x + y * y + z * z;
}

static int ob_in(const OBall *B, const double *p) {
  return B->r2 >= 0 && dist2(p, B->c) <= B->r2 * (1.0 + 1e-12);
}

static OBall ob_two(const double *a, const double *b) {
  OBall B;
  for (int k = 0; k < 3; ++k) B.c[k] = 0.5 * (a[k] + b[k]);
  B.r2 = 0.25 * dist2(a, b);
  return B;
}

/* smallest ball with a, b, c on its boundary (the circumcircle in their
 * plane); for (nearly) collinear points the ball of the farthest pair */
static OBall ob_three(const double *a, const double *b, const double *c) {
  double u[3], v[3], w[3];
  for (int k = 0; k < 3; ++k) { u[k] = b[k] - a[k]; v[k] = c[k] - a[k]; }
  w[0] = u[1] * v[2] - u[2] * v[1];
  w[1] = u[2] * v[0] - u[0] * v[2];
  w[2] = u[0] * v[1] - u[1] * v[0];
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  if (ww <= 1e-24 * uu * vv) {
    const double dab = dist2(a, b), dac = dist2(a, c), dbc = dist2(b, c);
    if (dab >= dac && dab >= dbc) return ob_two(a, b);
    return dac >= dbc ? ob_two(a, c) : ob_two(b, c);
  }
  /* centre = a + ((uu v - vv u) x w) / (2 ww) */
  double t[3];
  for (int k = 0; k < 3; ++k) t[k] = uu * v[k] - vv * u[k];
  OBall B;
  B.c[0] = a[0] + (t[1] * w[2] - t[2] * w[1]) / (2 * ww);
  B.c[1] = a[1] + (t[2] * w[0] - t[0] * w[2]) / (2 * ww);
  B.c[2] = a[2] + (t[0] * w[1] - t[1] * w[0]) / (2 * ww);
  B.r2 = dist2(a, B.c);
  return B;
}

/* the sphere through a, b, c, d; for (nearly) coplanar points the smallest
 * of the balls of three or two of them that holds all four */
static OBall ob_four(const double *a, const double *b, const double *c, const double *d) {
  double u[3], v[3], t[3];
  for (int k = 0; k < 3; ++k) { u[k] = b[k] - a[k]; v[k] = c[k] - a[k]; t[k] = d[k] - a[k]; }
  const double det = u[0] * (v[1] * t[2] - v[2] * t[1]) - u[1] * (v[0] * t[2] - v[2] * t[0]) +
                     u[2] * (v[0] * t[1] - v[1] * t[0]);
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  if (fabs(det) <= 1e-12 * sqrt(uu * vv * tt)) {
    const double *P[4] = {a, b, c, d};
    OBall best;
    best.r2 = -1;
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j) {
        OBall cand[3];
        int nc = 0;
        cand[nc++] = ob_two(P[i], P[j]);
        for (int k = j + 1; k < 4; ++k) cand[nc++] = ob_three(P[i], P[j], P[k]);
        for (int q = 0; q < nc; ++q) {
          int ok = 1;
          for (int m = 0; m < 4; ++m) ok &= ob_in(&cand[q], P[m]);
          if (ok && (best.r2 < 0 || cand[q].r2 < best.r2)) best = cand[q];
        }
      }
    return best;
  }
  /* solve 2 [u; v; t] x = [uu; vv; tt] for the centre offset x (Cramer) */
  const double r0 = 0.5 * uu, r1 = 0.5 * vv, r2 = 0.5 * tt;
  OBall B;
  double x[3];
  x[0] = (r0 * (v[1] * t[2] - v[2] * t[1]) - u[1] * (r1 * t[2] - v[2] * r2) +
          u[2] * (r1 * t[1] - v[1] * r2)) / det;
  x[1] = (u[0] * (r1 * t[2] - v[2] * r2) - r0 * (v[0] * t[2] - v[2] * t[0]) +
          u[2] * (v[0] * r2 - r1 * t[0])) / det;
  x[2] = (u[0] * (v[1] * r2 - r1 * t[1]) - u[1] * (v[0] * r2 - r1 * t[0]) +
          r0 * (v[0] * t[1] - v[1] * t[0])) / det;
  for (int k = 0; k < 3; ++k) B.c[k] = a[k] + x[k];
  B.r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
  return B;
}

static OBall ob_support(const double **R, int nr) {
  OBall B;
  switch (nr) {
    case 0: B.c[0] = B.c[1] = B.c[2] = 0; B.r2 = -1; return B;
    case 1: for (int k = 0; k < 3; ++k) B.c[k] = R[0][k]; B.r2 = 0; return B;
    case 2: return ob_two(R[0], R[1]);
    case 3: return ob_three(R[0], R[1], R[2]);
    default: return ob_four(R[0], R[1], R[2], R[3]);
  }
}

/* Welzl: the smallest ball holding P[0..n) with R[0..nr) on its boundary */
static OBall ob_welzl(const double **P, int n, const double **R, int nr) {
  if (n == 0 || nr == 4) return ob_support(R, nr);
  OBall B = ob_welzl(P, n - 1, R, nr);
  if (ob_in(&B, P[n - 1])) return B;
  const double *R2[4];
  for (int k = 0; k < nr; ++k) R2[k] = R[k];
  R2[nr] = P[n - 1];
  return ob_welzl(P, n - 1, R2, nr + 1);
}

static double ob_radius(const double *const *P, int n, const double c[3]) {
  double r = 0;
  for (int q = 0; q < n; ++q) {
    const double d = sqrt(dist2(P[q], c));
    if (d > r) r = d;
  }
  return r;
}

static void group_ball(const double **P, int n, const double *mass, int kind, double out[4]) {
  double c[3];
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) lo[a] = hi[a] = P[0][a];
  for (int q = 0; q < n; ++q)
    for (int a = 0; a < 3; ++a) {
      if (P[q][a] < lo[a]) lo[a] = P[q][a];
      if (P[q][a] > hi[a]) hi[a] = P[q][a];
    }
  double geo[3];
  for (int a = 0; a < 3; ++a) geo[a] = 0.5 * (lo[a] + hi[a]);
  if (kind == 1) {
    const double *R[4];
    OBall B = ob_welzl(P, n, R, 0);
    for (int a = 0; a < 3; ++a) c[a] = B.c[a];
  } else if (kind == 2) {
    int y = 0, z = 0;
    for (int q = 0; q < n; ++q) if (dist2(P[q], P[0]) > dist2(P[y], P[0])) y = q;
    for (int q = 0; q < n; ++q) if (dist2(P[q], P[y]) > dist2(P[z], P[y])) z = q;
    double r = 0.5 * sqrt(dist2(P[y], P[z]));
    for (int a = 0; a < 3; ++a) c[a] = 0.5 * (P[y][a] + P[z][a]);
    for (int q = 0; q < n; ++q) {
      const double d = sqrt(dist2(P[q], c));
      if (d > r) {  /* grow: the new ball holds the old one and P[q] */
        const double rn = 0.5 * (r + d);
        for (int a = 0; a < 3; ++a) c[a] += (P[q][a] - c[a]) * (rn - r) / d;
        r = rn;
      }
    }
  } else if (kind == 3 || kind == 4) {
    double M = 0, s[3] = {0, 0, 0};
    for (int q = 0; q < n; ++q) {
      M += mass[q];
      for (int a = 0; a < 3; ++a) s[a] += mass[q] * P[q][a];
    }
    for (int a = 0; a < 3; ++a) c[a] = M > 0 ? s[a] / M : geo[a];
    if (kind == 4 && !(ob_radius(P, n, c) < ob_radius(P, n, geo) * (1.0 - 1e-5)))
      for (int a = 0; a < 3; ++a) c[a] = geo[a];
  } else {
    for (int a = 0; a < 3; ++a) c[a] = geo[a];
  }
  for (int a = 0; a < 3; ++a) out[a] = c[a];
  out[3] = ob_radius(P, n, c);
}

/* plain smallest enclosing ball of points pts[n][3] (for tests) */
void orc_seb(int n, const double *pts, double out[4]) {
  const double **P = (const double **)malloc(sizeof(double *) * (size_t)(n > 0 ? n : 1));
  for (int q = 0; q < n; ++q) P[q] = pts + 3 * q;
  const double *R[4];
  OBall B = ob_welzl(P, n, R, 0);
  for (int a = 0; a < 3; ++a) out[a] = B.c[a];
  out[3] = ob_radius(P, n, B.c);
  free(P);
}

/* ---------------------------------------------------------------------- */
/* Groups (Sections 2.3-2.4): the active particles in key order.  Following
 * Section 2.4, two consecutive active particles farther apart than the
 * critical separation r_crit are never put in the same group (r_crit <= 0:
 * no such split); each run between such gaps is cut into groups of at most G
 * consecutive particles.  The gap test compares the float64 squared distance
 * of the (float32) positions with r_crit^2.  Each group gets a pseudo
 * i-particle (r_I, b_I): an enclosing ball of the kind `ball_kind` (see
 * group_ball; GEO by default).
 * act_sorted[k] = active flag of sorted particle k.  Outputs: alist (sorted
 * indices of active particles), gfirst/gcount into alist, ball[4g..] = r_I, b_I.
 * Returns the number of groups.                                              */
int64_t orc_groups(int64_t n, const uint8_t *act_sorted, const double *ps, int G,
                   double r_crit, uint32_t *alist, uint32_t *gfirst, uint32_t *gcount,
                   double *ball, int ball_kind) {
  int64_t na = 0;
  for (int64_t k = 0; k < n; ++k)
    if (act_sorted[k]) alist[na++] = (uint32_t)k;
  int64_t ng = 0, run_start = 0;
  for (int64_t a = 0; a < na; ++a) {
    int brk = (a == 0);
    if (!brk && r_crit > 0) {
      const double *p = ps + 4 * (int64_t)alist[a], *q = ps + 4 * (int64_t)alist[a - 1];
      const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
      brk = (dx * dx + dy * dy + dz * dz) > r_crit * r_crit;
    }
    if (brk) run_start = a;
    if ((a - run_start) % G == 0) gfirst[ng++] = (uint32_t)a;
  }
  for (int64_t g = 0; g < ng; ++g)
    gcount[g] = (uint32_t)((g + 1 < ng ? gfirst[g + 1] : na) - gfirst[g]);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < ng; ++g) {
    const int64_t s = gfirst[g];
    const int cnt = (int)gcount[g];
    const double *P[64];
    double m[64];
    for (int q = 0; q < cnt && q < 64; ++q) {
      P[q] = ps + 4 * (int64_t)alist[s + q];
      m[q] = ps[4 * (int64_t)alist[s + q] + 3];
    }
    group_ball(P, cnt < 64 ? cnt : 64, m, ball_kind, ball + 4 * g);
  }
  return ng;
}

/* ---------------------------------------------------------------------- */
/* Pair terms, y = r_i - r_J, R^2 = |y|^2 + eps^2.
 * Monopole (point mass):  a += -M y / R^3,  phi += -M / R.
 * Quadrupole (extension; the paper uses monopoles only): the second-order
 * Taylor term of the softened kernel about the centre of mass, with the raw
 * second moments S (the dipole vanishes about the centre of mass):
 *   phi += -(3/2) y.S.y / R^5 + (1/2) tr S / R^3
 *   a   +=  3 S.y / R^5 - (15/2) (y.S.y) y / R^7 + (3/2) tr S y / R^5          */
static void pair_mono(const double yi[3], const double rj[3], double M, double e2,
                      double acc[4]) {
  const double y0 = yi[0] - rj[0], y1 = yi[1] - rj[1], y2 = yi[2] - rj[2];
  const double R2 = y0 * y0 + y1 * y1 + y2 * y2 + e2;
  const double R = sqrt(R2);
  const double inv3 = 1.0 / (R2 * R);
  acc[0] -= M * y0 * inv3;
  acc[1] -= M * y1 * inv3;
  acc[2] -= M * y2 * inv3;
  acc[3] -= M / R;
}

static void pair_quad(const double yi[3], const double rj[3], const double S[6], double e2,
                      double acc[4]) {
  const double y[3] = {yi[0] - rj[0], yi[1] - rj[1], yi[2] - rj[2]};
  const double R2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + e2;
  const double R = sqrt(R2);
  const double R3 = R2 * R, R5 = R3 * R2, R7 = R5 * R2;
  const double Sy[3] = {S[0] * y[0] + S[3] * y[1] + S[4] * y[2],
                        S[3] * y[0] + S[1] * y[1] + S[5] * y[2],
                        S[4] * y[0] + S[5] * y[1] + S[2] * y[2]};
  const double q = y[0] * Sy[0] + y[1] * Sy[1] + y[2] * Sy[2];
  const double tr = S[0] + S[1] + S[2];
  for (int a = 0; a < 3; ++a)
    acc[a] += 3.0 * Sy[a] / R5 - 7.5 * q * y[a] / R7 + 1.5 * tr * y[a] / R5;
  acc[3] += -1.5 * q / R5 + 0.5 * tr / R3;
}

/* ---------------------------------------------------------------------- */
/* Tree walk (Sections 2.2-2.3).  For each group, breadth first from the root:
 * for a candidate pseudo j-particle J, r_JI = |r_J - r_I| and the distance to
 * the nearest possible i-particle is d = lambda r_JI with lambda = 1 - b_I/r_JI
 * when b_I < r_JI and 0 otherwise.  The opening-angle MAC b_J / d <= theta is
 * taken as b_J <= theta d (so d = 0 accepts only b_J = 0).  Accepted nodes
 * interact as pseudo particles; a rejected internal node queues its children;
 * a rejected leaf interacts through its member particles.  Every i of the
 * group then sums the same list.  The self pair of a particle gives zero force
 * and the potential term -m_i/eps, which is removed.  (For theta < 1 a node
 * holding an i of the group is never accepted unless b_J = 0, so the self pair
 * is always an explicit particle entry.)
 *
 * multipole: 1 monopole, 2 monopole + quadrupole for node entries.
 * Per group: cnt[3g+0] accepted node entries, cnt[3g+1] particle entries,
 * cnt[3g+2] near ties |b_J - theta d| <= tie_rel max(b_J, theta d) + tie_abs s,
 * s = |r_J|_1 + |r_I|_1 + b_I (the coordinate scale that bounds the absolute
 * rounding of a single-precision evaluation), among nodes with b_J > 0 (b_J = 0
 * is accepted at any distance);
 * mass[g] = summed mass of the list (mass closure).
 * gsel: optional subset of groups to evaluate (ngsel entries), NULL = all.
 * out: [n][4] in sorted order; rows of evaluated active particles written.   */
/* Multipole acceptance criteria of Section 2.2 for node J seen from a group
 * at lambda-distance d:
 *   mac 0  opening angle (Barnes & Hut):      b_J <= theta d
 *   mac 1  acceleration (Springel):           d >= (m_J b_J^2 / (Delta |a_old|))^(1/4)
 *          with |a_old| the smallest previous acceleration in the group
 *   mac 2  multipole (Warren & Salmon):       d >= b_J/2 + sqrt(b_J^2/4 + sqrt(3 B2 / Delta)),
 *          B2 = sum m |r - r_J|^2 (the trace of the second moments)
 * Reading: with mac 1 and 2 a node of positive size is also never accepted
 * when b_J >= d, i.e. when it may hold a member of the group (a node holding
 * group member i has d <= b_J, with equality when i is its farthest member);
 * so the self pair of every i-particle stays an explicit particle term.
 * Point nodes (b_J = 0) are exact and always pass this guard. */
static int mac_accept(int mac, double d, double bJ, double mJ, double B2, double theta,
                      double delta, double amin) {
  if (mac == 0) return bJ <= theta * d;
  if (bJ > 0.0 && bJ >= d) return 0;
  if (mac == 1) return mJ * bJ * bJ <= delta * amin * (d * d) * (d * d);
  return d >= 0.5 * bJ + sqrt(0.25 * bJ * bJ + sqrt(3.0 * B2 / delta));
}

void orc_walk(int64_t nn, const uint32_t *first, const uint32_t *count,
              const uint32_t *child_first, const uint8_t *n_child,
              const double *com, const double *b, const double *S,
              const double *ps, const uint32_t *alist, int64_t ng,
              const uint32_t *gfirst, const uint32_t *gcount, const double *ball,
              double eps, double theta, int multipole, double tie_rel, double tie_abs,
              const int64_t *gsel, int64_t ngsel, double *out, int64_t *cnt,
              double *mass, int mac, double delta, const double *amag,
              uint32_t *lists, int64_t lcap, uint32_t *lcount) {
  const double e2 = eps * eps;
  const int64_t nsel = gsel ? ngsel : ng;
#pragma omp parallel
  {
    uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nn > 0 ? nn : 1));
    uint32_t *lst = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nn > 0 ? nn : 1));
    size_t cap_p = 1024;
    uint32_t *plst = (uint32_t *)malloc(sizeof(uint32_t) * cap_p);
    uint32_t *leaf_of_entry = (uint32_t *)malloc(sizeof(uint32_t) * cap_p);
#pragma omp for schedule(dynamic, 4)
    for (int64_t t = 0; t < nsel; ++t) {
      const int64_t g = gsel ? gsel[t] : t;
      const double rI[3] = {ball[4 * g], ball[4 * g + 1], ball[4 * g + 2]};
      const double bI = ball[4 * g + 3];
      double amin = INFINITY;
      if (mac == 1)
        for (uint32_t a = gfirst[g]; a < gfirst[g] + gcount[g]; ++a)
          if (amag[alist[a]] < amin) amin = amag[alist[a]];
      int64_t nl = 0, np = 0, ties = 0, qh = 0, qt = 0;
      if (nn > 0) q[qt++] = 0;
      while (qh < qt) {
        const uint32_t J = q[qh++];
        const double dx = com[4 * J] - rI[0], dy = com[4 * J + 1] - rI[1],
                     dz = com[4 * J + 2] - rI[2];
        const double rJI = sqrt(dx * dx + dy * dy + dz * dz);
        const double lam = (bI < rJI) ? 1.0 - bI / rJI : 0.0;
        const double d = lam * rJI;
        const double td = theta * d;
        const double big = b[J] > td ? b[J] : td;
        const double scale = fabs(com[4 * J]) + fabs(com[4 * J + 1]) + fabs(com[4 * J + 2]) +
                             fabs(rI[0]) + fabs(rI[1]) + fabs(rI[2]) + bI;
        const double B2 = S[6 * J] + S[6 * J + 1] + S[6 * J + 2];
        const int acc = mac_accept(mac, d, b[J], com[4 * J + 3], B2, theta, delta, amin);
        if (mac == 0) {
          if (b[J] > 0 && fabs(b[J] - td) <= tie_rel * big + tie_abs * scale) ++ties;
        } else {
          /* a near tie: the decision changes within single-precision rounding of d */
          const double dlo = d * (1.0 - tie_rel) - tie_abs * scale;
          const double dhi = d * (1.0 + tie_rel) + tie_abs * scale;
          if (mac_accept(mac, dlo > 0 ? dlo : 0, b[J], com[4 * J + 3], B2, theta, delta, amin) !=
              mac_accept(mac, dhi, b[J], com[4 * J + 3], B2, theta, delta, amin))
            ++ties;
        }
        if (acc) {
          lst[nl++] = J;
        } else if (n_child[J] == 0) {
          if ((size_t)(np + count[J]) > cap_p) {
            while ((size_t)(np + count[J]) > cap_p) cap_p *= 2;
            plst = (uint32_t *)realloc(plst, sizeof(uint32_t) * cap_p);
            leaf_of_entry = (uint32_t *)realloc(leaf_of_entry, sizeof(uint32_t) * cap_p);
          }
          for (uint32_t j = first[J]; j < first[J] + count[J]; ++j) {
            leaf_of_entry[np] = J;
            plst[np++] = j;
          }
        } else {
          for (uint32_t c = 0; c < n_child[J]; ++c) q[qt++] = child_first[J] + c;
        }
      }
      double msum = 0;
      for (int64_t k = 0; k < nl; ++k) msum += com[4 * lst[k] + 3];
      for (int64_t k = 0; k < np; ++k) msum += ps[4 * plst[k] + 3];
      cnt[3 * g] = nl; cnt[3 * g + 1] = np; cnt[3 * g + 2] = ties;
      if (lists) {  /* the list itself: accepted nodes, then opened leaves | bit 31 */
        int64_t w = 0, nleaf = 0;
        for (int64_t k = 0; k < nl; ++k, ++w)
          if (w < lcap) lists[t * lcap + w] = lst[k];
        for (int64_t k = 0; k < np; k += (int64_t)count[leaf_of_entry[k]], ++nleaf, ++w)
          if (w < lcap) lists[t * lcap + w] = leaf_of_entry[k] | 0x80000000u;
        lcount[2 * t] = (uint32_t)nl;
        lcount[2 * t + 1] = (uint32_t)nleaf;
      }
      mass[g] = msum;
      for (uint32_t a = gfirst[g]; a < gfirst[g] + gcount[g]; ++a) {
        const uint32_t i = alist[a];
        const double yi[3] = {ps[4 * i], ps[4 * i + 1], ps[4 * i + 2]};
        double acc[4] = {0, 0, 0, 0};
        for (int64_t k = 0; k < nl; ++k) {
          const uint32_t J = lst[k];
          pair_mono(yi, com + 4 * J, com[4 * J + 3], e2, acc);
          if (multipole == 2) pair_quad(yi, com + 4 * J, S + 6 * J, e2, acc);
        }
        for (int64_t k = 0; k < np; ++k) {
          const uint32_t j = plst[k];
          pair_mono(yi, ps + 4 * j, ps[4 * j + 3], e2, acc);
        }
        acc[3] += ps[4 * i + 3] / eps; /* remove the self pair's -m_i/eps */
        for (int c = 0; c < 4; ++c) out[4 * (int64_t)i + c] = acc[c];
      }
    }
    free(q); free(lst); free(plst); free(leaf_of_entry);
  }
}

/* ---------------------------------------------------------------------- */
/* Check of another implementation's walk decisions (Sections 2.2-2.3), for
 * groups where single- and double-precision MAC decisions may legitimately
 * differ.  For each selected group g its interaction list is given as the
 * set of accepted nodes and the set of opened leaves (entries[k*cap ..],
 * nent[2k] accepted then nent[2k+1] leaves in any order; a leaf entry has bit
 * 31 set).  The tree is walked again from the group's root (groot[k], or node
 * 0 when groot is NULL), following the GIVEN decisions; at every visited node
 * the float64 MAC decision is taken as in orc_walk and compared:
 *   info[6k+0]  nodes visited
 *   info[6k+1]  decisions that differ from float64 inside the near-tie window
 *   info[6k+2]  decisions that differ outside it (an error)
 *   info[6k+3]  entries never reached by the walk (an error)
 *   info[6k+4]  inconsistent entries (a leaf neither accepted nor opened, an
 *               internal node listed as an opened leaf, a duplicate) (an error)
 *   info[6k+5]  list entries
 * mass[k] = summed mass of the list (mass closure); out[n][4] (sorted order)
 * = the float64 forces of the group's particles from the GIVEN list.          */
void orc_walk_replay(int64_t nn, const uint32_t *first, const uint32_t *count,
                     const uint32_t *child_first, const uint8_t *n_child,
                     const double *com, const double *b, const double *S,
                     const double *ps, const uint32_t *alist, const uint32_t *gfirst,
                     const uint32_t *gcount, const double *ball, double eps, double theta,
                     int multipole, double tie_rel, double tie_abs, int mac, double delta,
                     const double *amag, int64_t ngsel, const int64_t *gsel,
                     const uint32_t *groot, int64_t cap, const uint32_t *entries,
                     const uint32_t *nent, double *out, int64_t *info, double *mass) {
  const double e2 = eps * eps;
  uint8_t *mark = (uint8_t *)calloc((size_t)(nn > 0 ? nn : 1), 1);
  uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nn > 0 ? nn : 1));
  uint32_t *lst = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nn > 0 ? nn : 1));
  uint32_t *lf = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nn > 0 ? nn : 1));
  for (int64_t k = 0; k < ngsel; ++k) {
    const int64_t g = gsel[k];
    int64_t *inf = info + 6 * k;
    for (int c = 0; c < 6; ++c) inf[c] = 0;
    const uint32_t *e = entries + k * cap;
    const int64_t ne = (int64_t)nent[2 * k] + (int64_t)nent[2 * k + 1];
    inf[5] = ne;
    for (int64_t t = 0; t < ne; ++t) {
      const uint32_t J = e[t] & 0x7fffffffu;
      const uint8_t want = (e[t] & 0x80000000u) ? 2 : 1;
      if (J >= (uint64_t)nn || mark[J]) { ++inf[4]; continue; }
      mark[J] = want;
    }
    const double rI[3] = {ball[4 * g], ball[4 * g + 1], ball[4 * g + 2]};
    const double bI = ball[4 * g + 3];
    double amin = INFINITY;
    if (mac == 1)
      for (uint32_t a = gfirst[g]; a < gfirst[g] + gcount[g]; ++a)
        if (amag[alist[a]] < amin) amin = amag[alist[a]];
    int64_t qh = 0, qt = 0, nl = 0, np = 0, used = 0;
    if (nn > 0) q[qt++] = groot ? groot[k] : 0;
    while (qh < qt) {
      const uint32_t J = q[qh++];
      ++inf[0];
      const double dx = com[4 * J] - rI[0], dy = com[4 * J + 1] - rI[1], dz = com[4 * J + 2] - rI[2];
      const double rJI = sqrt(dx * dx + dy * dy + dz * dz);
      const double d = ((bI < rJI) ? 1.0 - bI / rJI : 0.0) * rJI;
      const double td = theta * d;
      const double big = b[J] > td ? b[J] : td;
      const double scale = fabs(com[4 * J]) + fabs(com[4 * J + 1]) + fabs(com[4 * J + 2]) +
                           fabs(rI[0]) + fabs(rI[1]) + fabs(rI[2]) + bI;
      const double B2 = S[6 * J] + S[6 * J + 1] + S[6 * J + 2];
      const int acc = mac_accept(mac, d, b[J], com[4 * J + 3], B2, theta, delta, amin);
      int tie;
      if (mac == 0) {
        tie = b[J] > 0 && fabs(b[J] - td) <= tie_rel * big + tie_abs * scale;
      } else {
        const double dlo = d * (1.0 - tie_rel) - tie_abs * scale;
        const double dhi = d * (1.0 + tie_rel) + tie_abs * scale;
        tie = mac_accept(mac, dlo > 0 ? dlo : 0, b[J], com[4 * J + 3], B2, theta, delta, amin) !=
              mac_accept(mac, dhi, b[J], com[4 * J + 3], B2, theta, delta, amin);
      }
      const int given = mark[J];
      const int given_acc = given == 1;
      if (given) ++used;
      mark[J] = 0;
      if (given == 2 && n_child[J] != 0) ++inf[4];
      if (given == 0 && n_child[J] == 0) { ++inf[4]; continue; }
      if (given_acc != acc) ++inf[tie ? 1 : 2];
      if (given_acc) lst[nl++] = J;
      else if (n_child[J] == 0) lf[np++] = J;
      else
        for (uint32_t c = 0; c < n_child[J]; ++c) q[qt++] = child_first[J] + c;
    }
    inf[3] = ne - inf[4] - used;
    for (int64_t t = 0; t < ne; ++t)
      if ((e[t] & 0x7fffffffu) < (uint64_t)nn) mark[e[t] & 0x7fffffffu] = 0;
    double msum = 0;
    for (int64_t t = 0; t < nl; ++t) msum += com[4 * lst[t] + 3];
    for (int64_t t = 0; t < np; ++t)
      for (uint32_t j = first[lf[t]]; j < first[lf[t]] + count[lf[t]]; ++j) msum += ps[4 * j + 3];
    mass[k] = msum;
    for (uint32_t a = gfirst[g]; a < gfirst[g] + gcount[g]; ++a) {
      const uint32_t i = alist[a];
      const double yi[3] = {ps[4 * i], ps[4 * i + 1], ps[4 * i + 2]};
      double acc4[4] = {0, 0, 0, 0};
      for (int64_t t = 0; t < nl; ++t) {
        const uint32_t J = lst[t];
        pair_mono(yi, com + 4 * J, com[4 * J + 3], e2, acc4);
        if (multipole == 2) pair_quad(yi, com + 4 * J, S + 6 * J, e2, acc4);
      }
      for (int64_t t = 0; t < np; ++t)
        for (uint32_t j = first[lf[t]]; j < first[lf[t]] + count[lf[t]]; ++j)
          pair_mono(yi, ps + 4 * j, ps[4 * j + 3], e2, acc4);
      acc4[3] += ps[4 * i + 3] / eps; /* remove the self pair's -m_i/eps */
      for (int c = 0; c < 4; ++c) out[4 * (int64_t)i + c] = acc4[c];
    }
  }
  free(mark); free(q); free(lst); free(lf);
}
