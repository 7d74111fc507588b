/*
 * Plain FP64 CPU oracle for the walk-on-stars (WoSt) estimator of
 * Sawhney, Miller, Gkioulekas and Crane, "Walk on Stars" (ACM TOG 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into oracle/liboracle.so
 * and is loaded only by the test-suite, by the smoke check and by the
 * benchmark's CPU-baseline leg.  The product path (the HIP library) never
 * links, loads or calls it, and it shares no code with that path.
 *
 * Everything here is slow on purpose: every geometric query is brute force
 * over all primitives (no acceleration structure), every quantity is a
 * double, and each function follows one definition of the paper:
 *
 *   problem           Sec. 3.2, Eq. (PoissonEquation)
 *   WoSt estimator    Sec. 4.3 (boxed estimator), Sec. 4.7 (final estimator),
 *                     Algorithm 1 (WalkOnStars)
 *   star radius       Sec. 4.4.2, Sec. 4.4.3 (minimum radius)
 *   directions        Sec. 4.4, Eq. (DirectionalSampling); hemisphere Sec. 4.4.4
 *   Neumann term      Sec. 4.5 and Sec. 5.2 (sampling by support extension)
 *   source term       Sec. 4.6
 *   silhouettes       Sec. 5.1, Eq. (SilhouetteDefinition)
 *   ball kernels      App. A.1, Eqs. (GreensFnsPoissonBall),
 *                     (GreensFnsNormPoissonBall)
 *
 * Readings taken where the paper is silent or inconsistent (each is listed
 * in the design notes of the repository):
 *   R1 sign: with Laplacian(u) = f, outward h = du/dn and the positive ball
 *      kernels of App. A.1, one step is  u_k = u_{k+1} + N - S.
 *   R2 closest silhouette: the minimum over all silhouette elements within
 *      the search radius (the plain definition of the closest silhouette
 *      point), not the first one met.
 *   R3 radius: r = min(d_D, max(r_min, d_sil)), so the ball never crosses
 *      the Dirichlet boundary; equal to the printed max(r_min, min(.)) when
 *      r_min <= eps.
 *   R4 on-boundary queries: when the walk sits on the Neumann boundary the
 *      silhouette query, the ray and the visibility ray start from
 *      x' = x - offset * n (the inward offset of the footnote in Sec. 4.4);
 *      the ray additionally skips the primitive the walk sits on.  The next
 *      point is the first point of that ray on the star boundary
 *      (Eq. DirectionalSampling applied to the offset ray): its Neumann
 *      crossing, or x' + r v when it has none.
 *   R5 2D: primitives are segments, silhouette elements are the vertices of
 *      the Neumann polyline.
 *   R6 random numbers: Philox4x32-10 keyed by the 64-bit seed, counter
 *      (point, walk, step, slot); a uniform is (u32 >> 8) * 2^-24.  Slot 0
 *      gives (direction, direction, source, source); slot 1 gives
 *      (pick, place, place, -) for the Neumann sample.
 *   R7 Neumann sample: a primitive that meets the ball B(x, r) is picked in
 *      proportion to its measure, then a point uniformly on it; the pdf is
 *      1 / (total measure of the primitives meeting the ball).  Any such
 *      sampler is unbiased by the support-extension argument of Sec. 4.5.
 *   R8 cap: a walk is stopped after max_steps steps, or when it is farther
 *      than escape_radius from the scene centre, returning g at the closest
 *      Dirichlet point; both events are counted.
 *   R10 screened Poisson (Sec. 3.2, Eq. ScreenedPoissonEquation; App. A.2):
 *      for Laplacian(u) - sigma u = f the step keeps the Poisson direction and
 *      source samplers; the Neumann term uses the screened ball Green's
 *      function G^{sigma,B}; the source term reweights the Poisson source
 *      sample by G^{sigma,B} / G^B; the continuation carries the factor
 *      Q^{sigma,B}(r = t, R = r) of Eq. (ScreenedPoissonKernelsSphere), applied
 *      as Russian roulette (the walk continues with probability Q, unweighted;
 *      the roulette uniform is the first of Philox slot 0xffffffff).  A
 *      Tikhonov switch (Sec. 3.4, pure Neumann) adds sigma_T to sigma from
 *      step K on.  Without a Dirichlet boundary the star radius is capped at
 *      the escape radius.
 *   R9 evaluation points on the Neumann boundary (Algorithm 1 with its
 *      on-boundary flag set at the start): the walk starts on the given
 *      Neumann primitive with that primitive's normal, i.e. in the same state
 *      as a walk that has just reached the boundary, so the first step samples
 *      the hemisphere and weights the Neumann term by 1 / alpha, alpha = 1/2.
 *   R12 implicit Dirichlet boundaries (Sec. 6, mixed representations; the
 *      closest-point query Q.1 is the only one a Dirichlet boundary takes
 *      part in): a scene may add analytic shapes -- balls, rounded boxes and
 *      capsules -- whose surfaces are Dirichlet boundary with the scene's g.
 *      Each bounds the domain from outside (the domain lies outside it) or,
 *      for a ball or a sharp box, from inside.  Q.1 returns the closest
 *      point over mesh primitives and shapes together; a shape's index is
 *      reported as n_prims + its position in the list.  The scene box (and
 *      so L, the offset and the escape radius) covers the shapes too.
 *   R11 double-sided boundaries (App. "Open Domains and Double-Sided
 *      Boundaries"): a primitive flagged double-sided carries data for both
 *      sides; "+" is the side its normal points away from (the inside of a
 *      closed, outward-oriented surface), "-" the other, with normal
 *      n- = -n+.  The walk keeps q = x_k - x_{k-1}.  At the end of a walk
 *      whose closest Dirichlet primitive is double-sided, g+ is used when
 *      q . n+ > 0 and g- otherwise; at step 0, q is the start side's
 *      normal for a boundary start and xbar - x0 (the side x0 lies on) for
 *      an interior start.  On reaching a double-sided Neumann primitive the
 *      walk's normal is n+ when q . n+ >= 0 and -n+ otherwise, and the
 *      hemisphere, the query offset and the next step use that normal.  The
 *      Neumann sample z on a double-sided primitive takes h+ when
 *      (z - x') . n+ > 0 and h- otherwise, x' the query origin: this is the
 *      appendix's rule for an interior x, and for x on the Neumann boundary
 *      it takes the data of the side the walk is on (the appendix's
 *      on-boundary sentence assigns h+ to a flipped normal, which would give
 *      a one-sided walk h- everywhere; it is read the other way).  h- as a
 *      normal derivative uses n-.
 *   R13 a walk on the boundary up to rounding: the walk's ray query also
 *      takes a crossing at -64 offset < t <= 0 (behind the origin) of a
 *      one-sided Neumann primitive that the ray leaves (v . n > 0) as a
 *      crossing at t = 0 when the origin lies outside the primitive's plane
 *      by less than offset/4, so the walk lands where it stands, on that
 *      primitive.  In exact
 *      arithmetic a walk is never outside the domain, so such a crossing can
 *      only come from a position that rounding has put on or just beyond the
 *      boundary (a step that ended by a miss within rounding of it); without
 *      the rule an outward ray from there would pass through the boundary and
 *      the walk would leave the domain.  The distance is measured across the
 *      plane, not along the ray: at grazing incidence a rounding-sized
 *      distance from the plane lies far back along the ray, hence the reach
 *      of 64 offsets in t (the device's tree search visits the boxes that
 *      the ray meets within that reach).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: Salmon, Moraes, Dror and Shaw, "Parallel random numbers:   */
/* as easy as 1, 2, 3", SC'11.  Ten rounds of two 32x32->64 multiplies, the  */
/* key bumped by the Weyl constants between rounds.                          */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u01(uint32_t u) { return (double)(u >> 8) * (1.0 / 16777216.0); }

/* the four uniforms of counter (point, walk, step, slot) */
void orc_uniforms(uint64_t seed, uint32_t point, uint32_t walk, uint32_t step, uint32_t slot,
                  double U[4]) {
  uint32_t ctr[4] = {point, walk, step, slot};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t o[4];
  orc_philox4x32_10(ctr, key, o);
  for (int i = 0; i < 4; ++i) U[i] = u01(o[i]);
}

/* ------------------------------------------------------------------------ */
/* small vector helpers (3-vectors; 2D data lives in the z = 0 plane)        */
/* ------------------------------------------------------------------------ */
static void vsub(const double a[3], const double b[3], double o[3]) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static double vdot(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void vcross(const double a[3], const double b[3], double o[3]) {
  double x = a[1] * b[2] - a[2] * b[1];
  double y = a[2] * b[0] - a[0] * b[2];
  double z = a[0] * b[1] - a[1] * b[0];
  o[0] = x; o[1] = y; o[2] = z;
}
static double vnorm(const double a[3]) { return sqrt(vdot(a, a)); }
static void vaxpy(const double x[3], double s, const double d[3], double o[3]) {
  o[0] = x[0] + s * d[0]; o[1] = x[1] + s * d[1]; o[2] = x[2] + s * d[2];
}
static void vcopy(const double a[3], double o[3]) { o[0] = a[0]; o[1] = a[1]; o[2] = a[2]; }

/* ------------------------------------------------------------------------ */
/* scene                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
  int kind;   /* 0 zero, 1 const, 2 poly2, 3 expcos, 4 per-corner */
  int as_nd;  /* 1: the field is grad(F) . n_prim */
  double coef[10];
  const float* per_corner; /* [n_prims][dim] */
} orc_fn;

/* an analytic Dirichlet shape (R12); p: centre or segment end a (0..2),
 * half extents or segment end b (3..5), radius or rounding (6) */
typedef struct {
  int kind;    /* 0 ball, 1 box (rounded by p[6]), 2 capsule */
  int inside;  /* 1: the domain is inside the shape */
  double p[8];
} orc_sdf;

typedef struct {
  int dim;
  long nv, np;
  long nsdf;
  orc_sdf* sdf;
  double* V;          /* [nv][3] */
  int* P;             /* [np][3] (third index unused in 2D) */
  unsigned char* bc;  /* 0 Dirichlet, 1 Neumann; 2, 3 the same, double-sided (R11) */
  double* nrm;        /* [np][3] unit outward normals */
  double* meas;       /* [np] length (2D) or area (3D) */
  /* silhouette elements: vertices (2D) / edges (3D) of the Neumann boundary */
  long ne;
  int* ev;            /* [ne][2] */
  int* eoff;          /* [ne + 1] CSR offsets into eadj */
  int* eadj;          /* adjacent Neumann primitives */
  orc_fn g, h, f;
  orc_fn gm, hm;      /* "-" side data of double-sided primitives (R11) */
  float* pc_g; float* pc_h; float* pc_f; float* pc_gm; float* pc_hm; /* owned per-corner data */
  double center[3], L;
  long nD, nN;
} orc_scene;

static void scene_box(orc_scene* s);
static int is_neumann(const orc_scene* s, long i) { return s->bc[i] & 1; }
static int double_sided(const orc_scene* s, long i) { return s->bc[i] >= 2; }

static float* dup_pc(const orc_fn* fn, long np, int dim) {
  if (!fn || fn->kind != 4 || !fn->per_corner) return NULL;
  float* p = (float*)malloc(sizeof(float) * np * dim);
  memcpy(p, fn->per_corner, sizeof(float) * np * dim);
  return p;
}

typedef struct { int a, b, prim; } orc_ekey;
static int ekey_cmp(const void* x, const void* y) {
  const orc_ekey* p = (const orc_ekey*)x;
  const orc_ekey* q = (const orc_ekey*)y;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  if (p->prim != q->prim) return p->prim < q->prim ? -1 : 1;
  return 0;
}

void orc_scene_free(orc_scene* s) {
  if (!s) return;
  free(s->V); free(s->P); free(s->bc); free(s->nrm); free(s->meas);
  free(s->ev); free(s->eoff); free(s->eadj);
  free(s->pc_g); free(s->pc_h); free(s->pc_f); free(s->pc_gm); free(s->pc_hm);
  free(s->sdf);
  free(s);
}

orc_scene* orc_scene_create(int dim, long nv, const float* V, long np, const int* P,
                            const unsigned char* bc, const orc_fn* g, const orc_fn* h,
                            const orc_fn* f, const orc_fn* gm, const orc_fn* hm) {
  if (dim != 2 && dim != 3) return NULL;
  orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
  s->dim = dim; s->nv = nv; s->np = np;
  s->V = (double*)calloc(nv * 3, sizeof(double));
  for (long i = 0; i < nv; ++i)
    for (int k = 0; k < dim; ++k) s->V[3 * i + k] = (double)V[dim * i + k];
  s->P = (int*)calloc(np * 3, sizeof(int));
  for (long i = 0; i < np; ++i)
    for (int k = 0; k < dim; ++k) s->P[3 * i + k] = P[dim * i + k];
  s->bc = (unsigned char*)malloc(np);
  memcpy(s->bc, bc, np);
  s->nrm = (double*)calloc(np * 3, sizeof(double));
  s->meas = (double*)calloc(np, sizeof(double));
  for (long i = 0; i < np; ++i) {
    const double* a = s->V + 3 * s->P[3 * i];
    const double* b = s->V + 3 * s->P[3 * i + 1];
    double e1[3], n[3];
    vsub(b, a, e1);
    if (dim == 2) {
      n[0] = e1[1]; n[1] = -e1[0]; n[2] = 0.0;
      s->meas[i] = vnorm(e1);
    } else {
      const double* c = s->V + 3 * s->P[3 * i + 2];
      double e2[3];
      vsub(c, a, e2);
      vcross(e1, e2, n);
      s->meas[i] = 0.5 * vnorm(n);
    }
    double ln = vnorm(n);
    for (int k = 0; k < 3; ++k) s->nrm[3 * i + k] = ln > 0 ? n[k] / ln : 0.0;
    if (is_neumann(s, i)) s->nN++; else s->nD++;
  }
  scene_box(s);
  /* silhouette elements and their adjacent Neumann primitives */
  long nk = s->nN * dim; /* 2D: 2 endpoints per segment; 3D: 3 edges per triangle */
  orc_ekey* K = (orc_ekey*)malloc(sizeof(orc_ekey) * (nk > 0 ? nk : 1));
  long m = 0;
  for (long i = 0; i < np; ++i) {
    if (!is_neumann(s, i)) continue;
    if (dim == 2) {
      for (int k = 0; k < 2; ++k) { K[m].a = K[m].b = s->P[3 * i + k]; K[m].prim = (int)i; ++m; }
    } else {
      for (int k = 0; k < 3; ++k) {
        int a = s->P[3 * i + k], b = s->P[3 * i + (k + 1) % 3];
        K[m].a = a < b ? a : b; K[m].b = a < b ? b : a; K[m].prim = (int)i; ++m;
      }
    }
  }
  qsort(K, m, sizeof(orc_ekey), ekey_cmp);
  long ne = 0;
  for (long i = 0; i < m; ++i)
    if (i == 0 || K[i].a != K[i - 1].a || K[i].b != K[i - 1].b) ++ne;
  s->ne = ne;
  s->ev = (int*)malloc(sizeof(int) * 2 * (ne > 0 ? ne : 1));
  s->eoff = (int*)malloc(sizeof(int) * (ne + 1));
  s->eadj = (int*)malloc(sizeof(int) * (m > 0 ? m : 1));
  long e = -1;
  for (long i = 0; i < m; ++i) {
    if (i == 0 || K[i].a != K[i - 1].a || K[i].b != K[i - 1].b) {
      ++e;
      s->ev[2 * e] = K[i].a; s->ev[2 * e + 1] = K[i].b;
      s->eoff[e] = (int)i;
    }
    s->eadj[i] = K[i].prim;
  }
  s->eoff[ne] = (int)m;
  free(K);
  if (g) { s->g = *g; s->pc_g = dup_pc(g, np, dim); s->g.per_corner = s->pc_g; }
  if (h) { s->h = *h; s->pc_h = dup_pc(h, np, dim); s->h.per_corner = s->pc_h; }
  if (f) { s->f = *f; s->pc_f = dup_pc(f, np, dim); s->f.per_corner = s->pc_f; }
  if (gm) { s->gm = *gm; s->pc_gm = dup_pc(gm, np, dim); s->gm.per_corner = s->pc_gm; }
  if (hm) { s->hm = *hm; s->pc_hm = dup_pc(hm, np, dim); s->hm.per_corner = s->pc_hm; }
  return s;
}

/* bounding box of the vertices and the analytic shapes (R12), its centre
 * and half-diagonal L */
static void scene_box(orc_scene* s) {
  const int dim = s->dim;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (long i = 0; i < s->nv; ++i)
    for (int k = 0; k < dim; ++k) {
      double x = s->V[3 * i + k];
      if (x < lo[k]) lo[k] = x;
      if (x > hi[k]) hi[k] = x;
    }
  for (long i = 0; i < s->nsdf; ++i) {
    const orc_sdf* f = &s->sdf[i];
    for (int k = 0; k < dim; ++k) {
      double a, b;
      if (f->kind == 0) { a = f->p[k] - f->p[6]; b = f->p[k] + f->p[6]; }
      else if (f->kind == 1) { a = f->p[k] - f->p[3 + k] - f->p[6]; b = f->p[k] + f->p[3 + k] + f->p[6]; }
      else { a = fmin(f->p[k], f->p[3 + k]) - f->p[6]; b = fmax(f->p[k], f->p[3 + k]) + f->p[6]; }
      if (a < lo[k]) lo[k] = a;
      if (b > hi[k]) hi[k] = b;
    }
  }
  double d2 = 0;
  for (int k = 0; k < 3; ++k) {
    if (k >= dim) { lo[k] = hi[k] = 0; }
    s->center[k] = 0.5 * (lo[k] + hi[k]);
    d2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
  }
  s->L = 0.5 * sqrt(d2);
}

/* adds the analytic Dirichlet shapes (R12) and recomputes the scene box */
void orc_scene_set_sdf(orc_scene* s, long n, const orc_sdf* f) {
  free(s->sdf);
  s->nsdf = n;
  s->sdf = (orc_sdf*)malloc(sizeof(orc_sdf) * (n > 0 ? n : 1));
  if (n > 0) memcpy(s->sdf, f, sizeof(orc_sdf) * n);
  scene_box(s);
}

double orc_scene_L(const orc_scene* s) { return s->L; }
void orc_scene_center(const orc_scene* s, double c[3]) { vcopy(s->center, c); }
long orc_scene_n_elements(const orc_scene* s) { return s->ne; }

/* ------------------------------------------------------------------------ */
/* boundary data f, g, h (Sec. 3.2: callbacks of the problem)                */
/* ------------------------------------------------------------------------ */
static double analytic_value(const orc_fn* fn, int dim, const double x[3]) {
  const double* c = fn->coef;
  switch (fn->kind) {
    case 0: return 0.0;
    case 1: return c[0];
    case 2:
      if (dim == 2)
        return c[0] + c[1] * x[0] + c[2] * x[1] + c[3] * x[0] * x[0] + c[4] * x[1] * x[1] +
               c[5] * x[0] * x[1];
      return c[0] + c[1] * x[0] + c[2] * x[1] + c[3] * x[2] + c[4] * x[0] * x[0] +
             c[5] * x[1] * x[1] + c[6] * x[2] * x[2] + c[7] * x[0] * x[1] + c[8] * x[1] * x[2] +
             c[9] * x[2] * x[0];
    case 3: return c[0] * exp(c[1] * x[0]) * cos(c[1] * x[1]);
    case 5: return c[0] * exp(c[1] * x[0] + c[2] * x[1] + c[3] * x[2]);
    default: return 0.0;
  }
}

static void analytic_grad(const orc_fn* fn, int dim, const double x[3], double gr[3]) {
  const double* c = fn->coef;
  gr[0] = gr[1] = gr[2] = 0.0;
  switch (fn->kind) {
    case 2:
      if (dim == 2) {
        gr[0] = c[1] + 2 * c[3] * x[0] + c[5] * x[1];
        gr[1] = c[2] + 2 * c[4] * x[1] + c[5] * x[0];
      } else {
        gr[0] = c[1] + 2 * c[4] * x[0] + c[7] * x[1] + c[9] * x[2];
        gr[1] = c[2] + 2 * c[5] * x[1] + c[7] * x[0] + c[8] * x[2];
        gr[2] = c[3] + 2 * c[6] * x[2] + c[8] * x[1] + c[9] * x[0];
      }
      break;
    case 3: {
      double e = c[0] * c[1] * exp(c[1] * x[0]);
      gr[0] = e * cos(c[1] * x[1]);
      gr[1] = -e * sin(c[1] * x[1]);
      break;
    }
    case 5: {
      double e = c[0] * exp(c[1] * x[0] + c[2] * x[1] + c[3] * x[2]);
      gr[0] = c[1] * e; gr[1] = c[2] * e; gr[2] = c[3] * e;
      break;
    }
    default: break;
  }
}

/* barycentric weights of point q on primitive `prim` (q assumed on it) */
static void prim_bary(const orc_scene* s, long prim, const double q[3], double w[3]) {
  const double* a = s->V + 3 * s->P[3 * prim];
  const double* b = s->V + 3 * s->P[3 * prim + 1];
  if (s->dim == 2) {
    double e[3], d[3];
    vsub(b, a, e); vsub(q, a, d);
    double t = vdot(d, e) / vdot(e, e);
    w[0] = 1 - t; w[1] = t; w[2] = 0;
    return;
  }
  const double* c = s->V + 3 * s->P[3 * prim + 2];
  double n[3], e1[3], e2[3], t1[3], t2[3], qa[3], qb[3], qc[3];
  vsub(b, a, e1); vsub(c, a, e2); vcross(e1, e2, n);
  double nn = vdot(n, n);
  vsub(a, q, qa); vsub(b, q, qb); vsub(c, q, qc);
  vcross(qb, qc, t1); w[0] = vdot(t1, n) / nn;
  vcross(qc, qa, t2); w[1] = vdot(t2, n) / nn;
  w[2] = 1 - w[0] - w[1];
}

/* value of a boundary field on primitive `prim` at point q (g, or h with its
 * normal derivative form, taken along sgn * n+: sgn = -1 on the "-" side of
 * a double-sided primitive) */
static double boundary_value(const orc_scene* s, const orc_fn* fn, long prim, const double q[3],
                             double sgn) {
  if (prim >= s->np) return analytic_value(fn, s->dim, q);   /* an analytic shape (R12) */
  if (fn->kind == 4) {
    double w[3];
    prim_bary(s, prim, q, w);
    double v = 0;
    for (int k = 0; k < s->dim; ++k) v += w[k] * (double)fn->per_corner[s->dim * prim + k];
    return v;
  }
  if (fn->as_nd) {
    double gr[3];
    analytic_grad(fn, s->dim, q, gr);
    return sgn * vdot(gr, s->nrm + 3 * prim);
  }
  return analytic_value(fn, s->dim, q);
}

int orc_has_source(const orc_scene* s) { return s->f.kind != 0; }
int orc_has_neumann_data(const orc_scene* s) { return s->h.kind != 0 || s->hm.kind != 0; }

/* ------------------------------------------------------------------------ */
/* closest points (plain definitions)                                        */
/* ------------------------------------------------------------------------ */
static void closest_on_segment(const double x[3], const double a[3], const double b[3], double o[3]) {
  double e[3], d[3];
  vsub(b, a, e); vsub(x, a, d);
  double ee = vdot(e, e);
  double t = ee > 0 ? vdot(d, e) / ee : 0.0;
  if (t < 0) t = 0;
  if (t > 1) t = 1;
  vaxpy(a, t, e, o);
}

/* q lies in triangle (a, b, c) (inclusive), given a normal n of its plane */
static int inside_triangle(const double q[3], const double a[3], const double b[3], const double c[3],
                           const double n[3]) {
  double e[3], d[3], t[3];
  vsub(b, a, e); vsub(q, a, d); vcross(e, d, t);
  if (vdot(t, n) < 0) return 0;
  vsub(c, b, e); vsub(q, b, d); vcross(e, d, t);
  if (vdot(t, n) < 0) return 0;
  vsub(a, c, e); vsub(q, c, d); vcross(e, d, t);
  if (vdot(t, n) < 0) return 0;
  return 1;
}

/* closest point of a triangle: the projection onto its plane when that lies
 * inside, otherwise the closest point on one of its three edges */
static void closest_on_triangle(const double x[3], const double a[3], const double b[3], const double c[3],
                                double o[3]) {
  double e1[3], e2[3], n[3], d[3], q[3];
  vsub(b, a, e1); vsub(c, a, e2); vcross(e1, e2, n);
  double nn = vdot(n, n);
  if (nn > 0) {
    vsub(x, a, d);
    vaxpy(x, -vdot(d, n) / nn, n, q);
    if (inside_triangle(q, a, b, c, n)) { vcopy(q, o); return; }
  }
  double best = INFINITY, p[3], t[3];
  const double* E[3][2] = {{a, b}, {b, c}, {c, a}};
  for (int k = 0; k < 3; ++k) {
    closest_on_segment(x, E[k][0], E[k][1], p);
    vsub(p, x, t);
    double dd = vdot(t, t);
    if (dd < best) { best = dd; vcopy(p, o); }
  }
}

static void closest_on_prim(const orc_scene* s, long i, const double x[3], double o[3]) {
  const double* a = s->V + 3 * s->P[3 * i];
  const double* b = s->V + 3 * s->P[3 * i + 1];
  if (s->dim == 2) closest_on_segment(x, a, b, o);
  else closest_on_triangle(x, a, b, s->V + 3 * s->P[3 * i + 2], o);
}

/* closest point o on the surface of an analytic shape (R12) and the
 * distance to it, from the plain definitions: a ball's surface point along
 * the ray from its centre; a box rounded by rho is the set of points within
 * rho of the sharp box, so from outside its closest point lies rho beyond the
 * sharp box's closest point (the clamp of x into it); from inside a sharp
 * box the closest point is on the nearest face; a capsule is the set of
 * points within its radius of a segment */
double orc_sdf_closest(int dim, const orc_sdf* f, const double x[3], double o[3]) {
  double v[3] = {0, 0, 0}, l;
  o[0] = o[1] = o[2] = 0.0;
  if (f->kind == 0) {
    for (int k = 0; k < dim; ++k) v[k] = x[k] - f->p[k];
    l = vnorm(v);
    const double dist = fabs(l - f->p[6]);
    if (l == 0.0) { v[0] = 1.0; l = 1.0; }   /* the centre: every surface point is closest */
    for (int k = 0; k < dim; ++k) o[k] = f->p[k] + f->p[6] * v[k] / l;
    return dist;
  }
  if (f->kind == 1 && f->inside) {
    int kmin = 0;
    double gmin = INFINITY;
    for (int k = 0; k < dim; ++k) {
      double g = f->p[3 + k] - fabs(x[k] - f->p[k]);
      if (g < gmin) { gmin = g; kmin = k; }
    }
    vcopy(x, o);
    o[kmin] = f->p[kmin] + (x[kmin] >= f->p[kmin] ? f->p[3 + kmin] : -f->p[3 + kmin]);
    return fabs(gmin);
  }
  double c[3] = {0, 0, 0};   /* closest point of the core (sharp box or segment) */
  if (f->kind == 1) {
    for (int k = 0; k < dim; ++k) c[k] = fmin(fmax(x[k], f->p[k] - f->p[3 + k]), f->p[k] + f->p[3 + k]);
  } else {
    double ab[3] = {0, 0, 0}, ax[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) { ab[k] = f->p[3 + k] - f->p[k]; ax[k] = x[k] - f->p[k]; }
    double t = vdot(ab, ab) > 0.0 ? vdot(ax, ab) / vdot(ab, ab) : 0.0;
    t = fmin(fmax(t, 0.0), 1.0);
    for (int k = 0; k < dim; ++k) c[k] = f->p[k] + t * ab[k];
  }
  vsub(x, c, v);
  l = vnorm(v);
  if (l == 0.0) { vcopy(c, o); return f->p[6]; }   /* on the core: outside the domain */
  for (int k = 0; k < dim; ++k) o[k] = c[k] + f->p[6] * v[k] / l;
  return fabs(l - f->p[6]);
}

/* Q.1 (Sec. 5): distance to the Dirichlet boundary, its closest point and
 * primitive (infinite distance and prim -1 when there is none); analytic
 * shapes take part as primitives n_prims + i (R12) */
double orc_closest_dirichlet(const orc_scene* s, const double x[3], double xbar[3], long* prim) {
  double best = INFINITY, p[3], t[3];
  *prim = -1;
  for (long i = 0; i < s->np; ++i) {
    if (is_neumann(s, i)) continue;
    closest_on_prim(s, i, x, p);
    vsub(p, x, t);
    double d = vnorm(t);
    if (d < best) { best = d; vcopy(p, xbar); *prim = i; }
  }
  for (long i = 0; i < s->nsdf; ++i) {
    double d = orc_sdf_closest(s->dim, &s->sdf[i], x, p);
    if (d < best) { best = d; vcopy(p, xbar); *prim = s->np + i; }
  }
  return best;
}

/* Q.2 (Sec. 5.1, Eq. SilhouetteDefinition): distance from x to the closest
 * point of the visibility silhouette of the Neumann boundary within rmax.
 * An element (edge / vertex) with a single adjacent Neumann primitive is
 * always a silhouette; otherwise it is one when (v.n_a)(v.n_b) <= 0 for some
 * pair (a, b) of adjacent primitives, v = closest point on the element - x. */
double orc_silhouette(const orc_scene* s, const double x[3], double rmax) {
  double best = rmax, p[3], v[3];
  for (long e = 0; e < s->ne; ++e) {
    const double* a = s->V + 3 * s->ev[2 * e];
    const double* b = s->V + 3 * s->ev[2 * e + 1];
    if (s->dim == 2) vcopy(a, p);
    else closest_on_segment(x, a, b, p);
    vsub(p, x, v);
    double d = vnorm(v);
    if (!(d < best)) continue;
    int n_adj = s->eoff[e + 1] - s->eoff[e];
    int sil = (n_adj == 1);
    for (int i = s->eoff[e]; i < s->eoff[e + 1] && !sil; ++i)
      for (int j = i + 1; j < s->eoff[e + 1] && !sil; ++j) {
        double da = vdot(v, s->nrm + 3 * s->eadj[i]);
        double db = vdot(v, s->nrm + 3 * s->eadj[j]);
        if (da * db <= 0.0) sil = 1;
      }
    if (sil) best = d;
  }
  return best;
}

/* ray o + t v against one primitive: the parameter t of the crossing (of
 * either sign), or -INFINITY when the ray's line misses it */
static double ray_prim(const orc_scene* s, long i, const double o[3], const double v[3]) {
  const double* a = s->V + 3 * s->P[3 * i];
  const double* b = s->V + 3 * s->P[3 * i + 1];
  if (s->dim == 2) {
    /* solve o + t v = a + u (b - a) by Cramer's rule */
    double e0 = b[0] - a[0], e1 = b[1] - a[1];
    double w0 = a[0] - o[0], w1 = a[1] - o[1];
    double det = -v[0] * e1 + e0 * v[1];
    if (det == 0.0) return -INFINITY;
    double t = (-w0 * e1 + e0 * w1) / det;
    double u = (v[0] * w1 - v[1] * w0) / det;
    if (u < 0.0 || u > 1.0) return -INFINITY;
    return t;
  }
  const double* c = s->V + 3 * s->P[3 * i + 2];
  double e1[3], e2[3], n[3], w[3], q[3];
  vsub(b, a, e1); vsub(c, a, e2); vcross(e1, e2, n);
  double den = vdot(n, v);
  if (den == 0.0) return -INFINITY;
  vsub(a, o, w);
  double t = vdot(n, w) / den;
  vaxpy(o, t, v, q);
  if (!inside_triangle(q, a, b, c, n)) return -INFINITY;
  return t;
}

/* signed distance of y from the plane (line, 2D) of primitive i, positive on
 * the side its outward normal points to */
static double plane_distance(const orc_scene* s, long i, const double y[3]) {
  const double* a = s->V + 3 * s->P[3 * i];
  double w[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < s->dim; ++k) w[k] = y[k] - a[k];
  double m = 0.0;
  for (int k = 0; k < s->dim; ++k) m += w[k] * s->nrm[3 * i + k];
  return m;
}

/* Q.3 (Sec. 5): first crossing of the ray o + t v, 0 < t <= tmax, with the
 * Neumann boundary, skipping primitives skip0 and skip1; returns the
 * primitive (or -1) and t.  With behind > 0 (reading R13) a crossing at
 * -256 behind < t <= 0 of a one-sided primitive that the ray leaves
 * (v . n > 0, n the outward normal, v a unit vector) counts as a crossing at
 * t = 0 when o lies outside the primitive's plane by less than behind.  Ties
 * go to the lowest primitive index. */
long orc_ray_neumann(const orc_scene* s, const double o[3], const double v[3], double tmax,
                     long skip0, long skip1, double behind, double* t_out) {
  long best = -1;
  double bt = tmax;
  for (long i = 0; i < s->np; ++i) {
    if (!is_neumann(s, i) || i == skip0 || i == skip1) continue;
    double t = ray_prim(s, i, o, v);
    if (!(t > 0.0) && behind > 0.0 && t > -256.0 * behind && !double_sided(s, i) &&
        vdot(v, s->nrm + 3 * i) > 0.0 && plane_distance(s, i, o) < behind)
      t = 0.0;
    else if (!(t > 0.0))
      continue;
    if (t <= bt && (best < 0 || t < bt)) { best = i; bt = t; }
  }
  *t_out = best >= 0 ? bt : tmax;
  return best;
}

/* ------------------------------------------------------------------------ */
/* decision margins                                                          */
/* ------------------------------------------------------------------------ */
/* A query answered in FP32 may pick a different discrete outcome than the
 * FP64 definitions above (a silhouette or not, a crossing or not) only where
 * one of the quantities that decide it lies near its threshold.  These two
 * functions return, for a reported result, the smallest distance (in length
 * units) of any deciding quantity from its threshold, so that a parity check
 * can tell such a near-tie from a wrong answer.  INFINITY: no decision near
 * the result. */

/* Q.2: the silhouette decisions that could yield distance d from x with
 * search radius rmax.  Over every silhouette element whose distance from x
 * is within tol of d: |distance - rmax| (the within-radius test) and, for an
 * element with two or more adjacent Neumann primitives, |v . n_i| for each of
 * them (v = closest point on the element - x), since the sign of
 * (v . n_a)(v . n_b) can only change where one factor vanishes. */
double orc_silhouette_margin(const orc_scene* s, const double x[3], double rmax, double d, double tol) {
  double m = INFINITY, p[3], v[3];
  for (long e = 0; e < s->ne; ++e) {
    const double* a = s->V + 3 * s->ev[2 * e];
    const double* b = s->V + 3 * s->ev[2 * e + 1];
    if (s->dim == 2) vcopy(a, p);
    else closest_on_segment(x, a, b, p);
    vsub(p, x, v);
    const double de = vnorm(v);
    if (!(fabs(de - d) <= tol)) continue;
    double me = fabs(de - rmax);
    if (s->eoff[e + 1] - s->eoff[e] >= 2)
      for (int i = s->eoff[e]; i < s->eoff[e + 1]; ++i) me = fmin(me, fabs(vdot(v, s->nrm + 3 * s->eadj[i])));
    m = fmin(m, me);
  }
  return m;
}

/* distance from y to the rim of primitive i: its end points (2D) or its
 * three edges (3D) */
static double prim_rim_distance(const orc_scene* s, long i, const double y[3]) {
  const double* a = s->V + 3 * s->P[3 * i];
  const double* b = s->V + 3 * s->P[3 * i + 1];
  double t[3], p[3];
  if (s->dim == 2) {
    vsub(y, a, t);
    double m = vnorm(t);
    vsub(y, b, t);
    return fmin(m, vnorm(t));
  }
  const double* c = s->V + 3 * s->P[3 * i + 2];
  const double* E[3][2] = {{a, b}, {b, c}, {c, a}};
  double m = INFINITY;
  for (int k = 0; k < 3; ++k) {
    closest_on_segment(y, E[k][0], E[k][1], p);
    vsub(p, y, t);
    m = fmin(m, vnorm(t));
  }
  return m;
}

/* Q.3: the crossing decisions that could yield parameter t on the ray
 * o + t v (0 < t <= tmax, skipping skip0 and skip1): |t - tmax| |v| (the
 * clip to the star radius), t |v| (the t > 0 test), and, for every Neumann
 * primitive within tol of y = o + t v, the distance from y to its rim (a
 * crossing near an edge or end point, where the FP32 test may call it a
 * miss or give it to the neighbour). */
double orc_ray_margin(const orc_scene* s, const double o[3], const double v[3], double tmax, double t,
                      long skip0, long skip1, double tol) {
  const double vl = vnorm(v);
  double m = fmin(fabs(t - tmax) * vl, fabs(t) * vl);
  double y[3], p[3], w[3];
  vaxpy(o, t, v, y);
  for (long i = 0; i < s->np; ++i) {
    if (!is_neumann(s, i) || i == skip0 || i == skip1) continue;
    closest_on_prim(s, i, y, p);
    vsub(p, y, w);
    if (!(vnorm(w) <= tol)) continue;
    m = fmin(m, prim_rim_distance(s, i, y));
  }
  return m;
}

/* ------------------------------------------------------------------------ */
/* samplers                                                                  */
/* ------------------------------------------------------------------------ */
/* uniform direction on the unit circle / sphere (Sec. 4.4): 2D angle
 * 2 pi U0; 3D Archimedes' map z = 1 - 2 U0, phi = 2 pi U1 */
void orc_sample_direction(int dim, double U0, double U1, double v[3]) {
  if (dim == 2) {
    double th = 2.0 * ORC_PI * U0;
    v[0] = cos(th); v[1] = sin(th); v[2] = 0.0;
    return;
  }
  double z = 1.0 - 2.0 * U0, phi = 2.0 * ORC_PI * U1;
  double rr = sqrt(fmax(0.0, 1.0 - z * z));
  v[0] = rr * cos(phi); v[1] = rr * sin(phi); v[2] = z;
}

/* distance fraction s = t / r of the source sample (Sec. 4.6): density
 * proportional to G^B(x, x + s r v) times the radial measure s^(N-1),
 * i.e. 6 s (1 - s) in 3D and -4 s ln s in 2D.  3D inverts
 * F(s) = 3 s^2 - 2 s^3 with the trigonometric root of the cubic; 2D takes
 * the square root of a product of two uniforms. */
double orc_source_fraction(int dim, double U2, double U3) {
  if (dim == 2) return sqrt(U2 * U3);
  return 0.5 + cos((acos(1.0 - 2.0 * U2) - 2.0 * ORC_PI) / 3.0);
}

/* ball Green's function G^B(x, y) with |y - x| = rho, ball radius R (App. A.1) */
double orc_green_ball(int dim, double rho, double R) {
  if (dim == 2) return log(R / rho) / (2.0 * ORC_PI);
  return (1.0 / rho - 1.0 / R) / (4.0 * ORC_PI);
}

/* its integral over the ball (App. A.1) */
double orc_green_ball_norm(int dim, double R) {
  return dim == 2 ? R * R / 4.0 : R * R / 6.0;
}

/* ---- screened Poisson (App. A.2) ---------------------------------------- */
/* Modified Bessel functions, exponentially scaled: orc_bessel_ie(n, x) =
 * e^-x I_n(x) from the power series sum_k (x/2)^(2k+n) / (k! (k+n)!), and
 * orc_bessel_ke(n, x) = e^x K_n(x) from the integral representation
 * K_n(x) = int_0^inf exp(-x cosh u) cosh(n u) du (trapezoid rule, whose
 * error decays exponentially for this analytic, doubly decaying integrand). */
double orc_bessel_ie(int n, double x) {
  double term = 1.0, sum = 0.0;
  for (int k = 1; k <= n; ++k) term *= (x / 2.0) / k;   /* (x/2)^n / n! */
  const double q = x * x / 4.0;
  for (int k = 0; k < 2000; ++k) {
    sum += term;
    term *= q / ((k + 1.0) * (k + 1.0 + n));
    if (term < 1e-18 * sum) break;
  }
  return sum * exp(-x);
}

double orc_bessel_ke(int n, double x) {
  /* integrand exp(-x (cosh u - 1)) cosh(n u), negligible once
     x (cosh u - 1) > 745 */
  const double umax = acosh(1.0 + 745.0 / x) + 1.0;
  const int m = (int)ceil(umax / 0.02);   /* node spacing 0.02 */
  const double h = umax / m;
  double sum = 0.5;   /* u = 0 */
  for (int i = 1; i <= m; ++i) {
    const double u = i * h;
    sum += exp(-x * (cosh(u) - 1.0)) * cosh(n * u);
  }
  return sum * h;
}

/* Q^{sigma,B}(r; R) of Eq. (ScreenedPoissonKernelsSphere): the factor by which
 * the screened ball Poisson kernel differs from the free-space one at a
 * boundary point at distance r of a ball of radius R */
double orc_screened_q(int dim, double sigma, double r, double R) {
  if (!(sigma > 0.0)) return 1.0;
  const double a = sqrt(sigma), zr = r * a, zR = R * a;
  if (dim == 2) {
    if (zr < 1e-12) return 1.0;
    /* (K1(zr) + I1(zr) K0(zR) / I0(zR)) zr, with scaled functions */
    const double k1 = orc_bessel_ke(1, zr) * exp(-zr);
    const double ratio = orc_bessel_ke(0, zR) / orc_bessel_ie(0, zR) * exp(-2.0 * zR);
    const double i1 = orc_bessel_ie(1, zr) * exp(zr);
    return (k1 + i1 * ratio) * zr;
  }
  /* e^-zr (zr + 1) + (cosh(zr) zr - sinh(zr)) e^-zR / sinh(zR) */
  return exp(-zr) * (zr + 1.0) + (cosh(zr) * zr - sinh(zr)) * exp(-zR) / sinh(zR);
}

/* screened ball Green's function G^{sigma,B} at distance rho, radius R */
double orc_green_ball_screened(int dim, double sigma, double rho, double R) {
  if (!(sigma > 0.0)) return orc_green_ball(dim, rho, R);
  const double a = sqrt(sigma), zr = rho * a, zR = R * a;
  if (dim == 2) {
    const double k0 = orc_bessel_ke(0, zr) * exp(-zr);
    const double i0 = orc_bessel_ie(0, zr) * exp(zr);
    const double ratio = orc_bessel_ke(0, zR) / orc_bessel_ie(0, zR) * exp(-2.0 * zR);
    return (k0 - i0 * ratio) / (2.0 * ORC_PI);
  }
  return sinh((R - rho) * a) / (4.0 * ORC_PI * rho * sinh(zR));
}

/* its integral over the ball */
double orc_green_ball_norm_screened(int dim, double sigma, double R) {
  if (!(sigma > 0.0)) return orc_green_ball_norm(dim, R);
  const double a = sqrt(sigma), zR = R * a;
  if (dim == 2) return (1.0 - exp(-zR) / orc_bessel_ie(0, zR)) / sigma;
  return (1.0 - zR / sinh(zR)) / sigma;
}

/* point on primitive i from two uniforms: linear in 2D; in 3D the
 * square-root barycentric map (uniform in area) */
static void point_on_prim(const orc_scene* s, long i, double U5, double U6, double z[3]) {
  const double* a = s->V + 3 * s->P[3 * i];
  const double* b = s->V + 3 * s->P[3 * i + 1];
  if (s->dim == 2) {
    double e[3];
    vsub(b, a, e);
    vaxpy(a, U5, e, z);
    return;
  }
  const double* c = s->V + 3 * s->P[3 * i + 2];
  double r1 = sqrt(U5);
  double wa = 1.0 - r1, wb = r1 * (1.0 - U6), wc = r1 * U6;
  for (int k = 0; k < 3; ++k) z[k] = wa * a[k] + wb * b[k] + wc * c[k];
}

/* Q.4 (Sec. 5.2), plain version of reading R7: returns the primitive (or -1
 * when no Neumann primitive meets B(x, r)), the point z and its pdf */
long orc_neumann_sample(const orc_scene* s, const double x[3], double r, double U4, double U5,
                        double U6, double z[3], double* pdf) {
  double total = 0.0, p[3], t[3];
  for (long i = 0; i < s->np; ++i) {
    if (!is_neumann(s, i)) continue;
    closest_on_prim(s, i, x, p);
    vsub(p, x, t);
    if (vnorm(t) < r) total += s->meas[i];
  }
  *pdf = 0.0;
  if (!(total > 0.0)) return -1;
  double target = U4 * total, cum = 0.0;
  long pick = -1;
  for (long i = 0; i < s->np; ++i) {
    if (!is_neumann(s, i)) continue;
    closest_on_prim(s, i, x, p);
    vsub(p, x, t);
    if (!(vnorm(t) < r)) continue;
    pick = i;
    cum += s->meas[i];
    if (cum > target) break;
  }
  point_on_prim(s, pick, U5, U6, z);
  *pdf = 1.0 / total;
  return pick;
}

/* ------------------------------------------------------------------------ */
/* one step of Algorithm 1                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  double eps, rmin, offset, escape_radius;
  int max_steps;
  uint64_t seed;
  double sigma;       /* screening coefficient (0: Poisson) */
  double tik_sigma;   /* Tikhonov switch: sigma_T added from step tik_steps on */
  int tik_steps;
} orc_params;

typedef struct {
  double x[3];
  double n[3];  /* on the Neumann boundary: the normal of the walk's side */
  int onN;
  int cur;      /* Neumann primitive the walk sits on, or -1 */
  double q[3];  /* x_k - x_{k-1} (R11); the start side's normal at a boundary start */
  int q_set;    /* 0 at an interior start, where q is not defined */
} orc_state;

typedef struct {
  double x[3];
  int onN, cur;
  double dD, xbar[3];
  int primD;
  int term;      /* 0 continue, 1 eps-shell, 2 capped, 3 escaped */
  double g_term; /* g(xbar) when the walk ends here */
  double dsil, r, v[3];
  int hit, hit_prim;
  double t, p[3];
  int n_prim, valid;
  double z[3], pdf, Nhat;
  double s_frac, Shat;
  double q;         /* screened continuation factor Q (1 for Poisson) */
  int roulette;     /* 1: the walk was ended by Russian roulette here */
  int side_g;       /* R11: +1 / -1 side of g at a double-sided end, else 0 */
  int side_h;       /* R11: +1 / -1 side of h for an accepted sample on a
                       double-sided primitive, else 0 */
} orc_step_rec;

/* Executes step k of walk (point, walk) from `st`; writes the record and the
 * next state; returns the contribution to the walk estimate. */
double orc_step(const orc_scene* s, const orc_params* P, uint32_t point, uint32_t walk,
                uint32_t k, const orc_state* st, orc_step_rec* rec, orc_state* next) {
  const int dim = s->dim;
  memset(rec, 0, sizeof(*rec));
  vcopy(st->x, rec->x);
  rec->onN = st->onN; rec->cur = st->cur;
  rec->hit_prim = -1; rec->n_prim = -1;
  *next = *st;

  /* Q.1 and the eps-shell test (Alg. 1; Sec. 3.4.2) */
  long primD;
  double xbar[3] = {0, 0, 0};
  double dD = orc_closest_dirichlet(s, st->x, xbar, &primD);
  rec->dD = dD; vcopy(xbar, rec->xbar); rec->primD = (int)primD;
  double gx = 0.0;
  if (primD >= 0) {
    /* double-sided: the side the walk approached from (R11) */
    int minus = 0;
    if (primD < s->np && double_sided(s, primD)) {
      double qd[3];
      if (st->q_set) vcopy(st->q, qd);
      else vsub(xbar, st->x, qd);
      minus = !(vdot(qd, s->nrm + 3 * primD) > 0.0);
      rec->side_g = minus ? -1 : 1;
    }
    gx = minus ? boundary_value(s, &s->gm, primD, xbar, -1.0) : boundary_value(s, &s->g, primD, xbar, 1.0);
  }
  double dc[3];
  vsub(st->x, s->center, dc);
  if (dD < P->eps) rec->term = 1;
  else if ((int)k >= P->max_steps) rec->term = 2;
  else if (vnorm(dc) > P->escape_radius) rec->term = 3;
  if (rec->term) { rec->g_term = gx; return gx; }

  /* query origin (reading R4) */
  double xq[3];
  if (st->onN) vaxpy(st->x, -P->offset, st->n, xq);
  else vcopy(st->x, xq);

  /* Q.2 and the star radius (Sec. 4.4.2-4.4.3, reading R3; without a
     Dirichlet boundary, capped at the escape radius, reading R10) */
  double dsil = orc_silhouette(s, xq, dD);
  double r = fmin(fmin(dD, fmax(P->rmin, dsil)), P->escape_radius);
  /* screening of this step: sigma, plus sigma_T once the Tikhonov switch is
     reached (reading R10) */
  const double sig = P->sigma + ((P->tik_sigma > 0.0 && (int)k >= P->tik_steps) ? P->tik_sigma : 0.0);
  rec->dsil = dsil; rec->r = r;

  /* direction, hemisphere flip (Sec. 4.4.4) */
  double U[4];
  orc_uniforms(P->seed, point, walk, k, 0, U);
  double v[3];
  orc_sample_direction(dim, U[0], U[1], v);
  if (st->onN && vdot(st->n, v) > 0.0) { v[0] = -v[0]; v[1] = -v[1]; v[2] = -v[2]; }
  vcopy(v, rec->v);

  /* Q.3 clipped to r; the sphere part of the star boundary on a miss */
  double t;
  long hp = orc_ray_neumann(s, xq, v, r, st->onN ? st->cur : -1, -1, 0.25 * P->offset, &t);
  double p[3];
  if (hp < 0) t = r;
  vaxpy(xq, t, v, p);   /* on the tested ray, from the query origin (R4) */
  rec->hit = hp >= 0; rec->hit_prim = (int)hp; rec->t = t; vcopy(p, rec->p);

  /* Neumann contribution (Sec. 4.5, reading R7) */
  double Nhat = 0.0;
  if (orc_has_neumann_data(s)) {
    double V4[4], z[3], pdf;
    orc_uniforms(P->seed, point, walk, k, 1, V4);
    long zp = orc_neumann_sample(s, st->x, r, V4[0], V4[1], V4[2], z, &pdf);
    rec->n_prim = (int)zp;
    if (zp >= 0) {
      vcopy(z, rec->z); rec->pdf = pdf;
      double dz[3], d[3], tv;
      vsub(z, st->x, dz);
      double rho = vnorm(dz);
      int valid = pdf > 0.0 && rho > 0.0 && rho < r;
      if (valid) {
        vsub(z, xq, d);
        long blk = orc_ray_neumann(s, xq, d, 1.0 - 1e-6, zp, -1, 0.0, &tv);
        valid = blk < 0;
      }
      rec->valid = valid;
      if (valid) {
        double alpha = st->onN ? 0.5 : 1.0;
        /* double-sided: the side of zp that the query origin sees (R11) */
        int minus = 0;
        if (double_sided(s, zp)) {
          minus = !(vdot(d, s->nrm + 3 * zp) > 0.0);
          rec->side_h = minus ? -1 : 1;
        }
        double hz = minus ? boundary_value(s, &s->hm, zp, z, -1.0) : boundary_value(s, &s->h, zp, z, 1.0);
        Nhat = orc_green_ball_screened(dim, sig, rho, r) * hz / (alpha * pdf);
      }
    }
  }
  rec->Nhat = Nhat;

  /* source contribution (Sec. 4.6), reusing the direction v */
  double Shat = 0.0;
  if (s->f.kind != 0) {
    double sf = orc_source_fraction(dim, U[2], U[3]);
    double ts = r * sf, y[3];
    vaxpy(st->x, ts, v, y);
    rec->s_frac = sf;
    if (ts < t) {
      Shat = orc_green_ball_norm(dim, r) * analytic_value(&s->f, dim, y);
      /* screened: reweight the Poisson-density sample (reading R10); the
         ratio tends to 1 at the centre */
      if (sig > 0.0 && ts > 0.0)
        Shat *= orc_green_ball_screened(dim, sig, ts, r) / orc_green_ball(dim, ts, r);
    }
  }
  rec->Shat = Shat;

  /* continuation factor Q, as Russian roulette (reading R10) */
  rec->q = orc_screened_q(dim, sig, t, r);
  if (sig > 0.0) {
    double Ur[4];
    orc_uniforms(P->seed, point, walk, k, 0xffffffffu, Ur);
    if (Ur[0] >= rec->q) {
      rec->roulette = 1;
      rec->term = 4;
    }
  }

  /* advance (reading R1 for the sign) */
  vcopy(p, next->x);
  vsub(p, st->x, next->q);
  next->q_set = 1;
  next->onN = hp >= 0;
  next->cur = (int)hp;
  if (hp >= 0) {
    vcopy(s->nrm + 3 * hp, next->n);
    /* double-sided: the normal of the side the walk arrives on (R11) */
    if (double_sided(s, hp) && vdot(next->q, next->n) < 0.0)
      for (int k = 0; k < 3; ++k) next->n[k] = -next->n[k];
  } else {
    next->n[0] = next->n[1] = next->n[2] = 0.0;
  }
  return Nhat - Shat;
}

/* one whole walk; returns the estimate, the number of steps (Q.1 calls) and
 * the way it ended (1 eps-shell, 2 capped, 3 escaped); optionally records up
 * to max_rec steps.  start_prim >= 0 (a Neumann primitive x0 lies on) starts
 * the walk on the boundary (reading R9), on the "+" side of a double-sided
 * primitive; start_prim = -2 - p starts it on the "-" side of the
 * double-sided primitive p (R11). */
double orc_walk_from(const orc_scene* s, const orc_params* P, const double x0[3], long start_prim,
                     uint32_t point, uint32_t walk, int* n_steps, int* how, orc_step_rec* recs,
                     int max_rec) {
  orc_state st, nx;
  memset(&st, 0, sizeof(st));
  vcopy(x0, st.x);
  st.cur = -1;
  const int minus = start_prim <= -2;
  const long sp = minus ? -2 - start_prim : start_prim;
  if (sp >= 0 && sp < s->np && is_neumann(s, sp) && (!minus || double_sided(s, sp))) {
    st.onN = 1;
    st.cur = (int)sp;
    for (int k = 0; k < 3; ++k) st.n[k] = (minus ? -1.0 : 1.0) * s->nrm[3 * sp + k];
    vcopy(st.n, st.q);
    st.q_set = 1;
  }
  double acc = 0.0;
  orc_step_rec rec;
  for (uint32_t k = 0;; ++k) {
    double c = orc_step(s, P, point, walk, k, &st, &rec, &nx);
    if (recs && (int)k < max_rec) recs[k] = rec;
    acc += c;
    if (rec.term) {
      *n_steps = (int)k + 1;
      *how = rec.term;
      return acc;
    }
    st = nx;
  }
}

double orc_walk(const orc_scene* s, const orc_params* P, const double x0[3], uint32_t point,
                uint32_t walk, int* n_steps, int* how, orc_step_rec* recs, int max_rec) {
  return orc_walk_from(s, P, x0, -1, point, walk, n_steps, how, recs, max_rec);
}

/* ------------------------------------------------------------------------ */
/* Monte Carlo aggregation (Sec. 3.4.1): per point, the mean of W walk       */
/* estimates and their unbiased sample variance, two passes in FP64.         */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_scene* s;
  const orc_params* P;
  const float* points;
  const uint32_t* point_ids;
  const int* start_prims;   /* optional [n]: Neumann primitive of a boundary point, or -1 */
  long n;
  int W;
  uint32_t walk_base;       /* RNG walk index of walk 0 */
  int nthreads, tid;
  double* values;           /* [n][W] */
  long steps, capped, escaped;
} orc_job;

/* the walks (point i, walk w) with i * W + w = tid (mod nthreads) */
static void* orc_worker(void* arg) {
  orc_job* J = (orc_job*)arg;
  const int dim = J->s->dim;
  const long total = J->n * (long)J->W;
  for (long j = J->tid; j < total; j += J->nthreads) {
    const long i = j / J->W;
    const int w = (int)(j - i * J->W);
    double x0[3] = {0, 0, 0};
    for (int k = 0; k < dim; ++k) x0[k] = (double)J->points[dim * i + k];
    uint32_t pid = J->point_ids ? J->point_ids[i] : (uint32_t)i;
    int ns, how;
    const long sp = J->start_prims ? J->start_prims[i] : -1;
    J->values[j] = orc_walk_from(J->s, J->P, x0, sp, pid, J->walk_base + (uint32_t)w, &ns, &how, NULL, 0);
    J->steps += ns;
    if (how == 2) J->capped++;
    if (how == 3) J->escaped++;
  }
  return NULL;
}

/* points [n][dim] float; point_ids (optional) gives the RNG point index of
 * each point; start_prims (optional) the Neumann primitive of each boundary
 * point or -1; the walks of a point have RNG walk indices walk_base ..
 * walk_base + W - 1; values (optional) receives every walk estimate [n][W];
 * stats_out = {steps, capped, escaped} */
int orc_solve_from(const orc_scene* s, const orc_params* P, const float* points,
                   const uint32_t* point_ids, const int* start_prims, long n, int W, uint32_t walk_base,
                   int nthreads, double* mean, double* var, double* values, long* stats_out) {
  if (nthreads < 1) nthreads = 1;
  double* vals = values ? values : (double*)malloc(sizeof(double) * (n * (long)W > 0 ? n * (long)W : 1));
  orc_job* J = (orc_job*)calloc(nthreads, sizeof(orc_job));
  pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
  for (int t = 0; t < nthreads; ++t) {
    J[t].s = s; J[t].P = P; J[t].points = points; J[t].point_ids = point_ids;
    J[t].start_prims = start_prims;
    J[t].n = n; J[t].W = W; J[t].walk_base = walk_base; J[t].nthreads = nthreads; J[t].tid = t;
    J[t].values = vals;
    pthread_create(&th[t], NULL, orc_worker, &J[t]);
  }
  long st[3] = {0, 0, 0};
  for (int t = 0; t < nthreads; ++t) {
    pthread_join(th[t], NULL);
    st[0] += J[t].steps; st[1] += J[t].capped; st[2] += J[t].escaped;
  }
  /* per point: mean and unbiased variance, two passes in walk order */
  for (long i = 0; i < n; ++i) {
    const double* v = vals + (long)W * i;
    double sum = 0.0, ss = 0.0;
    for (int w = 0; w < W; ++w) sum += v[w];
    const double m = sum / W;
    for (int w = 0; w < W; ++w) ss += (v[w] - m) * (v[w] - m);
    mean[i] = m;
    var[i] = W > 1 ? ss / (W - 1) : 0.0;
  }
  if (stats_out) { stats_out[0] = st[0]; stats_out[1] = st[1]; stats_out[2] = st[2]; }
  if (!values) free(vals);
  free(J); free(th);
  return 0;
}

int orc_solve(const orc_scene* s, const orc_params* P, const float* points, const uint32_t* point_ids,
              long n, int W, int nthreads, double* mean, double* var, double* values,
              long* stats_out) {
  return orc_solve_from(s, P, points, point_ids, NULL, n, W, 0, nthreads, mean, var, values, stats_out);
}
