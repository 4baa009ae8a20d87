/*
 * FP64 CPU oracle of the ANI-style neural-network-potential energy and forces
 * (Deep-HP paper, arXiv 2207.14276, section "Neural Network Potentials" and
 * "ANI models").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg load it.  It
 * shares no code, header or constant with the GPU library: every parameter
 * (cutoffs, shifts, widths, weights) arrives as an argument.
 *
 * What it computes, in the paper's order:
 *   1. neighbours of each centre atom, by brute force over every atom and
 *      every periodic image within the cutoff ("pair list of indices",
 *      section "Massive Parallelism within Tinker-HP");
 *   2. the cosine cutoff f_c (equation for f_c in "ANI models");
 *   3. the radial symmetry functions (radial equation in "ANI models"),
 *      one block of shifts per neighbour species;
 *   4. the ANI angular symmetry functions (angular equation in "ANI models"),
 *      one block per unordered species pair;
 *   5. one feed-forward network per element (section "Neural Network
 *      Potentials"), averaged over an ensemble of networks;
 *   6. the total energy as the sum of atomic energies (energy-decomposition
 *      equation);
 *   7. forces and virial as the exact analytic gradient of that total.
 * A second descriptor kind replaces steps 2-4 with the DeepPot local-frame
 * environment of section "DeePMD Models" (species-sorted neighbours, local
 * axes, {1/R, x/R, y/R, z/R}); steps 1 and 5-7 are shared.
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes): the radial term carries a 0.25 prefactor; the angular sum runs over
 * unordered neighbour pairs j < k, each counted once; theta enters through
 * cos(theta - theta_s) = cos(theta)cos(theta_s) + sin(theta)sin(theta_s) with
 * sin(theta) taken from |d_j x d_k|; the sin-derivative is taken as zero for
 * exactly collinear triplets; features are laid out as radial[species][shift]
 * then angular[pair][radial shift][angle shift] (angle shift fastest); the
 * network output is the atomic energy in kcal/mol with no self-energy; the
 * hidden activation is CELU; every periodic image inside the cutoff counts as
 * a distinct neighbour (self-images included).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int n_species;
  double rc_rad, eta_rad;
  int n_shf_rad;
  const double *shf_rad;
  double rc_ang, eta_ang, zeta;
  int n_shf_ang;
  const double *shf_ang;
  int n_shf_z;
  const double *shf_z;
  double radial_scale;
} orc_aev_params;

/* DeepPot-style descriptor (section "DeePMD Models"): neighbours inside rc,
 * grouped by species and ordered nearest first, at most sel[s] of species s
 * kept; each kept neighbour contributes {1/R, x/R, y/R, z/R} in the centre's
 * local frame. */
typedef struct {
  int n_species;
  double rc;
  const int *sel;        /* [n_species] neighbours kept per species */
} orc_dp_params;

enum { ORC_ANI = 0, ORC_DP = 1 };

typedef struct {
  orc_aev_params aev;    /* descriptor of kind ORC_ANI */
  int n_ensemble;
  const int *n_layers;   /* [n_species] linear layers per network */
  const int *widths;     /* per species: n_layers + 1 widths, concatenated */
  const double *weights; /* (member, species, layer): W[out][in] then b[out] */
  double celu_alpha;
  int kind;              /* ORC_ANI or ORC_DP */
  orc_dp_params dp;      /* descriptor of kind ORC_DP */
} orc_model;

typedef struct {
  int j;          /* neighbour atom index */
  int n[3];       /* lattice image */
  double d[3];    /* r_j + n*L - r_i */
  double r;       /* |d| */
} orc_nbr;

/* ---------------------------------------------------------------- helpers */

static int orc_omp_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int orc_threads(void) { return orc_omp_threads(); }

/* Threads used by later calls (n >= 1); returns the previous count.  Only
 * the timing of the baseline depends on it, never a result. */
int orc_set_threads(int n) {
  const int prev = orc_omp_threads();
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
  return prev;
}

int orc_aev_dim(const orc_aev_params *p) {
  int s = p->n_species;
  return s * p->n_shf_rad + (s * (s + 1) / 2) * p->n_shf_ang * p->n_shf_z;
}

/* Cosine cutoff: 0.5 cos(pi R / Rc) + 0.5 inside the cutoff, else 0. */
static double fc(double r, double rc) {
  return r < rc ? 0.5 * cos(M_PI * r / rc) + 0.5 : 0.0;
}

static double dfc(double r, double rc) {
  return r < rc ? -0.5 * M_PI / rc * sin(M_PI * r / rc) : 0.0;
}

/* Index of the unordered species pair (a, b), a <= b, in row-major upper
 * triangle order: (0,0), (0,1), ..., (0,S-1), (1,1), ... */
static int pair_index(int a, int b, int S) {
  if (a > b) { int t = a; a = b; b = t; }
  return a * S - a * (a - 1) / 2 + (b - a);
}

/* --------------------------------------------------------- 1. neighbours */

/* Every (j, image) with |r_j + n L - r_i| < rc, excluding (i, 0).  Brute
 * force over all atoms; along a periodic axis, all images within
 * ceil(rc / L) + 1 of the nearest one are scanned, which covers every image
 * inside the cutoff whatever the coordinates.  Returns the count; writes at
 * most `cap` entries. */
static int centre_neighbours(int n, const double *xyz, const double *box, int i,
                             double rc, orc_nbr *out, int cap) {
  int cnt = 0;
  int K[3], per[3];
  for (int a = 0; a < 3; ++a) {
    per[a] = box[a] > 0.0;
    K[a] = per[a] ? (int)ceil(rc / box[a]) + 1 : 0;
  }
  const double rc2 = rc * rc;
  for (int j = 0; j < n; ++j) {
    double base[3];
    int n0[3];
    for (int a = 0; a < 3; ++a) {
      base[a] = xyz[3 * j + a] - xyz[3 * i + a];
      n0[a] = per[a] ? -(int)lround(base[a] / box[a]) : 0;
    }
    for (int nx = n0[0] - K[0]; nx <= n0[0] + K[0]; ++nx)
      for (int ny = n0[1] - K[1]; ny <= n0[1] + K[1]; ++ny)
        for (int nz = n0[2] - K[2]; nz <= n0[2] + K[2]; ++nz) {
          if (j == i && nx == 0 && ny == 0 && nz == 0) continue;
          double d[3] = {base[0] + nx * box[0], base[1] + ny * box[1],
                         base[2] + nz * box[2]};
          double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          if (r2 < rc2) {
            if (cnt < cap) {
              orc_nbr *e = &out[cnt];
              e->j = j;
              e->n[0] = nx; e->n[1] = ny; e->n[2] = nz;
              e->d[0] = d[0]; e->d[1] = d[1]; e->d[2] = d[2];
              e->r = sqrt(r2);
            }
            ++cnt;
          }
        }
  }
  return cnt;
}

/* Neighbour list of a single centre, for tests: j and image triples. */
int orc_neighbours(int n, const double *xyz, const double *box, double rc,
                   int i, int cap, int *js, int *images) {
  orc_nbr *buf = (orc_nbr *)malloc(sizeof(orc_nbr) * (cap > 0 ? cap : 1));
  int cnt = centre_neighbours(n, xyz, box, i, rc, buf, cap);
  int w = cnt < cap ? cnt : cap;
  for (int e = 0; e < w; ++e) {
    js[e] = buf[e].j;
    for (int a = 0; a < 3; ++a) images[3 * e + a] = buf[e].n[a];
  }
  free(buf);
  return cnt;
}

/* Neighbours of centre i with a list that grows until it holds them all. */
static orc_nbr *neighbours_alloc(int n, const double *xyz, const double *box,
                                 int i, double rc, int *count) {
  int cap = 256;
  for (;;) {
    orc_nbr *buf = (orc_nbr *)malloc(sizeof(orc_nbr) * cap);
    int cnt = centre_neighbours(n, xyz, box, i, rc, buf, cap);
    if (cnt <= cap) { *count = cnt; return buf; }
    free(buf);
    cap = cnt;
  }
}

/* ------------------------------------------------- 2-4. the AEV of a centre */

static void centre_aev(const orc_nbr *nb, int nn, const int *species,
                       const orc_aev_params *p, double *G) {
  const int S = p->n_species;
  const int D = orc_aev_dim(p);
  const int rad_len = S * p->n_shf_rad;
  const int blk = p->n_shf_ang * p->n_shf_z;
  memset(G, 0, sizeof(double) * D);

  /* radial: sum over neighbours j of 0.25 exp(-eta (R - Rs)^2) fc(R) */
  for (int e = 0; e < nn; ++e) {
    double R = nb[e].r;
    if (!(R < p->rc_rad)) continue;
    int sj = species[nb[e].j];
    for (int m = 0; m < p->n_shf_rad; ++m) {
      double t = R - p->shf_rad[m];
      G[sj * p->n_shf_rad + m] +=
          p->radial_scale * exp(-p->eta_rad * t * t) * fc(R, p->rc_rad);
    }
  }

  /* angular: unordered pairs {j, k} of neighbours inside the angular cutoff */
  const double pref = pow(2.0, 1.0 - p->zeta);
  for (int e1 = 0; e1 < nn; ++e1) {
    if (!(nb[e1].r < p->rc_ang)) continue;
    for (int e2 = e1 + 1; e2 < nn; ++e2) {
      if (!(nb[e2].r < p->rc_ang)) continue;
      const double *dj = nb[e1].d, *dk = nb[e2].d;
      double Rj = nb[e1].r, Rk = nb[e2].r;
      double dot = dj[0] * dk[0] + dj[1] * dk[1] + dj[2] * dk[2];
      double cx = dj[1] * dk[2] - dj[2] * dk[1];
      double cy = dj[2] * dk[0] - dj[0] * dk[2];
      double cz = dj[0] * dk[1] - dj[1] * dk[0];
      double cr = sqrt(cx * cx + cy * cy + cz * cz);
      double cos_t = dot / (Rj * Rk);
      double sin_t = cr / (Rj * Rk);
      double fcc = fc(Rj, p->rc_ang) * fc(Rk, p->rc_ang);
      double Rbar = 0.5 * (Rj + Rk);
      int base = rad_len + blk * pair_index(species[nb[e1].j], species[nb[e2].j], S);
      for (int r = 0; r < p->n_shf_ang; ++r) {
        double u = Rbar - p->shf_ang[r];
        double f2 = exp(-p->eta_ang * u * u);
        for (int a = 0; a < p->n_shf_z; ++a) {
          double c = cos_t * cos(p->shf_z[a]) + sin_t * sin(p->shf_z[a]);
          double one_c = 1.0 + c;
          if (one_c < 0.0) one_c = 0.0;
          double f1 = pref * pow(one_c, p->zeta);
          G[base + r * p->n_shf_z + a] += f1 * f2 * fcc;
        }
      }
    }
  }
}

int orc_aev(int n, const double *xyz, const int *species, const double *box,
            const orc_aev_params *p, double *aev) {
  const int D = orc_aev_dim(p);
  int bad = 0;
  #pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
  for (int i = 0; i < n; ++i) {
    int nn;
    orc_nbr *nb = neighbours_alloc(n, xyz, box, i, p->rc_rad, &nn);
    if (!nb) { bad |= 1; continue; }
    centre_aev(nb, nn, species, p, aev + (size_t)i * D);
    free(nb);
  }
  return bad ? -1 : 0;
}

/* ------------------------------------- 2'-4'. the DeepPot descriptor of a centre
 *
 * Section "DeePMD Models".  Readings where the paper is silent:
 *   - "sorted by species and inverse distance": species ascending, then
 *     inverse distance descending (nearest first); exact distance ties are
 *     broken by neighbour index, then by lattice image (x, y, z) ascending;
 *     the distance is compared through R^2 = (dx dx + dy dy) + dz dz in
 *     float64, d = (r_j - r_i) + n L;
 *   - at most sel[s] neighbours of species s are kept (the nearest ones);
 *     their features fill slots sel[0] + ... + sel[s-1] + rank, slots past
 *     the last neighbour of a species stay zero;
 *   - the local frame: e_x along the nearest neighbour a, e_y along the
 *     part of the second-nearest neighbour b orthogonal to e_x, and
 *     e_z = e_x x e_y; with a single neighbour, or when b is collinear with
 *     a (|u|^2 <= 1e-12 |d_b|^2), e_y = e_z = 0;
 *   - no smoothing function at the cutoff (the paper gives none), so the
 *     energy is continuous only away from the cutoff and from changes of
 *     the neighbour order. */

typedef struct {
  const orc_nbr *e;
  double r2;
  int s;
} dp_item;

typedef struct {
  int a, b;                    /* nb indices of the axis neighbours, or -1 */
  double ex[3], ey[3], ez[3];  /* local axes (e_y = e_z = 0 when undefined) */
  double ra;                   /* |d_a| */
  double nu;                   /* |u|, u = d_b - (d_b . e_x) e_x; 0: e_y undefined */
} dp_frame;

int orc_dp_dim(const orc_dp_params *p) {
  int k = 0;
  for (int s = 0; s < p->n_species; ++s) k += p->sel[s];
  return 4 * k;
}

static double dp_r2(const orc_nbr *e) {
  return e->d[0] * e->d[0] + e->d[1] * e->d[1] + e->d[2] * e->d[2];
}

/* distance order: R^2, then neighbour index, then image */
static int dp_cmp_dist(const dp_item *a, const dp_item *b) {
  if (a->r2 != b->r2) return a->r2 < b->r2 ? -1 : 1;
  if (a->e->j != b->e->j) return a->e->j < b->e->j ? -1 : 1;
  for (int k = 0; k < 3; ++k)
    if (a->e->n[k] != b->e->n[k]) return a->e->n[k] < b->e->n[k] ? -1 : 1;
  return 0;
}

static int dp_cmp_species(const void *pa, const void *pb) {
  const dp_item *a = (const dp_item *)pa, *b = (const dp_item *)pb;
  if (a->s != b->s) return a->s < b->s ? -1 : 1;
  return dp_cmp_dist(a, b);
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

static void dp_axes(const orc_nbr *nb, dp_frame *f) {
  memset(f->ex, 0, sizeof f->ex);
  memset(f->ey, 0, sizeof f->ey);
  memset(f->ez, 0, sizeof f->ez);
  f->ra = 0.0;
  f->nu = 0.0;
  if (f->a < 0) return;
  const double *da = nb[f->a].d;
  f->ra = nb[f->a].r;
  for (int k = 0; k < 3; ++k) f->ex[k] = da[k] / f->ra;
  if (f->b < 0) return;
  const double *db = nb[f->b].d;
  const double t = dot3(db, f->ex);
  double u[3];
  for (int k = 0; k < 3; ++k) u[k] = db[k] - t * f->ex[k];
  const double uu = dot3(u, u);
  if (!(uu > 1e-12 * dot3(db, db))) return;   /* collinear: e_y, e_z undefined */
  f->nu = sqrt(uu);
  for (int k = 0; k < 3; ++k) f->ey[k] = u[k] / f->nu;
  cross3(f->ex, f->ey, f->ez);
}

/* Descriptor G[4 * sum(sel)] of one centre; slot[e] receives the slot of
 * neighbour entry e (-1: not kept) and *fr the local frame. */
static void centre_dp(const orc_nbr *nb, int nn, const int *species, const orc_dp_params *p,
                      double *G, int *slot, dp_frame *fr) {
  memset(G, 0, sizeof(double) * orc_dp_dim(p));
  dp_item *it = (dp_item *)malloc(sizeof(dp_item) * (nn > 0 ? nn : 1));
  for (int e = 0; e < nn; ++e) {
    it[e].e = &nb[e];
    it[e].r2 = dp_r2(&nb[e]);
    it[e].s = species[nb[e].j];
    slot[e] = -1;
  }
  /* the frame: the two nearest neighbours in distance order */
  fr->a = fr->b = -1;
  for (int e = 0; e < nn; ++e) {
    if (fr->a < 0 || dp_cmp_dist(&it[e], &it[fr->a]) < 0) {
      fr->b = fr->a;
      fr->a = e;
    } else if (fr->b < 0 || dp_cmp_dist(&it[e], &it[fr->b]) < 0) {
      fr->b = e;
    }
  }
  dp_axes(nb, fr);
  /* species blocks, nearest first; the first sel[s] of species s are kept */
  qsort(it, (size_t)nn, sizeof(dp_item), dp_cmp_species);
  int first_slot = 0, prev_s = -1, rank = 0;
  for (int k = 0; k < nn; ++k) {
    const int s = it[k].s;
    if (s != prev_s) {
      first_slot = 0;
      for (int q = 0; q < s; ++q) first_slot += p->sel[q];
      rank = 0;
      prev_s = s;
    }
    if (rank < p->sel[s]) {
      const int e = (int)(it[k].e - nb);
      const double *d = nb[e].d, R = nb[e].r;
      const int q = first_slot + rank;
      slot[e] = q;
      G[4 * q + 0] = 1.0 / R;
      G[4 * q + 1] = dot3(d, fr->ex) / R;
      G[4 * q + 2] = dot3(d, fr->ey) / R;
      G[4 * q + 3] = dot3(d, fr->ez) / R;
    }
    ++rank;
  }
  free(it);
}

/* Given g = dE/dG of the centre, writes gd[e] = dE/dd_e for each neighbour:
 * the explicit dependence of a kept neighbour's four features on its own
 * vector, plus the dependence of every x, y, z on the frame, which reaches
 * the axis neighbours a and b (e_x = d_a / |d_a|, e_y = u / |u| with
 * u = (I - e_x e_x^T) d_b, e_z = e_x x e_y). */
static void centre_dp_grad(const orc_nbr *nb, int nn, const int *slot, const dp_frame *fr,
                           const double *g, double (*gd)[3]) {
  double A[3][3] = {{0}};  /* A[c] = dE/de_c with the other axes fixed */
  for (int e = 0; e < nn; ++e) {
    gd[e][0] = gd[e][1] = gd[e][2] = 0.0;
    if (slot[e] < 0) continue;
    const double *gs = g + 4 * slot[e], *d = nb[e].d, R = nb[e].r;
    const double c[3] = {dot3(d, fr->ex), dot3(d, fr->ey), dot3(d, fr->ez)};
    /* d(1/R)/dd = -d/R^3; d(c/R)/dd = e_c/R - c d/R^3 */
    const double s = gs[0] + gs[1] * c[0] + gs[2] * c[1] + gs[3] * c[2];
    for (int k = 0; k < 3; ++k) {
      gd[e][k] += -s * d[k] / (R * R * R) + (gs[1] * fr->ex[k] + gs[2] * fr->ey[k] + gs[3] * fr->ez[k]) / R;
      for (int q = 0; q < 3; ++q) A[q][k] += gs[1 + q] * d[k] / R;
    }
  }
  if (fr->a < 0) return;
  double Bx[3] = {A[0][0], A[0][1], A[0][2]};
  if (fr->nu > 0.0) {
    double By[3] = {A[1][0], A[1][1], A[1][2]}, t[3];
    cross3(fr->ey, A[2], t);               /* e_z = e_x x e_y, through e_x */
    for (int k = 0; k < 3; ++k) Bx[k] += t[k];
    cross3(A[2], fr->ex, t);               /* ... and through e_y */
    for (int k = 0; k < 3; ++k) By[k] += t[k];
    const double *db = nb[fr->b].d;
    const double byy = dot3(By, fr->ey);
    double C[3];                            /* dE/du */
    for (int k = 0; k < 3; ++k) C[k] = (By[k] - byy * fr->ey[k]) / fr->nu;
    const double cx = dot3(C, fr->ex), bx = dot3(db, fr->ex);
    for (int k = 0; k < 3; ++k) {
      gd[fr->b][k] += C[k] - cx * fr->ex[k];
      Bx[k] += -cx * db[k] - bx * C[k];     /* u depends on e_x too */
    }
  }
  const double bxx = dot3(Bx, fr->ex);
  for (int k = 0; k < 3; ++k) gd[fr->a][k] += (Bx[k] - bxx * fr->ex[k]) / fr->ra;
}

int orc_dp_descriptor(int n, const double *xyz, const int *species, const double *box,
                      const orc_dp_params *p, double *out) {
  const int D = orc_dp_dim(p);
  int bad = 0;
  #pragma omp parallel for schedule(dynamic, 4) reduction(| : bad)
  for (int i = 0; i < n; ++i) {
    int nn;
    orc_nbr *nb = neighbours_alloc(n, xyz, box, i, p->rc, &nn);
    int *slot = (int *)malloc(sizeof(int) * (nn > 0 ? nn : 1));
    dp_frame fr;
    centre_dp(nb, nn, species, p, out + (size_t)i * D, slot, &fr);
    free(slot);
    free(nb);
  }
  return bad ? -1 : 0;
}

/* ----------------------------------------------------- 5. element networks */

/* Descriptor of either kind: species count, length and cutoff. */
static int model_species(const orc_model *m) { return m->kind == ORC_DP ? m->dp.n_species : m->aev.n_species; }
static int model_dim(const orc_model *m) { return m->kind == ORC_DP ? orc_dp_dim(&m->dp) : orc_aev_dim(&m->aev); }
static double model_rc(const orc_model *m) { return m->kind == ORC_DP ? m->dp.rc : m->aev.rc_rad; }

static double celu(double z, double alpha) {
  return z > 0.0 ? z : alpha * (exp(z / alpha) - 1.0);
}

static double dcelu(double z, double alpha) {
  return z > 0.0 ? 1.0 : exp(z / alpha);
}

/* Offset of the weights of (member, species) in the flat weight array. */
static size_t net_offset(const orc_model *m, int member, int species) {
  size_t per_member = 0, off_s = 0;
  int wo = 0;
  for (int s = 0; s < model_species(m); ++s) {
    size_t cnt = 0;
    for (int l = 0; l < m->n_layers[s]; ++l)
      cnt += (size_t)m->widths[wo + l] * m->widths[wo + l + 1] + m->widths[wo + l + 1];
    if (s < species) off_s += cnt;
    per_member += cnt;
    wo += m->n_layers[s] + 1;
  }
  return per_member * member + off_s;
}

static const int *net_widths(const orc_model *m, int species) {
  int wo = 0;
  for (int s = 0; s < species; ++s) wo += m->n_layers[s] + 1;
  return m->widths + wo;
}

/* Energy of one network on one AEV; if dEdG is given, adds scale * dE/dG. */
static double net_energy(const orc_model *m, int member, int species,
                         const double *G, double *dEdG, double scale) {
  const int L = m->n_layers[species];
  const int *w = net_widths(m, species);
  const double *W = m->weights + net_offset(m, member, species);
  int maxw = 0;
  for (int l = 0; l <= L; ++l) if (w[l] > maxw) maxw = w[l];
  /* z[l] keeps each layer's pre-activation for the backward pass */
  double *z = (double *)malloc(sizeof(double) * (size_t)maxw * (L + 1));
  double *h = (double *)malloc(sizeof(double) * maxw);
  double *g = (double *)malloc(sizeof(double) * maxw);
  double *g2 = (double *)malloc(sizeof(double) * maxw);
  const double **Wl = (const double **)malloc(sizeof(double *) * L);
  memcpy(h, G, sizeof(double) * w[0]);
  const double *p = W;
  for (int l = 0; l < L; ++l) {
    int n_in = w[l], n_out = w[l + 1];
    const double *Wm = p, *b = p + (size_t)n_out * n_in;
    Wl[l] = p;
    p += (size_t)n_out * n_in + n_out;
    double *zl = z + (size_t)l * maxw;
    for (int o = 0; o < n_out; ++o) {
      double acc = b[o];
      for (int k = 0; k < n_in; ++k) acc += Wm[(size_t)o * n_in + k] * h[k];
      zl[o] = acc;
    }
    if (l < L - 1)
      for (int o = 0; o < n_out; ++o) h[o] = celu(zl[o], m->celu_alpha);
  }
  double E = z[(size_t)(L - 1) * maxw];
  if (dEdG) {
    /* backward: g holds dE/dz of the current layer's output */
    g[0] = 1.0;
    for (int l = L - 1; l >= 0; --l) {
      int n_in = w[l], n_out = w[l + 1];
      const double *Wm = Wl[l];
      for (int k = 0; k < n_in; ++k) {
        double acc = 0.0;
        for (int o = 0; o < n_out; ++o) acc += Wm[(size_t)o * n_in + k] * g[o];
        g2[k] = acc;
      }
      if (l > 0) {
        const double *zp = z + (size_t)(l - 1) * maxw;
        for (int k = 0; k < n_in; ++k) g[k] = g2[k] * dcelu(zp[k], m->celu_alpha);
      } else {
        for (int k = 0; k < n_in; ++k) dEdG[k] += scale * g2[k];
      }
    }
  }
  free(z); free(h); free(g); free(g2); free((void *)Wl);
  return E;
}

/* Ensemble-averaged atomic energy and (optionally) its AEV gradient. */
static double atom_energy(const orc_model *m, int species, const double *G, double *dEdG) {
  const int D = model_dim(m);
  if (dEdG) memset(dEdG, 0, sizeof(double) * D);
  double E = 0.0;
  const double inv = 1.0 / m->n_ensemble;
  for (int mb = 0; mb < m->n_ensemble; ++mb)
    E += inv * net_energy(m, mb, species, G, dEdG, inv);
  return E;
}

/* Exported for tests: one network (member, species) on one AEV. */
double orc_net_energy(const orc_model *m, int member, int species,
                      const double *G, double *dEdG) {
  if (dEdG) memset(dEdG, 0, sizeof(double) * model_dim(m));
  return net_energy(m, member, species, G, dEdG, 1.0);
}

/* ------------------------------------ 7. gradient of a centre's AEV terms */

/* Given g = dE/dG of centre i, writes gd[e] = dE/dd_e for each neighbour. */
static void centre_aev_grad(const orc_nbr *nb, int nn, const int *species,
                            const orc_aev_params *p, const double *g,
                            double (*gd)[3]) {
  const int S = p->n_species;
  const int rad_len = S * p->n_shf_rad;
  const int blk = p->n_shf_ang * p->n_shf_z;
  for (int e = 0; e < nn; ++e) gd[e][0] = gd[e][1] = gd[e][2] = 0.0;

  for (int e = 0; e < nn; ++e) {
    double R = nb[e].r;
    if (!(R < p->rc_rad)) continue;
    int sj = species[nb[e].j];
    double f = fc(R, p->rc_rad), df = dfc(R, p->rc_rad);
    double dEdR = 0.0;
    for (int m = 0; m < p->n_shf_rad; ++m) {
      double t = R - p->shf_rad[m];
      double ex = exp(-p->eta_rad * t * t);
      dEdR += g[sj * p->n_shf_rad + m] * p->radial_scale *
              (ex * (-2.0 * p->eta_rad * t) * f + ex * df);
    }
    for (int a = 0; a < 3; ++a) gd[e][a] += dEdR * nb[e].d[a] / R;
  }

  const double pref = pow(2.0, 1.0 - p->zeta);
  for (int e1 = 0; e1 < nn; ++e1) {
    if (!(nb[e1].r < p->rc_ang)) continue;
    for (int e2 = e1 + 1; e2 < nn; ++e2) {
      if (!(nb[e2].r < p->rc_ang)) continue;
      const double *dj = nb[e1].d, *dk = nb[e2].d;
      double Rj = nb[e1].r, Rk = nb[e2].r;
      double dot = dj[0] * dk[0] + dj[1] * dk[1] + dj[2] * dk[2];
      double cx = dj[1] * dk[2] - dj[2] * dk[1];
      double cy = dj[2] * dk[0] - dj[0] * dk[2];
      double cz = dj[0] * dk[1] - dj[1] * dk[0];
      double cr = sqrt(cx * cx + cy * cy + cz * cz);
      double RR = Rj * Rk;
      double cos_t = dot / RR, sin_t = cr / RR;
      double fj = fc(Rj, p->rc_ang), fk = fc(Rk, p->rc_ang);
      double dfj = dfc(Rj, p->rc_ang), dfk = dfc(Rk, p->rc_ang);
      double Rbar = 0.5 * (Rj + Rk);
      int base = rad_len + blk * pair_index(species[nb[e1].j], species[nb[e2].j], S);
      double dVdcos = 0.0, dVdsin = 0.0, dVdRj = 0.0, dVdRk = 0.0;
      for (int r = 0; r < p->n_shf_ang; ++r) {
        double u = Rbar - p->shf_ang[r];
        double f2 = exp(-p->eta_ang * u * u);
        double df2 = -2.0 * p->eta_ang * u * f2; /* d f2 / d Rbar */
        for (int a = 0; a < p->n_shf_z; ++a) {
          double w = g[base + r * p->n_shf_z + a];
          double cs = cos(p->shf_z[a]), sn = sin(p->shf_z[a]);
          double one_c = 1.0 + cos_t * cs + sin_t * sn;
          if (one_c < 0.0) one_c = 0.0;
          double f1 = pref * pow(one_c, p->zeta);
          double df1 = pref * p->zeta * pow(one_c, p->zeta - 1.0);
          dVdcos += w * df1 * cs * f2 * fj * fk;
          dVdsin += w * df1 * sn * f2 * fj * fk;
          dVdRj += w * f1 * (0.5 * df2 * fj * fk + f2 * dfj * fk);
          dVdRk += w * f1 * (0.5 * df2 * fj * fk + f2 * fj * dfk);
        }
      }
      /* chain rule through cos(theta), sin(theta), R_j and R_k */
      double inv_cr = cr > 1e-12 * RR ? 1.0 / cr : 0.0;
      for (int a = 0; a < 3; ++a) {
        double dcos_j = dk[a] / RR - cos_t * dj[a] / (Rj * Rj);
        double dcos_k = dj[a] / RR - cos_t * dk[a] / (Rk * Rk);
        double dsin_j = (Rk * Rk * dj[a] - dot * dk[a]) * inv_cr / RR - sin_t * dj[a] / (Rj * Rj);
        double dsin_k = (Rj * Rj * dk[a] - dot * dj[a]) * inv_cr / RR - sin_t * dk[a] / (Rk * Rk);
        if (inv_cr == 0.0) { dsin_j = 0.0; dsin_k = 0.0; }
        gd[e1][a] += dVdcos * dcos_j + dVdsin * dsin_j + dVdRj * dj[a] / Rj;
        gd[e2][a] += dVdcos * dcos_k + dVdsin * dsin_k + dVdRk * dk[a] / Rk;
      }
    }
  }
}

/* One centre's descriptor and its gradient, for either kind.  slot and fr
 * carry the DeepPot slot assignment and frame from the forward to the
 * gradient (unused for the AEV). */
static void centre_desc(const orc_model *m, const orc_nbr *nb, int nn, const int *species,
                        double *G, int *slot, dp_frame *fr) {
  if (m->kind == ORC_DP) centre_dp(nb, nn, species, &m->dp, G, slot, fr);
  else centre_aev(nb, nn, species, &m->aev, G);
}

static void centre_desc_grad(const orc_model *m, const orc_nbr *nb, int nn, const int *species,
                             const int *slot, const dp_frame *fr, const double *g, double (*gd)[3]) {
  if (m->kind == ORC_DP) centre_dp_grad(nb, nn, slot, fr, g, gd);
  else centre_aev_grad(nb, nn, species, &m->aev, g, gd);
}

/* -------------------------------------- 6-7. energy, forces, virial of a system */

/* e_atom[n]: ensemble-mean atomic energies; forces[n][3] (nullable);
 * virial[9] (nullable) = -sum over neighbour terms of d (x) dE/dd, which for
 * a non-periodic system equals sum_i r_i (x) F_i.  Returns the total energy
 * through *energy (nullable). */
int orc_energy_forces(int n, const double *xyz, const int *species,
                      const double *box, const orc_model *m, double *e_atom,
                      double *energy, double *forces, double *virial) {
  const int D = model_dim(m);
  const int T = orc_omp_threads();
  const int need_grad = forces != NULL || virial != NULL;
  double *Fth = need_grad ? (double *)calloc((size_t)T * n * 3, sizeof(double)) : NULL;
  double *Wth = need_grad ? (double *)calloc((size_t)T * 9, sizeof(double)) : NULL;
  int bad = 0;
  #pragma omp parallel reduction(| : bad)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    double *G = (double *)malloc(sizeof(double) * D);
    double *g = need_grad ? (double *)malloc(sizeof(double) * D) : NULL;
    #pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      int nn;
      orc_nbr *nb = neighbours_alloc(n, xyz, box, i, model_rc(m), &nn);
      int *slot = (int *)malloc(sizeof(int) * (nn > 0 ? nn : 1));
      dp_frame fr;
      centre_desc(m, nb, nn, species, G, slot, &fr);
      e_atom[i] = atom_energy(m, species[i], G, g);
      if (need_grad) {
        double (*gd)[3] = (double (*)[3])malloc(sizeof(double) * 3 * (nn > 0 ? nn : 1));
        centre_desc_grad(m, nb, nn, species, slot, &fr, g, gd);
        double *F = Fth + (size_t)t * n * 3;
        double *W = Wth + (size_t)t * 9;
        for (int e = 0; e < nn; ++e) {
          for (int a = 0; a < 3; ++a) {
            F[3 * i + a] += gd[e][a];
            F[3 * nb[e].j + a] -= gd[e][a];
            for (int b = 0; b < 3; ++b) W[3 * a + b] -= nb[e].d[a] * gd[e][b];
          }
        }
        free(gd);
      }
      free(slot);
      free(nb);
    }
    free(G);
    free(g);
  }
  if (energy) {
    double E = 0.0;
    for (int i = 0; i < n; ++i) E += e_atom[i];
    *energy = E;
  }
  if (forces) {
    memset(forces, 0, sizeof(double) * 3 * n);
    for (int t = 0; t < T; ++t)
      for (size_t k = 0; k < (size_t)3 * n; ++k) forces[k] += Fth[(size_t)t * n * 3 + k];
  }
  if (virial) {
    memset(virial, 0, sizeof(double) * 9);
    for (int t = 0; t < T; ++t)
      for (int k = 0; k < 9; ++k) virial[k] += Wth[t * 9 + k];
  }
  free(Fth);
  free(Wth);
  return bad ? -1 : 0;
}

/* Atomic energies and forces of selected target atoms only.
 *
 * The force on atom t collects the derivative of every atomic energy whose
 * environment contains t: its own, and that of every centre c having some
 * image of t inside the descriptor's cutoff.  Each such centre is evaluated from
 * scratch, so the cost is independent of system size apart from the
 * brute-force neighbour scans.  e_t[nt], f_t[nt][3]. */
int orc_sampled(int n, const double *xyz, const int *species, const double *box,
                const orc_model *m, int nt, const int *targets, double *e_t,
                double *f_t) {
  const int D = model_dim(m);
  const double rc = model_rc(m);
  int bad = 0;
  #pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int q = 0; q < nt; ++q) {
    const int t = targets[q];
    double *G = (double *)malloc(sizeof(double) * D);
    double *g = (double *)malloc(sizeof(double) * D);
    int nt_nb;
    orc_nbr *tn = neighbours_alloc(n, xyz, box, t, rc, &nt_nb);
    /* unique centre list: t first, then every distinct neighbour index */
    int *centres = (int *)malloc(sizeof(int) * (nt_nb + 1));
    int nc = 0;
    centres[nc++] = t;
    for (int e = 0; e < nt_nb; ++e) {
      int j = tn[e].j, seen = 0;
      for (int k = 0; k < nc; ++k) if (centres[k] == j) { seen = 1; break; }
      if (!seen) centres[nc++] = j;
    }
    double F[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < nc; ++k) {
      int c = centres[k], nn;
      orc_nbr *nb = neighbours_alloc(n, xyz, box, c, rc, &nn);
      int *slot = (int *)malloc(sizeof(int) * (nn > 0 ? nn : 1));
      dp_frame fr;
      centre_desc(m, nb, nn, species, G, slot, &fr);
      double E = atom_energy(m, species[c], G, g);
      if (c == t) e_t[q] = E;
      double (*gd)[3] = (double (*)[3])malloc(sizeof(double) * 3 * (nn > 0 ? nn : 1));
      centre_desc_grad(m, nb, nn, species, slot, &fr, g, gd);
      for (int e = 0; e < nn; ++e) {
        for (int a = 0; a < 3; ++a) {
          if (c == t) F[a] += gd[e][a];
          if (nb[e].j == t) F[a] -= gd[e][a];
        }
      }
      free(gd);
      free(slot);
      free(nb);
    }
    for (int a = 0; a < 3; ++a) f_t[3 * q + a] = F[a];
    free(centres);
    free(tn);
    free(G);
    free(g);
  }
  return bad ? -1 : 0;
}
