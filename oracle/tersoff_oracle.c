/*
 * Tersoff potential: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header or table with the GPU
 * path.
 *
 * What it computes (the paper, Section III, Eqs. ters-1..ters-3, written out
 * with the standard Tersoff forms of f_C, f_R, f_A and g):
 *
 *   E   = 1/2 sum_i sum_{j != i} f_C(r_ij) [ f_R(r_ij) + b_ij f_A(r_ij) ]
 *   b_ij = (1 + (beta zeta_ij)^n)^(-1/(2n))
 *   zeta_ij = sum_{k != i,j} f_C(r_ik) g(theta_ijk) exp(lambda3^m (r_ij - r_ik)^m)
 *   F_a = -dE/dx_a,  W_ab = sum over terms of (x_a - x_i)_alpha f_a,beta
 *
 * The loop structure is the paper's Algorithm 2 (the plain triple loop): for
 * each i, for each j, a first k loop accumulates zeta_ij, then the pair term
 * and its forces are added, then a second k loop scatters dV/dzeta * dzeta/dx
 * onto i, j and k.  No derivative is stored between the two k loops.
 *
 * The factor 1/2 is Tersoff's own (the paper's Eq. ters-1 sums ordered pairs
 * without it); with it, diamond Si comes out at the published -4.63 eV/atom.
 *
 * Parameter table: P[ti][tj][tk][14] with fields, in order,
 *   m, gamma, lambda3, c, d, h(=cos theta0), n, beta, lambda2, B, R, D, lambda1, A
 * Pair quantities of (i,j) are read from P[ti][tj][tj]; the three-body
 * quantities of (i,j,k), and the cutoff of the (i,k) distance, from P[ti][tj][tk].
 *
 * Units: Angstrom, eV.  Box: orthorhombic, periodic in all three axes.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum {
  F_M = 0, F_GAMMA, F_LAM3, F_C, F_D, F_H, F_N, F_BETA, F_LAM2, F_B,
  F_R, F_DC, F_LAM1, F_A, NFIELD
};

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_BOX 2
#define ORC_ERR_OVERFLOW 3

static const double *prow(const double *table, int nt, int a, int b, int c) {
  return table + (((size_t)a * nt + b) * nt + c) * NFIELD;
}

/* Cutoff function f_C and its derivative (Tersoff 1988 form, LAMMPS R/D
 * parameterisation: smooth sine switch from 1 at R-D to 0 at R+D). */
static double fcut(double r, const double *p) {
  double R = p[F_R], D = p[F_DC];
  if (r < R - D) return 1.0;
  if (r > R + D) return 0.0;
  return 0.5 - 0.5 * sin(M_PI * (r - R) / (2.0 * D));
}
static double fcut_d(double r, const double *p) {
  double R = p[F_R], D = p[F_DC];
  if (r < R - D || r > R + D) return 0.0;
  return -(M_PI / (4.0 * D)) * cos(M_PI * (r - R) / (2.0 * D));
}

/* Angular function g(cos theta) = gamma (1 + c^2/d^2 - c^2/(d^2 + (cos - h)^2)).
 * Evaluated in the algebraically identical cancellation-free form
 * gamma (1 + c^2 t^2 / (d^2 (d^2 + t^2))), t = cos - h. */
static double gang(double cs, const double *p) {
  double c2 = p[F_C] * p[F_C], d2 = p[F_D] * p[F_D], t = cs - p[F_H];
  return p[F_GAMMA] * (1.0 + c2 * t * t / (d2 * (d2 + t * t)));
}
static double gang_d(double cs, const double *p) {
  double c2 = p[F_C] * p[F_C], d2 = p[F_D] * p[F_D], t = cs - p[F_H];
  double den = d2 + t * t;
  return p[F_GAMMA] * 2.0 * c2 * t / (den * den);
}

/* exp(lambda3^m (dr)^m) and its derivative wrt dr.  For the published
 * integer exponents m = 1, 3 this is (lambda3 dr)^m; any other m (used only
 * to differentiate with respect to m by finite differences) takes the
 * continuation sgn(u)|u|^m, u = lambda3 dr, which equals u^m at m = 1, 3. */
static double expo_arg(double u, double m) {
  if (m == 3.0) return u * u * u;
  if (m == 1.0) return u;
  if (u == 0.0) return 0.0;
  return copysign(pow(fabs(u), m), u);
}
static double expo(double dr, const double *p) {
  return exp(expo_arg(p[F_LAM3] * dr, p[F_M]));
}
static double expo_d(double dr, const double *p) {
  double l = p[F_LAM3];
  double u = l * dr;
  double m = p[F_M];
  double e = exp(expo_arg(u, m));
  if (m == 3.0) return 3.0 * l * u * u * e;
  if (m == 1.0) return l * e;
  if (u == 0.0) return 0.0;
  return m * l * pow(fabs(u), m - 1.0) * e;
}

/* Bond order b(zeta) and db/dzeta.  b = 1 when zeta == 0 (no third atom),
 * and the derivative is then taken as 0 because it multiplies an empty sum.
 * With s = n ln(beta zeta) and y = e^s = (beta zeta)^n, ln(1 + y) is formed as
 * s + ln(1 + e^-s) for s > 0 and y / (1 + y) as 1 / (1 + e^-s): y itself leaves
 * the FP64 range once s > 709, which close contacts reach (there the
 * three-body exponential makes zeta huge), and would turn b into 0 and
 * db/dzeta into inf / inf. */
static double log1p_exp(double s) { return s > 0.0 ? s + log1p(exp(-s)) : log1p(exp(s)); }
static double bond(double z, const double *p) {
  if (z <= 0.0) return 1.0;
  double n = p[F_N];
  double s = n * log(p[F_BETA] * z);
  return exp(-log1p_exp(s) / (2.0 * n));
}
static double bond_d(double z, const double *p) {
  if (z <= 0.0) return 0.0;
  double n = p[F_N];
  double s = n * log(p[F_BETA] * z);
  double b = exp(-log1p_exp(s) / (2.0 * n));
  double w = s > 0.0 ? 1.0 / (1.0 + exp(-s)) : exp(s) / (1.0 + exp(s)); /* y / (1 + y) */
  return -0.5 * b * w / z;
}

/* zeta(i,j,k) and its gradients wrt x_i, x_j, x_k.
 * dij, dik: displacement vectors x_j - x_i, x_k - x_i. */
static double zeta_term(const double *dij, double rij, const double *dik, double rik,
                        const double *p, double *gi, double *gj, double *gk) {
  double uij[3], uik[3];
  for (int a = 0; a < 3; ++a) { uij[a] = dij[a] / rij; uik[a] = dik[a] / rik; }
  double cs = uij[0] * uik[0] + uij[1] * uik[1] + uij[2] * uik[2];
  double fc = fcut(rik, p), dfc = fcut_d(rik, p);
  double g = gang(cs, p), dg = gang_d(cs, p);
  double e = expo(rij - rik, p), de = expo_d(rij - rik, p);
  if (gi) {
    for (int a = 0; a < 3; ++a) {
      double dcos_j = (uik[a] - cs * uij[a]) / rij;
      double dcos_k = (uij[a] - cs * uik[a]) / rik;
      gj[a] = fc * (dg * e * dcos_j + g * de * uij[a]);
      gk[a] = fc * dg * e * dcos_k + (dfc * g * e - fc * g * de) * uik[a];
      gi[a] = -(gj[a] + gk[a]);
    }
  }
  return fc * g * e;
}

static double norm3(const double *d) { return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]); }

/* Everything rooted at one centre atom i (Algorithm 2 for a fixed i).
 *   nn        : number of candidate neighbours (any set that contains every
 *               atom within the cutoff; others are skipped by the cutoff test)
 *   d[nn][3]  : displacement x_nb - x_i of each candidate
 *   tn[nn]    : species of each candidate
 *   fnb[nn][3]: force added onto each candidate (accumulated)
 *   fi[3]     : force added onto i (accumulated)
 *   *e        : energy of the terms rooted at i (accumulated)
 *   w[6]      : virial xx yy zz xy xz yz (accumulated) */
static void centre_terms(int ti, int nn, const double *d, const int *tn, int nt,
                         const double *table, double *e, double *fi, double *fnb, double *w) {
  for (int j = 0; j < nn; ++j) {
    const double *pij = prow(table, nt, ti, tn[j], tn[j]);
    const double *dij = d + 3 * j;
    double rij = norm3(dij);
    if (rij >= pij[F_R] + pij[F_DC]) continue;

    /* first k loop: zeta_ij */
    double zeta = 0.0;
    for (int k = 0; k < nn; ++k) {
      if (k == j) continue;
      const double *pijk = prow(table, nt, ti, tn[j], tn[k]);
      const double *dik = d + 3 * k;
      double rik = norm3(dik);
      if (rik >= pijk[F_R] + pijk[F_DC]) continue;
      zeta += zeta_term(dij, rij, dik, rik, pijk, NULL, NULL, NULL);
    }

    /* pair term V(i,j,zeta) */
    double fc = fcut(rij, pij), dfc = fcut_d(rij, pij);
    double fr = pij[F_A] * exp(-pij[F_LAM1] * rij);
    double dfr = -pij[F_LAM1] * fr;
    double fa = -pij[F_B] * exp(-pij[F_LAM2] * rij);
    double dfa = -pij[F_LAM2] * fa;
    double b = bond(zeta, pij), db = bond_d(zeta, pij);
    double v = fc * (fr + b * fa);
    double dvdr = dfc * (fr + b * fa) + fc * (dfr + b * dfa);
    *e += 0.5 * v;
    double fpair[3];
    for (int a = 0; a < 3; ++a) {
      fpair[a] = -0.5 * dvdr * dij[a] / rij; /* force on j; opposite on i */
      fnb[3 * j + a] += fpair[a];
      fi[a] -= fpair[a];
    }
    w[0] += dij[0] * fpair[0]; w[1] += dij[1] * fpair[1]; w[2] += dij[2] * fpair[2];
    w[3] += dij[0] * fpair[1]; w[4] += dij[0] * fpair[2]; w[5] += dij[1] * fpair[2];

    /* second k loop: dV/dzeta times dzeta(i,j,k)/dx */
    double dz = 0.5 * fc * fa * db;
    if (dz == 0.0) continue;
    for (int k = 0; k < nn; ++k) {
      if (k == j) continue;
      const double *pijk = prow(table, nt, ti, tn[j], tn[k]);
      const double *dik = d + 3 * k;
      double rik = norm3(dik);
      if (rik >= pijk[F_R] + pijk[F_DC]) continue;
      double gi[3], gj[3], gk[3];
      zeta_term(dij, rij, dik, rik, pijk, gi, gj, gk);
      double fj[3], fk[3];
      for (int a = 0; a < 3; ++a) {
        fi[a] -= dz * gi[a];
        fj[a] = -dz * gj[a];
        fk[a] = -dz * gk[a];
        fnb[3 * j + a] += fj[a];
        fnb[3 * k + a] += fk[a];
      }
      w[0] += dij[0] * fj[0] + dik[0] * fk[0];
      w[1] += dij[1] * fj[1] + dik[1] * fk[1];
      w[2] += dij[2] * fj[2] + dik[2] * fk[2];
      w[3] += dij[0] * fj[1] + dik[0] * fk[1];
      w[4] += dij[0] * fj[2] + dik[0] * fk[2];
      w[5] += dij[1] * fj[2] + dik[1] * fk[2];
    }
  }
}

static void min_image(double *d, const double *box) {
  for (int a = 0; a < 3; ++a) d[a] -= box[a] * nearbyint(d[a] / box[a]);
}

/* ---------------------------------------------------------------------------
 * Neighbour lists: N_i = { j != i : r_ij <= rlist } (the paper, Section II),
 * full (both orders), minimum image.  Output rows are sorted by j.
 * Return ORC_ERR_OVERFLOW (and the needed capacity in *need) if a row is
 * longer than cap, ORC_ERR_BOX if some box side is below 2*rlist.
 * ------------------------------------------------------------------------- */
int orc_neigh_brute(int n, const double *x, const double *box, double rlist, int cap,
                    int *count, int *list, int *need) {
  if (n < 0 || cap < 0) return ORC_ERR_ARG;
  for (int a = 0; a < 3; ++a) if (box[a] < 2.0 * rlist) return ORC_ERR_BOX;
  double rl2 = rlist * rlist;
  int worst = 0;
  for (int i = 0; i < n; ++i) {
    int c = 0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
      min_image(d, box);
      if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= rl2) {
        if (c < cap) list[(size_t)i * cap + c] = j;
        ++c;
      }
    }
    count[i] = c;
    if (c > worst) worst = c;
  }
  if (need) *need = worst;
  return worst > cap ? ORC_ERR_OVERFLOW : ORC_OK;
}

static int cmp_int(const void *a, const void *b) {
  int x = *(const int *)a, y = *(const int *)b;
  return (x > y) - (x < y);
}

/* Same list by binning atoms into cells of side >= rlist and scanning the 27
 * surrounding cells.  Falls back to the brute-force scan when a box side
 * holds fewer than 3 cells. */
int orc_neigh_cells(int n, const double *x, const double *box, double rlist, int cap,
                    int *count, int *list, int *need) {
  if (n < 0 || cap < 0) return ORC_ERR_ARG;
  for (int a = 0; a < 3; ++a) if (box[a] < 2.0 * rlist) return ORC_ERR_BOX;
  int nc[3];
  for (int a = 0; a < 3; ++a) nc[a] = (int)floor(box[a] / rlist);
  if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3)
    return orc_neigh_brute(n, x, box, rlist, cap, count, list, need);
  size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
  int *cell_of = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  int *head = (int *)malloc(sizeof(int) * ncell);
  int *next = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  for (size_t c = 0; c < ncell; ++c) head[c] = -1;
  for (int i = n - 1; i >= 0; --i) {
    int ci[3];
    for (int a = 0; a < 3; ++a) {
      double s = x[3 * i + a] / box[a];
      s -= floor(s);
      int q = (int)(s * nc[a]);
      if (q >= nc[a]) q = nc[a] - 1;
      if (q < 0) q = 0;
      ci[a] = q;
    }
    int c = (ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
    cell_of[i] = c;
    next[i] = head[c];
    head[c] = i;
  }
  double rl2 = rlist * rlist;
  int worst = 0;
  int *row = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) {
    int c = cell_of[i];
    int cx = c % nc[0], cy = (c / nc[0]) % nc[1], cz = c / (nc[0] * nc[1]);
    int m = 0;
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          int qx = (cx + ox + nc[0]) % nc[0], qy = (cy + oy + nc[1]) % nc[1], qz = (cz + oz + nc[2]) % nc[2];
          for (int j = head[(qz * nc[1] + qy) * nc[0] + qx]; j >= 0; j = next[j]) {
            if (j == i) continue;
            double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
            min_image(d, box);
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= rl2) row[m++] = j;
          }
        }
    qsort(row, (size_t)m, sizeof(int), cmp_int);
    for (int q = 0; q < m && q < cap; ++q) list[(size_t)i * cap + q] = row[q];
    count[i] = m;
    if (m > worst) worst = m;
  }
  free(row); free(cell_of); free(head); free(next);
  if (need) *need = worst;
  return worst > cap ? ORC_ERR_OVERFLOW : ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Energy, forces, virial over a full neighbour list (Algorithm 2).
 * The list may hold skin entries beyond the cutoff; they contribute nothing.
 * centre == NULL: all atoms are centres.  Otherwise only the ncentre listed
 * atoms are centres (used to get exact forces on sampled atoms: the force on
 * atom a is complete once a and all its neighbours are centres).
 * Outputs are accumulated (the caller zeroes them); any may be NULL.
 * ------------------------------------------------------------------------- */
int orc_tersoff(int n, const double *x, const int *type, const double *box, int nt,
                const double *table, const int *count, const int *list, int cap,
                int ncentre, const int *centre, double *energy, double *forces,
                double *virial, double *eatom) {
  if (n < 0 || nt <= 0) return ORC_ERR_ARG;
  double *d = (double *)malloc(sizeof(double) * 3 * (size_t)(cap > 0 ? cap : 1));
  double *fnb = (double *)malloc(sizeof(double) * 3 * (size_t)(cap > 0 ? cap : 1));
  int *tn = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
  int nc = centre ? ncentre : n;
  double etot = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
  for (int q = 0; q < nc; ++q) {
    int i = centre ? centre[q] : q;
    int nn = count[i] < cap ? count[i] : cap;
    for (int s = 0; s < nn; ++s) {
      int j = list[(size_t)i * cap + s];
      for (int a = 0; a < 3; ++a) d[3 * s + a] = x[3 * j + a] - x[3 * i + a];
      min_image(d + 3 * s, box);
      tn[s] = type[j];
      fnb[3 * s] = fnb[3 * s + 1] = fnb[3 * s + 2] = 0.0;
    }
    double e = 0.0, fi[3] = {0, 0, 0};
    centre_terms(type[i], nn, d, tn, nt, table, &e, fi, fnb, w);
    etot += e;
    if (eatom) eatom[i] += e;
    if (forces) {
      for (int a = 0; a < 3; ++a) forces[3 * i + a] += fi[a];
      for (int s = 0; s < nn; ++s) {
        int j = list[(size_t)i * cap + s];
        for (int a = 0; a < 3; ++a) forces[3 * j + a] += fnb[3 * s + a];
      }
    }
  }
  if (energy) *energy += etot;
  if (virial) for (int a = 0; a < 6; ++a) virial[a] += w[a];
  free(d); free(fnb); free(tn);
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Brute force without neighbour lists: every atom j and k in every periodic
 * image with shifts in [-nimg, nimg]^3 is a candidate (except i itself in the
 * home image); the cutoff test alone decides.  Valid for boxes of any size,
 * as long as nimg * min(box) exceeds the largest cutoff.
 * ------------------------------------------------------------------------- */
int orc_tersoff_images(int n, const double *x, const int *type, const double *box, int nt,
                       const double *table, int nimg, double *energy, double *forces,
                       double *virial, double *eatom) {
  if (n < 0 || nt <= 0 || nimg < 0) return ORC_ERR_ARG;
  int side = 2 * nimg + 1;
  size_t m = (size_t)n * side * side * side;
  double *d = (double *)malloc(sizeof(double) * 3 * (m > 0 ? m : 1));
  double *fnb = (double *)malloc(sizeof(double) * 3 * (m > 0 ? m : 1));
  int *tn = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
  int *owner = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
  double etot = 0.0, w[6] = {0, 0, 0, 0, 0, 0};
  for (int i = 0; i < n; ++i) {
    size_t nn = 0;
    for (int j = 0; j < n; ++j)
      for (int sz = -nimg; sz <= nimg; ++sz)
        for (int sy = -nimg; sy <= nimg; ++sy)
          for (int sx = -nimg; sx <= nimg; ++sx) {
            if (j == i && sx == 0 && sy == 0 && sz == 0) continue;
            d[3 * nn + 0] = x[3 * j + 0] + sx * box[0] - x[3 * i + 0];
            d[3 * nn + 1] = x[3 * j + 1] + sy * box[1] - x[3 * i + 1];
            d[3 * nn + 2] = x[3 * j + 2] + sz * box[2] - x[3 * i + 2];
            tn[nn] = type[j];
            owner[nn] = j;
            fnb[3 * nn] = fnb[3 * nn + 1] = fnb[3 * nn + 2] = 0.0;
            ++nn;
          }
    double e = 0.0, fi[3] = {0, 0, 0};
    centre_terms(type[i], (int)nn, d, tn, nt, table, &e, fi, fnb, w);
    etot += e;
    if (eatom) eatom[i] += e;
    if (forces) {
      for (int a = 0; a < 3; ++a) forces[3 * i + a] += fi[a];
      for (size_t s = 0; s < nn; ++s)
        for (int a = 0; a < 3; ++a) forces[3 * owner[s] + a] += fnb[3 * s + a];
    }
  }
  if (energy) *energy += etot;
  if (virial) for (int a = 0; a < 6; ++a) virial[a] += w[a];
  free(d); free(fnb); free(tn); free(owner);
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * The list-based evaluation above, with the centres shared among OpenMP
 * threads (each thread sums into its own force array, energy and virial,
 * added up at the end).  Same arithmetic per centre; only the order of the
 * final sums differs.  Built only for timing the oracle on the host's cores
 * (compiled with -fopenmp); without OpenMP it runs on one thread.  threads
 * > 0 caps the number of threads (0: all OpenMP offers).  Returns the number
 * of threads used.
 * ------------------------------------------------------------------------- */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_tersoff_threads(int n, const double *x, const int *type, const double *box, int nt,
                        const double *table, const int *count, const int *list, int cap,
                        int threads, double *energy, double *forces, double *virial) {
  if (n < 0 || nt <= 0) return -ORC_ERR_ARG;
  int nthr = 1;
#ifdef _OPENMP
  nthr = omp_get_max_threads();
  if (threads > 0 && threads < nthr) nthr = threads;
#endif
  double *fth = (double *)calloc((size_t)nthr * 3 * (size_t)(n > 0 ? n : 1), sizeof(double));
  double *eth = (double *)calloc((size_t)nthr * 7, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel num_threads(nthr)
#endif
  {
    int th = 0;
#ifdef _OPENMP
    th = omp_get_thread_num();
#endif
    double *f = fth + (size_t)th * 3 * (size_t)(n > 0 ? n : 1);
    double *ew = eth + 7 * th;
    double *d = (double *)malloc(sizeof(double) * 3 * (size_t)(cap > 0 ? cap : 1));
    double *fnb = (double *)malloc(sizeof(double) * 3 * (size_t)(cap > 0 ? cap : 1));
    int *tn = (int *)malloc(sizeof(int) * (size_t)(cap > 0 ? cap : 1));
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int i = 0; i < n; ++i) {
      int nn = count[i] < cap ? count[i] : cap;
      for (int s = 0; s < nn; ++s) {
        int j = list[(size_t)i * cap + s];
        for (int a = 0; a < 3; ++a) d[3 * s + a] = x[3 * j + a] - x[3 * i + a];
        min_image(d + 3 * s, box);
        tn[s] = type[j];
        fnb[3 * s] = fnb[3 * s + 1] = fnb[3 * s + 2] = 0.0;
      }
      double e = 0.0, fi[3] = {0, 0, 0};
      centre_terms(type[i], nn, d, tn, nt, table, &e, fi, fnb, ew + 1);
      ew[0] += e;
      for (int a = 0; a < 3; ++a) f[3 * i + a] += fi[a];
      for (int s = 0; s < nn; ++s) {
        int j = list[(size_t)i * cap + s];
        for (int a = 0; a < 3; ++a) f[3 * j + a] += fnb[3 * s + a];
      }
    }
    free(d); free(fnb); free(tn);
  }
  for (int t = 0; t < nthr; ++t) {
    if (energy) *energy += eth[7 * t];
    if (virial) for (int a = 0; a < 6; ++a) virial[a] += eth[7 * t + 1 + a];
    if (forces)
      for (size_t k = 0; k < 3 * (size_t)n; ++k) forces[k] += fth[(size_t)t * 3 * (size_t)(n > 0 ? n : 1) + k];
  }
  free(fth); free(eth);
  return nthr;
}
