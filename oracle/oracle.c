/*
 * FP64 checker for the combined force path.  TEST INFRASTRUCTURE ONLY:
 * nothing in the device library links, calls or includes this file; only the
 * tests, the smoke entry and the benchmark's CPU-baseline leg use it.
 *
 * Plain, serial-per-task sums written from the definitions:
 *  - gravity over a work request's interaction lists (Sec. 4.1: all particles
 *    of a bucket interact with the same nodes and particles), Plummer-softened,
 *    with monopole or monopole + quadrupole node terms;
 *  - brute-force all-pairs gravity;
 *  - node moments from member particles;
 *  - the reorganisation maps (Sec. 3.2): the sorted index array built by
 *    binary-search insertion in request order, the chare-table lookup, slot
 *    assignment, packed ranges, address lists and their sorted form;
 *  - Lennard-Jones over cell-pair compute objects (Sec. 4.2: one object per
 *    pair of patches updates both), and brute force with minimum image;
 *  - analytic vector-Jacobian products (gravity: direct + monopole or
 *    monopole + quadrupole with the node chain rule; Lennard-Jones: positions,
 *    masses, per-type eps/sigma);
 *  - the Ewald correction of periodic gravity (ChaNGa's second combined
 *    kernel, Sec. 4.1, Sec. 4.3): the pull of every periodic image of the box's
 *    total mass M at its centre of mass c (optionally expanded to the box's
 *    second moment about c), plus the neutralising background, minus the
 *    direct pull of the central copy that the tree walk computes.
 *  - the Barnes-Hut interaction lists of each bucket's work request (Sec. 4.1),
 *    a recursive descent from the definition of the opening test.
 *
 * Ewald (cubic box of side L, splitting parameter alpha; r = x - c taken to
 * the nearest image; real-space images n in {-nrep..nrep}^3; wave vectors
 * h in Z^3 with 0 < |h|^2 <= hmax2):
 *   phi(x) = -G M [ sum_{n != 0} erfc(alpha s_n)/s_n + (erfc(alpha s_0) - 1)/s_0
 *                  + 1/(pi L) sum_h exp(-pi^2 |h|^2/(alpha L)^2)/|h|^2 cos(2 pi h.r/L)
 *                  - pi/(alpha^2 L^3) ],   s_n = |r + n L|
 *   a(x) = -grad phi = G M [ sum_{n != 0} -(erfc(alpha s)/s^3 + 2 alpha/sqrt(pi) e^{-alpha^2 s^2}/s^2) s_vec
 *                           + (erf(alpha s)/s^3 - 2 alpha/sqrt(pi) e^{-alpha^2 s^2}/s^2) s_vec   (n = 0)
 *                           - 2/L^2 sum_h exp(-pi^2 |h|^2/(alpha L)^2)/|h|^2 sin(2 pi h.r/L) h ].
 * With the box's second moment S about c (optional), psi~ = -phi / (G M) above is expanded to
 * second order: phi -= G/2 S_ab d_a d_b psi~ and a += G/2 S_ab grad d_a d_b psi~, every image and
 * wave vector differentiated termwise.
 * The n = 0 terms take their Taylor series near s = 0 (erf(x)/x^3 - 2/sqrt(pi)
 * e^{-x^2}/x^2 = 2/sqrt(pi) (2/3 - 2/5 x^2 + 1/7 x^4 - 1/27 x^6 + 1/132 x^8 - ...),
 * (erfc(x) - 1)/x = -2/sqrt(pi) (1 - x^2/3 + x^4/10 - x^6/42 + ...)), where the
 * direct forms cancel.
 *
 * Formulas (G, softening eps):
 *   pair:      a_i += G m_j u / s^3,   u = x_j - x_i, s^2 = |u|^2 + eps^2, j != i
 *   monopole:  a_i += -G M d / r^3,    d = x_i - c,   r^2 = |d|^2 + eps^2
 *   quadrupole adds G [3 S d / r^5 - 15/2 (d.S.d) d / r^7 + 3/2 tr(S) d / r^5],
 *   the gradient of the second-order expansion about the centre of mass c of
 *   -G sum_k m_k / sqrt(|x - x_k|^2 + eps^2), S = sum_k m_k (x_k-c)(x_k-c)^T.
 *   LJ: q = sigma^2 / r^2, F_i += 24 eps (2 q^6 - q^3) / r^2 * d, d = x_i - x_j
 *   (minus the image shift), F_j -= the same; a = F / m; Lorentz-Berthelot
 *   mixing sigma_ij = (sigma_a + sigma_b)/2, eps_ij = sqrt(eps_a eps_b).
 *
 * The one decision taken in FP32: whether an LJ pair is inside the cutoff.
 * It is an integer outcome decided by floating point, so it is taken exactly
 * as the device takes it: d per component as (x_i - max(s,0)) - (x_j + min(s,0))
 * in FP32, r^2 = fma(dz, dz, fma(dy, dy, dx*dx)) in FP32, inside iff r^2 < rc^2
 * with rc^2 rounded to FP32.  Everything else is FP64.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* gravity                                                                  */
/* ------------------------------------------------------------------------ */

/* Acceleration on a target at x from source (xs, m), Plummer softening. */
static void pair_acc(const double* x, const double* xs, double m, double G, double eps2, double* a) {
  double u0 = xs[0] - x[0], u1 = xs[1] - x[1], u2 = xs[2] - x[2];
  double s2 = u0 * u0 + u1 * u1 + u2 * u2 + eps2;
  double s3 = s2 * sqrt(s2);
  a[0] += G * m * u0 / s3;
  a[1] += G * m * u1 / s3;
  a[2] += G * m * u2 / s3;
}

/* Node term: monopole (order 1) or monopole + quadrupole (order 2).
 * mom = (cx, cy, cz, M, Sxx, Syy, Szz, Sxy, Sxz, Syz). */
static void node_acc(const double* x, const double* mom, int order, double G, double eps2, double* a) {
  double d0 = x[0] - mom[0], d1 = x[1] - mom[1], d2 = x[2] - mom[2];
  double r2 = d0 * d0 + d1 * d1 + d2 * d2 + eps2;
  double r = sqrt(r2);
  double r3 = r2 * r, r5 = r3 * r2, r7 = r5 * r2;
  double M = mom[3];
  a[0] += -G * M * d0 / r3;
  a[1] += -G * M * d1 / r3;
  a[2] += -G * M * d2 / r3;
  if (order >= 2) {
    double Sxx = mom[4], Syy = mom[5], Szz = mom[6], Sxy = mom[7], Sxz = mom[8], Syz = mom[9];
    double Sd0 = Sxx * d0 + Sxy * d1 + Sxz * d2;
    double Sd1 = Sxy * d0 + Syy * d1 + Syz * d2;
    double Sd2 = Sxz * d0 + Syz * d1 + Szz * d2;
    double dSd = d0 * Sd0 + d1 * Sd1 + d2 * Sd2;
    double T = Sxx + Syy + Szz;
    a[0] += G * (3.0 * Sd0 / r5 - 7.5 * dSd * d0 / r7 + 1.5 * T * d0 / r5);
    a[1] += G * (3.0 * Sd1 / r5 - 7.5 * dSd * d1 / r7 + 1.5 * T * d1 / r5);
    a[2] += G * (3.0 * Sd2 / r5 - 7.5 * dSd * d2 / r7 + 1.5 * T * d2 / r5);
  }
}

/* Potential at x of a source (xs, m), Plummer softening: -G m / sqrt(|xs - x|^2 + eps^2). */
static double pair_pot(const double* x, const double* xs, double m, double G, double eps2) {
  double u0 = xs[0] - x[0], u1 = xs[1] - x[1], u2 = xs[2] - x[2];
  return -G * m / sqrt(u0 * u0 + u1 * u1 + u2 * u2 + eps2);
}

/* Potential of a node term, the function whose negative gradient node_acc adds: the second-order
 * Taylor expansion of the members' softened potential about their centre of mass,
 * -G [M / r + (3/2) d.S.d / r^5 - (1/2) T / r^3] (order 1: -G M / r). */
static double node_pot(const double* x, const double* mom, int order, double G, double eps2) {
  double d0 = x[0] - mom[0], d1 = x[1] - mom[1], d2 = x[2] - mom[2];
  double r2 = d0 * d0 + d1 * d1 + d2 * d2 + eps2;
  double r = sqrt(r2);
  double r3 = r2 * r, r5 = r3 * r2;
  double phi = mom[3] / r;
  if (order >= 2) {
    double Sxx = mom[4], Syy = mom[5], Szz = mom[6], Sxy = mom[7], Sxz = mom[8], Syz = mom[9];
    double dSd = d0 * (Sxx * d0 + Sxy * d1 + Sxz * d2) + d1 * (Sxy * d0 + Syy * d1 + Syz * d2) +
                 d2 * (Sxz * d0 + Syz * d1 + Szz * d2);
    double T = Sxx + Syy + Szz;
    phi += 1.5 * dSd / r5 - 0.5 * T / r3;
  }
  return -G * phi;
}

/* Sum over each task's lists.  pos: n x 3, mass: n, mom: nnodes x 10.
 * acc (n x 3) is written for every id in every task's target range; pot (optional, n) gets the
 * potential of the same terms (sources j != i). */
void or_grav_lists(int32_t ntasks, const int32_t* i_begin, const int32_t* i_count, const int32_t* n_first,
                   const int32_t* n_count, const int32_t* j_first, const int32_t* j_nr, const int32_t* node_idx,
                   const int32_t* ranges, const double* pos, const double* mass, const double* mom, int32_t order,
                   double G, double eps, double* acc, double* pot) {
  double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 4)
  for (int32_t t = 0; t < ntasks; ++t) {
    for (int32_t i = i_begin[t]; i < i_begin[t] + i_count[t]; ++i) {
      double a[3] = {0, 0, 0};
      double phi = 0.0;
      for (int32_t k = 0; k < n_count[t]; ++k) {
        const double* m = mom + 10 * (size_t)node_idx[n_first[t] + k];
        node_acc(pos + 3 * (size_t)i, m, order, G, eps2, a);
        if (pot) phi += node_pot(pos + 3 * (size_t)i, m, order, G, eps2);
      }
      for (int32_t r = 0; r < j_nr[t]; ++r) {
        int32_t b = ranges[2 * (size_t)(j_first[t] + r)], c = ranges[2 * (size_t)(j_first[t] + r) + 1];
        for (int32_t j = b; j < b + c; ++j)
          if (j != i) {
            pair_acc(pos + 3 * (size_t)i, pos + 3 * (size_t)j, mass[j], G, eps2, a);
            if (pot) phi += pair_pot(pos + 3 * (size_t)i, pos + 3 * (size_t)j, mass[j], G, eps2);
          }
      }
      acc[3 * (size_t)i] = a[0];
      acc[3 * (size_t)i + 1] = a[1];
      acc[3 * (size_t)i + 2] = a[2];
      if (pot) pot[i] = phi;
    }
  }
}

/* All pairs; pot (optional) gets the softened pair potential -G m_j / s summed over j != i. */
void or_grav_brute(int64_t n, const double* pos, const double* mass, double G, double eps, double* acc, double* pot) {
  double eps2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    double a[3] = {0, 0, 0}, p = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      pair_acc(pos + 3 * i, pos + 3 * j, mass[j], G, eps2, a);
      if (pot) {
        double u0 = pos[3 * j] - pos[3 * i], u1 = pos[3 * j + 1] - pos[3 * i + 1], u2 = pos[3 * j + 2] - pos[3 * i + 2];
        p += -G * mass[j] / sqrt(u0 * u0 + u1 * u1 + u2 * u2 + eps2);
      }
    }
    acc[3 * i] = a[0]; acc[3 * i + 1] = a[1]; acc[3 * i + 2] = a[2];
    if (pot) pot[i] = p;
  }
}

/* Node acceleration at arbitrary points (for closed-form and convergence checks). */
void or_node_acc_points(int64_t npts, const double* x, const double* mom, int32_t order, double G, double eps,
                        double* acc) {
  for (int64_t p = 0; p < npts; ++p) {
    double a[3] = {0, 0, 0};
    node_acc(x + 3 * p, mom, order, G, eps * eps, a);
    memcpy(acc + 3 * p, a, sizeof a);
  }
}

/* Moments of each node from its member id range: (cx, cy, cz, M, S6). */
void or_node_moments(int32_t nnodes, const int32_t* node_range, const double* pos, const double* mass, double* mom) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t k = 0; k < nnodes; ++k) {
    int32_t b = node_range[2 * k], c = node_range[2 * k + 1];
    double M = 0, cx = 0, cy = 0, cz = 0;
    for (int32_t i = b; i < b + c; ++i) {
      M += mass[i];
      cx += mass[i] * pos[3 * (size_t)i];
      cy += mass[i] * pos[3 * (size_t)i + 1];
      cz += mass[i] * pos[3 * (size_t)i + 2];
    }
    cx /= M; cy /= M; cz /= M;
    double S[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t i = b; i < b + c; ++i) {
      double m = mass[i], dx = pos[3 * (size_t)i] - cx, dy = pos[3 * (size_t)i + 1] - cy, dz = pos[3 * (size_t)i + 2] - cz;
      S[0] += m * dx * dx; S[1] += m * dy * dy; S[2] += m * dz * dz;
      S[3] += m * dx * dy; S[4] += m * dx * dz; S[5] += m * dy * dz;
    }
    double* o = mom + 10 * (size_t)k;
    o[0] = cx; o[1] = cy; o[2] = cz; o[3] = M;
    memcpy(o + 4, S, sizeof S);
  }
}

/* ------------------------------------------------------------------------ */
/* reorganisation maps                                                      */
/* ------------------------------------------------------------------------ */

/* Insert id into the sorted array arr[0..*n) unless present (binary search). */
static void sorted_insert(int32_t* arr, int64_t* n, int32_t id) {
  int64_t lo = 0, hi = *n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (arr[mid] < id) lo = mid + 1;
    else hi = mid;
  }
  if (lo < *n && arr[lo] == id) return;
  memmove(arr + lo + 1, arr + lo, sizeof(int32_t) * (size_t)(*n - lo));
  arr[lo] = id;
  (*n)++;
}

/* The sorted index array over a combined request: for every task in order,
 * its target ids then its direct ids, each inserted by binary search.
 * U must hold n_ids entries; returns |U|. */
int64_t or_union_insert(int32_t ntasks, const int32_t* i_begin, const int32_t* i_count, const int32_t* j_first,
                        const int32_t* j_nr, const int32_t* ranges, int32_t* U) {
  int64_t n = 0;
  for (int32_t t = 0; t < ntasks; ++t) {
    for (int32_t i = i_begin[t]; i < i_begin[t] + i_count[t]; ++i) sorted_insert(U, &n, i);
    for (int32_t r = 0; r < j_nr[t]; ++r) {
      int32_t b = ranges[2 * (size_t)(j_first[t] + r)], c = ranges[2 * (size_t)(j_first[t] + r) + 1];
      for (int32_t j = b; j < b + c; ++j) sorted_insert(U, &n, j);
    }
  }
  return n;
}

/* Full map set for one combined request against a pool state.
 *  mode: 0 REDUNDANT, 1 INDIRECT, 2 SORTED, 3 PACK.
 *  slot_of[n_ids] is updated in place (missing ids get slots) except in REDUNDANT mode.
 *  Outputs (caller-sized):
 *   U[n_ids], pos[n_ids] (-1 where not in U), missing[n_ids], new_slot[n_ids]
 *   pranges[2*n_ranges] and pi_begin[ntasks]   (REDUNDANT / PACK: positions in U order)
 *   ilist[sum i_count], jlist[sum direct ids]  (INDIRECT / SORTED: pool slots; SORTED sorts jlist per task)
 *  counts[0] = |U|, counts[1] = #missing.  Returns 0, or 3 if the pool has too few free slots. */
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

int32_t or_maps(int32_t ntasks, const int32_t* i_begin, const int32_t* i_count, const int32_t* j_first,
                const int32_t* j_nr, const int32_t* ranges, int32_t n_ranges, int32_t n_ids, int32_t capacity,
                int32_t* slot_of, int32_t mode, int32_t* U, int32_t* pos, int32_t* missing, int32_t* new_slot,
                int32_t* pranges, int32_t* pi_begin, int32_t* ilist, int32_t* jlist, int64_t* counts) {
  int64_t nu = or_union_insert(ntasks, i_begin, i_count, j_first, j_nr, ranges, U);
  for (int32_t i = 0; i < n_ids; ++i) pos[i] = -1;
  for (int64_t k = 0; k < nu; ++k) pos[U[k]] = (int32_t)k;
  int64_t nm = 0;
  if (mode != 0) {
    /* chare-table lookup: ids of the union not resident, ascending */
    for (int64_t k = 0; k < nu; ++k)
      if (slot_of[U[k]] < 0) missing[nm++] = U[k];
    /* free slots ascending; the k-th missing id takes the k-th free slot */
    char* used = (char*)calloc((size_t)capacity, 1);
    for (int32_t i = 0; i < n_ids; ++i)
      if (slot_of[i] >= 0) used[slot_of[i]] = 1;
    int64_t k = 0;
    for (int32_t s = 0; s < capacity && k < nm; ++s)
      if (!used[s]) new_slot[k++] = s;
    free(used);
    if (k < nm) return 3;
    for (int64_t q = 0; q < nm; ++q) slot_of[missing[q]] = new_slot[q];
  } else {
    for (int64_t q = 0; q < nu; ++q) missing[q] = U[q];
    nm = nu;
  }
  counts[0] = nu;
  counts[1] = nm;
  if (mode == 0 || mode == 3) {
    for (int32_t r = 0; r < n_ranges; ++r) {
      pranges[2 * r] = pos[ranges[2 * r]];
      pranges[2 * r + 1] = ranges[2 * r + 1];
    }
    for (int32_t t = 0; t < ntasks; ++t) pi_begin[t] = pos[i_begin[t]];
  } else {
    int64_t qi = 0, qj = 0;
    for (int32_t t = 0; t < ntasks; ++t) {
      for (int32_t i = i_begin[t]; i < i_begin[t] + i_count[t]; ++i) ilist[qi++] = slot_of[i];
      int64_t q0 = qj;
      for (int32_t r = 0; r < j_nr[t]; ++r) {
        int32_t b = ranges[2 * (size_t)(j_first[t] + r)], c = ranges[2 * (size_t)(j_first[t] + r) + 1];
        for (int32_t j = b; j < b + c; ++j) jlist[qj++] = slot_of[j];
      }
      if (mode == 2) qsort(jlist + q0, (size_t)(qj - q0), sizeof(int32_t), cmp_i32);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Lennard-Jones                                                            */
/* ------------------------------------------------------------------------ */

static int inside_cutoff_f32(const float* xi, const float* xj, const float* sh, float rc2) {
  float d[3];
  for (int c = 0; c < 3; ++c) {
    float a = sh[c] > 0.0f ? sh[c] : 0.0f;
    float b = sh[c] < 0.0f ? sh[c] : 0.0f;
    d[c] = (xi[c] - a) - (xj[c] + b);
  }
  float r2 = fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0]));
  return r2 < rc2;
}

/* Pair force factor f (force on i = f d) and potential for one LJ pair at r^2. */
static void lj_pair(double r2, double eps, double sig, double* f, double* u) {
  double q = sig * sig / r2;
  double q3 = q * q * q, q6 = q3 * q3;
  *f = 24.0 * eps * (2.0 * q6 - q3) / r2;
  if (u) *u = 4.0 * eps * (q6 - q3);
}

/* Cell-pair tasks.  rec32: FP32 records (x, y, z, type); force (n x 3) accumulated, then
 * acc = F / m_type.  pot (optional): per-atom half-shared potential energy. */
void or_lj_tasks(int32_t ntasks, const int32_t* i_begin, const int32_t* i_count, const int32_t* j_begin,
                 const int32_t* j_count, const int32_t* self_flag, const float* shift, const float* rec32,
                 int64_t n, int32_t ntypes, const double* eps_t, const double* sig_t, const double* mass_t,
                 double rcut, double* acc, double* pot, int64_t* n_inside) {
  (void)ntypes;
  float rc2 = (float)(rcut * rcut);
  double* F = (double*)calloc((size_t)(3 * n), sizeof(double));
  int64_t cnt = 0;
  for (int32_t t = 0; t < ntasks; ++t) {
    const float* sh = shift + 3 * (size_t)t;
    for (int32_t i = i_begin[t]; i < i_begin[t] + i_count[t]; ++i) {
      int32_t j0 = self_flag[t] ? i + 1 : j_begin[t];
      for (int32_t j = j0; j < j_begin[t] + j_count[t]; ++j) {
        const float* xi = rec32 + 4 * (size_t)i;
        const float* xj = rec32 + 4 * (size_t)j;
        if (!inside_cutoff_f32(xi, xj, sh, rc2)) continue;
        ++cnt;
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = ((double)xi[c] - (double)xj[c]) - (double)sh[c];
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        int ti = (int)xi[3], tj = (int)xj[3];
        double e = sqrt(eps_t[ti] * eps_t[tj]), s = 0.5 * (sig_t[ti] + sig_t[tj]);
        double f, u;
        lj_pair(r2, e, s, &f, &u);
        for (int c = 0; c < 3; ++c) {
          F[3 * (size_t)i + c] += f * d[c];
          F[3 * (size_t)j + c] -= f * d[c];
        }
        if (pot) { pot[i] += 0.5 * u; pot[j] += 0.5 * u; }
      }
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    double m = mass_t[(int)rec32[4 * i + 3]];
    for (int c = 0; c < 3; ++c) acc[3 * i + c] = F[3 * i + c] / m;
  }
  if (n_inside) *n_inside = cnt;
  free(F);
}

/* All pairs with minimum image in the box L; same FP32 cutoff decision with the
 * image shift s = L * round((x_i - x_j) / L) taken per component in FP64. */
void or_lj_brute(int64_t n, const float* rec32, const double* L, const double* eps_t, const double* sig_t,
                 const double* mass_t, double rcut, double* acc, double* pot) {
  float rc2 = (float)(rcut * rcut);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    double Fi[3] = {0, 0, 0}, p = 0;
    const float* xi = rec32 + 4 * i;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const float* xj = rec32 + 4 * j;
      float sh[3];
      double d[3];
      for (int c = 0; c < 3; ++c) {
        double raw = (double)xi[c] - (double)xj[c];
        sh[c] = (float)(L[c] * nearbyint(raw / L[c]));
        d[c] = raw - (double)sh[c];
      }
      if (!inside_cutoff_f32(xi, xj, sh, rc2)) continue;
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      int ti = (int)xi[3], tj = (int)xj[3];
      double e = sqrt(eps_t[ti] * eps_t[tj]), s = 0.5 * (sig_t[ti] + sig_t[tj]);
      double f, u;
      lj_pair(r2, e, s, &f, &u);
      for (int c = 0; c < 3; ++c) Fi[c] += f * d[c];
      p += 0.5 * u;
    }
    double m = mass_t[(int)xi[3]];
    for (int c = 0; c < 3; ++c) acc[3 * i + c] = Fi[c] / m;
    if (pot) pot[i] = p;
  }
}

/* ------------------------------------------------------------------------ */
/* vector-Jacobian products                                                 */
/* ------------------------------------------------------------------------ */

/* L = sum_i g_i . a_i over the lists (direct + monopole nodes), lists frozen,
 * node moments a function of their members.  Outputs gpos (n x 3), gmass (n). */
/* L = sum_i g_i . a_i over each task's lists (direct + node terms of `order`), lists frozen.
 * Node gradients reach members through c = sum m_k x_k / M, M = sum m_k and
 * S = sum m_k e_k e_k^T (e_k = x_k - c; sum m_k e_k = 0, so S depends on c not at all):
 *   dL/dx_k += (m_k / M) dL/dc + m_k (GS + GS^T) e_k,
 *   dL/dm_k += dL/dM + e_k . dL/dc / M + e_k^T GS e_k,
 * with GS = dL/dS over the nine entries of S (T = tr S included).  For the quadrupole term
 * a_q = G [3 S d / r^5 - 15/2 q d / r^7 + 3/2 T d / r^5], q = d^T S d:
 *   d(g.a_q)/dd = G [3 (S g / r^5 - 5 (g.Sd) d / r^7)
 *                    - 15/2 (2 (g.d) S d / r^7 + q g / r^7 - 7 q (g.d) d / r^9)
 *                    + 3/2 T (g / r^5 - 5 (g.d) d / r^7)],
 *   GS_ab = G [3 g_a d_b / r^5 - 15/2 (g.d) d_a d_b / r^7 + 3/2 (g.d) delta_ab / r^5]. */
void or_vjp_grav(int32_t ntasks, const int32_t* i_begin, const int32_t* i_count, const int32_t* n_first,
                 const int32_t* n_count, const int32_t* j_first, const int32_t* j_nr, const int32_t* node_idx,
                 const int32_t* ranges, int32_t nnodes, const int32_t* node_range, const double* pos,
                 const double* mass, const double* mom, int32_t order, double G, double eps, const double* g,
                 int64_t n, double* gpos, double* gmass) {
  double eps2 = eps * eps;
  double* gc = (double*)calloc((size_t)(3 * nnodes), sizeof(double));
  double* gM = (double*)calloc((size_t)nnodes, sizeof(double));
  double* gS = (double*)calloc((size_t)(9 * nnodes), sizeof(double));
  memset(gpos, 0, sizeof(double) * 3 * (size_t)n);
  memset(gmass, 0, sizeof(double) * (size_t)n);
  for (int32_t t = 0; t < ntasks; ++t) {
    for (int32_t i = i_begin[t]; i < i_begin[t] + i_count[t]; ++i) {
      const double* x = pos + 3 * (size_t)i;
      const double* gi = g + 3 * (size_t)i;
      for (int32_t r = 0; r < j_nr[t]; ++r) {
        int32_t b = ranges[2 * (size_t)(j_first[t] + r)], c = ranges[2 * (size_t)(j_first[t] + r) + 1];
        for (int32_t j = b; j < b + c; ++j) {
          if (j == i) continue;
          const double* xs = pos + 3 * (size_t)j;
          double u[3] = {xs[0] - x[0], xs[1] - x[1], xs[2] - x[2]};
          double s2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + eps2;
          double s = sqrt(s2), s3 = s2 * s, s5 = s3 * s2;
          double gu = gi[0] * u[0] + gi[1] * u[1] + gi[2] * u[2];
          for (int q = 0; q < 3; ++q) {
            double w = G * mass[j] * (gi[q] / s3 - 3.0 * gu * u[q] / s5);
            gpos[3 * (size_t)j + q] += w;
            gpos[3 * (size_t)i + q] -= w;
          }
          gmass[j] += G * gu / s3;
        }
      }
      for (int32_t k = 0; k < n_count[t]; ++k) {
        int32_t nd = node_idx[n_first[t] + k];
        const double* m = mom + 10 * (size_t)nd;
        double d[3] = {x[0] - m[0], x[1] - m[1], x[2] - m[2]};
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
        double r = sqrt(r2), r3 = r2 * r, r5 = r3 * r2, r7 = r5 * r2, r9 = r7 * r2;
        double gd = gi[0] * d[0] + gi[1] * d[1] + gi[2] * d[2];
        double v[3];
        for (int q = 0; q < 3; ++q) v[q] = -G * m[3] * (gi[q] / r3 - 3.0 * gd * d[q] / r5);
        if (order >= 2) {
          const double S[3][3] = {{m[4], m[7], m[8]}, {m[7], m[5], m[9]}, {m[8], m[9], m[6]}};
          double Sd[3], Sg[3];
          for (int a = 0; a < 3; ++a) {
            Sd[a] = S[a][0] * d[0] + S[a][1] * d[1] + S[a][2] * d[2];
            Sg[a] = S[a][0] * gi[0] + S[a][1] * gi[1] + S[a][2] * gi[2];
          }
          double q = d[0] * Sd[0] + d[1] * Sd[1] + d[2] * Sd[2];
          double gSd = gi[0] * Sd[0] + gi[1] * Sd[1] + gi[2] * Sd[2];
          double T = m[4] + m[5] + m[6];
          for (int a = 0; a < 3; ++a) {
            v[a] += G * (3.0 * (Sg[a] / r5 - 5.0 * gSd * d[a] / r7) -
                         7.5 * (2.0 * gd * Sd[a] / r7 + q * gi[a] / r7 - 7.0 * q * gd * d[a] / r9) +
                         1.5 * T * (gi[a] / r5 - 5.0 * gd * d[a] / r7));
            for (int bb = 0; bb < 3; ++bb)
              gS[9 * (size_t)nd + 3 * a + bb] +=
                  G * (3.0 * gi[a] * d[bb] / r5 - 7.5 * gd * d[a] * d[bb] / r7 + (a == bb ? 1.5 * gd / r5 : 0.0));
          }
        }
        for (int q = 0; q < 3; ++q) {
          gpos[3 * (size_t)i + q] += v[q];
          gc[3 * (size_t)nd + q] -= v[q];
        }
        gM[nd] += -G * gd / r3;
      }
    }
  }
  /* node -> members */
  for (int32_t nd = 0; nd < nnodes; ++nd) {
    const double* m = mom + 10 * (size_t)nd;
    const double* GS = gS + 9 * (size_t)nd;
    for (int32_t k = node_range[2 * nd]; k < node_range[2 * nd] + node_range[2 * nd + 1]; ++k) {
      double e[3], dc = 0, eGe = 0;
      for (int q = 0; q < 3; ++q) e[q] = pos[3 * (size_t)k + q] - m[q];
      for (int q = 0; q < 3; ++q) {
        double sym = 0;
        for (int bb = 0; bb < 3; ++bb) {
          sym += (GS[3 * q + bb] + GS[3 * bb + q]) * e[bb];
          eGe += e[q] * GS[3 * q + bb] * e[bb];
        }
        gpos[3 * (size_t)k + q] += mass[k] / m[3] * gc[3 * (size_t)nd + q] + mass[k] * sym;
        dc += e[q] * gc[3 * (size_t)nd + q];
      }
      gmass[k] += gM[nd] + dc / m[3] + eGe;
    }
  }
  free(gc);
  free(gM);
  free(gS);
}

/* The direct + monopole case of or_vjp_grav. */
void or_vjp_grav_mono(int32_t ntasks, const int32_t* i_begin, const int32_t* i_count, const int32_t* n_first,
                      const int32_t* n_count, const int32_t* j_first, const int32_t* j_nr, const int32_t* node_idx,
                      const int32_t* ranges, int32_t nnodes, const int32_t* node_range, const double* pos,
                      const double* mass, const double* mom, double G, double eps, const double* g, int64_t n,
                      double* gpos, double* gmass) {
  or_vjp_grav(ntasks, i_begin, i_count, n_first, n_count, j_first, j_nr, node_idx, ranges, nnodes, node_range, pos,
              mass, mom, 1, G, eps, g, n, gpos, gmass);
}

/* L = sum_i g_i . a_i over the cell-pair tasks.  pos (n x 3, FP64) is the
 * differentiation point; rec32 supplies types and the FP32 cutoff decisions
 * (frozen).  mass (n) per atom.  Outputs gpos (n x 3), gmass (n),
 * geps_t / gsig_t (ntypes). */
void or_vjp_lj(int32_t ntasks, const int32_t* i_begin, const int32_t* i_count, const int32_t* j_begin,
               const int32_t* j_count, const int32_t* self_flag, const float* shift, const float* rec32,
               const double* pos, const double* mass, int64_t n, int32_t ntypes, const double* eps_t,
               const double* sig_t, double rcut, const double* g, double* gpos, double* gmass, double* geps_t,
               double* gsig_t) {
  float rc2 = (float)(rcut * rcut);
  double* F = (double*)calloc((size_t)(3 * n), sizeof(double));
  memset(gpos, 0, sizeof(double) * 3 * (size_t)n);
  memset(gmass, 0, sizeof(double) * (size_t)n);
  memset(geps_t, 0, sizeof(double) * (size_t)ntypes);
  memset(gsig_t, 0, sizeof(double) * (size_t)ntypes);
  for (int32_t t = 0; t < ntasks; ++t) {
    const float* sh = shift + 3 * (size_t)t;
    for (int32_t i = i_begin[t]; i < i_begin[t] + i_count[t]; ++i) {
      int32_t j0 = self_flag[t] ? i + 1 : j_begin[t];
      for (int32_t j = j0; j < j_begin[t] + j_count[t]; ++j) {
        if (!inside_cutoff_f32(rec32 + 4 * (size_t)i, rec32 + 4 * (size_t)j, sh, rc2)) continue;
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = (pos[3 * (size_t)i + c] - pos[3 * (size_t)j + c]) - (double)sh[c];
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        int ti = (int)rec32[4 * (size_t)i + 3], tj = (int)rec32[4 * (size_t)j + 3];
        double e = sqrt(eps_t[ti] * eps_t[tj]), s = 0.5 * (sig_t[ti] + sig_t[tj]);
        double f;
        lj_pair(r2, e, s, &f, NULL);
        double s2 = s * s, s6 = s2 * s2 * s2, s12 = s6 * s6;
        double r4 = r2 * r2, r8 = r4 * r4, r10 = r8 * r2, r14 = r10 * r4, r16 = r8 * r8;
        double fp = 24.0 * e * (-14.0 * s12 / r16 + 4.0 * s6 / r10);   /* df / d(r^2) */
        double hi[3], hj[3], p = 0;
        for (int c = 0; c < 3; ++c) {
          hi[c] = g[3 * (size_t)i + c] / mass[i];
          hj[c] = g[3 * (size_t)j + c] / mass[j];
          p += (hi[c] - hj[c]) * d[c];
        }
        for (int c = 0; c < 3; ++c) {
          double w = f * (hi[c] - hj[c]) + 2.0 * fp * p * d[c];
          gpos[3 * (size_t)i + c] += w;
          gpos[3 * (size_t)j + c] -= w;
          F[3 * (size_t)i + c] += f * d[c];
          F[3 * (size_t)j + c] -= f * d[c];
        }
        double dLde = p * f / e;
        double dLds = p * 24.0 * e * (24.0 * s12 / s / r14 - 6.0 * s6 / s / r8);
        /* eps_ij = sqrt(eps_a eps_b), sigma_ij = (sigma_a + sigma_b) / 2 */
        geps_t[ti] += dLde * eps_t[tj] / (2.0 * e);
        geps_t[tj] += dLde * eps_t[ti] / (2.0 * e);
        gsig_t[ti] += 0.5 * dLds;
        gsig_t[tj] += 0.5 * dLds;
      }
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    double gf = 0;
    for (int c = 0; c < 3; ++c) gf += g[3 * i + c] * F[3 * i + c];
    gmass[i] = -gf / (mass[i] * mass[i]);
  }
  free(F);
}

/* Total LJ potential energy (unshifted) at FP64 positions over frozen decisions. */
double or_lj_energy_at(int32_t ntasks, const int32_t* i_begin, const int32_t* i_count, const int32_t* j_begin,
                       const int32_t* j_count, const int32_t* self_flag, const float* shift, const float* rec32,
                       const double* pos, const double* eps_t, const double* sig_t, double rcut) {
  float rc2 = (float)(rcut * rcut);
  double U = 0;
  for (int32_t t = 0; t < ntasks; ++t) {
    const float* sh = shift + 3 * (size_t)t;
    for (int32_t i = i_begin[t]; i < i_begin[t] + i_count[t]; ++i) {
      int32_t j0 = self_flag[t] ? i + 1 : j_begin[t];
      for (int32_t j = j0; j < j_begin[t] + j_count[t]; ++j) {
        if (!inside_cutoff_f32(rec32 + 4 * (size_t)i, rec32 + 4 * (size_t)j, sh, rc2)) continue;
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = (pos[3 * (size_t)i + c] - pos[3 * (size_t)j + c]) - (double)sh[c];
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        int ti = (int)rec32[4 * (size_t)i + 3], tj = (int)rec32[4 * (size_t)j + 3];
        double f, u;
        lj_pair(r2, sqrt(eps_t[ti] * eps_t[tj]), 0.5 * (sig_t[ti] + sig_t[tj]), &f, &u);
        U += u;
      }
    }
  }
  return U;
}

/* LJ forces at FP64 positions over frozen decisions (for finite differences of or_vjp_lj). */
void or_lj_tasks_at(int32_t ntasks, const int32_t* i_begin, const int32_t* i_count, const int32_t* j_begin,
                    const int32_t* j_count, const int32_t* self_flag, const float* shift, const float* rec32,
                    const double* pos, const double* mass, int64_t n, const double* eps_t, const double* sig_t,
                    double rcut, double* acc) {
  float rc2 = (float)(rcut * rcut);
  double* F = (double*)calloc((size_t)(3 * n), sizeof(double));
  for (int32_t t = 0; t < ntasks; ++t) {
    const float* sh = shift + 3 * (size_t)t;
    for (int32_t i = i_begin[t]; i < i_begin[t] + i_count[t]; ++i) {
      int32_t j0 = self_flag[t] ? i + 1 : j_begin[t];
      for (int32_t j = j0; j < j_begin[t] + j_count[t]; ++j) {
        if (!inside_cutoff_f32(rec32 + 4 * (size_t)i, rec32 + 4 * (size_t)j, sh, rc2)) continue;
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = (pos[3 * (size_t)i + c] - pos[3 * (size_t)j + c]) - (double)sh[c];
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        int ti = (int)rec32[4 * (size_t)i + 3], tj = (int)rec32[4 * (size_t)j + 3];
        double f;
        lj_pair(r2, sqrt(eps_t[ti] * eps_t[tj]), 0.5 * (sig_t[ti] + sig_t[tj]), &f, NULL);
        for (int c = 0; c < 3; ++c) {
          F[3 * (size_t)i + c] += f * d[c];
          F[3 * (size_t)j + c] -= f * d[c];
        }
      }
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) acc[3 * i + c] = F[3 * i + c] / mass[i];
  free(F);
}

/* ------------------------------------------------------------------------ */
/* Ewald correction of periodic gravity                                     */
/* ------------------------------------------------------------------------ */

/* x * (erf(a s)/s^3 - 2a/sqrt(pi) e^{-a^2 s^2}/s^2) / a^3 = f(a s) and (erfc(a s) - 1)/s / a = g(a s). */
static double ew_f0(double x) {
  const double c = 2.0 / sqrt(M_PI);
  if (x < 0.1) {
    double x2 = x * x;
    return c * (2.0 / 3.0 + x2 * (-2.0 / 5.0 + x2 * (1.0 / 7.0 + x2 * (-1.0 / 27.0 + x2 * (1.0 / 132.0)))));
  }
  return erf(x) / (x * x * x) - c * exp(-x * x) / (x * x);
}
static double ew_g0(double x) {
  const double c = 2.0 / sqrt(M_PI);
  if (x < 0.1) {
    double x2 = x * x;
    return -c * (1.0 + x2 * (-1.0 / 3.0 + x2 * (1.0 / 10.0 + x2 * (-1.0 / 42.0))));
  }
  return (erfc(x) - 1.0) / x;
}

/* v_out = S v for a symmetric S stored as (xx, yy, zz, xy, xz, yz). */
static void quad_apply(const double* S, const double* v, double* out) {
  out[0] = S[0] * v[0] + S[3] * v[1] + S[4] * v[2];
  out[1] = S[3] * v[0] + S[1] * v[1] + S[5] * v[2];
  out[2] = S[4] * v[0] + S[5] * v[1] + S[2] * v[2];
}

/* Radial derivatives of the Ewald kernels, B_l = (-(1/s) d/ds)^l B_0 for l = 1..3, so that
 * d_a B_0 = -B_1 s_a, d_a d_b B_0 = -delta_ab B_1 + s_a s_b B_2 and
 * d_a d_b d_c B_0 = (delta_ab s_c + delta_ac s_b + delta_bc s_a) B_2 - s_a s_b s_c B_3.
 * Differentiating B_0 = erfc(alpha s)/s once more each time gives the recursion
 * B_l = ((2l - 1) B_{l-1} + (2 alpha^2)^l / (alpha sqrt(pi)) e^{-alpha^2 s^2}) / s^2.
 * For the central copy the kernel is -erf(alpha s)/s (erfc - 1: its direct 1/s removed), which
 * obeys the same recursion (1/s alone obeys it without the exponential) but cancels near s = 0;
 * there it takes its series, from erf's: -(2/sqrt(pi)) 2^l alpha^{2l+1}
 * sum_j (-1)^j x^{2j} / (j! (2j + 2l + 1)), x = alpha s. */
static void ew_radial(double s, double alpha, int central, double B[4]) {
  const double x = alpha * s;
  if (central && x < 1.0) {
    for (int l = 0; l < 4; ++l) {
      double sum = 0.0, term = 1.0; /* term = (-1)^j x^{2j} / j! */
      for (int j = 0; j < 40; ++j) {
        sum += term / (2 * j + 2 * l + 1);
        term *= -x * x / (j + 1);
      }
      B[l] = -(2.0 / sqrt(M_PI)) * pow(2.0, l) * pow(alpha, 2 * l + 1) * sum;
    }
    return;
  }
  const double e = exp(-x * x) / (alpha * sqrt(M_PI));
  B[0] = central ? -erf(x) / s : erfc(x) / s;
  double t = 1.0;
  for (int l = 1; l < 4; ++l) {
    t *= 2.0 * alpha * alpha;
    B[l] = ((2 * l - 1) * B[l - 1] + t * e) / (s * s);
  }
}

/* acc (n x 3) = the Ewald correction at each position; pot (optional, n) its potential phi.
 * S (optional, xx yy zz xy xz yz) = the box's second moment about c, sum_j m_j d_j d_j^T: the
 * potential kernel psi~ (the sum above, per unit mass) is expanded to second order about c,
 * phi = -G (M psi~ + 1/2 S_ab d_a d_b psi~), a = G grad(M psi~ + 1/2 S_ab d_a d_b psi~), the
 * images taking the derivatives of the same real-space and wave-vector terms. */
void or_ewald(int64_t n, const double* pos, double L, double G, double M, const double* c, const double* S,
              double alpha, int32_t nrep, int32_t hmax2, double* acc, double* pot) {
  const double sp = 2.0 / sqrt(M_PI);
  int hm = 0;
  while ((hm + 1) * (hm + 1) <= hmax2) ++hm;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    double r[3];
    for (int d = 0; d < 3; ++d) {
      r[d] = pos[3 * i + d] - c[d];
      r[d] -= L * nearbyint(r[d] / L);
    }
    double a[3] = {0, 0, 0}, p = 0;
    double aq[3] = {0, 0, 0}, pq = 0; /* the second-moment terms, without G */
    for (int nx = -nrep; nx <= nrep; ++nx)
      for (int ny = -nrep; ny <= nrep; ++ny)
        for (int nz = -nrep; nz <= nrep; ++nz) {
          double sv[3] = {r[0] + nx * L, r[1] + ny * L, r[2] + nz * L};
          double s = sqrt(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]);
          double k, q;
          if (nx == 0 && ny == 0 && nz == 0) {
            k = alpha * alpha * alpha * ew_f0(alpha * s);
            q = alpha * ew_g0(alpha * s);
          } else {
            k = -(erfc(alpha * s) / (s * s * s) + sp * alpha * exp(-alpha * alpha * s * s) / (s * s));
            q = erfc(alpha * s) / s;
          }
          for (int d = 0; d < 3; ++d) a[d] += k * sv[d];
          p += q;
          if (S) {
            double B[4];
            ew_radial(s, alpha, nx == 0 && ny == 0 && nz == 0, B);
            double Ss[3];
            quad_apply(S, sv, Ss);
            const double sSs = sv[0] * Ss[0] + sv[1] * Ss[1] + sv[2] * Ss[2], tr = S[0] + S[1] + S[2];
            for (int d = 0; d < 3; ++d) aq[d] += 0.5 * (tr * sv[d] + 2.0 * Ss[d]) * B[2] - 0.5 * sSs * sv[d] * B[3];
            pq += 0.5 * (-tr * B[1] + sSs * B[2]);
          }
        }
    for (int hx = -hm; hx <= hm; ++hx)
      for (int hy = -hm; hy <= hm; ++hy)
        for (int hz = -hm; hz <= hm; ++hz) {
          int h2 = hx * hx + hy * hy + hz * hz;
          if (h2 == 0 || h2 > hmax2) continue;
          double w = exp(-M_PI * M_PI * h2 / (alpha * alpha * L * L)) / h2;
          double th = 2.0 * M_PI * (hx * r[0] + hy * r[1] + hz * r[2]) / L;
          double sn = sin(th);
          a[0] += -2.0 / (L * L) * w * sn * hx;
          a[1] += -2.0 / (L * L) * w * sn * hy;
          a[2] += -2.0 / (L * L) * w * sn * hz;
          p += w * cos(th) / (M_PI * L);
          if (S) {
            const double hv[3] = {hx, hy, hz};
            double Sh[3];
            quad_apply(S, hv, Sh);
            const double hSh = hx * Sh[0] + hy * Sh[1] + hz * Sh[2];
            for (int d = 0; d < 3; ++d) aq[d] += 4.0 * M_PI * M_PI / (L * L * L * L) * w * hSh * sn * hv[d];
            pq += -2.0 * M_PI / (L * L * L) * w * hSh * cos(th);
          }
        }
    p -= M_PI / (alpha * alpha * L * L * L);
    for (int d = 0; d < 3; ++d) acc[3 * i + d] = G * M * a[d] + G * aq[d];
    if (pot) pot[i] = -G * M * p - G * pq;
  }
}

/* ---- Barnes-Hut interaction lists: the lists of a bucket's work request (Sec. 4.1) ----
 *
 * A bucket is a leaf of the tree; its work request holds a node list and a direct list of id
 * ranges.  From the root, children in ascending node index (their octant order), a node N is
 * taken into bucket B's node list when theta > 0, N's id range does not overlap B's and
 * side(N) < theta * dist(com(N), box(B)) strictly; box(B) is the tight bounding box of B's
 * positions (FP32 values taken exactly into FP64) and dist the Euclidean distance from a point
 * to the box (zero inside), per axis e = lo - c below, c - hi above, else 0, summed as
 * (e_x^2 + e_y^2) + e_z^2 before the square root.  A node that is not taken is, if a leaf, added
 * to the direct list as its id range, and otherwise opened.  Children come from the parent array.
 * Without node_idx / ranges the walk only counts (n_count, r_count per bucket); with them it
 * writes each bucket's lists at n_off[b] and r_off[b].
 */
typedef struct {
  const int32_t* range;
  const double* side;
  const double* com;
  const int32_t* cfirst;
  const int32_t* clist;
  double theta;
  int32_t bf, bc;
  double lo[3], hi[3];
  int32_t* nodes;
  int32_t* ranges;
  int64_t nn, nr;
} walk_state;

static void walk_visit(walk_state* w, int32_t k) {
  const int32_t f = w->range[2 * k], c = w->range[2 * k + 1];
  const int disjoint = f + c <= w->bf || w->bf + w->bc <= f;
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double x = w->com[3 * (size_t)k + d];
    double e = 0.0;
    if (x < w->lo[d]) e = w->lo[d] - x;
    else if (x > w->hi[d]) e = x - w->hi[d];
    s += e * e;
  }
  if (w->theta > 0 && disjoint && w->side[k] < w->theta * sqrt(s)) {
    if (w->nodes) w->nodes[w->nn] = k;
    w->nn++;
  } else if (w->cfirst[k] == w->cfirst[k + 1]) {
    if (w->ranges) {
      w->ranges[2 * w->nr] = f;
      w->ranges[2 * w->nr + 1] = c;
    }
    w->nr++;
  } else {
    for (int32_t q = w->cfirst[k]; q < w->cfirst[k + 1]; ++q) walk_visit(w, w->clist[q]);
  }
}

void or_bh_walk(int32_t n_nodes, const int32_t* node_range, const int32_t* node_parent, const double* side,
                const double* com, const float* rec, int32_t n_buckets, const int32_t* bucket_node, double theta,
                int32_t* n_count, int32_t* r_count, const int64_t* n_off, const int64_t* r_off, int32_t* node_idx,
                int32_t* ranges) {
  int32_t* cfirst = (int32_t*)calloc((size_t)n_nodes + 1, sizeof(int32_t));
  int32_t* clist = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_nodes > 1 ? n_nodes : 1));
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_nodes > 0 ? n_nodes : 1));
  for (int32_t k = 1; k < n_nodes; ++k) cfirst[node_parent[k] + 1]++;
  for (int32_t k = 0; k < n_nodes; ++k) cfirst[k + 1] += cfirst[k];
  for (int32_t k = 0; k < n_nodes; ++k) fill[k] = cfirst[k];
  for (int32_t k = 1; k < n_nodes; ++k) clist[fill[node_parent[k]]++] = k;
#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t b = 0; b < n_buckets; ++b) {
    walk_state w;
    w.range = node_range; w.side = side; w.com = com; w.cfirst = cfirst; w.clist = clist; w.theta = theta;
    w.bf = node_range[2 * bucket_node[b]];
    w.bc = node_range[2 * bucket_node[b] + 1];
    for (int d = 0; d < 3; ++d) { w.lo[d] = INFINITY; w.hi[d] = -INFINITY; }
    for (int32_t i = w.bf; i < w.bf + w.bc; ++i)
      for (int d = 0; d < 3; ++d) {
        const double v = rec[4 * (size_t)i + d];
        if (v < w.lo[d]) w.lo[d] = v;
        if (v > w.hi[d]) w.hi[d] = v;
      }
    w.nodes = node_idx ? node_idx + n_off[b] : NULL;
    w.ranges = ranges ? ranges + 2 * r_off[b] : NULL;
    w.nn = w.nr = 0;
    if (n_nodes > 0) walk_visit(&w, 0);
    if (n_count) n_count[b] = (int32_t)w.nn;
    if (r_count) r_count[b] = (int32_t)w.nr;
  }
  free(cfirst);
  free(clist);
  free(fill);
}
