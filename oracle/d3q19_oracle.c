/*
 * d3q19_oracle.c -- plain FP64 CPU oracle: D3Q19 BGK lattice Boltzmann with
 * the on-site velocity boundary condition of Hecht & Harting
 * (arXiv:0811.4593).
 *
 * The pressure (density) variant of the same boundary condition (eq_rhoin,
 * eq_buried_rho) is included.
 *
 * TEST INFRASTRUCTURE ONLY: called from tests/, __graft_entry__.smoke() and
 * bench.py's cpu_baseline leg.  Shares nothing with the HIP library.
 *
 * Written for reading against the paper, not for speed: populations are kept
 * in 1-based arrays f[1..19] so that every boundary formula below reads like
 * the paper's equation it cites.  Readings of passages that are silent,
 * ambiguous or garbled are marked "Reading:".
 */
#include "d3q19_oracle.h"

#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <string.h>

/* Lattice vectors c_i: the columns of the matrix M (Sec. II, eq_deffs).
 * Entry 0 is unused so that indices match the paper. */
static const int CX[20] = {0, 1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0};
static const int CY[20] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0};
static const int CZ[20] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, 0};

/* Lattice weights (eq_weights). */
static double weight(int i) {
  if (i <= 6) return 2.0 / 36.0;
  if (i <= 18) return 1.0 / 36.0;
  return 12.0 / 36.0;
}

/* Index i of the lattice vector (cx, cy, cz); 0 if it is not one. */
static int vector_index(int cx, int cy, int cz) {
  for (int i = 1; i <= 19; ++i)
    if (CX[i] == cx && CY[i] == cy && CZ[i] == cz) return i;
  return 0;
}

/* Index of the opposite vector, c_{-i} = -c_i. */
static int opposite(int i) { return vector_index(-CX[i], -CY[i], -CZ[i]); }

static int dot_c(int i, const int n[3]) { return CX[i] * n[0] + CY[i] * n[1] + CZ[i] * n[2]; }

/* Inward unit normal of each face (faces: x=0, x=nx-1, y=0, y=ny-1, z=0, z=nz-1). */
static const int NORMAL[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

void oracle_tables(int c[19][3], double w[19]) {
  for (int i = 1; i <= 19; ++i) {
    c[i - 1][0] = CX[i];
    c[i - 1][1] = CY[i];
    c[i - 1][2] = CZ[i];
    w[i - 1] = weight(i);
  }
}

/* Second-order equilibrium, c_s^2 = 1/3 (eq_feq):
 * f_i^eq = w_i rho [1 + c.u/cs^2 + (c.u)^2/(2 cs^4) - u^2/(2 cs^2)]. */
static void feq_paper(double rho, const double u[3], double feq[20]) {
  const double cs2 = 1.0 / 3.0;
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 1; i <= 19; ++i) {
    const double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    feq[i] = weight(i) * rho * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
  }
}

void oracle_feq(double rho, const double u[3], double feq[19]) {
  double e[20];
  feq_paper(rho, u, e);
  for (int i = 1; i <= 19; ++i) feq[i - 1] = e[i];
}

/* ------------------------------------------------------------------------ */
/* Face rules: Sec. IV (bottom plane, eq_uin, eq_f5, eq_f9-eq_f17, eq_Nx,     */
/* eq_Ny) and the Appendix (top, left, right, front, back).  In each rule the */
/* density and the transverse momentum corrections N use known populations */
/* only (in-plane and outgoing), so the unknowns can be assigned after.      */
/*                                                                          */
/* B is the bracket of eq_uin: in-plane populations plus twice the outgoing */
/* ones.  Velocity face (rho0 == NULL): all three velocity components are   */
/* given and rho = B / (1 - v.n) (eq_uin and the Appendix forms).  Pressure */
/* face (rho0 != NULL): rho = rho0 and the tangential components are given; */
/* the normal component follows from B (eq_rhoin, Sec. IV; eq_voutx,         */
/* eq_uinx, eq_uiny, eq_uouty and the top-plane form in the Appendix).  The */
/* unknowns are then computed by the same formulas in both cases.           */
/* ------------------------------------------------------------------------ */

/* z = 0, inward normal +z (Sec. IV). */
static void face_bottom(double *f, double vx, double vy, double vz, const double *rho0, int noN) {
  const double B = f[1] + f[2] + f[3] + f[4] + f[7] + f[8] + f[11] + f[12] + f[19] +
                   2.0 * (f[6] + f[10] + f[14] + f[16] + f[18]);
  double rho;
  if (rho0) {
    rho = *rho0;
    vz = 1.0 - B / rho; /* eq_rhoin */
  } else {
    rho = B / (1.0 - vz); /* eq_uin */
  }
  double Nzx = 0.5 * (f[1] + f[7] + f[8] - (f[2] + f[11] + f[12])) - rho * vx / 3.0;  /* eq_Nx */
  double Nzy = 0.5 * (f[3] + f[7] + f[11] - (f[4] + f[8] + f[12])) - rho * vy / 3.0;  /* eq_Ny */
  if (noN) Nzx = Nzy = 0.0; /* eq_f9NoNs-eq_f17NoNs: no transverse correction */
  f[5] = f[6] + rho * vz / 3.0;                          /* eq_f5 */
  f[9] = f[14] + rho / 6.0 * (vz + vx) - Nzx;            /* eq_f9 */
  f[13] = f[10] + rho / 6.0 * (vz - vx) + Nzx;           /* eq_f13 */
  f[15] = f[18] + rho / 6.0 * (vz + vy) - Nzy;           /* eq_f15 */
  f[17] = f[16] + rho / 6.0 * (vz - vy) + Nzy;           /* eq_f17 */
}

/* z = nz-1, inward normal -z (Appendix, top plane). */
static void face_top(double *f, double vx, double vy, double vz, const double *rho0, int noN) {
  const double B = f[1] + f[2] + f[3] + f[4] + f[7] + f[11] + f[12] + f[8] + f[19] +
                   2.0 * (f[5] + f[9] + f[13] + f[15] + f[17]);
  double rho;
  if (rho0) {
    rho = *rho0;
    vz = -1.0 + B / rho;
  } else {
    rho = B / (vz + 1.0);
  }
  double Nzx = 0.5 * (f[1] + f[7] + f[8] - (f[2] + f[11] + f[12])) - rho * vx / 3.0;
  double Nzy = 0.5 * (f[3] + f[7] + f[11] - (f[4] + f[8] + f[12])) - rho * vy / 3.0;
  if (noN) Nzx = Nzy = 0.0; /* eq_f9NoNs-eq_f17NoNs: no transverse correction */
  f[6] = f[5] - rho * vz / 3.0;
  f[10] = f[13] + rho / 6.0 * (-vz + vx) - Nzx;
  f[14] = f[9] + rho / 6.0 * (-vz - vx) + Nzx;
  f[16] = f[17] + rho / 6.0 * (-vz + vy) - Nzy;
  f[18] = f[15] + rho / 6.0 * (-vz - vy) + Nzy;
}

/* x = 0, inward normal +x (Appendix, left boundary; eq_rhooutx, eq_Nxy, eq_Nxz). */
static void face_left(double *f, double vx, double vy, double vz, const double *rho0, int noN) {
  const double B = f[3] + f[4] + f[5] + f[6] + f[15] + f[16] + f[17] + f[18] + f[19] +
                   2.0 * (f[2] + f[11] + f[12] + f[13] + f[14]);
  double rho;
  if (rho0) {
    rho = *rho0;
    vx = 1.0 - B / rho; /* eq_voutx */
  } else {
    rho = B / (1.0 - vx); /* eq_rhooutx */
  }
  double Nxy = 0.5 * (f[3] + f[15] + f[16] - (f[4] + f[17] + f[18])) - rho * vy / 3.0;
  double Nxz = 0.5 * (f[5] + f[17] + f[15] - (f[6] + f[16] + f[18])) - rho * vz / 3.0;
  if (noN) Nxy = Nxz = 0.0; /* eq_f9NoNs-eq_f17NoNs: no transverse correction */
  f[1] = f[2] + rho * vx / 3.0;
  f[8] = f[11] + rho / 6.0 * (vx - vy) + Nxy;
  f[7] = f[12] + rho / 6.0 * (vx + vy) - Nxy;
  f[9] = f[14] + rho / 6.0 * (vx + vz) - Nxz;
  f[10] = f[13] + rho / 6.0 * (vx - vz) + Nxz;
}

/* x = nx-1, inward normal -x (Appendix, right boundary; eq_rhoinx). */
static void face_right(double *f, double vx, double vy, double vz, const double *rho0, int noN) {
  const double B = f[3] + f[4] + f[5] + f[6] + f[15] + f[16] + f[17] + f[18] + f[19] +
                   2.0 * (f[1] + f[7] + f[8] + f[9] + f[10]);
  double rho;
  if (rho0) {
    rho = *rho0;
    vx = -1.0 + B / rho; /* eq_uinx */
  } else {
    rho = B / (vx + 1.0); /* eq_rhoinx */
  }
  double Nxy = 0.5 * (f[3] + f[15] + f[16] - (f[4] + f[17] + f[18])) - rho * vy / 3.0;
  double Nxz = 0.5 * (f[5] + f[17] + f[15] - (f[6] + f[16] + f[18])) - rho * vz / 3.0;
  if (noN) Nxy = Nxz = 0.0; /* eq_f9NoNs-eq_f17NoNs: no transverse correction */
  f[2] = f[1] - rho * vx / 3.0;
  f[11] = f[8] + rho / 6.0 * (-vx + vy) - Nxy;
  f[12] = f[7] + rho / 6.0 * (-vx - vy) + Nxy;
  f[14] = f[9] + rho / 6.0 * (-vx - vz) + Nxz;
  f[13] = f[10] + rho / 6.0 * (-vx + vz) - Nxz;
}

/* y = 0, inward normal +y (Appendix, front boundary; eq_rhoiny, eq_Nyx, eq_Nyz). */
static void face_front(double *f, double vx, double vy, double vz, const double *rho0, int noN) {
  const double B = f[1] + f[2] + f[5] + f[6] + f[9] + f[10] + f[13] + f[14] + f[19] +
                   2.0 * (f[4] + f[8] + f[12] + f[17] + f[18]);
  double rho;
  if (rho0) {
    rho = *rho0;
    vy = 1.0 - B / rho; /* eq_uiny */
  } else {
    rho = B / (1.0 - vy); /* eq_rhoiny */
  }
  double Nyx = 0.5 * (f[1] + f[9] + f[10] - (f[2] + f[13] + f[14])) - rho * vx / 3.0;
  double Nyz = 0.5 * (f[5] + f[9] + f[13] - (f[6] + f[10] + f[14])) - rho * vz / 3.0;
  if (noN) Nyx = Nyz = 0.0; /* eq_f9NoNs-eq_f17NoNs: no transverse correction */
  f[3] = f[4] + rho * vy / 3.0;
  f[7] = f[12] + rho / 6.0 * (vy + vx) - Nyx;
  f[11] = f[8] + rho / 6.0 * (vy - vx) + Nyx;
  f[15] = f[18] + rho / 6.0 * (vy + vz) - Nyz;
  f[16] = f[17] + rho / 6.0 * (vy - vz) + Nyz;
}

/* y = ny-1, inward normal -y (Appendix, back boundary; eq_rhoouty). */
static void face_back(double *f, double vx, double vy, double vz, const double *rho0, int noN) {
  const double B = f[1] + f[2] + f[5] + f[6] + f[9] + f[10] + f[13] + f[14] + f[19] +
                   2.0 * (f[3] + f[7] + f[11] + f[15] + f[16]);
  double rho;
  if (rho0) {
    rho = *rho0;
    /* eq_uouty.  Reading: the paper labels this component v_x; on the back
     * plane (normal along y) the component fixed by the density is v_y. */
    vy = -1.0 + B / rho;
  } else {
    rho = B / (vy + 1.0); /* eq_rhoouty */
  }
  double Nyx = 0.5 * (f[1] + f[9] + f[10] - (f[2] + f[13] + f[14])) - rho * vx / 3.0;
  double Nyz = 0.5 * (f[5] + f[9] + f[13] - (f[6] + f[10] + f[14])) - rho * vz / 3.0;
  if (noN) Nyx = Nyz = 0.0; /* eq_f9NoNs-eq_f17NoNs: no transverse correction */
  f[4] = f[3] - rho * vy / 3.0;
  f[12] = f[7] + rho / 6.0 * (-vy - vx) + Nyx;
  f[8] = f[11] + rho / 6.0 * (-vy + vx) - Nyx;
  f[18] = f[15] + rho / 6.0 * (-vy - vz) + Nyz;
  f[17] = f[16] + rho / 6.0 * (-vy + vz) - Nyz;
}

/* rho0 == NULL: velocity face; else pressure face with density *rho0 (the
 * normal component of v is then not used).  noN: comparison variant without
 * the transverse corrections (Sec. IV, eq_f9NoNs-eq_f17NoNs: non-equilibrium
 * bounce-back of every unknown, an over-determined system). */
static void face_rule_paper(int face, const double v[3], const double *rho0, int noN, double *f) {
  switch (face) {
    case 0: face_left(f, v[0], v[1], v[2], rho0, noN); break;
    case 1: face_right(f, v[0], v[1], v[2], rho0, noN); break;
    case 2: face_front(f, v[0], v[1], v[2], rho0, noN); break;
    case 3: face_back(f, v[0], v[1], v[2], rho0, noN); break;
    case 4: face_bottom(f, v[0], v[1], v[2], rho0, noN); break;
    case 5: face_top(f, v[0], v[1], v[2], rho0, noN); break;
  }
}

/* ------------------------------------------------------------------------ */
/* Edge rule, no-slip (Sec. V: eq_Nxzy, eq_edge, eq_buried).                 */
/* n1, n2: inward normals of the two planes meeting at the edge.  rho0:      */
/* NULL, or the prescribed density where the edge borders a pressure plane  */
/* (eq_buried_rho).                                                          */
/* ------------------------------------------------------------------------ */
static void edge_rule_paper(const int n1[3], const int n2[3], const double *rho0, double *f) {
  /* Edge direction n1 x n2. */
  const int e[3] = {n1[1] * n2[2] - n1[2] * n2[1], n1[2] * n2[0] - n1[0] * n2[2],
                    n1[0] * n2[1] - n1[1] * n2[0]};
  int bounced[20] = {0};
  int buried[20] = {0};
  /* Buried link: c = +-(n1 - n2); its opposite also points out of the domain. */
  buried[vector_index(n1[0] - n2[0], n1[1] - n2[1], n1[2] - n2[2])] = 1;
  buried[vector_index(n2[0] - n1[0], n2[1] - n1[1], n2[2] - n1[2])] = 1;

  /* Step 1: bounce back every population whose source lies outside the
   * domain (c.n1 > 0 or c.n2 > 0), buried links excepted. */
  for (int i = 1; i <= 18; ++i) {
    const int unknown = dot_c(i, n1) > 0 || dot_c(i, n2) > 0;
    if (unknown && !buried[i]) {
      f[i] = f[opposite(i)];
      bounced[i] = 1;
    }
  }

  /* Step 2: transverse momentum correction along the edge (eq_Nxzy):
   * N = (f_{+e} - f_{-e}) / 4, spread over the four bounced populations with
   * c.e != 0.  Reading: the correction is subtracted, N (c.e), so that the
   * momentum along the edge vanishes (the no-slip the correction is for); adding it as the
   * text literally says would double that momentum instead. */
  const double N = 0.25 * (f[vector_index(e[0], e[1], e[2])] - f[vector_index(-e[0], -e[1], -e[2])]);
  for (int i = 1; i <= 18; ++i)
    if (bounced[i] && dot_c(i, e) != 0) f[i] -= N * dot_c(i, e);

  /* Step 3: buried links and rest population (eq_buried).  Reading of the
   * bracket: 1 - (1 - |c.(n1 x n2)|)(1 - |c.(n1+n2)|/|c|^2), which is 0 for
   * the buried pair and 1 for the other 16 moving populations (6 of weight
   * 2/36 and 10 of weight 1/36, 22/36 in all). */
  const int s[3] = {n1[0] + n2[0], n1[1] + n2[1], n1[2] + n2[2]};
  double sum = 0.0;
  for (int i = 1; i <= 18; ++i) {
    const double c2 = (double)(CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]);
    const double bracket = 1.0 - (1.0 - fabs((double)dot_c(i, e))) * (1.0 - fabs((double)dot_c(i, s) / c2));
    if (bracket != 0.0) sum += f[i] * bracket; /* a zero bracket drops the (unknown) term */
  }
  double fb = sum / 22.0;
  /* Edge of a pressure plane (eq_buried_rho): the buried pair and the rest
   * population take what the prescribed density leaves, in the ratio of
   * their weights, 1 : 1 : 12 (14/36 in all).  Reading: f^(1,2) inside
   * eq_buried_rho is the value eq_buried gives, so 22 f^(1,2) is the sum of
   * the other 16 moving populations and the node's density becomes rho0. */
  if (rho0) fb = (*rho0 - 22.0 * fb) / 14.0;
  for (int i = 1; i <= 18; ++i)
    if (buried[i]) f[i] = fb;
  f[19] = 12.0 * fb; /* w_19 / w_7 = 12 */
}

/* ------------------------------------------------------------------------ */
/* Corner rule, no-slip (Sec. V, eq_corner); rho0 as for the edge rule.    */
/* ------------------------------------------------------------------------ */
static void corner_rule_paper(const int n1[3], const int n2[3], const int n3[3], const double *rho0,
                              double *f) {
  const int s[3] = {n1[0] + n2[0] + n3[0], n1[1] + n2[1] + n3[1], n1[2] + n2[2] + n3[2]};
  /* Bounce back the populations coming from outside whose opposite is known;
   * the six buried vectors are those with c.(n1+n2+n3) = 0. */
  for (int i = 1; i <= 18; ++i) {
    const int unknown = dot_c(i, n1) > 0 || dot_c(i, n2) > 0 || dot_c(i, n3) > 0;
    if (unknown && dot_c(i, s) != 0) f[i] = f[opposite(i)];
  }
  /* eq_corner: weight |c.(n1+n2+n3)| / |c|^2 -- 1 for the six axis vectors
   * and the six non-buried diagonals (18/36 in all), 0 for the buried six. */
  double sum = 0.0;
  for (int i = 1; i <= 18; ++i) {
    const double c2 = (double)(CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]);
    const double weight_i = fabs((double)dot_c(i, s) / c2);
    if (weight_i != 0.0) sum += f[i] * weight_i; /* buried (unknown) terms drop out */
  }
  double fb = sum / 18.0;
  /* Corner of a pressure plane: f~ = rho0/18 - f^(1..6).  Reading: f^(1..6)
   * is the eq_corner value, so the six buried links and the rest population
   * (18/36 of weight in all) take what the prescribed density leaves. */
  if (rho0) fb = *rho0 / 18.0 - fb;
  for (int i = 1; i <= 18; ++i)
    if (dot_c(i, s) == 0) f[i] = fb;
  f[19] = 12.0 * fb;
  /* No momentum correction on corners (Sec. V). */
}

/* ------------------------------------------------------------------------ */
/* Convex edge (Sec. V, eq_edge2).  n1, n2: normals of the two solid faces,   */
/* pointing into the fluid; the fluid surrounds the edge on three sides.    */
/* ------------------------------------------------------------------------ */
static void convex_edge_rule_paper(const int n1[3], const int n2[3], double *f) {
  const int e[3] = {n1[1] * n2[2] - n1[2] * n2[1], n1[2] * n2[0] - n1[0] * n2[2],
                    n1[0] * n2[1] - n1[1] * n2[0]};
  /* Only the population arriving from the solid's interior, along n1 + n2,
   * is unknown: bounce it back (its opposite left into the fluid). */
  const int i_in = vector_index(n1[0] + n2[0], n1[1] + n2[1], n1[2] + n2[2]);
  f[i_in] = f[opposite(i_in)];
  /* eq_edge2: the momentum along the edge, sum_j f_j c_j.e, is spread as
   * -(c_i.e) N, N = (1/4) sum_j f_j c_j.e, over the four populations with
   * c_i.e != 0 that travel into the bulk (c_i = +-e + n1 or +-e + n2).
   * Reading: as for the concave edge, the correction removes the momentum
   * along the edge (slip is reduced, not doubled). */
  double P = 0.0;
  for (int j = 1; j <= 18; ++j) P += f[j] * dot_c(j, e);
  const double N = 0.25 * P;
  for (int i = 1; i <= 18; ++i)
    if (dot_c(i, e) != 0 && dot_c(i, n1) + dot_c(i, n2) == 1) f[i] -= N * dot_c(i, e);
}

/* ------------------------------------------------------------------------ */
/* Any other wall node (Sec. V, points where an edge meets a plane; also     */
/* thin features): bounce back every unknown population whose opposite is   */
/* known; the buried ones (opposite unknown too) and the rest population    */
/* take the mass of the others in the ratio of their lattice weights.       */
/* Reading: the paper sets the rest population of an edge-plane point to     */
/* (12/36) times the sum of the moving populations; that does not return a  */
/* fluid at rest unchanged (it needs w_19 / sum of the moving weights = 1/2),*/
/* so the weight-ratio closure that gives eq_buried's 1/22 and eq_corner's  */
/* 1/18 is used here as well.                                               */
/* ------------------------------------------------------------------------ */
static void general_rule_paper(const int unknown[20], double *f) {
  int buried[20] = {0};
  for (int i = 1; i <= 18; ++i) buried[i] = unknown[i] && unknown[opposite(i)];
  for (int i = 1; i <= 18; ++i)
    if (unknown[i] && !buried[i]) f[i] = f[opposite(i)];
  double sum = 0.0, wsum = 0.0;
  for (int i = 1; i <= 18; ++i)
    if (!buried[i]) {
      sum += f[i];
      wsum += weight(i);
    }
  for (int i = 1; i <= 18; ++i)
    if (buried[i]) f[i] = weight(i) / wsum * sum;
  f[19] = weight(19) / wsum * sum;
}

/* Unknown set and rule kind of a wall node (Sec. V; the per-node normal
 * index of the paper is derived here from the geometry): a plane with
 * inward normal n is a wall of the node when every population arriving
 * along c.n > 0 is unknown. */
static int classify_node(const oracle_lattice *L, int x, int y, int z, int unknown[20], int walls[3], int *nwalls) {
  const int size[3] = {L->nx, L->ny, L->nz};
  int nunk = 0;
  for (int i = 0; i <= 19; ++i) unknown[i] = 0;
  for (int i = 1; i <= 18; ++i) {
    int s[3] = {x - CX[i], y - CY[i], z - CZ[i]};
    for (int a = 0; a < 3; ++a) s[a] = (s[a] + size[a]) % size[a];
    const size_t src = (size_t)s[0] + (size_t)L->nx * ((size_t)s[1] + (size_t)L->ny * s[2]);
    if (L->cell[src] == 2) {
      unknown[i] = 1;
      ++nunk;
    }
  }
  *nwalls = 0;
  int covered[20] = {0};
  for (int fc = 0; fc < 6; ++fc) {
    int all = 1;
    for (int i = 1; i <= 18; ++i)
      if (dot_c(i, NORMAL[fc]) > 0 && !unknown[i]) all = 0;
    if (!all) continue;
    if (*nwalls < 3) walls[*nwalls] = fc;
    ++*nwalls;
    for (int i = 1; i <= 18; ++i)
      if (dot_c(i, NORMAL[fc]) > 0) covered[i] = 1;
  }
  int exact = 1; /* the unknown set is exactly the union of the walls' sets */
  for (int i = 1; i <= 18; ++i)
    if (covered[i] != unknown[i]) exact = 0;
  if (nunk == 0) return ORACLE_NODE_FLUID;
  if (exact && *nwalls >= 1 && *nwalls <= 3) {
    int orth = 1; /* walls on distinct axes */
    for (int p = 0; p < *nwalls; ++p)
      for (int q = p + 1; q < *nwalls; ++q)
        if (walls[p] / 2 == walls[q] / 2) orth = 0;
    if (orth) return *nwalls == 1 ? ORACLE_NODE_FACE : (*nwalls == 2 ? ORACLE_NODE_EDGE : ORACLE_NODE_CORNER);
  }
  if (*nwalls == 0 && nunk == 1) {
    for (int i = 7; i <= 18; ++i)
      if (unknown[i]) {
        /* the unknown diagonal is n1 + n2 */
        int k = 0;
        const int comp[3] = {CX[i], CY[i], CZ[i]};
        for (int a = 0; a < 3; ++a)
          if (comp[a] != 0) walls[k++] = 2 * a + (comp[a] > 0 ? 0 : 1);
        *nwalls = 2;
        return ORACLE_NODE_CONVEX_EDGE;
      }
  }
  return ORACLE_NODE_GENERAL;
}

int oracle_classify(const oracle_lattice *L, int x, int y, int z, unsigned *unknown) {
  if (!L->cell) return -1;
  const size_t n = (size_t)x + (size_t)L->nx * ((size_t)y + (size_t)L->ny * z);
  if (L->cell[n] != 1) return -1;
  int unk[20], walls[3], nw;
  const int kind = classify_node(L, x, y, z, unk, walls, &nw);
  if (unknown) {
    *unknown = 0;
    for (int i = 1; i <= 18; ++i)
      if (unk[i]) *unknown |= 1u << (i - 1);
  }
  return kind;
}

/* ------------------------------------------------------------------------ */
/* Public node-rule entry points (k-ordered arrays).                         */
/* ------------------------------------------------------------------------ */
void oracle_face_rule(int face, const double v[3], double fk[19]) {
  double f[20];
  f[0] = 0.0;
  memcpy(f + 1, fk, 19 * sizeof(double));
  face_rule_paper(face, v, NULL, 0, f);
  memcpy(fk, f + 1, 19 * sizeof(double));
}

void oracle_face_rule_no_transverse(int face, const double v[3], double fk[19]) {
  double f[20];
  f[0] = 0.0;
  memcpy(f + 1, fk, 19 * sizeof(double));
  face_rule_paper(face, v, NULL, 1, f);
  memcpy(fk, f + 1, 19 * sizeof(double));
}

void oracle_edge_rule(int face_a, int face_b, double fk[19]) {
  double f[20];
  f[0] = 0.0;
  memcpy(f + 1, fk, 19 * sizeof(double));
  edge_rule_paper(NORMAL[face_a], NORMAL[face_b], NULL, f);
  memcpy(fk, f + 1, 19 * sizeof(double));
}

void oracle_corner_rule(int face_a, int face_b, int face_c, double fk[19]) {
  double f[20];
  f[0] = 0.0;
  memcpy(f + 1, fk, 19 * sizeof(double));
  corner_rule_paper(NORMAL[face_a], NORMAL[face_b], NORMAL[face_c], NULL, f);
  memcpy(fk, f + 1, 19 * sizeof(double));
}

void oracle_convex_edge_rule(int face_a, int face_b, double fk[19]) {
  double f[20];
  f[0] = 0.0;
  memcpy(f + 1, fk, 19 * sizeof(double));
  convex_edge_rule_paper(NORMAL[face_a], NORMAL[face_b], f);
  memcpy(fk, f + 1, 19 * sizeof(double));
}

void oracle_general_rule(unsigned unknown, double fk[19]) {
  double f[20];
  int unk[20] = {0};
  f[0] = 0.0;
  memcpy(f + 1, fk, 19 * sizeof(double));
  for (int i = 1; i <= 18; ++i) unk[i] = (unknown >> (i - 1)) & 1u;
  general_rule_paper(unk, f);
  memcpy(fk, f + 1, 19 * sizeof(double));
}

void oracle_face_rule_pressure(int face, double rho0, const double v[3], double fk[19]) {
  double f[20];
  f[0] = 0.0;
  memcpy(f + 1, fk, 19 * sizeof(double));
  face_rule_paper(face, v, &rho0, 0, f);
  memcpy(fk, f + 1, 19 * sizeof(double));
}

void oracle_edge_rule_pressure(int face_a, int face_b, double rho0, double fk[19]) {
  double f[20];
  f[0] = 0.0;
  memcpy(f + 1, fk, 19 * sizeof(double));
  edge_rule_paper(NORMAL[face_a], NORMAL[face_b], &rho0, f);
  memcpy(fk, f + 1, 19 * sizeof(double));
}

void oracle_corner_rule_pressure(int face_a, int face_b, int face_c, double rho0, double fk[19]) {
  double f[20];
  f[0] = 0.0;
  memcpy(f + 1, fk, 19 * sizeof(double));
  corner_rule_paper(NORMAL[face_a], NORMAL[face_b], NORMAL[face_c], &rho0, f);
  memcpy(fk, f + 1, 19 * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Lattice bookkeeping.                                                      */
/* ------------------------------------------------------------------------ */
static int lattice_valid(const oracle_lattice *L) {
  const int n[3] = {L->nx, L->ny, L->nz};
  if (L->nx < 1 || L->ny < 1 || L->nz < 1) return 0;
  if (!(L->tau > 0.5)) return 0;
  if (L->cell) {
    if (L->solid) return 0;
    for (int f = 0; f < 6; ++f)
      if (L->bc_set[f]) return 0; /* the geometry carries every wall */
  }
  int pressure_axis = -1;
  for (int a = 0; a < 3; ++a) {
    if (L->bc_set[2 * a] != L->bc_set[2 * a + 1]) return 0;
    if (L->bc_set[2 * a] && n[a] < 3) return 0;
    for (int s = 0; s < 2; ++s) {
      const int face = 2 * a + s;
      if (!L->bc_pressure[face]) continue;
      if (!L->bc_set[face] || !(L->rho_bc[face] > 0.0)) return 0;
      if (L->face_v[face]) return 0; /* per-node velocities are for velocity faces */
      /* Reading: the paper gives edge and corner rules for a pressure plane
       * (in- or outlet) meeting no-slip walls; two pressure planes meeting at
       * an edge are not covered, so pressure planes lie on one axis. */
      if (pressure_axis >= 0 && pressure_axis != a) return 0;
      pressure_axis = a;
    }
  }
  return 1;
}

int oracle_update_node(const oracle_lattice *L, int x, int y, int z, const double pulled[19],
                       double out[19], double u_pre[3]) {
  if (!lattice_valid(L)) return -1;
  double f[20];
  f[0] = 0.0;
  memcpy(f + 1, pulled, 19 * sizeof(double));

  /* Node class: the set of boundary planes the node lies on.  Reading: a
   * plane of a periodic axis is not a boundary; an edge or corner exists only
   * where two or three boundary planes meet, and edges and corners always
   * take the no-slip rules (Sec. IV end, Sec. V: the inflow must decay to
   * zero at the edges), also next to an inflow plane; next to a pressure
   * plane their buried links and rest population take the pressure closure
   * (eq_buried_rho, and its corner form in Sec. V). */
  int faces[3], nf = 0;
  const int coord[3] = {x, y, z};
  const int size[3] = {L->nx, L->ny, L->nz};
  for (int a = 0; a < 3; ++a) {
    if (L->bc_set[2 * a] && coord[a] == 0) faces[nf++] = 2 * a;
    if (L->bc_set[2 * a + 1] && coord[a] == size[a] - 1) faces[nf++] = 2 * a + 1;
  }
  if (L->cell && L->cell[(size_t)x + (size_t)L->nx * ((size_t)y + (size_t)L->ny * z)] == 1) {
    /* Wall node of a complex geometry (Sec. V): the rule follows from the
     * node's unknown populations; every wall is at rest. */
    int unk[20], walls[3], nw;
    const double zero[3] = {0.0, 0.0, 0.0};
    switch (classify_node(L, x, y, z, unk, walls, &nw)) {
      case ORACLE_NODE_FACE: face_rule_paper(walls[0], zero, NULL, 0, f); break;
      case ORACLE_NODE_EDGE: edge_rule_paper(NORMAL[walls[0]], NORMAL[walls[1]], NULL, f); break;
      case ORACLE_NODE_CORNER:
        corner_rule_paper(NORMAL[walls[0]], NORMAL[walls[1]], NORMAL[walls[2]], NULL, f);
        break;
      case ORACLE_NODE_CONVEX_EDGE: convex_edge_rule_paper(NORMAL[walls[0]], NORMAL[walls[1]], f); break;
      case ORACLE_NODE_GENERAL: general_rule_paper(unk, f); break;
      default: break;
    }
    nf = 0; /* no box faces with cells */
  }
  /* The density of the node's pressure plane, if it lies on one (at most
   * one: pressure planes lie on one axis). */
  const double *rho0 = NULL;
  for (int q = 0; q < nf; ++q)
    if (L->bc_pressure[faces[q]]) rho0 = &L->rho_bc[faces[q]];
  if (nf == 1) {
    /* Velocity of the face: uniform, or this node's entry of a per-node
     * field (e.g. the parabolic inflow of eq_pois, Sec. VI). */
    const double *v = L->v[faces[0]];
    const double *fld = L->face_v[faces[0]];
    if (fld) {
      const int a = faces[0] / 2;
      const size_t idx = a == 0 ? (size_t)y + (size_t)L->ny * z
                                : (a == 1 ? (size_t)x + (size_t)L->nx * z : (size_t)x + (size_t)L->nx * y);
      v = fld + 3 * idx;
    }
    face_rule_paper(faces[0], v, rho0, L->no_transverse, f);
  }
  if (nf == 2) edge_rule_paper(NORMAL[faces[0]], NORMAL[faces[1]], rho0, f);
  if (nf == 3) corner_rule_paper(NORMAL[faces[0]], NORMAL[faces[1]], NORMAL[faces[2]], rho0, f);

  /* Moments (eq_rho, eq_vel), then BGK towards f^eq (eq_bgk, eq_feq).  With a
   * body force the velocity inside f^eq is shifted by tau F / rho
   * (eq_gravity). */
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 1; i <= 19; ++i) {
    rho += f[i];
    j[0] += f[i] * CX[i];
    j[1] += f[i] * CY[i];
    j[2] += f[i] * CZ[i];
  }
  const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  if (u_pre) {
    u_pre[0] = u[0];
    u_pre[1] = u[1];
    u_pre[2] = u[2];
  }
  const double ueq[3] = {u[0] + L->tau * L->force[0] / rho, u[1] + L->tau * L->force[1] / rho,
                         u[2] + L->tau * L->force[2] / rho};
  double feq[20];
  feq_paper(rho, ueq, feq);
  for (int i = 1; i <= 19; ++i) out[i - 1] = f[i] - (f[i] - feq[i]) / L->tau;
  return 0;
}

void oracle_init(const oracle_lattice *L, double rho0, const double u0[3], double *f) {
  const size_t N = (size_t)L->nx * L->ny * L->nz;
  double feq[20];
  feq_paper(rho0, u0, feq);
  for (int i = 1; i <= 19; ++i)
    for (size_t n = 0; n < N; ++n) f[(size_t)(i - 1) * N + n] = feq[i];
}

int oracle_step(const oracle_lattice *L, const double *fin, double *fout, double *u_pre, int nthreads) {
  if (!lattice_valid(L)) return -1;
  const int nx = L->nx, ny = L->ny, nz = L->nz;
  const size_t N = (size_t)nx * ny * nz;
  const int periodic[3] = {!L->bc_set[0], !L->bc_set[2], !L->bc_set[4]};
  const int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
  /* Nodes are independent within a step, so the result does not depend on
   * the thread count. */
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int z = 0; z < nz; ++z) {
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        /* Streaming (Sec. II; Sec. III for periodic planes): the population
         * arriving along c_i comes from x - c_i.  A source outside a boundary
         * plane does not exist; its value is unknown (NaN here, so that any
         * use of it would show). */
        double pulled[19];
        for (int i = 1; i <= 19; ++i) {
          int s[3] = {x - CX[i], y - CY[i], z - CZ[i]};
          const int size[3] = {nx, ny, nz};
          int inside = 1;
          for (int a = 0; a < 3; ++a) {
            if (s[a] < 0 || s[a] >= size[a]) {
              if (periodic[a])
                s[a] = (s[a] + size[a]) % size[a];
              else
                inside = 0;
            }
          }
          const size_t src = (size_t)s[0] + (size_t)nx * ((size_t)s[1] + (size_t)ny * s[2]);
          const size_t here = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
          if (!inside || (L->cell && L->cell[src] == 2))
            pulled[i - 1] = NAN; /* unknown: outside the domain or inside a solid */
          else if (L->solid && L->solid[src])
            /* Mid-grid bounce-back (Sec. III): the population sent towards
             * the solid neighbour returns reversed after one step. */
            pulled[i - 1] = fin[(size_t)(opposite(i) - 1) * N + here];
          else
            pulled[i - 1] = fin[(size_t)(i - 1) * N + src];
        }
        const size_t n = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
        if ((L->solid && L->solid[n]) || (L->cell && L->cell[n] == 2)) {
          /* Solid node: not part of the fluid; its populations stay as they are. */
          for (int k = 0; k < 19; ++k) fout[(size_t)k * N + n] = fin[(size_t)k * N + n];
          if (u_pre) u_pre[n] = u_pre[N + n] = u_pre[2 * N + n] = 0.0;
          continue;
        }
        double out[19], up[3];
        oracle_update_node(L, x, y, z, pulled, out, up);
        for (int k = 0; k < 19; ++k) fout[(size_t)k * N + n] = out[k];
        if (u_pre) {
          u_pre[n] = up[0];
          u_pre[N + n] = up[1];
          u_pre[2 * N + n] = up[2];
        }
      }
    }
  }
  return 0;
}

void oracle_moments(const oracle_lattice *L, const double *f, double *rho, double *u) {
  const size_t N = (size_t)L->nx * L->ny * L->nz;
  for (size_t n = 0; n < N; ++n) {
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 1; i <= 19; ++i) {
      const double fi = f[(size_t)(i - 1) * N + n];
      r += fi;
      j[0] += fi * CX[i];
      j[1] += fi * CY[i];
      j[2] += fi * CZ[i];
    }
    if (rho) rho[n] = r;
    if (u) {
      u[n] = j[0] / r;
      u[N + n] = j[1] / r;
      u[2 * N + n] = j[2] / r;
    }
  }
}

void oracle_totals(const oracle_lattice *L, const double *f, double *mass, double mom[3]) {
  const size_t N = (size_t)L->nx * L->ny * L->nz;
  double m = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (size_t n = 0; n < N; ++n) {
    for (int i = 1; i <= 19; ++i) {
      const double fi = f[(size_t)(i - 1) * N + n];
      m += fi;
      j[0] += fi * CX[i];
      j[1] += fi * CY[i];
      j[2] += fi * CZ[i];
    }
  }
  *mass = m;
  mom[0] = j[0];
  mom[1] = j[1];
  mom[2] = j[2];
}
