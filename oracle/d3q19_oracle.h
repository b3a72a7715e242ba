/*
 * d3q19_oracle.h -- plain FP64 CPU oracle for the D3Q19 BGK lattice Boltzmann
 * step with the on-site Zou-He velocity boundary condition of Hecht & Harting,
 * "Implementation of on-site velocity boundary conditions for D3Q19 lattice
 * Boltzmann" (arXiv:0811.4593), and its pressure (density) variant.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP path; it is
 * called from tests/, from __graft_entry__.smoke() and from bench.py's
 * cpu_baseline leg, and from nothing else.  It shares no code, header, table
 * or helper with the HIP library.
 *
 * Conventions (the oracle's own; chosen to match the library's public ABI so
 * that arrays can be compared element by element):
 *   node index   n = x + nx*(y + ny*z)
 *   population   k = i - 1, where i = 1..19 is the paper's numbering of the
 *                lattice vectors (Sec. II, eq. eq_deffs); k = 18 is the rest
 *                population i = 19
 *   state array  f[k*N + n], N = nx*ny*nz  (structure of arrays)
 *   faces        0: x=0, 1: x=nx-1, 2: y=0, 3: y=ny-1, 4: z=0, 5: z=nz-1
 *                (paper names: left, right, front, back, bottom, top)
 */
#ifndef D3Q19_ORACLE_H
#define D3Q19_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nx, ny, nz;
  double tau;          /* BGK relaxation time (eq_bgk) */
  int bc_set[6];       /* 1: face carries an on-site velocity BC; an axis with
                          no face set is periodic.  Both faces of an axis must
                          agree. */
  double v[6][3];      /* prescribed velocity per face (v = 0: no-slip) */
  double force[3];     /* body force F, applied as the velocity shift
                          tau*F/rho inside f^eq (eq_gravity); 0 for the plain
                          method */
  int bc_pressure[6];  /* 1: the face (with bc_set) is a pressure face: its
                          density rho_bc is prescribed and v gives the
                          tangential velocity only (eq_rhoin).  Pressure
                          faces must all lie on one axis. */
  double rho_bc[6];    /* prescribed density of a pressure face (> 0) */
  const unsigned char *solid; /* NULL, or [N] flags: 1 = solid node.  A
                          population whose streaming source is a solid node
                          is bounced back at the fluid node (mid-grid
                          bounce-back, Sec. III); solid nodes keep their
                          populations unchanged. */
  const double *face_v[6]; /* NULL, or the per-node velocity of a velocity
                          face, [n_face][3]; face node order: x faces
                          y + ny*z, y faces x + nx*z, z faces x + nx*y */
  int no_transverse;   /* 1: face rule without the transverse corrections N
                          (eq_f9NoNs-eq_f17NoNs; comparison variant) */
  const unsigned char *cell; /* NULL, or [N] node types for complex geometry
                          (Sec. V): 0 fluid, 1 wall node (on-site no-slip),
                          2 solid interior (no populations: a population
                          streaming from it is unknown at the receiving wall
                          node).  With cells, every axis must be periodic
                          (the geometry carries all walls) and solid (the
                          mid-grid option) must be NULL. */
} oracle_lattice;

/* Rule kinds of a wall node, from its set of unknown populations. */
enum {
  ORACLE_NODE_FLUID = 0,       /* no unknowns: no rule */
  ORACLE_NODE_FACE = 1,        /* unknowns of one plane (eq_bbshort, v = 0) */
  ORACLE_NODE_EDGE = 2,        /* concave edge (eq_edge, eq_buried) */
  ORACLE_NODE_CORNER = 3,      /* concave corner (eq_corner) */
  ORACLE_NODE_CONVEX_EDGE = 4, /* convex edge (eq_edge2) */
  ORACLE_NODE_GENERAL = 5      /* any other set, e.g. an edge meeting a plane */
};

/* Lattice tables as the oracle holds them: c[k][3], w[k]. */
void oracle_tables(int c[19][3], double w[19]);

/* f^eq_k(rho, u) (eq_feq, eq_weights), k-ordered. */
void oracle_feq(double rho, const double u[3], double feq[19]);

/* Node rules, applied in place to the 19 post-streaming populations of one
 * node (k-ordered).  Unknown entries may hold anything (NaN included); they
 * are overwritten and never read. */
void oracle_face_rule(int face, const double v[3], double f[19]);
/* Comparison variant of the face rule without the transverse corrections N
 * (eq_f9NoNs-eq_f17NoNs). */
void oracle_face_rule_no_transverse(int face, const double v[3], double f[19]);
void oracle_edge_rule(int face_a, int face_b, double f[19]);
void oracle_corner_rule(int face_a, int face_b, int face_c, double f[19]);

/* The same rules for a pressure face (eq_rhoin and the Appendix forms: the
 * normal velocity follows from rho0; v gives the tangential components) and
 * for edges and corners bordering a pressure face (eq_buried_rho, Sec. V). */
void oracle_face_rule_pressure(int face, double rho0, const double v[3], double f[19]);
void oracle_edge_rule_pressure(int face_a, int face_b, double rho0, double f[19]);
void oracle_corner_rule_pressure(int face_a, int face_b, int face_c, double rho0, double f[19]);

/* Rule kind of the wall node (x, y, z) of a lattice with cells, and its
 * unknown set (bit k: population k).  Returns -1 if the lattice has no
 * cells or the node is not a wall node. */
int oracle_classify(const oracle_lattice *L, int x, int y, int z, unsigned *unknown);

/* The convex-edge and general rules on one node's populations (k-ordered,
 * in place): n1, n2 are the inward normals (face ids) of the two planes;
 * unknown is the bit set of unknown populations. */
void oracle_convex_edge_rule(int face_a, int face_b, double f[19]);
void oracle_general_rule(unsigned unknown, double f[19]);

/* One node: classification, boundary rule, moments, BGK.  pulled[k] is the
 * value streamed into the node along c_k; out[k] the post-collision value.
 * If u_pre is non-NULL it receives the post-boundary, pre-collision velocity
 * sum_k f_k c_k / rho. Returns 0, or -1 if the lattice description is invalid. */
int oracle_update_node(const oracle_lattice *L, int x, int y, int z,
                       const double pulled[19], double out[19], double u_pre[3]);

/* f = f^eq(rho0, u0) at every node. */
void oracle_init(const oracle_lattice *L, double rho0, const double u0[3], double *f);

/* One time step: pull streaming, boundary rules, BGK.  fin and fout are
 * distinct [19][N] arrays.  u_pre (optional, [3][N]) receives the
 * post-boundary, pre-collision velocity of every node.  nthreads <= 0 uses
 * the OpenMP default.  Returns 0, or -1 on an invalid lattice. */
int oracle_step(const oracle_lattice *L, const double *fin, double *fout,
                double *u_pre, int nthreads);

/* rho[n] and u[3][n] of a stored state (eq_rho, eq_vel); either may be NULL. */
void oracle_moments(const oracle_lattice *L, const double *f, double *rho, double *u);

/* Total mass and momentum, summed node by node in index order. */
void oracle_totals(const oracle_lattice *L, const double *f, double *mass, double mom[3]);

#ifdef __cplusplus
}
#endif
#endif
