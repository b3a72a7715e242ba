// d3q19.hpp -- D3Q19 lattice constants and the per-node rules of the sweep,
// as device functions for gfx950.
//
// Population k = i - 1 where i numbers the lattice vectors as the columns of
// the matrix M (Sec. II, eq_deffs); weights from eq_weights.  Every rule is a
// template over the boundary normals, so after unrolling all population
// indices and lattice-vector components are compile-time constants: the 19
// populations of a node live in registers and are never indexed at run time.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

__host__ __device__ constexpr int cx(int k) {
  constexpr int t[19] = {1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0};
  return t[k];
}
__host__ __device__ constexpr int cy(int k) {
  constexpr int t[19] = {0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0};
  return t[k];
}
__host__ __device__ constexpr int cz(int k) {
  constexpr int t[19] = {0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, 0};
  return t[k];
}
// Weight numerators over 36 (eq_weights).
__host__ __device__ constexpr int w36(int k) { return k < 6 ? 2 : (k < 18 ? 1 : 12); }

__host__ __device__ constexpr int index_of(int x, int y, int z) {
  for (int k = 0; k < 19; ++k)
    if (cx(k) == x && cy(k) == y && cz(k) == z) return k;
  return -1;
}
__host__ __device__ constexpr int opp(int k) { return index_of(-cx(k), -cy(k), -cz(k)); }

template <class T>
__device__ __forceinline__ T weight(int k) {
  return T(w36(k)) / T(36);
}

// c_k . n for an integer vector n = (nx, ny, nz).
__host__ __device__ constexpr int dotn(int k, int nx, int ny, int nz) {
  return cx(k) * nx + cy(k) * ny + cz(k) * nz;
}

// Bit mask (bit k) of the populations whose streaming source lies outside the
// domain at a node on boundary face f: c_k . n_f > 0, n_f the inward normal
// of face f (x=0, x=nx-1, y=0, y=ny-1, z=0, z=nz-1).
__host__ __device__ constexpr int face_normal(int f, int axis) {
  return (f / 2 == axis) ? ((f % 2 == 0) ? 1 : -1) : 0;
}
__host__ __device__ constexpr unsigned unknown_mask(int f) {
  unsigned m = 0;
  for (int k = 0; k < 19; ++k)
    if (dotn(k, face_normal(f, 0), face_normal(f, 1), face_normal(f, 2)) > 0) m |= 1u << k;
  return m;
}

// Face velocities in the compute type, indexed by face id (x0,x1,y0,y1,z0,z1).
template <class T>
struct FaceVel {
  T v[6][3];
};

// Per-lattice parameters of the node update.
template <class T>
struct NodeParams {
  unsigned bc_mask;  // bit f: face f is bounded (velocity or pressure BC)
  unsigned p_mask;   // bit f: face f is a pressure face (subset of bc_mask)
  T omega;           // 1 / tau
  T tau_f[3];        // tau * F: velocity shift times rho inside f^eq (body force F)
  FaceVel<T> fv;     // velocity faces: the velocity; pressure faces: the
                     // tangential velocity (normal component zero)
  T rho_p[6];        // prescribed density of each pressure face
  unsigned rule_flags;  // kRuleNoTransverse: face rule without the corrections N
};

// Comparison variant of the face rule: non-equilibrium bounce-back of every
// unknown without the transverse corrections N (Sec. IV, eq_f9NoNs-eq_f17NoNs).
constexpr unsigned kRuleNoTransverse = 1u;

// Velocity (velocity face) or tangential velocity and density (pressure face)
// of the face a node with the single-face mask m lies on.
template <class T>
__device__ __forceinline__ void face_values(unsigned m, const NodeParams<T> &p, T &vx, T &vy, T &vz, T &r0) {
  vx = T(0);
  vy = T(0);
  vz = T(0);
  r0 = T(1);
#pragma unroll
  for (int b = 0; b < 6; ++b)
    if (m == (1u << b)) {
      vx = p.fv.v[b][0];
      vy = p.fv.v[b][1];
      vz = p.fv.v[b][2];
      r0 = p.rho_p[b];
    }
}

// ---------------------------------------------------------------------------
// All rules below act on deviations d_k = f_k - w_k from the rest state.
// Opposite populations have equal weights and the weights of any set of
// links closed under c -> -c or lying in a lattice plane have zero first
// moment, so every rule of the paper keeps its form in d (bounce-back,
// the corrections N, the buried-link averages); only the density picks up
// the weight sum, rho = 1 + sum_k d_k.  Working in d keeps the FP32 and FP16
// forms accurate: the stored numbers are the small deviations, not f ~ w.
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Boundary rules of one node.  m has bit f set when the node lies on boundary
// face f (at most one bit per axis).  The face rule is instantiated per face
// (its unknowns and normal are constants); the edge and corner rule is
// written once for all of them, with the set of unknown populations U, the
// normals and the edge direction as per-lane values and each update a
// select.  Every population index is a compile-time constant, so the 19
// populations stay in registers and are never indexed at run time.  A wave
// whose lanes lie on one or two faces (the ends of x-rows) runs only those
// faces' rules.
//
// Face (one bit; Sec. IV, Appendix; general form of eq_bbshort):
//   rho (1 - v.n) = sum_{c.n=0} f + 2 sum_{c.n<0} f                       (eq_uin)
//                 = 1 + sum_{c.n<=0} d + sum_{c.n<0} d
//   for every unknown j (c_j.n > 0), i = -j:
//   f_j = f_i - 6 w_i rho (c_i.v) - (rho/3) (t_i.v) + 1/2 t_i.M           (eq_bbshort)
//   with t_i = c_i - (c_i.n) n = c_i + n and M = sum_{c.n=0} f c (the
//   in-plane momentum; t_i.M = c_i.M as M is normal to n).  The factor 6 w_i
//   is rho/3 on the normal link (eq_f5) and rho/6 on the diagonals
//   (eq_f9-eq_f17); the last two terms are the corrections N (eq_Nx, eq_Ny).
// Pressure face (Sec. IV eq_rhoin; Appendix): rho = rho0 is prescribed with
// the tangential velocity, and the normal component follows from the same
// bracket, v.n = 1 - (1 + sum_{c.n<=0} d + sum_{c.n<0} d) / rho0; the
// unknowns then take the same formula as above.
// Edge (two bits; Sec. V, eq_Nxzy, eq_edge, eq_buried) and corner (three
// bits; eq_corner), both no-slip:
//   buried links: unknown populations whose opposite is unknown as well
//   (the pair +-(n1 - n2) on an edge, the six c.(n1+n2+n3) = 0 on a corner);
//   every other unknown is bounced back, f_k = f_{-k}; on an edge the four
//   bounced links with c.e != 0 (e the edge direction) also get
//   -(c.e)(f_{+e} - f_{-e})/4, which removes the momentum along the edge;
//   buried links = (sum of the other moving populations) / D with D = 22
//   (edge) or 18 (corner) -- in deviations, the weights' share 22/36 or
//   18/36 cancels against the buried links' own weight 1/36; rest
//   population = 12 times that.  On an edge or corner of a pressure face the
//   buried links and the rest population instead take what the prescribed
//   density leaves, in the ratio of their weights (eq_buried_rho; Sec. V
//   corner form): in deviations (rho0 - 1 - s) / 14 (edge) or / 18 (corner),
//   s the sum of the other moving populations.
// ---------------------------------------------------------------------------
// Face rule of face b (one bit of m; b a compile-time constant, so the set of
// unknowns U, the normal n and every population index are constants and only
// the unknowns' updates are computed).  (vx, vy, vz, r0): the face values
// (the face's parameters, or a per-node field); pressure: b is a pressure
// face.  The sums run in population order and skip only terms that are
// exactly +0 in the masked form of the rule, so the result does not depend
// on whether the face is known at compile time.
template <class T, int b>
__device__ __forceinline__ void face_rule(T (&d)[19], bool pressure, T keep_n, T vx, T vy, T vz, T r0) {
  constexpr unsigned U = unknown_mask(b);
  constexpr int sx = face_normal(b, 0), sy = face_normal(b, 1), sz = face_normal(b, 2);
  T s_known = T(0), s_out = T(0), Mx = T(0), My = T(0), Mz = T(0);
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const bool unk = (U >> k) & 1u;
    const bool out = (U >> opp(k)) & 1u;  // c_k.n < 0
    const bool in_plane = !unk && !out;
    if (!unk) s_known += d[k];
    if (out) s_out += d[k];
    if (cx(k) && in_plane) Mx += T(cx(k)) * d[k];
    if (cy(k) && in_plane) My += T(cy(k)) * d[k];
    if (cz(k) && in_plane) Mz += T(cz(k)) * d[k];
  }
  const T B = T(1) + s_known + s_out;
  T rho = r0;
  if (pressure) {
    const T vn_p = T(1) - B / r0;  // normal velocity from rho0
    vx = vx + T(sx) * vn_p;
    vy = vy + T(sy) * vn_p;
    vz = vz + T(sz) * vn_p;
  }
  const T vn = T(sx) * vx + T(sy) * vy + T(sz) * vz;
  if (!pressure) rho = B / (T(1) - vn);
  const T rho3 = rho / T(3);
#pragma unroll
  for (int j = 0; j < 18; ++j) {
    if (!((U >> j) & 1u)) continue;
    const int i = opp(j);
    const T civ = T(cx(i)) * vx + T(cy(i)) * vy + T(cz(i)) * vz;
    const T ciM = T(cx(i)) * Mx + T(cy(i)) * My + T(cz(i)) * Mz;
    d[j] = d[i] - T(6 * w36(i)) / T(36) * rho * civ + keep_n * (T(0.5) * ciM - rho3 * (civ + vn));
  }
}

// Edge (two bits of m) or corner (three bits), no-slip; the density of a
// bordering pressure face (pmask: the pressure faces among m's faces; at
// most one, as pressure faces lie on one axis) when there is one.
template <class T>
__device__ __forceinline__ void edge_corner_rule(T (&d)[19], unsigned m, const NodeParams<T> &p, unsigned pmask) {
  unsigned U = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b)
    if (m & (1u << b)) U |= unknown_mask(b);
  // Sum of inward normals, one component per axis.
  const int sx = int(m & 1u) - int((m >> 1) & 1u);
  const int sy = int((m >> 2) & 1u) - int((m >> 3) & 1u);
  const int sz = int((m >> 4) & 1u) - int((m >> 5) & 1u);
  const int nb = __popc(m);
  const unsigned pm = m & pmask;
  T r0 = T(1);
#pragma unroll
  for (int b = 0; b < 6; ++b)
    if (pm & (1u << b)) r0 = p.rho_p[b];
  const int ex = (nb == 2 && sx == 0) ? 1 : 0;
  const int ey = (nb == 2 && sy == 0) ? 1 : 0;
  const int ez = (nb == 2 && sz == 0) ? 1 : 0;
  const T Pq = T(0.25) * (T(ex) * (d[0] - d[1]) + T(ey) * (d[2] - d[3]) + T(ez) * (d[4] - d[5]));
  unsigned bur = 0;
#pragma unroll
  for (int k = 0; k < 18; ++k) bur |= ((U >> k) & (U >> opp(k)) & 1u) << k;
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    const bool bounced = ((U & ~bur) >> k) & 1u;
    const int ce = cx(k) * ex + cy(k) * ey + cz(k) * ez;
    const T dk = d[opp(k)] - T(ce) * Pq;
    d[k] = bounced ? dk : d[k];
  }
  T s = T(0);
#pragma unroll
  for (int k = 0; k < 18; ++k) s += ((bur >> k) & 1u) ? T(0) : d[k];
  const T db_v = s / (nb == 2 ? T(22) : T(18));
  const T db_p = (r0 - T(1) - s) / (nb == 2 ? T(14) : T(18));
  const T db = pm ? db_p : db_v;
#pragma unroll
  for (int k = 0; k < 18; ++k) d[k] = ((bur >> k) & 1u) ? db : d[k];
  d[18] = T(12) * db;
}

// Boundary rule of a node with face mask m and given face values (a
// per-node velocity field, or the walls of a complex geometry): each lane
// runs the rule of its own face, edge or corner; a wave runs only the face
// rules its lanes need.  (vx, vy, vz, r0): the face values of a face node;
// not used on edges and corners.  pmask: the pressure faces among m's faces
// (p.p_mask for box faces, 0 for the walls of a complex geometry).
template <class T>
__device__ __forceinline__ void boundary_rule(T (&d)[19], unsigned m, const NodeParams<T> &p, unsigned pmask, T vx,
                                              T vy, T vz, T r0) {
  const T keep_n = (p.rule_flags & kRuleNoTransverse) ? T(0) : T(1);
  if (m == 1u) face_rule<T, 0>(d, (pmask & 1u) != 0u, keep_n, vx, vy, vz, r0);
  if (m == 2u) face_rule<T, 1>(d, (pmask & 2u) != 0u, keep_n, vx, vy, vz, r0);
  if (m == 4u) face_rule<T, 2>(d, (pmask & 4u) != 0u, keep_n, vx, vy, vz, r0);
  if (m == 8u) face_rule<T, 3>(d, (pmask & 8u) != 0u, keep_n, vx, vy, vz, r0);
  if (m == 16u) face_rule<T, 4>(d, (pmask & 16u) != 0u, keep_n, vx, vy, vz, r0);
  if (m == 32u) face_rule<T, 5>(d, (pmask & 32u) != 0u, keep_n, vx, vy, vz, r0);
  if (m & (m - 1u)) edge_corner_rule<T>(d, m, p, pmask);
}

// Boundary rule of a node of a box whose faces take the lattice's face
// parameters (velocity, or tangential velocity and density of a pressure
// face): as boundary_rule, with the face values read directly.
template <class T>
__device__ __forceinline__ void box_boundary_rule(T (&d)[19], unsigned m, const NodeParams<T> &p) {
  const T keep_n = (p.rule_flags & kRuleNoTransverse) ? T(0) : T(1);
#define LBM_FACE(b)                                                                                        \
  if (m == (1u << (b)))                                                                                    \
    face_rule<T, b>(d, ((p.p_mask >> (b)) & 1u) != 0u, keep_n, p.fv.v[b][0], p.fv.v[b][1], p.fv.v[b][2], \
                    p.rho_p[b]);
  LBM_FACE(0)
  LBM_FACE(1)
  LBM_FACE(2)
  LBM_FACE(3)
  LBM_FACE(4)
  LBM_FACE(5)
#undef LBM_FACE
  if (m & (m - 1u)) edge_corner_rule<T>(d, m, p, p.p_mask);
}

// ---------------------------------------------------------------------------
// Wall nodes of a complex geometry (Sec. V) that are not plane, concave-edge
// or corner nodes.  U: bit set of the unknown populations.
//
// Convex edge (eq_edge2): U is the single diagonal n1 + n2 (n1, n2 the
// normals of the two solid faces, pointing into the fluid).  It is bounced
// back; then the momentum along the edge e = n1 x n2, P = sum_j d_j c_j.e,
// is removed from the four populations travelling into the bulk with
// c.e != 0 (c = +-e + n1, +-e + n2): d_c -= (c.e) P / 4.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void convex_edge_rule(T (&d)[19], unsigned U) {
  int sx = 0, sy = 0, sz = 0;  // n1 + n2
#pragma unroll
  for (int k = 6; k < 18; ++k)
    if ((U >> k) & 1u) {
      sx = cx(k);
      sy = cy(k);
      sz = cz(k);
    }
  // e is the axis with no component in n1 + n2 (its sign does not matter).
  const int ex = sx == 0 ? 1 : 0, ey = sy == 0 ? 1 : 0, ez = sz == 0 ? 1 : 0;
  // (+ 0: a select between two plain array elements would be turned into a
  // load through a selected address, which forces the array into scratch.)
#pragma unroll
  for (int k = 6; k < 18; ++k) d[k] = ((U >> k) & 1u) ? d[opp(k)] + T(0) : d[k];
  T P = T(0);
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    const int ce = cx(k) * ex + cy(k) * ey + cz(k) * ez;
    if (ce != 0) P += T(ce) * d[k];
  }
  const T Pq = T(0.25) * P;
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    const int ce = cx(k) * ex + cy(k) * ey + cz(k) * ez;
    const int cs = cx(k) * sx + cy(k) * sy + cz(k) * sz;
    d[k] = (ce != 0 && cs == 1) ? d[k] - T(ce) * Pq : d[k];
  }
}

// Any other wall node (an edge meeting a plane, thin features): bounce back
// every unknown whose opposite is known; the buried links (opposite unknown
// as well) and the rest population take the others' mass in the ratio of the
// lattice weights -- in deviations d_b = w36_b * s / W36, s the sum of the
// non-buried moving deviations, W36 their weight sum in units of 1/36 (22 on
// a concave edge, 18 on a corner, 24 when nothing is buried).
template <class T>
__device__ __forceinline__ void general_wall_rule(T (&d)[19], unsigned U) {
  unsigned bur = 0;
#pragma unroll
  for (int k = 0; k < 18; ++k) bur |= ((U >> k) & (U >> opp(k)) & 1u) << k;
#pragma unroll
  for (int k = 0; k < 18; ++k) d[k] = (((U & ~bur) >> k) & 1u) ? d[opp(k)] + T(0) : d[k];  // + 0: see above
  T s = T(0);
  int W = 0;
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    const bool b = (bur >> k) & 1u;
    s += b ? T(0) : d[k];
    W += b ? 0 : w36(k);
  }
  const T per = s / T(W);
#pragma unroll
  for (int k = 0; k < 18; ++k) d[k] = ((bur >> k) & 1u) ? T(w36(k)) * per : d[k];
  d[18] = T(12) * per;
}

// BGK collision towards the second-order equilibrium (eq_bgk, eq_feq), in
// deviations: rho = 1 + sum d, rho u = sum d c,
//   d_k^eq = f_k^eq - w_k = w_k (rho - 1) + w_k rho (3 c.u + 4.5 (c.u)^2 - 1.5 u^2),
//   d_k <- d_k + omega (d_k^eq - d_k), omega = 1/tau, c_s^2 = 1/3.
// A body force F enters as the velocity shift tau F / rho inside f^eq
// (eq_gravity): u = (sum d c + tau F) / rho.
template <class T>
__device__ __forceinline__ void bgk_collide(T (&d)[19], T omega, const T (&tau_f)[3]) {
  // Moments: partial sums over the populations with c_a = +1, -1 (and, for
  // x, 0); each starts from its first term (0 + x is not foldable under
  // signed zeros, so a zero start would cost an instruction).
  static_assert(cx(0) == 1 && cx(1) == -1 && cy(2) == 1 && cy(3) == -1 && cz(4) == 1 && cz(5) == -1 &&
                    cx(2) == 0 && cx(3) == 0 && cx(4) == 0 && cx(5) == 0,
                "axis populations first (paper order, Sec. II)");
  T xp = d[0], xm = d[1], yp = d[2], ym = d[3], zp = d[4], zm = d[5];
  T x0 = (d[2] + d[3]) + (d[4] + d[5]);
#pragma unroll
  for (int k = 6; k < 19; ++k) {
    if (cx(k) > 0) xp += d[k];
    if (cx(k) < 0) xm += d[k];
    if (cx(k) == 0) x0 += d[k];
    if (cy(k) > 0) yp += d[k];
    if (cy(k) < 0) ym += d[k];
    if (cz(k) > 0) zp += d[k];
    if (cz(k) < 0) zm += d[k];
  }
  const T drho = (xp + xm) + x0;
  const T rho = T(1) + drho;
  // 1 / rho: correctly rounded in double; in float (the FP16 forms, whose
  // storage keeps 11 bits) the hardware reciprocal, within about 1 ulp, in
  // one instruction instead of the ten of a rounded division
  T ir;
  if constexpr (sizeof(T) == 4)
    ir = __builtin_amdgcn_rcpf(rho);
  else
    ir = T(1) / rho;
  const T ux = (xp - xm + tau_f[0]) * ir, uy = (yp - ym + tau_f[1]) * ir, uz = (zp - zm + tau_f[2]) * ir;
  // d_eq = w (drho + rho (3 cu + 4.5 cu^2 - 1.5 u^2)) = w (C + cu (B + A cu)), and
  // d + omega (d_eq - d) = (1 - omega) d + (omega w) (C + cu (B + A cu)).
  const T A = T(4.5) * rho, B = T(3) * rho;
  const T C = drho - T(1.5) * rho * (ux * ux + uy * uy + uz * uz);
  const T keep = T(1) - omega;
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const T ow = omega * weight<T>(k);
    T t = C;
    if (k != 18) {
      // c.u from the non-zero components only
      T cu = cx(k) ? T(cx(k)) * ux : T(cy(k)) * uy;
      if (cx(k) && cy(k)) cu += T(cy(k)) * uy;
      if (cz(k)) cu = (cx(k) || cy(k)) ? cu + T(cz(k)) * uz : T(cz(k)) * uz;
      t = (A * cu + B) * cu + C;
    }
    d[k] = keep * d[k] + ow * t;
  }
}

}  // namespace lbm
