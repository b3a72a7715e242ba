// lbm_capi.hip -- the C ABI declared in include/lbm.h: handle management,
// argument and state validation, and the launches on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_internal.hpp"
#include "lbm_launch_defaults.hpp"

namespace {

thread_local char g_err[512] = "";

}  // namespace

lbm_status lbm::set_error(lbm_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

namespace {

#define fail lbm::set_error

lbm_status hip_fail(hipError_t e, const char *what) {
  return fail(LBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define LBM_HIP(call, what)                      \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr int kPartialBlocks = 1024;  // fixed grid of the reduction: deterministic order
constexpr size_t kChunkNodes = size_t(1) << 22;  // host transfers are staged in chunks
constexpr int kMaxPlacementBuffers = 8;          // pool size limit of lbm_tune_placement

}  // namespace

struct lbm_lattice {
  int nx, ny, nz;
  size_t N;      // nodes
  size_t pitch;      // population stride in elements (N rounded up to 64)
  size_t buf_elems;  // capacity of each of the two buffers, in elements (>= the layout's need)
  int layout;        // LBM_LAYOUT_* of the state
  lbm::PopLayout lay;
  double tau;
  int storage;
  size_t esize;
  hipStream_t stream;
  void *buf[2];
  int cur;
  bool owns;
  unsigned bc_mask;
  unsigned p_mask;  // pressure faces (subset of bc_mask)
  double v[6][3];
  double rho_p[6];
  double force[3];
  unsigned rule_flags;
  unsigned *d_solid;       // [N] solid words on the device (NodeExt), or nullptr
  double *d_face_v[6];     // per-node face velocities on the device, or nullptr
  unsigned *d_geo;         // complex-geometry node codes on the device, or nullptr
  int block_x, npt, xcd;
  int pass_steps;  // 1 or 2 steps per pass over HBM
  int zc;          // z-planes per workgroup of the two-step pass
  int tile_rows;   // interior rows of its tiles (0: the form's default)
  unsigned long long steps;  // steps taken since creation (its low 32 bits key the stochastic rounding)
  double *d_partials;  // [kPartialBlocks * 4]
  double *d_totals;    // [4]
  double *d_stage;     // [19 * kChunkNodes] doubles, allocated on first use
};

extern "C" {

const char *lbm_last_error(void) { return g_err; }

size_t lbm_population_pitch(size_t nodes) { return lbm::population_pitch(nodes); }

size_t lbm_buffer_elements(int nx, int ny, int nz, lbm_storage storage, int layout) {
  const size_t esize = lbm_element_bytes(storage);
  if (nx < 1 || ny < 1 || nz < 1 || esize == 0) return 0;
  if (layout != LBM_LAYOUT_POPULATION_MAJOR && layout != LBM_LAYOUT_ROW_MAJOR) return 0;
  return lbm::buffer_elements(layout, nx, ny, nz, esize);
}

size_t lbm_element_bytes(lbm_storage storage) {
  switch (storage) {
    case LBM_STORE_F64: return 8;
    case LBM_STORE_F32: return 4;
    case LBM_STORE_F16_DEV: return 2;
    case LBM_STORE_F16_DEV_SR: return 2;
  }
  return 0;
}

static lbm_status validate_create(int nx, int ny, int nz, double tau, double rho0, lbm_storage storage,
                                  lbm_lattice **out) {
  if (!out) return fail(LBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1) return fail(LBM_ERR_ARG, "lattice sizes must be >= 1 (got %d x %d x %d)", nx, ny, nz);
  const double n = double(nx) * double(ny) * double(nz);
  if (n >= 2147483648.0) return fail(LBM_ERR_ARG, "lattice has %.0f nodes; at most 2^31 - 1 are supported", n);
  if (!(tau > 0.5) || !std::isfinite(tau)) return fail(LBM_ERR_ARG, "tau must be > 1/2 (got %g)", tau);
  if (!(rho0 > 0.0) || !std::isfinite(rho0)) return fail(LBM_ERR_ARG, "rho0 must be > 0 (got %g)", rho0);
  if (lbm_element_bytes(storage) == 0) return fail(LBM_ERR_ARG, "invalid storage form %d", int(storage));
  return LBM_OK;
}

static constexpr int kDefaultZPlanes = 64;

static void default_launch(lbm_lattice *L) {
  // One node per thread, each XCD on its own eighth of the lattice, the
  // block width by row length (256 threads is the fastest shape measured on
  // the 1024 x 512 x 512 duct).  lbm_set_launch and lbm_autotune override it.
  L->block_x = lbm::default_block_x(L->nx);
  L->npt = 1;
  L->xcd = LBM_XCD_SLABS;
  L->pass_steps = 1;
  L->zc = kDefaultZPlanes;
  L->tile_rows = 0;
}

static lbm_status finish_create(lbm_lattice *L, double rho0, const double u0[3], lbm_lattice **out) {
  const double zero[3] = {0.0, 0.0, 0.0};
  if (!u0) u0 = zero;
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(u0[d])) return fail(LBM_ERR_ARG, "u0 is not finite");
  hipError_t e = hipMalloc(&L->d_partials, sizeof(double) * (kPartialBlocks * 4 + 4));
  if (e != hipSuccess) return fail(LBM_ERR_OOM, "hipMalloc of reduction scratch failed: %s", hipGetErrorString(e));
  L->d_totals = L->d_partials + kPartialBlocks * 4;
  e = lbm::launch_init(L->storage, L->buf[0], L->N, L->lay, rho0, u0, L->stream);
  if (e != hipSuccess) return hip_fail(e, "init launch");
  e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "init");
  *out = L;
  g_err[0] = '\0';
  return LBM_OK;
}

lbm_status lbm_create(int nx, int ny, int nz, double tau, double rho0, const double u0[3], lbm_storage storage,
                      void *hip_stream, lbm_lattice **out) {
  lbm_status st = validate_create(nx, ny, nz, tau, rho0, storage, out);
  if (st != LBM_OK) return st;
  lbm_lattice *L = new (std::nothrow) lbm_lattice();
  if (!L) return fail(LBM_ERR_OOM, "host allocation failed");
  L->nx = nx;
  L->ny = ny;
  L->nz = nz;
  L->N = size_t(nx) * ny * nz;
  L->pitch = lbm::population_pitch(L->N);
  L->tau = tau;
  L->storage = int(storage);
  L->esize = lbm_element_bytes(storage);
  L->stream = static_cast<hipStream_t>(hip_stream);
  L->owns = true;
  // The library's buffers start row-major (rows padded to cache lines, the
  // faster layout for the sweep) and hold either layout.
  L->layout = LBM_LAYOUT_ROW_MAJOR;
  L->lay = lbm::row_major(nx, L->esize);
  L->buf_elems = std::max(19 * L->pitch, lbm::buffer_elements(LBM_LAYOUT_ROW_MAJOR, nx, ny, nz, L->esize));
  default_launch(L);
  const size_t bytes = L->buf_elems * L->esize;
  for (int i = 0; i < 2; ++i) {
    hipError_t e = hipMalloc(&L->buf[i], bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      lbm_destroy(L);
      return fail(LBM_ERR_OOM, "hipMalloc of %zu bytes for populations failed: %s", bytes, hipGetErrorString(e));
    }
  }
  st = finish_create(L, rho0, u0, out);
  if (st != LBM_OK) lbm_destroy(L);
  return st;
}

lbm_status lbm_create_on_buffers(int nx, int ny, int nz, double tau, double rho0, const double u0[3],
                                 lbm_storage storage, void *hip_stream, void *buf_a, void *buf_b, size_t buf_bytes,
                                 lbm_lattice **out) {
  lbm_status st = validate_create(nx, ny, nz, tau, rho0, storage, out);
  if (st != LBM_OK) return st;
  const size_t need = 19 * lbm::population_pitch(size_t(nx) * ny * nz) * lbm_element_bytes(storage);
  if (!buf_a || !buf_b || buf_a == buf_b) return fail(LBM_ERR_ARG, "two distinct device buffers are required");
  if (buf_bytes < need) return fail(LBM_ERR_ARG, "buffers hold %zu bytes, %zu needed", buf_bytes, need);
  if ((reinterpret_cast<uintptr_t>(buf_a) | reinterpret_cast<uintptr_t>(buf_b)) & 255u)
    return fail(LBM_ERR_ARG, "buffers must be 256-byte aligned");
  lbm_lattice *L = new (std::nothrow) lbm_lattice();
  if (!L) return fail(LBM_ERR_OOM, "host allocation failed");
  L->nx = nx;
  L->ny = ny;
  L->nz = nz;
  L->N = size_t(nx) * ny * nz;
  L->pitch = lbm::population_pitch(L->N);
  L->layout = LBM_LAYOUT_POPULATION_MAJOR;  // the caller's buffers: k*P + n until lbm_set_layout
  L->lay = lbm::population_major(L->N, nx);
  L->tau = tau;
  L->storage = int(storage);
  L->esize = lbm_element_bytes(storage);
  L->stream = static_cast<hipStream_t>(hip_stream);
  L->owns = false;
  L->buf_elems = buf_bytes / L->esize;
  L->buf[0] = buf_a;
  L->buf[1] = buf_b;
  default_launch(L);
  st = finish_create(L, rho0, u0, out);
  if (st != LBM_OK) lbm_destroy(L);
  return st;
}

void lbm_destroy(lbm_lattice *L) {
  if (!L) return;
  if (L->stream) (void)hipStreamSynchronize(L->stream);
  else (void)hipDeviceSynchronize();
  if (L->owns) {
    for (int i = 0; i < 2; ++i)
      if (L->buf[i]) (void)hipFree(L->buf[i]);
  }
  if (L->d_partials) (void)hipFree(L->d_partials);
  if (L->d_solid) (void)hipFree(L->d_solid);
  if (L->d_geo) (void)hipFree(L->d_geo);
  for (int f = 0; f < 6; ++f)
    if (L->d_face_v[f]) (void)hipFree(L->d_face_v[f]);
  if (L->d_stage) (void)hipFree(L->d_stage);
  delete L;
}

static const int kNormal[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

static void drop_face_field(lbm_lattice *L, int f) {
  if (L->d_face_v[f]) (void)hipFree(L->d_face_v[f]);
  L->d_face_v[f] = nullptr;
}

lbm_status lbm_set_velocity_bc(lbm_lattice *L, lbm_face face, const double u[3]) {
  if (!L || !u) return fail(LBM_ERR_ARG, "NULL argument");
  const int f = int(face);
  if (f < 0 || f > 5) return fail(LBM_ERR_ARG, "invalid face %d", f);
  const int size[3] = {L->nx, L->ny, L->nz};
  if (size[f / 2] < 3) return fail(LBM_ERR_ARG, "a bounded axis needs at least 3 nodes (axis %d has %d)", f / 2, size[f / 2]);
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(u[d])) return fail(LBM_ERR_ARG, "velocity is not finite");
  const double un = u[0] * kNormal[f][0] + u[1] * kNormal[f][1] + u[2] * kNormal[f][2];
  if (std::fabs(un) >= 1.0) return fail(LBM_ERR_ARG, "|u.n| = %g >= 1: the boundary density diverges", std::fabs(un));
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  if (uu >= 1.0 / 3.0) return fail(LBM_ERR_ARG, "|u| = %g is not below the speed of sound 1/sqrt(3)", std::sqrt(uu));
  L->bc_mask |= 1u << f;
  L->p_mask &= ~(1u << f);
  L->rho_p[f] = 0.0;
  for (int d = 0; d < 3; ++d) L->v[f][d] = u[d];
  drop_face_field(L, f);
  return LBM_OK;
}

lbm_status lbm_set_pressure_bc(lbm_lattice *L, lbm_face face, double rho0, const double u_t[3]) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  const int f = int(face);
  if (f < 0 || f > 5) return fail(LBM_ERR_ARG, "invalid face %d", f);
  const int size[3] = {L->nx, L->ny, L->nz};
  if (size[f / 2] < 3) return fail(LBM_ERR_ARG, "a bounded axis needs at least 3 nodes (axis %d has %d)", f / 2, size[f / 2]);
  if (!std::isfinite(rho0) || !(rho0 > 0.0)) return fail(LBM_ERR_ARG, "density %g is not a positive finite number", rho0);
  double t[3] = {0.0, 0.0, 0.0};
  if (u_t) {
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(u_t[d])) return fail(LBM_ERR_ARG, "velocity is not finite");
    // Keep the tangential part; the normal component is computed each step.
    const double un = u_t[0] * kNormal[f][0] + u_t[1] * kNormal[f][1] + u_t[2] * kNormal[f][2];
    for (int d = 0; d < 3; ++d) t[d] = u_t[d] - un * kNormal[f][d];
  }
  const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  if (tt >= 1.0 / 3.0) return fail(LBM_ERR_ARG, "|u_t| = %g is not below the speed of sound 1/sqrt(3)", std::sqrt(tt));
  L->bc_mask |= 1u << f;
  L->p_mask |= 1u << f;
  L->rho_p[f] = rho0;
  for (int d = 0; d < 3; ++d) L->v[f][d] = t[d];
  drop_face_field(L, f);
  return LBM_OK;
}

lbm_status lbm_clear_bc(lbm_lattice *L, lbm_face face) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  const int f = int(face);
  if (f < 0 || f > 5) return fail(LBM_ERR_ARG, "invalid face %d", f);
  L->bc_mask &= ~(1u << f);
  L->p_mask &= ~(1u << f);
  L->rho_p[f] = 0.0;
  for (int d = 0; d < 3; ++d) L->v[f][d] = 0.0;
  drop_face_field(L, f);
  return LBM_OK;
}

static size_t face_nodes(const lbm_lattice *L, int f) {
  const int a = f / 2;
  return a == 0 ? size_t(L->ny) * L->nz : (a == 1 ? size_t(L->nx) * L->nz : size_t(L->nx) * L->ny);
}

lbm_status lbm_set_velocity_field(lbm_lattice *L, lbm_face face, const double *v) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  const int f = int(face);
  if (f < 0 || f > 5) return fail(LBM_ERR_ARG, "invalid face %d", f);
  if (!v) {
    drop_face_field(L, f);
    return LBM_OK;
  }
  const int size[3] = {L->nx, L->ny, L->nz};
  if (size[f / 2] < 3) return fail(LBM_ERR_ARG, "a bounded axis needs at least 3 nodes (axis %d has %d)", f / 2, size[f / 2]);
  const size_t nf = face_nodes(L, f);
  for (size_t i = 0; i < nf; ++i) {
    const double *u = v + 3 * i;
    if (!std::isfinite(u[0]) || !std::isfinite(u[1]) || !std::isfinite(u[2]))
      return fail(LBM_ERR_ARG, "velocity of face node %zu is not finite", i);
    const double un = u[0] * kNormal[f][0] + u[1] * kNormal[f][1] + u[2] * kNormal[f][2];
    if (std::fabs(un) >= 1.0 || u[0] * u[0] + u[1] * u[1] + u[2] * u[2] >= 1.0 / 3.0)
      return fail(LBM_ERR_ARG, "velocity of face node %zu out of range (|u.n| < 1 and |u| < 1/sqrt(3) required)", i);
  }
  if (!L->d_face_v[f]) {
    hipError_t e = hipMalloc(&L->d_face_v[f], sizeof(double) * 3 * nf);
    if (e != hipSuccess) {
      L->d_face_v[f] = nullptr;
      return fail(LBM_ERR_OOM, "hipMalloc of a face velocity field failed: %s", hipGetErrorString(e));
    }
  }
  hipError_t e = hipMemcpyAsync(L->d_face_v[f], v, sizeof(double) * 3 * nf, hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "face velocity upload");
  L->bc_mask |= 1u << f;
  L->p_mask &= ~(1u << f);
  L->rho_p[f] = 0.0;
  return LBM_OK;
}

lbm_status lbm_set_solid_mask(lbm_lattice *L, const unsigned char *solid) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (!solid) {
    if (L->d_solid) (void)hipFree(L->d_solid);
    L->d_solid = nullptr;
    return LBM_OK;
  }
  if (!L->d_solid) {
    hipError_t e = hipMalloc(&L->d_solid, L->N * sizeof(unsigned));
    if (e != hipSuccess) {
      L->d_solid = nullptr;
      return fail(LBM_ERR_OOM, "hipMalloc of the solid mask failed: %s", hipGetErrorString(e));
    }
  }
  // One word per node: which of its 18 moving populations stream in from a
  // solid node (source at -c_k, periodic wrap, as the sweep's gather), and
  // whether it is solid itself (any non-zero flag counts).
  const int nx = L->nx, ny = L->ny, nz = L->nz;
  std::vector<unsigned> words(L->N);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t n = size_t(x) + size_t(nx) * (size_t(y) + size_t(ny) * size_t(z));
        unsigned w = solid[n] ? (1u << lbm::kSolidSelfBit) : 0u;
        for (int k = 0; k < 18; ++k) {
          int xs = x - lbm::cx(k), ys = y - lbm::cy(k), zs = z - lbm::cz(k);
          xs += xs < 0 ? nx : (xs >= nx ? -nx : 0);
          ys += ys < 0 ? ny : (ys >= ny ? -ny : 0);
          zs += zs < 0 ? nz : (zs >= nz ? -nz : 0);
          if (solid[size_t(xs) + size_t(nx) * (size_t(ys) + size_t(ny) * size_t(zs))]) w |= 1u << k;
        }
        words[n] = w;
      }
  hipError_t e = hipMemcpyAsync(L->d_solid, words.data(), L->N * sizeof(unsigned), hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "solid mask upload");
  return LBM_OK;
}

static lbm_status check_cells(const unsigned char *cell, size_t N) {
  for (size_t n = 0; n < N; ++n)
    if (cell[n] > 2) return fail(LBM_ERR_ARG, "node type %d at node %zu (0 fluid, 1 wall, 2 solid)", int(cell[n]), n);
  return LBM_OK;
}

lbm_status lbm_classify_geometry(int nx, int ny, int nz, const unsigned char *cell, unsigned *code,
                                 long long counts[5]) {
  if (!cell || !code) return fail(LBM_ERR_ARG, "NULL argument");
  if (nx < 1 || ny < 1 || nz < 1) return fail(LBM_ERR_ARG, "lattice sizes must be >= 1");
  if (double(nx) * ny * nz >= 2147483648.0) return fail(LBM_ERR_ARG, "at most 2^31 - 1 nodes");
  const lbm_status st = check_cells(cell, size_t(nx) * ny * nz);
  if (st != LBM_OK) return st;
  lbm::classify_geometry(nx, ny, nz, cell, code, counts);
  return LBM_OK;
}

lbm_status lbm_set_geometry(lbm_lattice *L, const unsigned char *cell) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (!cell) {
    if (L->d_geo) (void)hipFree(L->d_geo);
    L->d_geo = nullptr;
    return LBM_OK;
  }
  const lbm_status st = check_cells(cell, L->N);
  if (st != LBM_OK) return st;
  std::vector<unsigned> code(L->N);
  lbm::classify_geometry(L->nx, L->ny, L->nz, cell, code.data(), nullptr);
  if (!L->d_geo) {
    hipError_t e = hipMalloc(&L->d_geo, sizeof(unsigned) * L->N);
    if (e != hipSuccess) {
      L->d_geo = nullptr;
      return fail(LBM_ERR_OOM, "hipMalloc of the geometry codes failed: %s", hipGetErrorString(e));
    }
  }
  hipError_t e = hipMemcpyAsync(L->d_geo, code.data(), sizeof(unsigned) * L->N, hipMemcpyHostToDevice, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e, "geometry upload");
  return LBM_OK;
}

lbm_status lbm_set_rule_options(lbm_lattice *L, unsigned flags) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (flags & ~unsigned(LBM_RULE_NO_TRANSVERSE)) return fail(LBM_ERR_ARG, "unknown rule option bits 0x%x", flags);
  L->rule_flags = flags;
  return LBM_OK;
}

lbm_status lbm_set_body_force(lbm_lattice *L, const double F[3]) {
  if (!L || !F) return fail(LBM_ERR_ARG, "NULL argument");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(F[d])) return fail(LBM_ERR_ARG, "force is not finite");
  for (int d = 0; d < 3; ++d) L->force[d] = F[d];
  return LBM_OK;
}

static lbm::SweepConfig sweep_config(const lbm_lattice *L) {
  lbm::SweepConfig c;
  c.storage = L->storage;
  c.nx = L->nx;
  c.ny = L->ny;
  c.nz = L->nz;
  c.layout = L->lay;
  c.tau = L->tau;
  c.bc_mask = L->bc_mask;
  c.p_mask = L->p_mask;
  std::memcpy(c.v, L->v, sizeof(c.v));
  std::memcpy(c.rho_p, L->rho_p, sizeof(c.rho_p));
  std::memcpy(c.force, L->force, sizeof(c.force));
  c.rule_flags = L->rule_flags;
  c.solid = L->d_solid;
  c.geo_code = L->d_geo;
  for (int f = 0; f < 6; ++f) c.face_v[f] = L->d_face_v[f];
  c.block_x = L->block_x;
  c.nodes_per_thread = L->npt;
  c.xcd_remap = L->xcd;
  c.step = unsigned(L->steps);
  return c;
}

lbm_status lbm_step(lbm_lattice *L, int nsteps) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps must be >= 0");
  for (int a = 0; a < 3; ++a) {
    const unsigned bits = (L->bc_mask >> (2 * a)) & 3u;
    if (bits == 1u || bits == 2u)
      return fail(LBM_ERR_STATE, "axis %d has a BC on one face only; set both faces or none", a);
  }
  if (L->d_geo && L->bc_mask)
    return fail(LBM_ERR_STATE, "a lattice with a complex geometry carries its walls in the geometry; clear the face BCs");
  if (L->d_geo && L->d_solid) return fail(LBM_ERR_STATE, "a complex geometry and a solid mask cannot be combined");
  int p_axes = 0;
  for (int a = 0; a < 3; ++a) p_axes += ((L->p_mask >> (2 * a)) & 3u) != 0u;
  if (p_axes > 1)
    return fail(LBM_ERR_STATE, "pressure faces on %d axes: edges between two pressure faces are not defined", p_axes);
  lbm::SweepConfig c = sweep_config(L);
  const bool ext = L->d_solid || L->d_geo || L->d_face_v[0] || L->d_face_v[1] || L->d_face_v[2] ||
                   L->d_face_v[3] || L->d_face_v[4] || L->d_face_v[5];
  const bool two = L->pass_steps == 2 && L->layout == LBM_LAYOUT_ROW_MAJOR && !ext;
  for (int s = 0; s < nsteps;) {
    c.step = unsigned(L->steps);
    const bool pair = two && nsteps - s >= 2;
    hipError_t e = pair ? lbm::launch_sweep2(c, L->zc, L->tile_rows, L->buf[L->cur], L->buf[L->cur ^ 1], L->stream)
                        : lbm::launch_sweep(c, L->buf[L->cur], L->buf[L->cur ^ 1], false, L->stream);
    if (e != hipSuccess) return hip_fail(e, pair ? "two-step sweep launch" : "sweep launch");
    L->cur ^= 1;
    L->steps += pair ? 2 : 1;
    s += pair ? 2 : 1;
  }
  return LBM_OK;
}

static lbm_status ensure_stage(lbm_lattice *L) {
  if (L->d_stage) return LBM_OK;
  hipError_t e = hipMalloc(&L->d_stage, sizeof(double) * 19 * kChunkNodes);
  if (e != hipSuccess) {
    L->d_stage = nullptr;
    return fail(LBM_ERR_OOM, "hipMalloc of the staging buffer failed: %s", hipGetErrorString(e));
  }
  return LBM_OK;
}

lbm_status lbm_moments(lbm_lattice *L, double *rho, double *u, int dst_on_device) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (!rho && !u) return LBM_OK;
  const void *f = L->buf[L->cur];
  if (dst_on_device) {
    LBM_HIP(lbm::launch_moments(L->storage, f, L->lay, 0, L->N, rho, u, nullptr, kPartialBlocks, L->stream),
            "moments launch");
    LBM_HIP(hipStreamSynchronize(L->stream), "moments");
    return LBM_OK;
  }
  lbm_status st = ensure_stage(L);
  if (st != LBM_OK) return st;
  for (size_t n0 = 0; n0 < L->N; n0 += kChunkNodes) {
    const size_t cnt = (L->N - n0) < kChunkNodes ? (L->N - n0) : kChunkNodes;
    double *drho = L->d_stage, *du = L->d_stage + cnt;
    LBM_HIP(lbm::launch_moments(L->storage, f, L->lay, n0, cnt, rho ? drho : nullptr, u ? du : nullptr, nullptr,
                                kPartialBlocks, L->stream),
            "moments launch");
    if (rho) LBM_HIP(hipMemcpyAsync(rho + n0, drho, cnt * sizeof(double), hipMemcpyDeviceToHost, L->stream), "copy rho");
    if (u)
      for (int a = 0; a < 3; ++a)
        LBM_HIP(hipMemcpyAsync(u + a * L->N + n0, du + a * cnt, cnt * sizeof(double), hipMemcpyDeviceToHost,
                               L->stream),
                "copy u");
    LBM_HIP(hipStreamSynchronize(L->stream), "moments");
  }
  return LBM_OK;
}

lbm_status lbm_totals(lbm_lattice *L, double *mass, double momentum[3]) {
  if (!L || !mass || !momentum) return fail(LBM_ERR_ARG, "NULL argument");
  LBM_HIP(lbm::launch_moments(L->storage, L->buf[L->cur], L->lay, 0, L->N, nullptr, nullptr, L->d_partials,
                              kPartialBlocks, L->stream),
          "totals launch");
  LBM_HIP(lbm::launch_reduce(L->d_partials, kPartialBlocks, L->d_totals, L->stream), "reduce launch");
  double h[4];
  LBM_HIP(hipMemcpyAsync(h, L->d_totals, sizeof(h), hipMemcpyDeviceToHost, L->stream), "copy totals");
  LBM_HIP(hipStreamSynchronize(L->stream), "totals");
  *mass = h[0];
  momentum[0] = h[1];
  momentum[1] = h[2];
  momentum[2] = h[3];
  for (int c = 0; c < 4; ++c)
    if (!std::isfinite(h[c])) return fail(LBM_ERR_NONFINITE, "the state holds NaN or Inf (totals not finite)");
  return LBM_OK;
}

lbm_status lbm_get_populations(lbm_lattice *L, double *f) {
  if (!L || !f) return fail(LBM_ERR_ARG, "NULL argument");
  lbm_status st = ensure_stage(L);
  if (st != LBM_OK) return st;
  for (size_t n0 = 0; n0 < L->N; n0 += kChunkNodes) {
    const size_t cnt = (L->N - n0) < kChunkNodes ? (L->N - n0) : kChunkNodes;
    LBM_HIP(lbm::launch_to_double(L->storage, L->buf[L->cur], L->lay, n0, cnt, L->d_stage, L->stream),
            "convert launch");
    for (int k = 0; k < 19; ++k)
      LBM_HIP(hipMemcpyAsync(f + size_t(k) * L->N + n0, L->d_stage + size_t(k) * cnt, cnt * sizeof(double),
                             hipMemcpyDeviceToHost, L->stream),
              "copy populations");
    LBM_HIP(hipStreamSynchronize(L->stream), "get populations");
  }
  return LBM_OK;
}

lbm_status lbm_set_populations(lbm_lattice *L, const double *f) {
  if (!L || !f) return fail(LBM_ERR_ARG, "NULL argument");
  lbm_status st = ensure_stage(L);
  if (st != LBM_OK) return st;
  for (size_t n0 = 0; n0 < L->N; n0 += kChunkNodes) {
    const size_t cnt = (L->N - n0) < kChunkNodes ? (L->N - n0) : kChunkNodes;
    for (int k = 0; k < 19; ++k)
      LBM_HIP(hipMemcpyAsync(L->d_stage + size_t(k) * cnt, f + size_t(k) * L->N + n0, cnt * sizeof(double),
                             hipMemcpyHostToDevice, L->stream),
              "copy populations");
    LBM_HIP(lbm::launch_from_double(L->storage, L->buf[L->cur], L->lay, n0, cnt, L->d_stage, L->stream),
            "convert launch");
    LBM_HIP(hipStreamSynchronize(L->stream), "set populations");
  }
  return LBM_OK;
}

lbm_status lbm_set_layout(lbm_lattice *L, int layout) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (layout != LBM_LAYOUT_POPULATION_MAJOR && layout != LBM_LAYOUT_ROW_MAJOR)
    return fail(LBM_ERR_ARG, "layout must be LBM_LAYOUT_POPULATION_MAJOR or LBM_LAYOUT_ROW_MAJOR (got %d)", layout);
  if (layout == L->layout) return LBM_OK;
  const lbm::PopLayout to =
      layout == LBM_LAYOUT_ROW_MAJOR ? lbm::row_major(L->nx, L->esize) : lbm::population_major(L->N, L->nx);
  const size_t need = lbm::buffer_elements(layout, L->nx, L->ny, L->nz, L->esize);
  if (need > L->buf_elems)  // only caller-owned buffers can be too small: the library's hold either layout
    return fail(LBM_ERR_STATE, "the row-major layout needs %zu bytes per buffer; the caller's buffers hold %zu "
                               "(lbm_buffer_elements gives the size)", need * L->esize, L->buf_elems * L->esize);
  // the state moves into the other buffer in the new layout
  LBM_HIP(lbm::launch_relayout(int(L->esize), L->buf[L->cur], L->lay, L->buf[L->cur ^ 1], to, L->N, L->stream),
          "relayout launch");
  L->cur ^= 1;
  L->layout = layout;
  L->lay = to;
  return LBM_OK;
}

lbm_status lbm_get_layout(const lbm_lattice *L, int *layout) {
  if (!L || !layout) return fail(LBM_ERR_ARG, "NULL argument");
  *layout = L->layout;
  return LBM_OK;
}

lbm_status lbm_state_buffer(const lbm_lattice *L, void **dev_ptr) {
  if (!L || !dev_ptr) return fail(LBM_ERR_ARG, "NULL argument");
  *dev_ptr = L->buf[L->cur];
  return LBM_OK;
}

lbm_status lbm_set_launch(lbm_lattice *L, int block_x, int nodes_per_thread, int xcd_remap) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (block_x != 64 && block_x != 128 && block_x != 256 && block_x != 512)
    return fail(LBM_ERR_ARG, "block_x must be 64, 128, 256 or 512 (got %d)", block_x);
  if (nodes_per_thread != 1 && nodes_per_thread != 2 && nodes_per_thread != 4)
    return fail(LBM_ERR_ARG, "nodes_per_thread must be 1, 2 or 4 (got %d)", nodes_per_thread);
  if (xcd_remap != LBM_XCD_NONE && xcd_remap != LBM_XCD_SLABS && xcd_remap != LBM_XCD_ROWS)
    return fail(LBM_ERR_ARG, "xcd_remap must be 0, 1 or 2 (got %d)", xcd_remap);
  L->block_x = block_x;
  L->npt = nodes_per_thread;
  L->xcd = xcd_remap;
  return LBM_OK;
}

lbm_status lbm_get_launch(const lbm_lattice *L, int *block_x, int *nodes_per_thread, int *xcd_remap) {
  if (!L || !block_x || !nodes_per_thread || !xcd_remap) return fail(LBM_ERR_ARG, "NULL argument");
  *block_x = L->block_x;
  *nodes_per_thread = L->npt;
  *xcd_remap = L->xcd;
  return LBM_OK;
}

lbm_status lbm_set_steps_per_pass(lbm_lattice *L, int steps_per_pass, int z_planes, int tile_rows) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (steps_per_pass != 1 && steps_per_pass != 2)
    return fail(LBM_ERR_ARG, "steps_per_pass must be 1 or 2 (got %d)", steps_per_pass);
  if (z_planes < 0) return fail(LBM_ERR_ARG, "z_planes must be >= 0 (got %d)", z_planes);
  if (tile_rows != 0 && tile_rows != 5 && tile_rows != 12)
    return fail(LBM_ERR_ARG, "tile_rows must be 0, 5 or 12 (got %d)", tile_rows);
  L->pass_steps = steps_per_pass;
  L->zc = z_planes == 0 ? kDefaultZPlanes : z_planes;
  L->tile_rows = tile_rows;
  return LBM_OK;
}

lbm_status lbm_get_steps_per_pass(const lbm_lattice *L, int *steps_per_pass, int *z_planes, int *tile_rows) {
  if (!L || !steps_per_pass || !z_planes || !tile_rows) return fail(LBM_ERR_ARG, "NULL argument");
  *steps_per_pass = L->pass_steps;
  *z_planes = L->zc;
  *tile_rows = L->tile_rows;
  return LBM_OK;
}

lbm_status lbm_get_size(const lbm_lattice *L, int *nx, int *ny, int *nz) {
  if (!L || !nx || !ny || !nz) return fail(LBM_ERR_ARG, "NULL argument");
  *nx = L->nx;
  *ny = L->ny;
  *nz = L->nz;
  return LBM_OK;
}

lbm_status lbm_get_step(const lbm_lattice *L, unsigned long long *steps) {
  if (!L || !steps) return fail(LBM_ERR_ARG, "NULL argument");
  *steps = L->steps;
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_lattice *L, int trial_steps, int *block_x, int *nodes_per_thread, int *xcd_remap) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (trial_steps < 1) return fail(LBM_ERR_ARG, "trial_steps must be >= 1");
  const lbm_status st = lbm_step(L, 0);  // the state checks of lbm_step
  if (st != LBM_OK) return st;
  // Candidate shapes of the single sweep: blocks no wider than the row
  // rounded up to a power of two (at least 64); one node per thread for the
  // extended sweep.  In the row-major layout without extended options also
  // the two-step pass: z ranges of 16, 32 or 64 planes, tiles of the form's
  // default rows, 5 or 12 rows, slab or dispatch-order placement.
  const bool ext = L->d_solid || L->d_geo || L->d_face_v[0] || L->d_face_v[1] || L->d_face_v[2] ||
                   L->d_face_v[3] || L->d_face_v[4] || L->d_face_v[5];
  int row = 64;
  while (row < L->nx && row < 512) row *= 2;
  struct Cand {
    int pass, bx, npt, xcd, zc, rows;
  };
  std::vector<Cand> cands;
  static const int shape[][2] = {{64, 1}, {128, 1}, {256, 1}, {512, 1}, {128, 2}, {256, 2}, {128, 4}, {256, 4}};
  static const int place[] = {LBM_XCD_SLABS, LBM_XCD_NONE, LBM_XCD_ROWS};
  for (const auto &sh : shape)
    for (int xcd : place) {
      if (sh[0] * sh[1] > row || (ext && sh[1] != 1)) continue;
      // with one block per row the rows placement is the dispatch order
      if (xcd == LBM_XCD_ROWS && sh[0] * sh[1] >= L->nx) continue;
      cands.push_back({1, sh[0], sh[1], xcd, 0, 0});
    }
  if (L->layout == LBM_LAYOUT_ROW_MAJOR && !ext)
    for (int zc : {16, 32, 64})
      for (int rows : {0, 5, 12}) {
        if (rows != 0 && L->storage == LBM_STORE_F64) continue;  // FP64 tiles have 5 rows either way
        for (int xcd : {LBM_XCD_SLABS, LBM_XCD_NONE}) cands.push_back({2, L->block_x, L->npt, xcd, zc, rows});
      }
  const int old[6] = {L->block_x, L->npt, L->xcd, L->pass_steps, L->zc, L->tile_rows};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(hipGetLastError(), "event creation");
  }
  float best_ms = 0.0f;
  int best = -1;
  lbm_status result = LBM_OK;
  for (int i = 0; i < int(cands.size()); ++i) {
    const Cand &c = cands[i];
    L->block_x = c.bx;
    L->npt = c.npt;
    L->xcd = c.xcd;
    L->pass_steps = c.pass;
    L->zc = c.pass == 2 ? c.zc : old[4];
    L->tile_rows = c.pass == 2 ? c.rows : old[5];
    // untimed launches, then timed ones (all of them real steps); the pass
    // takes pairs of steps
    const int n = c.pass == 2 ? 2 * trial_steps : trial_steps;
    result = lbm_step(L, c.pass);
    if (result == LBM_OK && hipEventRecord(e0, L->stream) != hipSuccess) result = hip_fail(hipGetLastError(), "event");
    if (result == LBM_OK) result = lbm_step(L, n);
    if (result == LBM_OK && hipEventRecord(e1, L->stream) != hipSuccess) result = hip_fail(hipGetLastError(), "event");
    float ms = 0.0f;
    if (result == LBM_OK && hipEventSynchronize(e1) != hipSuccess) result = hip_fail(hipGetLastError(), "event");
    if (result == LBM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) result = hip_fail(hipGetLastError(), "timing");
    if (result != LBM_OK) break;
    ms /= float(n);  // per step
    if (best < 0 || ms < best_ms) {
      best_ms = ms;
      best = i;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (result != LBM_OK || best < 0) {
    L->block_x = old[0];
    L->npt = old[1];
    L->xcd = old[2];
    L->pass_steps = old[3];
    L->zc = old[4];
    L->tile_rows = old[5];
    return result != LBM_OK ? result : fail(LBM_ERR_STATE, "no launch shape to try");
  }
  const Cand &c = cands[best];
  L->block_x = c.bx;
  L->npt = c.npt;
  L->xcd = c.xcd;
  L->pass_steps = c.pass;
  L->zc = c.pass == 2 ? c.zc : old[4];
  L->tile_rows = c.pass == 2 ? c.rows : old[5];
  if (block_x) *block_x = L->block_x;
  if (nodes_per_thread) *nodes_per_thread = L->npt;
  if (xcd_remap) *xcd_remap = L->xcd;
  return LBM_OK;
}

lbm_status lbm_tune_placement(lbm_lattice *L, int max_buffers, int trial_steps, int *buffers_tried,
                              double *ms_before, double *ms_after) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (!L->owns) return fail(LBM_ERR_STATE, "the lattice runs on caller-owned buffers; their placement is the caller's");
  if (max_buffers < 2 || max_buffers > kMaxPlacementBuffers)
    return fail(LBM_ERR_ARG, "max_buffers must be 2..%d (got %d)", kMaxPlacementBuffers, max_buffers);
  if (trial_steps < 1) return fail(LBM_ERR_ARG, "trial_steps must be >= 1");
  lbm_status result = lbm_step(L, 0);  // the state checks of lbm_step
  if (result != LBM_OK) return result;
  const size_t bytes = L->buf_elems * L->esize;
  // The pool: the state buffer, its partner, then new buffers while the device
  // keeps at least 1/8 of its memory (and 1 GiB) free.  All stay allocated
  // until the choice is made, so each new one lands on memory of its own.
  void *pool[kMaxPlacementBuffers] = {L->buf[L->cur], L->buf[L->cur ^ 1]};
  int n = 2;
  while (n < max_buffers) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      (void)hipGetLastError();
      break;
    }
    const size_t reserve = total_b / 8 > (size_t(1) << 30) ? total_b / 8 : (size_t(1) << 30);
    if (free_b < bytes + reserve) break;
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      break;
    }
    pool[n++] = p;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    result = hip_fail(hipGetLastError(), "event creation");
  }
  // Every unordered pair (i, j), i < j, with the state in pool[i]: two
  // untimed and 2 * trial_steps timed steps (an even count, so the state is
  // back in pool[i]).  L->buf always holds the state buffer and its partner.
  float first_ms = -1.0f, best_ms = 0.0f;
  int bi = 0, bj = 1;
  for (int i = 0; i + 1 < n && result == LBM_OK; ++i) {
    for (int j = i + 1; j < n && result == LBM_OK; ++j) {
      void *state = L->buf[L->cur];
      if (state != pool[i]) {
        hipError_t e = hipMemcpyAsync(pool[i], state, bytes, hipMemcpyDeviceToDevice, L->stream);
        if (e != hipSuccess) {
          result = hip_fail(e, "state copy");
          break;
        }
      }
      L->buf[0] = pool[i];
      L->buf[1] = pool[j];
      L->cur = 0;
      result = lbm_step(L, 2);
      if (result == LBM_OK && hipEventRecord(e0, L->stream) != hipSuccess) result = hip_fail(hipGetLastError(), "event");
      if (result == LBM_OK) result = lbm_step(L, 2 * trial_steps);
      if (result == LBM_OK && hipEventRecord(e1, L->stream) != hipSuccess) result = hip_fail(hipGetLastError(), "event");
      float ms = 0.0f;
      if (result == LBM_OK && hipEventSynchronize(e1) != hipSuccess) result = hip_fail(hipGetLastError(), "event");
      if (result == LBM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) result = hip_fail(hipGetLastError(), "timing");
      if (result != LBM_OK) break;
      ms /= float(2 * trial_steps);
      if (first_ms < 0.0f) first_ms = best_ms = ms;  // the lattice's own pair, measured first
      if (ms < best_ms) {
        best_ms = ms;
        bi = i;
        bj = j;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (result == LBM_OK) {
    // move the state into the first buffer of the fastest pair
    void *state = L->buf[L->cur];
    if (state != pool[bi]) {
      hipError_t e = hipMemcpyAsync(pool[bi], state, bytes, hipMemcpyDeviceToDevice, L->stream);
      if (e != hipSuccess) result = hip_fail(e, "state copy");
    }
    if (result == LBM_OK) {
      L->buf[0] = pool[bi];
      L->buf[1] = pool[bj];
      L->cur = 0;
    }
  }
  // Free every pool buffer the lattice does not hold (after the stream has
  // finished with them).
  if (hipStreamSynchronize(L->stream) != hipSuccess && result == LBM_OK)
    result = hip_fail(hipGetLastError(), "placement");
  for (int k = 0; k < n; ++k)
    if (pool[k] != L->buf[0] && pool[k] != L->buf[1]) (void)hipFree(pool[k]);
  if (result != LBM_OK) return result;
  if (buffers_tried) *buffers_tried = n;
  if (ms_before) *ms_before = double(first_ms);
  if (ms_after) *ms_after = double(best_ms);
  return LBM_OK;
}

lbm_status lbm_probe(lbm_lattice *L, int kind, int nrep) {
  if (!L) return fail(LBM_ERR_ARG, "NULL handle");
  if (kind != 0 && kind != 1) return fail(LBM_ERR_ARG, "probe kind must be 0 or 1");
  if (nrep < 0) return fail(LBM_ERR_ARG, "nrep must be >= 0");
  const void *src = L->buf[L->cur];
  void *dst = L->buf[L->cur ^ 1];
  const lbm::SweepConfig c = sweep_config(L);
  for (int r = 0; r < nrep; ++r) {
    hipError_t e = kind == 0 ? lbm::launch_copy_probe(src, dst, L->buf_elems * L->esize & ~size_t(15), L->stream)
                             : lbm::launch_sweep(c, src, dst, true, L->stream);
    if (e != hipSuccess) return hip_fail(e, "probe launch");
  }
  return LBM_OK;
}

}  // extern "C"
