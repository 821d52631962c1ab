// Plan lifetime, validation, footprints, export and error reporting.
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "srt_internal.h"

namespace srt {

namespace {
thread_local std::string g_last_error;

// Makes `device` current for the scope and restores the caller's device.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool finite_all(const double *v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

Status validate_plan(const srt_plan *p) {
  if (!p) return fail(SRT_EINVAL, "plan is NULL");
  if (p->magic != kPlanMagic) return fail(SRT_EINVAL, "plan is not a live plan (destroyed?)");
  return Status{};
}

srt_status finish(const Status &s) { return s.code; }

void destroy_contents(srt_plan *p) {
  clear_timing(p);
  release_operators(p);
  (void)hipFree(p->d_geom);
  (void)hipFree(p->own_ws);
  p->d_geom = nullptr;
  p->own_ws = nullptr;
}

bool strictly_increasing_positive(const double *v, int32_t n) {
  if (v[0] <= 0) return false;
  for (int32_t i = 1; i < n; ++i)
    if (!(v[i] > v[i - 1])) return false;
  return true;
}

// col_xy: host [na][2] column centres (x, y). rho: host [nr] radial grid of
// the stage-2 image, or NULL for the radii themselves.
Status create(const srt_grid *grid, int32_t basis, const double *col_xy, int32_t na,
              const double *zpos, int32_t nh, const double *radii, int32_t nl,
              const double *rho, int32_t nr, srt_dtype vdt, srt_dtype wdt, srt_opmode mode,
              int32_t device, hipStream_t s, srt_plan **out) {
  if (!out) return fail(SRT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grid || !col_xy || !zpos || !radii) return fail(SRT_EINVAL, "NULL argument");
  if (basis != SRT_BASIS_CONSTANT && basis != SRT_BASIS_LINEAR)
    return fail(SRT_EINVAL, "unknown basis");
  const bool own_rho = rho != nullptr;
  if (!own_rho) {
    rho = radii;
    nr = nl;
  }
  if (grid->ms <= 0 || grid->mz <= 0) return fail(SRT_EINVAL, "grid sizes must be positive");
  if (!(std::isfinite(grid->x0) && std::isfinite(grid->z0) && std::isfinite(grid->dxy) &&
        std::isfinite(grid->dz)) || grid->dxy <= 0 || grid->dz <= 0)
    return fail(SRT_EINVAL, "grid origin and pitch must be finite, pitch > 0");
  if (na <= 0 || nh <= 0 || nl <= 0 || nr <= 0)
    return fail(SRT_EINVAL, "sample counts must be positive");
  if (!finite_all(col_xy, 2 * (int64_t)na) || !finite_all(zpos, nh) || !finite_all(radii, nl) ||
      !finite_all(rho, nr))
    return fail(SRT_EINVAL, "sample positions must be finite");
  if (radii[0] <= 0) return fail(SRT_EINVAL, "radii must be > 0");
  for (int32_t i = 1; i < nl; ++i)
    if (!(radii[i] > radii[i - 1])) return fail(SRT_EINVAL, "radii must be strictly increasing");
  if (own_rho && !strictly_increasing_positive(rho, nr))
    return fail(SRT_EINVAL, "rho grid must be > 0 and strictly increasing");
  const bool pair_ok = (vdt == SRT_F32 && (wdt == SRT_F32 || wdt == SRT_BF16 || wdt == SRT_F16)) ||
                       (vdt == SRT_F64 && wdt == SRT_F64);
  if (!pair_ok) return fail(SRT_EINVAL, "unsupported (value, weight) dtype pair");
  if (mode != SRT_OP_AUTO && mode != SRT_OP_STORED && mode != SRT_OP_ONTHEFLY)
    return fail(SRT_EINVAL, "unknown mode");
  // Index ranges: every dense index below must fit in int32 rows/cols.
  const int64_t npix = (int64_t)grid->ms * grid->ms;
  if (npix > INT32_MAX || (int64_t)na * nl > INT32_MAX || (int64_t)nh * nl > INT32_MAX ||
      (int64_t)na * nr > INT32_MAX || (int64_t)nr * grid->mz > INT32_MAX ||
      npix * grid->mz > ((int64_t)1 << 40))
    return fail(SRT_ENOTSUP, "problem too large for 32-bit operator indices");
  int ndev = 0;
  SRT_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(SRT_EINVAL, "device ordinal out of range");
  DeviceGuard dg(device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");

  srt_plan *p = new (std::nothrow) srt_plan();
  if (!p) return fail(SRT_ENOMEM, "host allocation failed");
  p->device = device;
  p->vdtype = vdt;
  p->wdtype = wdt;
  auto bail = [&](Status st) {
    destroy_contents(p);
    delete p;
    return st;
  };
  // device copy: cx[na], cy[na], zpos[nh], radii[nl], rho[nr]
  const size_t ngeom = 2 * (size_t)na + nh + nl + nr;
  if (hipMalloc(&p->d_geom, sizeof(double) * ngeom) != hipSuccess)
    return bail(fail(SRT_ENOMEM, "device allocation for geometry failed"));
  std::vector<double> h(ngeom);
  for (int32_t a = 0; a < na; ++a) {
    h[a] = col_xy[2 * a];
    h[na + a] = col_xy[2 * a + 1];
  }
  std::memcpy(h.data() + 2 * na, zpos, sizeof(double) * nh);
  std::memcpy(h.data() + 2 * na + nh, radii, sizeof(double) * nl);
  std::memcpy(h.data() + 2 * na + nh + nl, rho, sizeof(double) * nr);
  hipError_t e = hipMemcpyAsync(p->d_geom, h.data(), sizeof(double) * h.size(),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bail(hip_fail(e, "upload of sample positions"));

  Geometry &g = p->geo;
  g.ms = grid->ms;
  g.mz = grid->mz;
  g.x0 = grid->x0;
  g.z0 = grid->z0;
  g.dxy = grid->dxy;
  g.dz = grid->dz;
  g.na = na;
  g.nh = nh;
  g.nl = nl;
  g.cx = p->d_geom;
  g.cy = p->d_geom + na;
  g.zpos = p->d_geom + 2 * na;
  g.radii = p->d_geom + 2 * na + nh;
  g.rho = p->d_geom + 2 * na + nh + nl;
  g.nr = nr;
  g.basis = basis;

  Status st = build_operators(p, s, kAllTiles);
  if (st.ok()) {
    p->nnz12 = p->a12.nnz;
    p->nnz34 = p->a34.nnz;
    p->scale12 = p->a12.scale;
    p->scale34 = p->a34.scale;
    p->op_bytes = operator_bytes(p);
    // AUTO keeps the operators resident unless they would take more than
    // half of the device's memory: regenerating them in an apply costs most
    // of a plan build (a 128^3 forward measured 0.36 ms stored, 52 ms on the
    // fly), so a plan that fits stays stored.
    srt_opmode m = mode;
    if (m == SRT_OP_AUTO) {
      size_t free_b = 0, total_b = 0;
      m = hipMemGetInfo(&free_b, &total_b) == hipSuccess && p->op_bytes > total_b / 2
              ? SRT_OP_ONTHEFLY
              : SRT_OP_STORED;
    }
    p->mode = m;
    if (m == SRT_OP_ONTHEFLY) {
      SRT_HIP(hipStreamSynchronize(s));
      release_operators(p);
    }
  }
  if (!st.ok()) return bail(st);
  p->magic = kPlanMagic;
  *out = p;
  return Status{};
}

}  // namespace

void set_error(const std::string &msg) { g_last_error = msg; }

Status fail(srt_status code, const std::string &msg) {
  set_error(msg);
  Status s;
  s.code = code;
  return s;
}

Status hip_fail(hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    return fail(SRT_ENOMEM, std::string(what) + ": out of device memory");
  }
  return fail(SRT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void clear_timing(srt_plan *p) {
  for (auto &list : p->timed) {
    for (auto &rec : list)
      for (auto &e : rec.ev) (void)hipEventDestroy(e);
    list.clear();
  }
}

size_t dtype_size(srt_dtype t) {
  switch (t) {
    case SRT_F64: return 8;
    case SRT_F32: return 4;
    default: return 2;
  }
}

size_t operator_bytes(const srt_plan *p) {
  return p->a12.bytes() + p->a12t.bytes() + p->a34.bytes() + p->a34t.bytes() + p->t12.bytes() +
         p->t12t.bytes() + p->t34.bytes() + p->t34t.bytes();
}

void release_operators(srt_plan *p) {
  p->a12.release();
  p->a12t.release();
  p->a34.release();
  p->a34t.release();
  p->t12.release();
  p->t12t.release();
  p->t34.release();
  p->t34t.release();
}

Status build_operators(srt_plan *p, hipStream_t s, unsigned tiles) {
  const Geometry &g = p->geo;
  const int64_t na = g.na, nh = g.nh, nl = g.nl, nr = g.nr;
  const int64_t npix = (int64_t)g.ms * g.ms;
  const srt_dtype wdt = p->wdtype;
  Coo pieces;
  auto free_pieces = [&]() {
    (void)hipFree(pieces.keys);
    (void)hipFree(pieces.vals);
    pieces = Coo{};
  };
  Status st = a12_pieces(g, s, &pieces);
  if (st.ok()) st = compact_a12(&pieces, (int32_t)nr, npix, s, &p->live);
  if (st.ok())
    st = build_csr_pair(&pieces, na * p->live, npix, wdt, s, &p->a12, &p->a12t);
  free_pieces();
  if (st.ok()) st = a34_pieces(g, p->live, s, &pieces);
  if (st.ok())
    st = build_csr_pair(&pieces, nh * nl, (int64_t)p->live * g.mz, wdt, s, &p->a34, &p->a34t);
  free_pieces();
  // Row-blocked copies for the applies: compact blocks of kRB rows whose
  // arcs share cells (at kRB = 128: 8 columns x 16 radii, 16 heights x 8
  // radii, 16 x 8 rho-z cells, 8 x 16 pixels). Rows processed side by side
  // get equal work per chunk: one radius at 8 columns (A12), one radius at 8
  // heights (A34), 4 rho-neighbouring cells at one z (A34^T), 4
  // y-neighbouring pixels (A12^T). Shapes, slot order and block numbering
  // tiles (2 column groups for A12, 2 height groups for A34, 4 rho groups
  // for A34^T, plain row-major for A12^T) were measured at 256^3 under the
  // kernels' work order. The forward operators cut their blocks' columns into
  // chunks in polar order about the block (sectors of the block's arcs).
  const int64_t L = p->live;
  const int me = p->vdtype == SRT_F64 ? kE64 : kE32;
  const int64_t bh = kRB / 16;  // 16 or 8
  ColumnOrder o12, o34, plain;
  o12.kind = 1;
  o12.cx = g.cx;
  o12.cy = g.cy;
  o12.ms = g.ms;
  o12.x0 = g.x0;
  o12.dxy = g.dxy;
  o34.kind = 2;
  o34.zpos = g.zpos;
  o34.rho = g.rho;
  o34.mz = g.mz;
  o34.z0 = g.z0;
  o34.dz = g.dz;
  if (st.ok() && (tiles & kTileA12))
    st = build_tiled(p->a12, RowGrid{na, L, 8, kRB / 8, true, 2}, me, o12, s, &p->t12);
  if (st.ok() && (tiles & kTileA12t))
    st = build_tiled(p->a12t, RowGrid{g.ms, g.ms, bh, 16, true, 1}, me, plain, s, &p->t12t);
  if (st.ok() && (tiles & kTileA34))
    st = build_tiled(p->a34, RowGrid{nh, nl, 16, bh, true, 2}, me, o34, s, &p->t34);
  if (st.ok() && (tiles & kTileA34t))
    st = build_tiled(p->a34t, RowGrid{L, g.mz, 16, bh, true, 4}, me, plain, s, &p->t34t);
  if (!st.ok()) release_operators(p);
  return st;
}

}  // namespace srt

using namespace srt;

namespace {
// Column positions of a cylinder aperture: column a stands at
// (R cos angles[a], R sin angles[a]).
Status cylinder_columns(double cyl_radius, const double *angles, int32_t n_angles,
                        std::vector<double> *xy) {
  if (!angles) return fail(SRT_EINVAL, "NULL argument");
  if (!std::isfinite(cyl_radius) || cyl_radius < 0)
    return fail(SRT_EINVAL, "cylinder radius must be finite and >= 0");
  if (n_angles <= 0) return fail(SRT_EINVAL, "sample counts must be positive");
  if (!finite_all(angles, n_angles)) return fail(SRT_EINVAL, "sample positions must be finite");
  xy->resize(2 * (size_t)n_angles);
  for (int32_t a = 0; a < n_angles; ++a) {
    (*xy)[2 * a] = cyl_radius * std::cos(angles[a]);
    (*xy)[2 * a + 1] = cyl_radius * std::sin(angles[a]);
  }
  return Status{};
}
}  // namespace

extern "C" {

srt_status srt_plan_create(const srt_grid *grid, double cyl_radius, const double *angles,
                           int32_t n_angles, const double *z_pos, int32_t n_z,
                           const double *radii, int32_t n_radii, srt_dtype value_dtype,
                           srt_dtype weight_dtype, srt_opmode mode, int32_t device,
                           void *hip_stream, srt_plan **out) {
  try {
    if (out) *out = nullptr;
    std::vector<double> xy;
    Status st = cylinder_columns(cyl_radius, angles, n_angles, &xy);
    if (!st.ok()) return finish(st);
    return finish(create(grid, SRT_BASIS_CONSTANT, xy.data(), n_angles, z_pos, n_z, radii,
                         n_radii, nullptr, 0, value_dtype, weight_dtype, mode, device,
                         (hipStream_t)hip_stream, out));
  } catch (...) {
    return finish(fail(SRT_ENOMEM, "host exception during plan creation"));
  }
}

srt_status srt_plan_create_columns(const srt_grid *grid, const double *col_xy, int32_t n_cols,
                                   const double *z_pos, int32_t n_z, const double *radii,
                                   int32_t n_radii, srt_dtype value_dtype,
                                   srt_dtype weight_dtype, srt_opmode mode, int32_t device,
                                   void *hip_stream, srt_plan **out) {
  try {
    return finish(create(grid, SRT_BASIS_CONSTANT, col_xy, n_cols, z_pos, n_z, radii, n_radii,
                         nullptr, 0, value_dtype, weight_dtype, mode, device,
                         (hipStream_t)hip_stream, out));
  } catch (...) {
    return finish(fail(SRT_ENOMEM, "host exception during plan creation"));
  }
}

srt_status srt_plan_create_desc(const srt_plan_desc *desc, void *hip_stream, srt_plan **out) {
  try {
    if (out) *out = nullptr;
    if (!desc) return finish(fail(SRT_EINVAL, "NULL argument"));
    const srt_plan_desc &d = *desc;
    if ((d.angles == nullptr) == (d.col_xy == nullptr))
      return finish(fail(SRT_EINVAL, "exactly one of angles and col_xy must be given"));
    if ((d.rho == nullptr) != (d.n_rho == 0))
      return finish(fail(SRT_EINVAL, "rho and n_rho must both be given or both be absent"));
    std::vector<double> xy;
    const double *col_xy = d.col_xy;
    if (d.angles) {
      Status st = cylinder_columns(d.cyl_radius, d.angles, d.n_cols, &xy);
      if (!st.ok()) return finish(st);
      col_xy = xy.data();
    }
    return finish(create(&d.grid, (int32_t)d.basis, col_xy, d.n_cols, d.z_pos, d.n_z, d.radii,
                         d.n_radii, d.rho, d.n_rho, d.value_dtype, d.weight_dtype, d.mode,
                         d.device, (hipStream_t)hip_stream, out));
  } catch (...) {
    return finish(fail(SRT_ENOMEM, "host exception during plan creation"));
  }
}

srt_status srt_plan_destroy(srt_plan *plan) {
  if (!plan) return SRT_OK;
  if (plan->magic != kPlanMagic) return finish(fail(SRT_EINVAL, "plan is not a live plan"));
  DeviceGuard dg(plan->device);
  plan->magic = 0;
  destroy_contents(plan);
  delete plan;
  return SRT_OK;
}

srt_status srt_plan_footprint(const srt_plan *plan, int32_t batch, size_t *resident,
                              size_t *workspace) {
  Status st = validate_plan(plan);
  if (!st.ok()) return finish(st);
  if (batch <= 0) return finish(fail(SRT_EINVAL, "batch must be >= 1"));
  const size_t geom = sizeof(double) * (2 * (size_t)plan->geo.na + plan->geo.nh +
                                        plan->geo.nl + plan->geo.nr);
  // an on-the-fly plan holds only its geometry; each apply regenerates its
  // operators, at most all of op_bytes, beside the workspace
  const bool otf = plan->mode == SRT_OP_ONTHEFLY;
  if (resident) *resident = geom + (otf ? 0 : plan->op_bytes);
  if (workspace) *workspace = workspace_bytes(plan, batch);
  return SRT_OK;
}

srt_status srt_plan_get_info(const srt_plan *plan, srt_plan_info *info) {
  Status st = validate_plan(plan);
  if (!st.ok()) return finish(st);
  if (!info) return finish(fail(SRT_EINVAL, "info is NULL"));
  info->nnz_a12 = plan->nnz12;
  info->nnz_a34 = plan->nnz34;
  info->live_radii = plan->live;
  info->n_angles = plan->geo.na;
  info->n_z = plan->geo.nh;
  info->n_radii = plan->geo.nl;
  info->weight_scale_a12 = plan->scale12;
  info->weight_scale_a34 = plan->scale34;
  info->basis = plan->geo.basis;
  info->n_rho = plan->geo.nr;
  info->mode = plan->mode;
  info->operator_bytes = (int64_t)plan->op_bytes;
  return SRT_OK;
}

srt_status srt_plan_export_coo(const srt_plan *plan, int32_t which, int64_t capacity,
                               int64_t *nnz, int32_t *rows, int32_t *cols, double *vals) {
  Status st = validate_plan(plan);
  if (!st.ok()) return finish(st);
  if (which < 0 || which > 3) return finish(fail(SRT_EINVAL, "which must be 0..3"));
  if (!nnz) return finish(fail(SRT_EINVAL, "nnz is NULL"));
  const int64_t n = which == 0 || which == 2 ? plan->nnz12 : plan->nnz34;
  *nnz = n;
  if (capacity == 0) return SRT_OK;
  if (capacity < n) return finish(fail(SRT_EINVAL, "capacity smaller than nnz"));
  if (!rows || !cols || !vals) return finish(fail(SRT_EINVAL, "NULL output array"));
  DeviceGuard dg(plan->device);
  if (dg.err != hipSuccess) return finish(hip_fail(dg.err, "hipSetDevice"));
  // an on-the-fly plan regenerates its CSR operators for the copy (the
  // plan's observable state does not change)
  srt_plan *mp = const_cast<srt_plan *>(plan);
  struct Regen {
    srt_plan *p = nullptr;
    ~Regen() {
      if (p) release_operators(p);
    }
  } regen;
  if (plan->mode == SRT_OP_ONTHEFLY) {
    regen.p = mp;
    st = build_operators(mp, nullptr, 0);
    if (!st.ok()) return finish(st);
  }
  const Csr *m = which == 0 ? &plan->a12 : which == 1 ? &plan->a34 : which == 2 ? &plan->a12t
                                                                               : &plan->a34t;
  std::vector<int32_t> rp((size_t)m->nrows + 1);
  const size_t wsz = dtype_size(m->wdtype);
  std::vector<unsigned char> raw(wsz * (size_t)m->nnz);
  hipError_t e = hipMemcpy(rp.data(), m->rowptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess && m->nnz)
    e = hipMemcpy(cols, m->cols, sizeof(int32_t) * m->nnz, hipMemcpyDeviceToHost);
  if (e == hipSuccess && m->nnz) e = hipMemcpy(raw.data(), m->vals, raw.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return finish(hip_fail(e, "export copy"));
  for (int64_t r = 0; r < m->nrows; ++r)
    for (int32_t k = rp[r]; k < rp[r + 1]; ++k) rows[k] = (int32_t)r;
  // A12 rows are stored as a * live + m; report them as a * n_rho + m.
  const int64_t L = plan->live, NL = plan->geo.nr;
  if (which == 0)
    for (int64_t k = 0; k < m->nnz; ++k) rows[k] = (int32_t)((rows[k] / L) * NL + rows[k] % L);
  if (which == 2)
    for (int64_t k = 0; k < m->nnz; ++k) cols[k] = (int32_t)((cols[k] / L) * NL + cols[k] % L);
  for (int64_t k = 0; k < m->nnz; ++k) {
    double v;
    const unsigned char *b = raw.data() + wsz * k;
    if (m->wdtype == SRT_F64) {
      std::memcpy(&v, b, 8);
    } else if (m->wdtype == SRT_F32) {
      float f;
      std::memcpy(&f, b, 4);
      v = f;
    } else if (m->wdtype == SRT_BF16) {
      uint32_t u = (uint32_t)(b[0] | (b[1] << 8)) << 16;
      float f;
      std::memcpy(&f, &u, 4);
      v = f;
    } else {
      _Float16 hv;
      std::memcpy(&hv, b, 2);
      v = (double)(float)hv;
    }
    vals[k] = v / m->scale;
  }
  return SRT_OK;
}

srt_status srt_plan_set_timing(srt_plan *plan, int32_t enable) {
  Status st = validate_plan(plan);
  if (!st.ok()) return finish(st);
  DeviceGuard dg(plan->device);
  clear_timing(plan);
  plan->timing = enable != 0;
  return SRT_OK;
}

srt_status srt_plan_stage_times(const srt_plan *plan, int32_t adjoint, int32_t n_stages,
                                double *total_ms, int32_t *n_calls) {
  Status st = validate_plan(plan);
  if (!st.ok()) return finish(st);
  if (!total_ms || !n_calls || n_stages < 0 || n_stages > kStages)
    return finish(fail(SRT_EINVAL, "bad output arguments"));
  DeviceGuard dg(plan->device);
  const auto &list = plan->timed[adjoint ? 1 : 0];
  for (int32_t i = 0; i < n_stages; ++i) total_ms[i] = 0.0;
  for (const auto &rec : list) {
    for (int32_t i = 0; i < n_stages; ++i) {
      float ms = 0.f;
      hipError_t e = hipEventElapsedTime(&ms, rec.ev[i], rec.ev[i + 1]);
      if (e == hipErrorNotReady) return finish(fail(SRT_EINVAL, "timed applies have not completed"));
      if (e != hipSuccess) return finish(hip_fail(e, "hipEventElapsedTime"));
      total_ms[i] += ms;
    }
  }
  *n_calls = (int32_t)list.size();
  return SRT_OK;
}

const char *srt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
