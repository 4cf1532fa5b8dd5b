// Host helpers: descriptor validation, device layout of an instance, tile
// work-list construction, autotune table, parameter marshalling.
#include "fv_runtime.h"

#include <new>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>

namespace fvrt {

thread_local std::string t_err;

int set_error(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_err = buf;
  return status;
}

static int face_ext(const fv_block_desc& b, int d) { return d == 0 ? b.ni : (d == 1 ? b.nj : b.nk); }
static void trans(const fv_block_desc& b, int d, int& n1, int& n2) {
  if (d == 0) { n1 = b.nj; n2 = b.nk; }
  else if (d == 1) { n1 = b.ni; n2 = b.nk; }
  else { n1 = b.ni; n2 = b.nj; }
}

static int validate_and_copy_impl(const fv_grid_desc* d, HostGrid& g) {
  if (!d) return set_error(FV_E_INVAL, "null grid descriptor");
  if (d->ndim != 2 && d->ndim != 3) return set_error(FV_E_INVAL, "ndim must be 2 or 3 (got %d)", d->ndim);
  if (d->nblocks <= 0 || !d->blocks) return set_error(FV_E_INVAL, "no blocks");
  if (!(d->gamma > 1.0) || !std::isfinite(d->gamma)) return set_error(FV_E_INVAL, "gamma must be > 1");
  g = HostGrid();
  g.ndim = d->ndim;
  g.nv = d->ndim + 2;
  g.nblocks = d->nblocks;
  g.gamma = d->gamma;
  g.blocks.assign(d->blocks, d->blocks + d->nblocks);
  g.xs.resize(d->nblocks);
  g.ys.resize(d->nblocks);
  g.zs.resize(d->nblocks);
  if (d->with_source != 0 && d->with_source != 1)
    return set_error(FV_E_INVAL, "with_source must be 0 or 1 (got %d)", d->with_source);
  g.with_source = d->with_source == 1;
  const long long kMaxDim = 1 << 20;
  for (int b = 0; b < g.nblocks; ++b) {
    fv_block_desc& B = g.blocks[b];
    if (g.ndim == 2) {
      if (B.nk == 0) B.nk = 1;
      if (B.nk != 1) return set_error(FV_E_INVAL, "block %d: nk must be 1 in 2D", b);
    }
    if (B.ni <= 0 || B.nj <= 0 || B.nk <= 0 || B.ni > kMaxDim || B.nj > kMaxDim || B.nk > kMaxDim)
      return set_error(FV_E_INVAL, "block %d: bad extents %d x %d x %d", b, B.ni, B.nj, B.nk);
    // the 3D stage kernels address a cell within its k-plane by a 32-bit byte
    // offset: a plane of one variable must stay below 4 GiB
    if (g.ndim == 3 && (long long)B.ni * B.nj * 8LL >= (1LL << 32))
      return set_error(FV_E_UNSUPPORTED,
                       "block %d: a k-plane of %d x %d cells exceeds the 3D kernels' 32-bit "
                       "in-plane offsets (ni * nj must stay below 2^29)", b, B.ni, B.nj);
    if (g.ndim == 3 && (B.x || B.y || B.z) && !(B.x && B.y && B.z))
      return set_error(FV_E_INVAL, "block %d: give x, y and z or none of them", b);
    if (g.ndim == 2 && ((B.x == nullptr) != (B.y == nullptr)))
      return set_error(FV_E_INVAL, "block %d: give both x and y or neither", b);
    if (g.ndim == 2 && B.z) return set_error(FV_E_INVAL, "block %d: z must be NULL in 2D", b);
    if (!B.x) {
      for (int a = 0; a < g.ndim; ++a)
        if (!(B.h[a] > 0.0) || !std::isfinite(B.h[a]))
          return set_error(FV_E_INVAL, "block %d: spacing h[%d] must be > 0", b, a);
    } else {
      const size_t nn = (size_t)(B.ni + 1) * (size_t)(B.nj + 1) * (size_t)(g.ndim == 3 ? B.nk + 1 : 1);
      g.xs[b].assign(B.x, B.x + nn);
      g.ys[b].assign(B.y, B.y + nn);
      if (g.ndim == 3) g.zs[b].assign(B.z, B.z + nn);
      for (size_t q = 0; q < nn; ++q)
        if (!std::isfinite(g.xs[b][q]) || !std::isfinite(g.ys[b][q]) ||
            (g.ndim == 3 && !std::isfinite(g.zs[b][q])))
          return set_error(FV_E_INVAL, "block %d: non-finite node coordinate", b);
      B.x = g.xs[b].data();
      B.y = g.ys[b].data();
      B.z = g.ndim == 3 ? g.zs[b].data() : nullptr;
      g.node_doubles += (g.ndim == 3 ? 3 : 2) * (long long)nn;
      if (g.ndim == 3) g.gen3 = true;
    }
    g.ncells += (long long)B.ni * B.nj * B.nk;
  }
  for (int b = 0; b < g.nblocks; ++b) {
    const fv_block_desc& B = g.blocks[b];
    for (int f = 0; f < 2 * g.ndim; ++f) {
      const fv_bc& bc = B.face[f];
      if (bc.kind < FV_BC_PERIODIC || bc.kind > FV_BC_NOSLIP)
        return set_error(FV_E_INVAL, "block %d face %d: unknown boundary kind %d", b, f, bc.kind);
      if (bc.kind == FV_BC_NOSLIP) {
        if (g.ndim != 2)
          return set_error(FV_E_UNSUPPORTED, "block %d face %d: no-slip walls are provided in 2D only", b, f);
        for (int a = 1; a <= 3; ++a)
          if (!std::isfinite(bc.prim_in[a]))
            return set_error(FV_E_INVAL, "block %d face %d: non-finite wall velocity", b, f);
        g.has_noslip = true;
      }
      if (bc.kind == FV_BC_BLOCK) {
        if (bc.nbr_block < 0 || bc.nbr_block >= g.nblocks)
          return set_error(FV_E_INVAL, "block %d face %d: neighbour block %d out of range", b, f, bc.nbr_block);
        if (g.ndim == 2 && (bc.nbr_face != (f ^ 1) || bc.orient != 0))
          return set_error(FV_E_INVAL, "block %d face %d: 2D links join opposite faces (neighbour face "
                           "%d, orient 0)", b, f, f ^ 1);
        if (bc.nbr_face < 0 || bc.nbr_face > 5)
          return set_error(FV_E_INVAL, "block %d face %d: neighbour face %d out of range", b, f, bc.nbr_face);
        if (bc.orient < 0 || bc.orient > 7)
          return set_error(FV_E_INVAL, "block %d face %d: orient %d out of range 0..7", b, f, bc.orient);
        int n1, n2, m1, m2;
        trans(B, f / 2, n1, n2);
        trans(g.blocks[bc.nbr_block], bc.nbr_face / 2, m1, m2);
        if (bc.orient & 1) std::swap(n1, n2);
        if (n1 != m1 || n2 != m2)
          return set_error(FV_E_INVAL, "block %d face %d: transverse size %dx%d (in the neighbour's "
                           "order) != neighbour's %dx%d", b, f, n1, n2, m1, m2);
        // the uniform 3D kernel reads its neighbours' opposite faces unoriented
        if (bc.nbr_face != (f ^ 1) || bc.orient != 0) g.gen3 = true;
      }
      // the two ghost layers of these rules are two distinct cells of the source block
      if (bc.kind == FV_BC_PERIODIC || bc.kind == FV_BC_SLIPWALL || bc.kind == FV_BC_BLOCK ||
          bc.kind == FV_BC_NOSLIP) {
        const fv_block_desc& S = bc.kind == FV_BC_BLOCK ? g.blocks[bc.nbr_block] : B;
        const int sd = bc.kind == FV_BC_BLOCK ? bc.nbr_face / 2 : f / 2;
        if (face_ext(S, sd) < 2)
          return set_error(FV_E_INVAL, "block %d face %d: this rule needs at least 2 cells across the face", b, f);
      }
      if (bc.kind == FV_BC_INFLOW) {
        if (!(bc.prim_in[0] > 0.0) || !(bc.prim_in[4] > 0.0))
          return set_error(FV_E_INVAL, "block %d face %d: inflow needs rho > 0 and p > 0", b, f);
      }
    }
  }
  g.state_size = g.ncells * g.nv;
  if (g.ndim == 3 && g.with_source) g.gen3 = true;
  return FV_OK;
}

// the host copies of a large grid can exhaust host memory: that is an error
// return, never an exception through the C interface
int validate_and_copy(const fv_grid_desc* d, HostGrid& g) {
  try {
    return validate_and_copy_impl(d, g);
  } catch (const std::bad_alloc&) {
    g = HostGrid();
    return set_error(FV_E_NOMEM, "host allocation failed while copying the grid descriptor");
  }
}

static const int kMinRows2D = 2, kMinPlanes3D = 4, kMinNy3D = 3;

long long max_tiles_of(const HostGrid& g) {
  long long t = 0;
  for (const auto& B : g.blocks) {
    const long long ci = (B.ni + 63) / 64;
    if (g.ndim == 2) t += ci * ((B.nj + kMinRows2D - 1) / kMinRows2D);
    else t += ci * ((B.nj + kMinNy3D - 1) / kMinNy3D) * ((B.nk + kMinPlanes3D - 1) / kMinPlanes3D);
  }
  return t;
}

void build_segs(const HostGrid& g, std::vector<fvk::GhostSeg>& segs) {
  segs.clear();
  long long cell = 0, out = 0;
  for (int b = 0; b < g.nblocks; ++b)
    for (int f = 0; f < 2 * g.ndim; ++f) {
      fvk::GhostSeg s;
      s.blk = b;
      s.face = f;
      trans(g.blocks[b], f / 2, s.n1, s.n2);
      s.cell_off = cell;
      s.out_off = out;
      const long long per = (long long)s.n1 * s.n2;
      cell += 2 * per;
      out += 2 * per * g.nv;
      segs.push_back(s);
    }
}

InstLayout layout_of(const HostGrid& g) {
  InstLayout L;
  L.max_tiles = max_tiles_of(g);
  std::vector<fvk::GhostSeg> segs;
  build_segs(g, segs);
  L.nseg = (int)segs.size();
  L.ghost_cells = 0;
  for (const auto& s : segs) L.ghost_cells += 2LL * s.n1 * s.n2;
  L.ghost_doubles = L.ghost_cells * g.nv;
  size_t off = 0;
  L.blocks = off; off += align_up(sizeof(fvk::DevBlock) * g.nblocks);
  L.inst = off;   off += align_up(sizeof(fvk::DevInstance));
  L.ntiles = off; off += align_up(sizeof(int) * 4);
  L.tiles = off;  off += align_up(sizeof(fvk::DevTile) * (size_t)L.max_tiles);
  L.part = off;   off += align_up(sizeof(double) * fvk::kPartStride * (size_t)L.max_tiles);
  L.segs = off;   off += align_up(sizeof(fvk::GhostSeg) * (size_t)L.nseg);
  L.nodes = off;  off += align_up(sizeof(double) * (size_t)g.node_doubles);
  L.src = off;    off += g.with_source ? align_up(sizeof(double) * (size_t)g.state_size) : 0;
  for (int s = 0; s < 3; ++s) {
    L.u[s] = off;
    off += align_up(sizeof(double) * (size_t)g.state_size);
  }
  L.total = off;
  return L;
}

void build_blocks(const HostGrid& g, char* base, const InstLayout& L, int inst_index,
                  std::vector<fvk::DevBlock>& out, int boff) {
  out.clear();
  long long soff = 0, noff = 0;
  for (int b = 0; b < g.nblocks; ++b) {
    const fv_block_desc& D = g.blocks[b];
    fvk::DevBlock B;
    std::memset(&B, 0, sizeof(B));
    B.ni = D.ni;
    B.nj = D.nj;
    B.nk = D.nk;
    B.inst = inst_index;
    B.ncell = (long long)D.ni * D.nj * D.nk;
    for (int a = 0; a < 3; ++a) B.org[a] = D.origin[a];
    for (int s = 0; s < 3; ++s) B.u[s] = (double*)(base + L.u[s]) + soff;
    B.out_off = soff;
    if (D.x) {
      const long long nn = (long long)(D.ni + 1) * (D.nj + 1) * (g.ndim == 3 ? D.nk + 1 : 1);
      B.xn = (const double*)(base + L.nodes) + noff;
      B.yn = B.xn + nn;
      if (g.ndim == 3) B.zn = B.yn + nn;
      noff += (g.ndim == 3 ? 3 : 2) * nn;
    }
    if (g.with_source) B.src = (const double*)(base + L.src) + soff;
    if (g.ndim == 2) {
      B.area[0] = D.h[1];
      B.area[1] = D.h[0];
      B.area[2] = 0.0;
      B.vol = D.h[0] * D.h[1];
    } else {
      B.area[0] = D.h[1] * D.h[2];
      B.area[1] = D.h[0] * D.h[2];
      B.area[2] = D.h[0] * D.h[1];
      B.vol = D.h[0] * D.h[1] * D.h[2];
    }
    for (int f = 0; f < 6; ++f) {
      const fv_bc& bc = D.face[f];
      B.bc_kind[f] = (f < 2 * g.ndim) ? bc.kind : FV_BC_PERIODIC;
      B.bc_nbr[f] = bc.kind == FV_BC_BLOCK ? bc.nbr_block + boff : -1;
      B.bc_link[f] = bc.kind == FV_BC_BLOCK ? bc.nbr_face | bc.orient << 3 : 0;
      if (bc.kind == FV_BC_INFLOW && f < 2 * g.ndim) {
        // conserved state of the prescribed primitive (rho, u, v, w, p)
        const double rho = bc.prim_in[0];
        double ke = 0.0;
        B.bc_q[f][0] = rho;
        for (int a = 0; a < g.ndim; ++a) {
          B.bc_q[f][1 + a] = rho * bc.prim_in[1 + a];
          ke += bc.prim_in[1 + a] * bc.prim_in[1 + a];
        }
        B.bc_q[f][g.ndim + 1] = bc.prim_in[4] / (g.gamma - 1.0) + 0.5 * rho * ke;
      }
      if (bc.kind == FV_BC_NOSLIP && f < 2 * g.ndim)
        for (int a = 1; a <= 3; ++a) B.bc_q[f][a] = bc.prim_in[a];  // wall velocity
    }
    out.push_back(B);
    soff += B.ncell * g.nv;
  }
}

hipError_t upload_nodes(const HostGrid& g, char* dst, hipStream_t s) {
  size_t off = 0;
  for (int b = 0; b < g.nblocks; ++b) {
    if (g.xs[b].empty()) continue;
    const size_t bytes = g.xs[b].size() * sizeof(double);
    const std::vector<double>* c[3] = {&g.xs[b], &g.ys[b], &g.zs[b]};
    for (int a = 0; a < (g.ndim == 3 ? 3 : 2); ++a) {
      const hipError_t e = hipMemcpyAsync(dst + off, c[a]->data(), bytes, hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return e;
      off += bytes;
    }
  }
  return hipSuccess;
}

TileShape default_shape(const HostGrid& g) {
  TileShape s;
  if (g.ndim == 2) {
    // aim for about 8 wavefronts per SIMD across the chip, 4..64 rows
    const long long cells = g.ncells;
    long long want = cells / (64LL * 8192);
    int rows = 4;
    while (rows < 64 && rows * 2 <= want) rows *= 2;
    s.rows = rows;
    s.ny = 1;
  } else if (g.gen3) {
    s.ny = 4;
    s.rows = 16;
  } else {
    s.ny = 7;
    s.rows = 32;
  }
  return s;
}

void build_tiles(const HostGrid& g, const TileShape& sh, int inst_index, int boff,
                 std::vector<fvk::DevTile>& out) {
  out.clear();
  int local = 0;
  for (int b = 0; b < g.nblocks - g.nphantom; ++b) {
    const fv_block_desc& B = g.blocks[b];
    if (g.ndim == 2) {
      // at most 64 rows: the right-edge fluxes of a tile are formed one row per lane
      const int R = std::min(64, std::max(kMinRows2D, sh.rows));
      for (int j0 = 0; j0 < B.nj; j0 += R)
        for (int i0 = 0; i0 < B.ni; i0 += 64) {
          fvk::DevTile t;
          std::memset(&t, 0, sizeof(t));
          t.blk = b + boff;
          t.inst = inst_index;
          t.local = local++;
          t.ncol = std::min(64, B.ni - i0);
          t.i0 = i0;
          t.j0 = j0;
          t.k0 = 0;
          t.n = std::min(R, B.nj - j0);
          t.ny = 1;
          t.curv = B.x != nullptr ? 1 : 0;
          out.push_back(t);
        }
    } else {
      // at most 64 planes: the kernel keeps a row's right-edge fluxes in 64 LDS slots, one per plane
      const int P = std::min(64, std::max(kMinPlanes3D, sh.rows));
      const int NY = g.gen3 ? 4 : (sh.ny >= 7 ? 7 : 3);
      for (int k0 = 0; k0 < B.nk; k0 += P)
        for (int j0 = 0; j0 < B.nj; j0 += NY)
          for (int i0 = 0; i0 < B.ni; i0 += 64) {
            fvk::DevTile t;
            std::memset(&t, 0, sizeof(t));
            t.blk = b + boff;
            t.inst = inst_index;
            t.local = local++;
            t.ncol = std::min(64, B.ni - i0);
            t.i0 = i0;
            t.j0 = j0;
            t.k0 = k0;
            t.n = std::min(P, B.nk - k0);
            t.ny = std::min(NY, B.nj - j0);
            out.push_back(t);
          }
    }
  }
}

int size_class(const HostGrid& g) {
  int c = 0;
  long long n = g.ncells;
  while (n > 1) {
    n >>= 1;
    ++c;
  }
  return c;
}

std::string tune_key(const HostGrid& g, int precision, bool ns) {
  char buf[96];
  snprintf(buf, sizeof(buf), "%dd_%s_c%d%s%s", g.ndim, precision == FV_FP32_FLUX ? "fp32flux" : "fp64",
           size_class(g), ns ? "_ns" : "", g.gen3 ? "_gen" : "");
  return buf;
}

static std::mutex g_tune_mu;

const char* tune_path(const char* given) {
  if (given && given[0]) return given;
  const char* e = getenv("FV_AUTOTUNE_CACHE");
  return (e && e[0]) ? e : nullptr;
}

// The table is a flat JSON object {"key": {"rows": r, "ny": y, "ms": t}, ...}
static std::map<std::string, std::pair<TileShape, double>> read_table(const char* path) {
  std::map<std::string, std::pair<TileShape, double>> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t p = 0;
  while ((p = s.find('"', p)) != std::string::npos) {
    const size_t q = s.find('"', p + 1);
    if (q == std::string::npos) break;
    const std::string key = s.substr(p + 1, q - p - 1);
    const size_t lb = s.find('{', q), rb = s.find('}', q);
    if (lb == std::string::npos || rb == std::string::npos || lb > rb) {
      p = q + 1;
      continue;
    }
    const std::string body = s.substr(lb, rb - lb + 1);
    TileShape sh;
    double ms = 0.0;
    auto num = [&](const char* name, double& v) {
      const size_t a = body.find(std::string("\"") + name + "\"");
      if (a == std::string::npos) return false;
      const size_t c = body.find(':', a);
      v = atof(body.c_str() + c + 1);
      return true;
    };
    double r = 0, y = 0;
    if (num("rows", r) && num("ny", y)) {
      num("ms", ms);
      sh.rows = (int)r;
      sh.ny = (int)y;
      m[key] = {sh, ms};
    }
    p = rb + 1;
  }
  return m;
}

bool tune_lookup(const char* path, const std::string& key, TileShape& sh) {
  if (!path) return false;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto m = read_table(path);
  auto it = m.find(key);
  if (it == m.end()) return false;
  sh = it->second.first;
  return true;
}

void tune_store(const char* path, const std::string& key, const TileShape& sh, double ms) {
  if (!path) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto m = read_table(path);
  m[key] = {sh, ms};
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t n = 0;
  for (auto& kv : m) {
    fprintf(f, "  \"%s\": {\"rows\": %d, \"ny\": %d, \"ms\": %.6f}%s\n", kv.first.c_str(),
            kv.second.first.rows, kv.second.first.ny, kv.second.second, ++n < m.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

int rk_of(const fv_params* p) { return p->rk == 0 ? 3 : p->rk; }

int check_params(const fv_params* p) {
  if (!p) return set_error(FV_E_INVAL, "null params");
  if (p->precision != FV_FP64 && p->precision != FV_FP32_FLUX)
    return set_error(FV_E_INVAL, "unknown precision %d", p->precision);
  if (p->limiter < FV_LIM_MINMOD || p->limiter > FV_FIRST_ORDER)
    return set_error(FV_E_INVAL, "unknown limiter %d", p->limiter);
  if (p->rk != 0 && p->rk != 2 && p->rk != 3 && p->rk != 4)
    return set_error(FV_E_UNSUPPORTED, "rk %d: the schemes are 3 (SSP-RK3), 2 and 4", p->rk);
  if (!(p->dt_fixed > 0.0) && !(p->cfl > 0.0)) return set_error(FV_E_INVAL, "need cfl > 0 or dt_fixed > 0");
  if (!std::isfinite(p->cfl) || !std::isfinite(p->dt_fixed) || !std::isfinite(p->t_end) ||
      !std::isfinite(p->eps) || !std::isfinite(p->kappa) || !(p->entropy_fix >= 0.0))
    return set_error(FV_E_INVAL, "non-finite parameter");
  if (!(p->mu >= 0.0) || !std::isfinite(p->mu))
    return set_error(FV_E_INVAL, "viscosity mu must be finite and >= 0");
  if (p->mu > 0.0 && (!(p->prandtl > 0.0) || !std::isfinite(p->prandtl)))
    return set_error(FV_E_INVAL, "a viscous run needs a Prandtl number > 0");
  return FV_OK;
}

void params_to_inst(const fv_params* p, double gamma, fvk::DevInstance& I) {
  I.cfl = p->cfl;
  I.dt_fixed = p->dt_fixed;
  I.t_end = p->t_end;
  I.eps = p->eps;
  I.kappa = p->kappa;
  I.efix = p->entropy_fix;
  I.gamma = gamma;
  for (int v = 0; v < 5; ++v) I.qref[v] = p->qref[v];
  I.limiter = p->limiter;
  // stage coefficients of the scheme (the StageKind table): SSP-RK3 uses
  // c0 = 1 for its first stage; the 2- and 4-stage second-order schemes
  // write U^n + c_k dt L at stage k, with c3 the last stage's
  I.rk = rk_of(p);
  I.rk_c[0] = I.rk == 2 ? 0.5 : (I.rk == 4 ? 0.25 : 1.0);
  I.rk_c[1] = 1.0 / 3.0;
  I.rk_c[2] = 0.5;
  I.rk_c[3] = 1.0;
  I.mu = p->mu;
  I.prandtl = p->mu > 0.0 ? p->prandtl : 0.0;
}

int device_cu_count() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cus = v;
  }
  return cus;
}

int occupancy_blocks(const void* kernel, int block_threads) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block_threads, 0) != hipSuccess || n <= 0)
    n = 1;
  return n * device_cu_count();
}

}  // namespace fvrt

extern "C" const char* fv_last_error(void) { return fvrt::t_err.c_str(); }

extern "C" const char* fv_strerror(int s) {
  switch (s) {
    case FV_OK: return "ok";
    case FV_PENDING: return "pending";
    case FV_E_INVAL: return "invalid argument";
    case FV_E_NOMEM: return "workspace or arena too small";
    case FV_E_DEVICE: return "device error";
    case FV_E_NONPHYSICAL: return "non-physical state";
    case FV_E_UNSUPPORTED: return "unsupported";
    case FV_E_BUSY: return "busy";
    case FV_E_NOTFOUND: return "not found";
    case FV_E_CANCELLED: return "cancelled";
    default: return "unknown status";
  }
}

extern "C" void fv_default_params(fv_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->cfl = 0.5;
  p->precision = FV_FP64;
  p->limiter = FV_LIM_MINMOD;
  p->eps = 1.0;
  p->kappa = -1.0;
  p->entropy_fix = 0.1;
  p->rk = 3;
  for (int v = 0; v < 5; ++v) p->qref[v] = 1.0;
  p->mu = 0.0;
  p->prandtl = 0.72;
}
