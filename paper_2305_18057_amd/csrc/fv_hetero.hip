// CPU-GPU heterogeneous stepping of one 2D block: the synchronous workflow of
// Sec. 4 with the 1D domain decomposition of Sec. 6, for the Euler and the
// Navier-Stokes solver (Sec. 8 runs both this way).  The GPU part runs the
// 2D stage kernels (Euler, or Navier-Stokes for a viscosity or a no-slip
// face) on columns [0, split) of the block, with a two-column block after it
// that its block link reads and nothing computes (its storage is the halo
// the host part sends).  The host part runs the same stage arithmetic (the
// flux formulas of fv_device.h compiled for the host) on columns [split, ni),
// its rows dealt to a pool of worker threads.  Every RK substep: the two
// columns on each side of the cut cross over, both parts compute, everybody
// synchronizes.  The step end combines norms and time-step bounds and the
// host sets the common time step.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "fv_grid_impl.h"
#include "fv_launch.h"

using namespace fvrt;

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Worker threads that run one task at a time, each worker on its own share;
// the calling thread is worker 0.  Idle workers spin briefly, then sleep.
class Pool {
 public:
  explicit Pool(int n) : n_(std::max(1, n)) {
    for (int w = 1; w < n_; ++w) th_.emplace_back([this, w] { loop(w); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      quit_.store(true, std::memory_order_release);
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  int size() const { return n_; }
  // all workers of the running task meet here (generation-counted spin barrier)
  void barrier() {
    if (n_ == 1) return;
    const long g = bar_gen_.load(std::memory_order_acquire);
    if (bar_count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
      bar_count_.store(0, std::memory_order_relaxed);
      bar_gen_.fetch_add(1, std::memory_order_release);
    } else {
      while (bar_gen_.load(std::memory_order_acquire) == g) std::this_thread::yield();
    }
  }
  // run f(w) on every worker w and return when all have finished
  void run(const std::function<void(int)>& f) {
    if (n_ == 1) {
      f(0);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(m_);
      task_ = &f;
      done_.store(0, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    f(0);
    while (done_.load(std::memory_order_acquire) < n_ - 1) std::this_thread::yield();
  }

 private:
  void loop(int w) {
    long seen = 0;
    for (;;) {
      for (int s = 0; s < 4000 && gen_.load(std::memory_order_acquire) == seen &&
                      !quit_.load(std::memory_order_acquire);
           ++s)
        std::this_thread::yield();
      const std::function<void(int)>* f = nullptr;
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] {
          return quit_.load(std::memory_order_acquire) || gen_.load(std::memory_order_acquire) != seen;
        });
        if (quit_.load(std::memory_order_acquire)) return;
        seen = gen_.load(std::memory_order_acquire);
        f = task_;
      }
      (*f)(w);
      done_.fetch_add(1, std::memory_order_acq_rel);
    }
  }
  int n_;
  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_;
  std::atomic<long> gen_{0};
  std::atomic<int> done_{0};
  const std::function<void(int)>* task_ = nullptr;
  std::atomic<bool> quit_{false};
  std::atomic<int> bar_count_{0};
  std::atomic<long> bar_gen_{0};
};

constexpr int NV = 4;  // 2D

// The host part: columns [s, ni) of the block, stored [var][j][c].
struct HostPart {
  int ni = 0, nj = 0, nc = 0, s = 0;
  double gamma = 1.4;
  bool curv = false;
  double hx = 1.0, hy = 1.0;
  std::vector<double> u[3];
  // area vectors of the i-faces (nj rows of nc+1) and j-faces (nj+1 rows of
  // nc), volumes and the time-step bound's mean area vectors (nj x nc)
  std::vector<double> six, siy, sjx, sjy, vol, sb;
  int bc_kind[4] = {0, 0, 0, 0};
  double bcq[4][NV] = {};  // INFLOW: conserved state; NOSLIP: wall velocity in [1..2]
  // Navier-Stokes: node coordinates of node columns [s-2, ni], rows [0, nj];
  // (u, v, p/rho) and centres of the cells in columns [s-1, ni] and rows
  // [-1, nj] (ghost centres by the rule of the stage kernel; corners unused)
  std::vector<double> nx, ny, cx, cy, W;
  double bound_mu = 0.0, bound_pr = 0.0;  // viscosity of the current time-step bound
  std::vector<double> P;       // padded stage input [var][nj+4][nc+4]
  std::vector<double> fi, fj;  // face fluxes times area: [var][j][nc+1], [var][nj+1][c]
  std::vector<double> rsum;    // per row: 4 norm sums, minimum, flag
  double sums[NV] = {0, 0, 0, 0};
  double raw_min = 0.0;
  int bad = 0;

  int pw() const { return nc + 4; }
  int cw() const { return nc + 2; }
  size_t nd(int i, int j) const { return (size_t)j * (nc + 3) + (i - (s - 2)); }
  size_t ce(int i, int j) const { return (size_t)(j + 1) * cw() + (i - (s - 1)); }
  double& w(int k, int i, int j) { return W[(size_t)k * (nj + 2) * cw() + ce(i, j)]; }
  double& p(int v, int jj, int cc) { return P[((size_t)v * (nj + 4) + jj) * pw() + cc]; }
  double& U(int b, int v, int j, int c) { return u[b][((size_t)v * nj + j) * nc + c]; }
};

// rows [lo, hi) of n split over the pool's workers
inline void share(int n, int w, int nw, int& lo, int& hi) {
  lo = (int)((long long)n * w / nw);
  hi = (int)((long long)n * (w + 1) / nw);
}

// momentum mirrored about the area vector (Sx, Sy), as the device kernels do
inline void mirror(double* q, double Sx, double Sy) {
  const double ms = q[1] * Sx + q[2] * Sy;
  const double ss = Sx * Sx + Sy * Sy;
  const double fct = 2.0 * ms / ss;
  q[1] -= fct * Sx;
  q[2] -= fct * Sy;
}

// area vector of the wall face of a j-face side f (2, 3) at column i (i in
// [s-2, ni-1]), or of the i-max face at row j
void jwall_vec(const HostPart& H, int f, int i, double& sx, double& sy) {
  if (!H.curv) {
    sx = 0.0;
    sy = 1.0;
    return;
  }
  const int r = f == 2 ? 0 : H.nj;
  sx = -(H.ny[H.nd(i + 1, r)] - H.ny[H.nd(i, r)]);
  sy = H.nx[H.nd(i + 1, r)] - H.nx[H.nd(i, r)];
}
void imax_wall_vec(const HostPart& H, int j, double& sx, double& sy) {
  if (!H.curv) {
    sx = 1.0;
    sy = 0.0;
    return;
  }
  const size_t f = (size_t)j * (H.nc + 1) + H.nc;
  sx = H.six[f];
  sy = H.siy[f];
}

// State of cell (i, j) of the block, columns [s-2, ni+1] and rows [-2, nj+1],
// in buffer bin: the i-face rule first (the block's i-max face; columns s-2
// and s-1 are the GPU part's, from gh: [var][j][2]), then the j-face rule of
// the block, then the two transforms in reverse order, as the stage kernels
// resolve ghost and corner cells.
void cell_at(const HostPart& H, int bin, const double* gh, int i, int j, double* q) {
  int si = i, ikind = -1;
  if (i >= H.ni) {
    const int g = i - H.ni + 1;
    ikind = H.bc_kind[1];
    if (ikind == FV_BC_INFLOW) {
      for (int v = 0; v < NV; ++v) q[v] = H.bcq[1][v];
      return;
    }
    si = ikind == FV_BC_EXTRAP ? H.ni - 1 : H.ni - g;  // extrapolation or a wall
  }
  int sj = j, jkind = -1, jface = 2;
  bool set = false;
  if (j < 0 || j >= H.nj) {
    const int side = j < 0 ? 0 : 1;
    const int g = side == 0 ? -j : j - H.nj + 1;
    jface = 2 + side;
    jkind = H.bc_kind[jface];
    if (jkind == FV_BC_INFLOW) {
      for (int v = 0; v < NV; ++v) q[v] = H.bcq[jface][v];
      set = true;
    } else if (jkind == FV_BC_PERIODIC) {
      sj = side == 0 ? H.nj - g : g - 1;
    } else if (jkind == FV_BC_EXTRAP) {
      sj = side == 0 ? 0 : H.nj - 1;
    } else {
      sj = side == 0 ? g - 1 : H.nj - g;  // slip or no-slip wall
    }
  }
  if (!set) {
    for (int v = 0; v < NV; ++v)
      q[v] = si >= H.s ? H.u[bin][((size_t)v * H.nj + sj) * H.nc + (si - H.s)]
                       : gh[((size_t)v * H.nj + sj) * 2 + (si - (H.s - 2))];
    if (jkind == FV_BC_SLIPWALL) {
      double sx, sy;
      jwall_vec(H, jface, si, sx, sy);
      mirror(q, sx, sy);
    } else if (jkind == FV_BC_NOSLIP) {
      fvk::noslip_mirror<2>(q, H.bcq[jface]);
    }
  }
  if (ikind == FV_BC_SLIPWALL) {
    double sx, sy;
    imax_wall_vec(H, std::min(std::max(j, 0), H.nj - 1), sx, sy);
    mirror(q, sx, sy);
  } else if (ikind == FV_BC_NOSLIP) {
    fvk::noslip_mirror<2>(q, H.bcq[1]);
  }
}

// centre of cell (i, j), i in [s-1, ni], j in [-1, nj], from the nodes; a
// ghost centre is the interior one reflected through the boundary face's
// midpoint, or across a periodic face its image moved by the offset between
// the two faces (the rule of the Navier-Stokes stage kernel)
void centre_at(const HostPart& H, int i, int j, double& cx, double& cy) {
  auto node = [&](int a, int b, double& x, double& y) {
    x = H.nx[H.nd(a, b)];
    y = H.ny[H.nd(a, b)];
  };
  auto interior = [&](int a, int b, double& x, double& y) {
    double x0, y0, x1, y1, x2, y2, x3, y3;
    node(a, b, x0, y0);
    node(a + 1, b, x1, y1);
    node(a, b + 1, x2, y2);
    node(a + 1, b + 1, x3, y3);
    x = 0.25 * (((x0 + x1) + x2) + x3);
    y = 0.25 * (((y0 + y1) + y2) + y3);
  };
  const bool iin = i < H.ni, jin = j >= 0 && j < H.nj;
  if (iin && jin) {
    interior(i, j, cx, cy);
    return;
  }
  if (!iin && !jin) {
    cx = cy = 0.0;
    return;
  }
  double x0, y0, x1, y1;
  if (!iin) {  // beyond the i-max face (never periodic or linked here)
    node(H.ni, j, x0, y0);
    node(H.ni, j + 1, x1, y1);
    double ix, iy;
    interior(H.ni - 1, j, ix, iy);
    cx = 2.0 * (0.5 * (x0 + x1)) - ix;
    cy = 2.0 * (0.5 * (y0 + y1)) - iy;
    return;
  }
  const int side = j < 0 ? 0 : 1;
  const int w = side == 0 ? 0 : H.nj;
  node(i, w, x0, y0);
  node(i + 1, w, x1, y1);
  const double mx = 0.5 * (x0 + x1), my = 0.5 * (y0 + y1);
  if (H.bc_kind[2 + side] == FV_BC_PERIODIC) {
    const int along = side == 0 ? H.nj - 1 : 0, wo = side == 0 ? H.nj : 0;
    node(i, wo, x0, y0);
    node(i + 1, wo, x1, y1);
    const double ox = 0.5 * (x0 + x1), oy = 0.5 * (y0 + y1);
    interior(i, along, cx, cy);
    cx += mx - ox;
    cy += my - oy;
  } else {
    interior(i, side == 0 ? 0 : H.nj - 1, cx, cy);
    cx = 2.0 * mx - cx;
    cy = 2.0 * my - cy;
  }
}

// input and output buffer and coefficient slot of a stage kind (StageKind)
template <int MODE>
void kind_of(int& bin, int& bout, int& coef) {
  bin = fvk::StageKind<MODE>::bin;
  bout = fvk::StageKind<MODE>::bout;
  coef = fvk::StageKind<MODE>::coef;
}
void stage_buffers(int mode, int& bin, int& bout, int& coef) {
  switch (mode) {
    case 1: kind_of<1>(bin, bout, coef); break;
    case 2: kind_of<2>(bin, bout, coef); break;
    case 3: kind_of<3>(bin, bout, coef); break;
    case 4: kind_of<4>(bin, bout, coef); break;
    case 5: kind_of<5>(bin, bout, coef); break;
    default: kind_of<6>(bin, bout, coef); break;
  }
}

struct StageCtx {
  int mode, bin, bout, lim;
  double dt;  // dt times the stage coefficient
  fvk::Recon<double> rc;
  fvk::FluxK<double> K;
  const double* gh;  // the GPU part's columns split-2, split-1: [var][j][2]
  double mu = 0.0, prandtl = 0.72, kq = 0.0;  // viscosity, Prandtl number, mu/Pr gamma/(gamma-1)
};

// flux times area across a face from its four cells along the face normal
inline void face_flux(const StageCtx& X, const HostPart& H, const double* c0, const double* c1,
                      const double* c2, const double* c3, double Sx, double Sy, int axis,
                      double* F) {
  double qL[NV], qR[NV];
  for (int v = 0; v < NV; ++v) {
    double ep, em, ep2, em2;
    fvk::extrap<-1, double>(X.rc, c1[v] - c0[v], c2[v] - c1[v], ep, em);
    fvk::extrap<-1, double>(X.rc, c2[v] - c1[v], c3[v] - c2[v], ep2, em2);
    qL[v] = c1[v] + ep;
    qR[v] = c2[v] - em2;
  }
  if (H.curv) {
    double A, h;
    fvk::M<double>::sqrt2(fvk::fmad(Sx, Sx, Sy * Sy), A, h);
    const double iA = 2.0 * h;
    const double n[2] = {Sx * iA, Sy * iA};
    fvk::roe_flux<double, 2, -1>(qL, qR, n, A, X.K, F);
  } else if (axis == 0) {
    fvk::roe_flux<double, 2, 0>(qL, qR, nullptr, H.hy, X.K, F);
  } else {
    fvk::roe_flux<double, 2, 1>(qL, qR, nullptr, H.hx, X.K, F);
  }
}

// one RK substep of the host part (the stage kinds of fv_device.h)
void host_stage(HostPart& H, Pool& pool, const StageCtx& X) {
  const int nj = H.nj, nc = H.nc, nw = pool.size();
  const int bin = X.bin;
  const bool visc = X.mu > 0.0;
  // F -= F_nu . S for the face between cells (iL, jL) and (iR, jR) whose
  // nodes A, B have B - A turned by -90 degrees equal to S; a node's value
  // is the mean of the four cells around it
  auto node_w = [&](int i, int j, double* o) {
    for (int k = 0; k < 3; ++k)
      o[k] = 0.25 * (((H.w(k, i - 1, j - 1) + H.w(k, i, j - 1)) + H.w(k, i - 1, j)) + H.w(k, i, j));
  };
  auto visc_face = [&](int iL, int jL, int iR, int jR, int iA, int jA, int iB, int jB, double Sx,
                       double Sy, double* F) {
    double wL[3], wR[3], wA[3], wB[3], Fv[4];
    for (int k = 0; k < 3; ++k) {
      wL[k] = H.w(k, iL, jL);
      wR[k] = H.w(k, iR, jR);
    }
    node_w(iA, jA, wA);
    node_w(iB, jB, wB);
    const double dx = H.cx[H.ce(iR, jR)] - H.cx[H.ce(iL, jL)];
    const double dy = H.cy[H.ce(iR, jR)] - H.cy[H.ce(iL, jL)];
    fvk::visc_flux<double>(wL, wR, wA, wB, dx, dy, Sx, Sy, X.mu, X.kq, Fv);
    for (int v = 0; v < NV; ++v) F[v] -= Fv[v];
  };
  const bool reads_un = X.mode >= 2, low = X.mode >= 4, norms = X.mode <= 1,
             cfl = X.mode == 3 || X.mode == 6;
  pool.run([&](int w) {
    int lo, hi;
    // 1. padded input: own cells, the GPU's two columns, i-max and j ghosts
    //    and the corner ghosts (the viscous flux reads those next to the
    //    part); then (u, v, p/rho) of the cells the viscous flux reads
    share(nj + 4, w, nw, lo, hi);
    for (int jj = lo; jj < hi; ++jj) {
      double q[NV];
      const int j = jj - 2;
      if (jj < 2 || jj >= nj + 2) {
        for (int c = 0; c < nc + 4; ++c) {
          cell_at(H, bin, X.gh, H.s - 2 + c, j, q);
          for (int v = 0; v < NV; ++v) H.p(v, jj, c) = q[v];
        }
        continue;
      }
      for (int v = 0; v < NV; ++v) {
        std::memcpy(&H.p(v, jj, 2), &H.U(bin, v, j, 0), sizeof(double) * nc);
        H.p(v, jj, 0) = X.gh[((size_t)v * nj + j) * 2 + 0];
        H.p(v, jj, 1) = X.gh[((size_t)v * nj + j) * 2 + 1];
      }
      for (int g = 1; g <= 2; ++g) {
        cell_at(H, bin, X.gh, H.ni - 1 + g, j, q);
        for (int v = 0; v < NV; ++v) H.p(v, jj, nc + 1 + g) = q[v];
      }
    }
    pool.barrier();
    if (visc) {
      share(nj + 2, w, nw, lo, hi);
      for (int r = lo; r < hi; ++r)
        for (int c = 0; c < nc + 2; ++c) {
          const int i = H.s - 1 + c, j = r - 1;
          const double rho = H.p(0, r + 1, c + 1);
          const double ir = 1.0 / rho;
          const double u = H.p(1, r + 1, c + 1) * ir, v = H.p(2, r + 1, c + 1) * ir;
          const double pr = (H.gamma - 1.0) * (H.p(3, r + 1, c + 1) - 0.5 * rho * (u * u + v * v));
          H.w(0, i, j) = u;
          H.w(1, i, j) = v;
          H.w(2, i, j) = pr * ir;
        }
      pool.barrier();
    }
    // 2. face fluxes: i-faces of rows, j-faces of face rows
    share(nj, w, nw, lo, hi);
    double c0[NV], c1[NV], c2[NV], c3[NV], F[NV];
    for (int j = lo; j < hi; ++j)
      for (int f = 0; f <= nc; ++f) {
        for (int v = 0; v < NV; ++v) {
          c0[v] = H.p(v, j + 2, f);
          c1[v] = H.p(v, j + 2, f + 1);
          c2[v] = H.p(v, j + 2, f + 2);
          c3[v] = H.p(v, j + 2, f + 3);
        }
        const size_t fx = (size_t)j * (nc + 1) + f;
        face_flux(X, H, c0, c1, c2, c3, H.curv ? H.six[fx] : 0.0, H.curv ? H.siy[fx] : 0.0, 0, F);
        if (visc) {
          const int i = H.s + f;  // the face at i - 1/2, nodes (i, j) and (i, j+1)
          visc_face(i - 1, j, i, j, i, j, i, j + 1, H.curv ? H.six[fx] : H.hy, H.curv ? H.siy[fx] : 0.0, F);
        }
        for (int v = 0; v < NV; ++v) H.fi[((size_t)v * nj + j) * (nc + 1) + f] = F[v];
      }
    share(nj + 1, w, nw, lo, hi);
    for (int r = lo; r < hi; ++r)
      for (int c = 0; c < nc; ++c) {
        for (int v = 0; v < NV; ++v) {
          c0[v] = H.p(v, r, c + 2);
          c1[v] = H.p(v, r + 1, c + 2);
          c2[v] = H.p(v, r + 2, c + 2);
          c3[v] = H.p(v, r + 3, c + 2);
        }
        const size_t fx = (size_t)r * nc + c;
        face_flux(X, H, c0, c1, c2, c3, H.curv ? H.sjx[fx] : 0.0, H.curv ? H.sjy[fx] : 0.0, 1, F);
        if (visc) {
          const int i = H.s + c;  // the face at j - 1/2 (j = r), nodes (i+1, j) and (i, j)
          visc_face(i, r - 1, i, r, i + 1, r, i, r, H.curv ? H.sjx[fx] : 0.0, H.curv ? H.sjy[fx] : H.hx, F);
        }
        for (int v = 0; v < NV; ++v) H.fj[((size_t)v * (nj + 1) + r) * nc + c] = F[v];
      }
    pool.barrier();
    // 3. residual and update, with per-row norm sums and time-step minima
    share(nj, w, nw, lo, hi);
    for (int j = lo; j < hi; ++j) {
      double acc[NV] = {0, 0, 0, 0}, mn = INFINITY;
      int bad = 0;
      for (int c = 0; c < nc; ++c) {
        const size_t cell = (size_t)j * nc + c;
        const double vol = H.vol[cell];
        const double iv = 1.0 / vol;
        const double f = X.dt * iv;
        double out[NV];
        for (int v = 0; v < NV; ++v) {
          const double* FI = &H.fi[((size_t)v * nj + j) * (nc + 1)];
          const double* FJ = &H.fj[(size_t)v * (nj + 1) * nc];
          const double R = (0.0 + (FI[c + 1] - FI[c])) + (FJ[(size_t)(j + 1) * nc + c] - FJ[(size_t)j * nc + c]);
          if (norms) {
            const double rv = R * iv;
            acc[v] = fvk::fmad(rv, rv, acc[v]);
          }
          const double un = reads_un ? H.U(0, v, j, c) : 0.0;
          if (low) {
            out[v] = fvk::fmad(-f, R, un);
          } else {
            const double us = fvk::fmad(-f, R, H.U(bin, v, j, c));
            if (X.mode == 1) out[v] = us;
            else if (X.mode == 2) out[v] = fvk::fmad(0.75, un, 0.25 * us);
            else out[v] = fvk::fmad(1.0 / 3.0, un, (2.0 / 3.0) * us);
          }
        }
        for (int v = 0; v < NV; ++v) H.U(X.bout, v, j, c) = out[v];
        if (cfl) {
          const double Sb[2][3] = {{H.sb[4 * cell + 0], H.sb[4 * cell + 1], 0.0},
                                   {H.sb[4 * cell + 2], H.sb[4 * cell + 3], 0.0}};
          mn = std::min(mn, visc ? fvk::cell_dt_limit_visc(out, Sb, vol, H.gamma, X.mu, X.prandtl, bad)
                                 : fvk::cell_dt_limit<2>(out, Sb, vol, H.gamma, bad));
        }
      }
      double* rs = &H.rsum[(size_t)j * 6];
      for (int v = 0; v < NV; ++v) rs[v] = acc[v];
      rs[4] = mn;
      rs[5] = bad;
    }
  });
  // rows combined in row order: the result does not depend on the workers
  if (norms)
    for (int v = 0; v < NV; ++v) {
      double s = 0.0;
      for (int j = 0; j < nj; ++j) s += H.rsum[(size_t)j * 6 + v];
      H.sums[v] = s;
    }
  if (cfl) {
    double mn = INFINITY;
    int bad = 0;
    for (int j = 0; j < nj; ++j) {
      mn = std::min(mn, H.rsum[(size_t)j * 6 + 4]);
      bad |= H.rsum[(size_t)j * 6 + 5] != 0.0;
    }
    H.raw_min = mn;
    H.bad = bad;
  }
}

// time-step bound and physical check of the host part's U^n (with the
// viscous term for mu > 0)
void host_bound(HostPart& H, double mu, double prandtl) {
  double mn = INFINITY;
  int bad = 0;
  for (int j = 0; j < H.nj; ++j)
    for (int c = 0; c < H.nc; ++c) {
      const size_t cell = (size_t)j * H.nc + c;
      double q[NV];
      for (int v = 0; v < NV; ++v) q[v] = H.U(0, v, j, c);
      const double Sb[2][3] = {{H.sb[4 * cell + 0], H.sb[4 * cell + 1], 0.0},
                               {H.sb[4 * cell + 2], H.sb[4 * cell + 3], 0.0}};
      mn = std::min(mn, mu > 0.0 ? fvk::cell_dt_limit_visc(q, Sb, H.vol[cell], H.gamma, mu, prandtl, bad)
                                 : fvk::cell_dt_limit<2>(q, Sb, H.vol[cell], H.gamma, bad));
    }
  H.raw_min = mn;
  H.bad = bad;
  H.bound_mu = mu;
  H.bound_pr = prandtl;
}

// the grid checks of the split; fills the GPU part's 2-block host grid
int split_grids(const fv_grid_desc* desc, int split, HostGrid& whole, HostGrid& gpu) {
  int st = validate_and_copy(desc, whole);
  if (st) return st;
  if (whole.ndim != 2 || whole.nblocks != 1)
    return set_error(FV_E_UNSUPPORTED, "the CPU-GPU split takes one 2D block");
  if (whole.with_source)
    return set_error(FV_E_UNSUPPORTED, "the CPU-GPU split takes no source term");
  const fv_block_desc& B = whole.blocks[0];
  for (int f = 0; f < 4; ++f) {
    const int k = B.face[f].kind;
    if (k == FV_BC_BLOCK || (f < 2 && k == FV_BC_PERIODIC))
      return set_error(FV_E_UNSUPPORTED, "the CPU-GPU split cuts along i: i-faces may not be periodic or linked, no face may be linked");
  }
  if (split < 2 || split > B.ni - 2)
    return set_error(FV_E_INVAL, "split %d: both parts need at least 2 columns (2 <= split <= %d)", split, B.ni - 2);
  // GPU part: block 0 = columns [0, split), block 1 = the 2-column halo
  fv_block_desc b[2];
  b[0] = B;
  b[1] = B;
  b[0].ni = split;
  b[1].ni = 2;
  std::vector<double> x0, y0, x1, y1;
  if (B.x) {
    const int w = B.ni + 1;
    for (int j = 0; j <= B.nj; ++j) {
      for (int i = 0; i <= split; ++i) {
        x0.push_back(B.x[(size_t)j * w + i]);
        y0.push_back(B.y[(size_t)j * w + i]);
      }
      for (int i = split; i <= split + 2; ++i) {
        x1.push_back(B.x[(size_t)j * w + i]);
        y1.push_back(B.y[(size_t)j * w + i]);
      }
    }
    b[0].x = x0.data();
    b[0].y = y0.data();
    b[1].x = x1.data();
    b[1].y = y1.data();
  }
  b[1].origin[0] = B.origin[0] + split * B.h[0];
  b[0].face[1].kind = FV_BC_BLOCK;
  b[0].face[1].nbr_block = 1;
  b[0].face[1].nbr_face = FV_IMIN;
  b[0].face[1].orient = 0;
  b[1].face[0].kind = FV_BC_BLOCK;
  b[1].face[0].nbr_block = 0;
  b[1].face[0].nbr_face = FV_IMAX;
  b[1].face[0].orient = 0;
  b[1].face[1].kind = FV_BC_EXTRAP;
  fv_grid_desc d = *desc;
  d.nblocks = 2;
  d.blocks = b;
  d.with_source = 0;
  st = validate_and_copy(&d, gpu);
  if (st) return st;
  gpu.nphantom = 1;
  gpu.phantom_cells = 2LL * B.nj;
  return FV_OK;
}

}  // namespace

struct fv_hetero {
  HostGrid whole;
  fv_grid* gpu = nullptr;
  HostPart H;
  Pool* pool = nullptr;
  // pinned exchange buffers, two of each (one stage's while the next fills):
  // gh the GPU columns split-2, split-1 of a stage input, ch the host columns
  // split, split+1; evd[x] marks the arrival of gh[x]
  double* gh[2] = {nullptr, nullptr};
  double* ch[2] = {nullptr, nullptr};
  hipEvent_t evd[2] = {nullptr, nullptr};
  hipEvent_t evk[4][2] = {};  // around each stage kernel of a step
  int split = 0, nj = 0, ni = 0;
  int have_state = 0;
  // marching state of the whole block
  double t = 0.0, dt_dev = 0.0, norm_first = 0.0;
  long long steps = 0;
  int have_first = 0;
  ~fv_hetero() {
    if (gpu) fv_destroy_grid(gpu);
    delete pool;
    for (int x = 0; x < 2; ++x) {
      if (gh[x]) (void)hipHostFree(gh[x]);
      if (ch[x]) (void)hipHostFree(ch[x]);
      if (evd[x]) (void)hipEventDestroy(evd[x]);
    }
    for (auto& p : evk)
      for (auto& e : p)
        if (e) (void)hipEventDestroy(e);
  }
};

extern "C" size_t fv_hetero_workspace_bytes(const fv_grid_desc* desc, int split) {
  HostGrid whole, gpu;
  if (split_grids(desc, split, whole, gpu) != FV_OK) return 0;
  return layout_of(gpu).total;
}

extern "C" int fv_hetero_create(const fv_grid_desc* desc, int split, int cpu_workers,
                                void* d_workspace, size_t bytes, void* hip_stream, fv_hetero** out) {
  if (!out) return set_error(FV_E_INVAL, "null output handle");
  *out = nullptr;
  if (cpu_workers < 1 || cpu_workers > 1024)
    return set_error(FV_E_INVAL, "cpu_workers must be 1..1024 (got %d)", cpu_workers);
  HostGrid whole, gpu;
  int st = split_grids(desc, split, whole, gpu);
  if (st) return st;
  fv_hetero* h = new (std::nothrow) fv_hetero();
  if (!h) return set_error(FV_E_NOMEM, "host allocation failed");
  h->whole = std::move(whole);
  st = fvgrid::create(std::move(gpu), d_workspace, bytes, hip_stream, &h->gpu);
  if (st) {
    delete h;
    return st;
  }
  const fv_block_desc& B = h->whole.blocks[0];
  h->split = split;
  h->ni = B.ni;
  h->nj = B.nj;
  HostPart& H = h->H;
  H.ni = B.ni;
  H.nj = B.nj;
  H.s = split;
  H.nc = B.ni - split;
  H.gamma = h->whole.gamma;
  H.curv = B.x != nullptr;
  H.hx = B.h[0];
  H.hy = B.h[1];
  const size_t ncell = (size_t)H.nj * H.nc;
  try {
    for (auto& u : H.u) u.assign(NV * ncell, 0.0);
    H.P.assign((size_t)NV * (H.nj + 4) * (H.nc + 4), 0.0);
    H.fi.assign((size_t)NV * H.nj * (H.nc + 1), 0.0);
    H.fj.assign((size_t)NV * (H.nj + 1) * H.nc, 0.0);
    H.rsum.assign((size_t)H.nj * 6, 0.0);
    H.nx.assign((size_t)(H.nj + 1) * (H.nc + 3), 0.0);
    H.ny.assign(H.nx.size(), 0.0);
    H.cx.assign((size_t)(H.nj + 2) * H.cw(), 0.0);
    H.cy.assign(H.cx.size(), 0.0);
    H.W.assign(3 * H.cx.size(), 0.0);
    H.vol.assign(ncell, 0.0);
    H.sb.assign(4 * ncell, 0.0);
    if (H.curv) {
      H.six.assign((size_t)H.nj * (H.nc + 1), 0.0);
      H.siy.assign(H.six.size(), 0.0);
      H.sjx.assign((size_t)(H.nj + 1) * H.nc, 0.0);
      H.sjy.assign(H.sjx.size(), 0.0);
    }
    h->pool = new Pool(cpu_workers);
  } catch (...) {
    delete h;
    return set_error(FV_E_NOMEM, "host allocation failed");
  }
  // geometry of the host part: the device kernels' formulas
  const int w = B.ni + 1;
  auto X = [&](int i, int j) { return B.x[(size_t)j * w + i]; };
  auto Y = [&](int i, int j) { return B.y[(size_t)j * w + i]; };
  for (int j = 0; j < H.nj; ++j)
    for (int c = 0; c < H.nc; ++c) {
      const size_t cell = (size_t)j * H.nc + c;
      const int i = split + c;
      if (H.curv) {
        const double xa = X(i, j), ya = Y(i, j), xb = X(i + 1, j), yb = Y(i + 1, j);
        const double xc = X(i, j + 1), yc = Y(i, j + 1), xd = X(i + 1, j + 1), yd = Y(i + 1, j + 1);
        H.vol[cell] = 0.5 * fvk::fmad(xd - xa, yc - yb, -((xc - xb) * (yd - ya)));
        H.sb[4 * cell + 0] = 0.5 * ((yc - ya) + (yd - yb));
        H.sb[4 * cell + 1] = -0.5 * ((xc - xa) + (xd - xb));
        H.sb[4 * cell + 2] = -0.5 * ((yb - ya) + (yd - yc));
        H.sb[4 * cell + 3] = 0.5 * ((xb - xa) + (xd - xc));
      } else {
        H.vol[cell] = B.h[0] * B.h[1];
        H.sb[4 * cell + 0] = B.h[1];
        H.sb[4 * cell + 3] = B.h[0];
      }
    }
  if (H.curv) {
    for (int j = 0; j < H.nj; ++j)
      for (int f = 0; f <= H.nc; ++f) {
        const int i = split + f;
        H.six[(size_t)j * (H.nc + 1) + f] = Y(i, j + 1) - Y(i, j);
        H.siy[(size_t)j * (H.nc + 1) + f] = -(X(i, j + 1) - X(i, j));
      }
    for (int r = 0; r <= H.nj; ++r)
      for (int c = 0; c < H.nc; ++c) {
        const int i = split + c;
        H.sjx[(size_t)r * H.nc + c] = -(Y(i + 1, r) - Y(i, r));
        H.sjy[(size_t)r * H.nc + c] = X(i + 1, r) - X(i, r);
      }
  }
  // nodes of columns [s-2, ni] (the uniform lattice as the stage kernels
  // form it) and the cell centres the viscous flux reads
  for (int j = 0; j <= H.nj; ++j)
    for (int i = split - 2; i <= B.ni; ++i) {
      H.nx[H.nd(i, j)] = H.curv ? X(i, j) : B.origin[0] + i * B.h[0];
      H.ny[H.nd(i, j)] = H.curv ? Y(i, j) : B.origin[1] + j * B.h[1];
    }
  for (int f = 0; f < 4; ++f) {
    H.bc_kind[f] = B.face[f].kind;
    if (B.face[f].kind == FV_BC_NOSLIP)
      for (int a = 1; a <= 3; ++a) H.bcq[f][a] = B.face[f].prim_in[a];  // wall velocity
    if (B.face[f].kind == FV_BC_INFLOW) {
      const double rho = B.face[f].prim_in[0];
      const double u = B.face[f].prim_in[1], v = B.face[f].prim_in[2];
      H.bcq[f][0] = rho;
      H.bcq[f][1] = rho * u;
      H.bcq[f][2] = rho * v;
      H.bcq[f][3] = B.face[f].prim_in[4] / (H.gamma - 1.0) + 0.5 * rho * (u * u + v * v);
    }
  }
  for (int j = -1; j <= H.nj; ++j)
    for (int i = split - 1; i <= B.ni; ++i) centre_at(H, i, j, H.cx[H.ce(i, j)], H.cy[H.ce(i, j)]);
  const size_t xb = sizeof(double) * NV * H.nj * 2;
  bool ok = true;
  for (int x = 0; x < 2; ++x)
    ok = ok && hipHostMalloc((void**)&h->gh[x], xb, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void**)&h->ch[x], xb, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&h->evd[x], hipEventDisableTiming) == hipSuccess;
  for (auto& p : h->evk)
    for (auto& e : p) ok = ok && hipEventCreate(&e) == hipSuccess;
  if (!ok) {
    delete h;
    return set_error(FV_E_DEVICE, "pinned exchange buffers or events could not be created");
  }
  *out = h;
  return FV_OK;
}

extern "C" int fv_hetero_destroy(fv_hetero* h) {
  if (!h) return FV_E_INVAL;
  delete h;
  return FV_OK;
}

extern "C" int fv_hetero_set_state(fv_hetero* h, const double* U) {
  if (!h || !U) return set_error(FV_E_INVAL, "null argument");
  const int ni = h->ni, nj = h->nj, s = h->split;
  // the GPU part: block 0 (columns [0, s)) and the halo block (s, s+1)
  std::vector<double> Ug((size_t)NV * nj * (s + 2));
  for (int v = 0; v < NV; ++v)
    for (int j = 0; j < nj; ++j) {
      const double* row = U + ((size_t)v * nj + j) * ni;
      std::memcpy(&Ug[((size_t)v * nj + j) * s], row, sizeof(double) * s);
      std::memcpy(&Ug[(size_t)NV * nj * s + ((size_t)v * nj + j) * 2], row + s, sizeof(double) * 2);
      std::memcpy(&h->H.U(0, v, j, 0), row + s, sizeof(double) * (ni - s));
    }
  int st = fv_set_state(h->gpu, Ug.data(), 0);
  if (st && st != FV_E_NONPHYSICAL) return st;
  host_bound(h->H, h->H.bound_mu, h->H.bound_pr);
  h->t = 0.0;
  h->steps = 0;
  h->have_first = 0;
  h->norm_first = 0.0;
  h->have_state = 1;
  if (st == FV_E_NONPHYSICAL || h->H.bad)
    return set_error(FV_E_NONPHYSICAL, "initial state has a cell with rho <= 0, p <= 0 or a non-finite value");
  return FV_OK;
}

extern "C" int fv_hetero_get_state(fv_hetero* h, double* U) {
  if (!h || !U) return set_error(FV_E_INVAL, "null argument");
  const int ni = h->ni, nj = h->nj, s = h->split;
  std::vector<double> Ug((size_t)NV * nj * (s + 2));
  const int st = fv_get_state(h->gpu, Ug.data(), 0);
  if (st) return st;
  for (int v = 0; v < NV; ++v)
    for (int j = 0; j < nj; ++j) {
      double* row = U + ((size_t)v * nj + j) * ni;
      std::memcpy(row, &Ug[((size_t)v * nj + j) * s], sizeof(double) * s);
      std::memcpy(row + s, &h->H.U(0, v, j, 0), sizeof(double) * (ni - s));
    }
  return FV_OK;
}

extern "C" int fv_hetero_step(fv_hetero* h, const fv_params* p, int nsteps, fv_step_info* info,
                              double times_ms[4]) {
  const auto t_call = Clock::now();
  if (!h) return set_error(FV_E_INVAL, "null handle");
  int st = check_params(p);
  if (st) return st;
  if (!h->have_state) return set_error(FV_E_INVAL, "no state set");
  if (nsteps < 0) return set_error(FV_E_INVAL, "negative step count");
  fv_grid* g = h->gpu;
  HostPart& H = h->H;
  const int nj = h->nj, s = h->split;
  const int rk = rk_of(p);
  static const int kStages3[] = {1, 2, 3}, kStages2[] = {1, 6}, kStages4[] = {1, 4, 5, 6};
  const int* modes = rk == 2 ? kStages2 : (rk == 4 ? kStages4 : kStages3);
  const int nst = rk == 2 ? 2 : (rk == 4 ? 4 : 3);
  // the GPU instance marches under the host's time step: no stop rule of its own
  params_to_inst(p, h->whole.gamma, g->hinst);
  g->hinst.dt_fixed = 0.0;
  g->hinst.t_end = 0.0;
  g->hinst.drop_tol = 0.0;
  g->hinst.step_limit = LLONG_MAX;
  if ((st = fvgrid::put_inst(g, false))) return st;
  if ((st = fvgrid::use_params(g, p))) return st;
  FV_HIP(fvk::launch_prepare(g->stream, g->d_inst, nullptr, 1));
  g->plan.rk = rk;
  g->plan.lim = p->limiter;
  const int fp32 = p->precision == FV_FP32_FLUX;
  StageCtx X;
  X.lim = p->limiter;
  X.rc.lim = p->limiter;
  X.rc.heps = 0.5 * p->eps;
  X.rc.c1 = 0.25 * p->eps * (1.0 - p->kappa);
  X.rc.c2 = 0.25 * p->eps * (1.0 + p->kappa);
  X.K.gm1 = H.gamma - 1.0;
  X.K.efix = p->entropy_fix;
  X.K.iefix = p->entropy_fix > 0.0 ? 1.0 / p->entropy_fix : 0.0;
  X.gh = nullptr;  // set per stage
  X.mu = p->mu;
  X.prandtl = p->prandtl;
  X.kq = p->mu > 0.0 ? p->mu / p->prandtl * H.gamma / (H.gamma - 1.0) : 0.0;
  // the host part's time-step bound of U^n with this viscosity, as the GPU
  // part forms its own again in use_params
  if (H.bound_mu != p->mu || H.bound_pr != p->prandtl) host_bound(H, p->mu, p->prandtl);
  const long long ncell_gpu = (long long)nj * s, ncell_all = (long long)nj * h->ni;
  double t_gpu = 0.0, t_cpu = 0.0, t_x = 0.0;
  int flags = 0;
  double dt = 0.0, nrm[5] = {0, 0, 0, 0, 0}, comb = 0.0, drop = 0.0;
  const size_t xbytes = sizeof(double) * NV * nj * 2;
  double* const halo_dev_off[3] = {g->d_u[0] + (size_t)NV * nj * s, g->d_u[1] + (size_t)NV * nj * s,
                                   g->d_u[2] + (size_t)NV * nj * s};
  int k = 0;
  for (; k < nsteps; ++k) {
    // the common time step from the bounds of both parts
    const double mn = std::min(g->hinst.raw_min, H.raw_min);
    dt = p->dt_fixed > 0.0 ? p->dt_fixed : p->cfl * mn;
    bool last = false;
    if (p->t_end > 0.0) {
      if (h->t >= p->t_end) {
        flags |= FV_FLAG_T_END;
        break;
      }
      if (dt >= p->t_end - h->t) {
        dt = p->t_end - h->t;
        last = true;
      }
    }
    h->dt_dev = dt;
    FV_HIP(hipMemcpyAsync((char*)g->d_inst + offsetof(fvk::DevInstance, dt), &h->dt_dev,
                          sizeof(double), hipMemcpyHostToDevice, g->stream));
    // The exchange is pipelined on the stream: the GPU's columns of a stage's
    // output go to the host right behind the stage kernel (while the host
    // part computes the same stage), and the host's columns go to the device
    // before the next stage kernel, in stream order.  Buffers alternate.
    auto d2h = [&](int bin, int x) -> int {
      FV_HIP(hipMemcpy2DAsync(h->gh[x], 2 * sizeof(double), g->d_u[bin] + (s - 2),
                              (size_t)s * sizeof(double), 2 * sizeof(double), (size_t)NV * nj,
                              hipMemcpyDeviceToHost, g->stream));
      FV_HIP(hipEventRecord(h->evd[x], g->stream));
      return FV_OK;
    };
    auto h2d = [&](int bin, int x) -> int {
      double* c = h->ch[x];
      for (int v = 0; v < NV; ++v)
        for (int j = 0; j < nj; ++j) {
          c[((size_t)v * nj + j) * 2 + 0] = H.U(bin, v, j, 0);
          c[((size_t)v * nj + j) * 2 + 1] = H.U(bin, v, j, 1);
        }
      FV_HIP(hipMemcpyAsync(halo_dev_off[bin], c, xbytes, hipMemcpyHostToDevice, g->stream));
      return FV_OK;
    };
    int bins[4], bouts[4], coefs[4];
    for (int m = 0; m < nst; ++m) stage_buffers(modes[m], bins[m], bouts[m], coefs[m]);
    int x = 0;
    auto t0 = Clock::now();
    if ((st = d2h(bins[0], x)) || (st = h2d(bins[0], x))) return st;
    t_x += ms_since(t0);
    for (int m = 0; m < nst; ++m) {
      X.mode = modes[m];
      X.bin = bins[m];
      X.bout = bouts[m];
      X.dt = coefs[m] < 0 ? dt : dt * g->hinst.rk_c[coefs[m]];
      FV_HIP(hipEventRecord(h->evk[m][0], g->stream));
      st = fvexec::enqueue_stage(g->plan, modes[m], fp32, nullptr, g->stream);
      if (st) return st;
      FV_HIP(hipEventRecord(h->evk[m][1], g->stream));
      if (m + 1 < nst && (st = d2h(bins[m + 1], x ^ 1))) return st;
      t0 = Clock::now();
      FV_HIP(hipEventSynchronize(h->evd[x]));
      t_x += ms_since(t0);
      X.gh = h->gh[x];
      t0 = Clock::now();
      host_stage(H, *h->pool, X);
      t_cpu += ms_since(t0);
      if (m + 1 < nst) {
        t0 = Clock::now();
        if ((st = h2d(bins[m + 1], x ^ 1))) return st;
        t_x += ms_since(t0);
      }
      x ^= 1;
    }
    // step end: the GPU part's reductions, then the whole block's
    t0 = Clock::now();
    FV_HIP(fvk::launch_finalize(g->stream, g->d_inst, nullptr, 1));
    if ((st = fvgrid::get_inst(g))) return st;
    t_x += ms_since(t0);
    for (int m = 0; m < nst; ++m) {
      float ms = 0.f;
      FV_HIP(hipEventElapsedTime(&ms, h->evk[m][0], h->evk[m][1]));
      t_gpu += ms;
    }
    const fvk::DevInstance& I = g->hinst;
    double cs = 0.0;
    for (int v = 0; v < 5; ++v) {
      if (v < NV) {
        const double sg = I.norms[v] * I.norms[v] * (double)ncell_gpu;
        nrm[v] = std::sqrt((sg + H.sums[v]) / (double)ncell_all);
        const double q = p->qref[v] != 0.0 ? p->qref[v] : 1.0;
        const double r = nrm[v] / q;
        cs += r * r;
      } else {
        nrm[v] = 0.0;
      }
    }
    comb = std::sqrt(cs);
    if (!h->have_first) {
      h->norm_first = comb;
      h->have_first = 1;
    }
    drop = h->norm_first > 0.0 ? comb / h->norm_first : 0.0;
    h->t = last ? p->t_end : h->t + dt;
    h->steps += 1;
    if ((I.flags & fvk::FLAG_NONPHYS) || H.bad) {
      flags |= FV_FLAG_NONPHYSICAL;
      ++k;
      break;
    }
    if (last) {
      flags |= FV_FLAG_T_END;
      ++k;
      break;
    }
  }
  if (k >= nsteps && !(flags & (FV_FLAG_NONPHYSICAL | FV_FLAG_T_END))) flags |= FV_FLAG_STEP_LIMIT;
  if (info) {
    info->steps = h->steps;
    info->t = h->t;
    info->dt_last = dt;
    for (int v = 0; v < 5; ++v) info->norms[v] = nrm[v];
    info->norm = comb;
    info->drop = drop;
    info->flags = flags;
  }
  if (times_ms) {
    times_ms[0] = t_gpu;
    times_ms[1] = t_cpu;
    times_ms[2] = t_x;
    times_ms[3] = ms_since(t_call);
  }
  if (flags & FV_FLAG_NONPHYSICAL)
    return set_error(FV_E_NONPHYSICAL, "state turned non-physical after %lld steps", h->steps);
  return FV_OK;
}
