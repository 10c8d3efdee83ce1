// Host runtime of libfdlb: problem set-up, device memory layout, binding,
// initial states, time marching, steady solves and outputs.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "fdlb_internal.h"

fdlb_problem::~fdlb_problem() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (pinned && own_pinned) (void)hipHostFree(pinned);
}

namespace fdlb {

namespace {

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

void rule_uncached(int kind, int n, std::vector<double>& x, std::vector<double>& w);

// Nodes and weights of a rule, computed once per (kind, n) for the process (the extended-
// precision construction costs ~1 ms; a batch of thousands of problems shares a few rules).
void rule(int kind, int n, std::vector<double>& x, std::vector<double>& w) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, std::pair<std::vector<double>, std::vector<double>>> cache;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find({kind, n});
        if (it != cache.end()) {
            x = it->second.first;
            w = it->second.second;
            return;
        }
    }
    rule_uncached(kind, n, x, w);
    std::lock_guard<std::mutex> lock(mu);
    cache.emplace(std::make_pair(kind, n), std::make_pair(x, w));
}

void rule_uncached(int kind, int n, std::vector<double>& x, std::vector<double>& w) {
    if (kind == FDLB_HALF) {
        if (n < 1 || n > 16) throw Error(FDLB_EINVAL, "half-range rule needs 1..16 nodes per half");
        x.resize(2 * n);
        w.resize(2 * n);
        quad_half_range(n, x.data(), w.data());
    } else if (kind == FDLB_FULL) {
        if (n < 1 || n > 32) throw Error(FDLB_EINVAL, "full-range rule needs 1..32 nodes");
        x.resize(n);
        w.resize(n);
        quad_full_range(n, x.data(), w.data());
    } else {
        throw Error(FDLB_EINVAL, "quadrature kind must be FDLB_HALF or FDLB_FULL");
    }
}

}  // namespace

bool tile_fits(const TileShape& t, int nx, int ny, bool periodic_x, bool periodic_y) {
    if (nx % t.vx) return false;
    if (!periodic_x && t.vx >= nx) return false;  // one lane must not hold both x walls
    if (!periodic_y && t.k >= ny) return false;   // nor both y walls
    if (t.lx == 1 && nx != 1) return false;       // column tiles are for single-cell-wide grids
    if (t.lx > 1 && nx == 1) return false;
    return true;
}

// Built-in choice of tile shape (the autotuner measures instead).  Among the shapes that fit:
// a grid with many cells (at least ~8 waves per CU without splitting the velocities) takes the
// widest vectors and the least idle lanes; a small grid takes the shape with the most waves (up
// to 8 per CU), splitting the velocities over several waves per tile.
int heuristic_tile_for(int precision, int nx, int ny, bool px, bool py) {
    const auto& shapes = tile_shapes(precision);
    const double cells = (double)nx * ny;
    const bool small = cells / (64.0 * 4.0) < 2048.0;  // < 8 waves/CU at 4 cells per lane
    int best = -1;
    double best_score = 1e300;
    for (size_t i = 0; i < shapes.size(); ++i) {
        const TileShape& t = shapes[i];
        if (!tile_fits(t, nx, ny, px, py)) continue;
        if (!small && t.wa != 1) continue;
        const int64_t tx = (nx + t.tile_w() - 1) / t.tile_w();
        const int64_t ty = (ny + t.tile_h() - 1) / t.tile_h();
        const double cover = (double)(tx * t.tile_w() * ty * t.tile_h()) / cells;
        double score;
        if (small) {
            const double waves = (double)(tx * ty) * t.wpb * t.wa;
            score = cover / std::min(waves, 2048.0);  // more than 8 waves per CU measured no faster
        } else {
            score = cover * (4.0 / t.vx) * (t.k > 1 ? 1.0 : 1.02);
        }
        if (score < best_score - 1e-12) {
            best_score = score;
            best = (int)i;
        }
    }
    if (best < 0) {  // small-grid shapes may not fit: any shape will do
        for (size_t i = 0; i < shapes.size(); ++i)
            if (tile_fits(shapes[i], nx, ny, px, py)) return (int)i;
        throw Error(FDLB_EINVAL, "no compiled tile shape fits this grid");
    }
    return best;
}

static int heuristic_tile(const fdlb_problem& p, int precision) {
    return heuristic_tile_for(precision, p.d.nx, p.d.ny, p.d.periodic_x, p.d.periodic_y);
}
static int heuristic_tile(const fdlb_problem& p) { return heuristic_tile(p, p.prec); }

template <class T>
std::vector<VelEntry<T>> vel_table(const fdlb_problem& p);

void build_problem(fdlb_problem& p, const fdlb_problem_desc& d) {
    if (d.nx < 1 || d.ny < 1) throw Error(FDLB_EINVAL, "nx and ny must be >= 1");
    if ((int64_t)d.nx * d.ny > (int64_t)1 << 28) throw Error(FDLB_EINVAL, "grid too large");
    if ((d.periodic_x && d.nx != 1) || (d.periodic_y && d.ny != 1))
        throw Error(FDLB_EINVAL, "a periodic axis must have exactly one cell");
    if (!d.periodic_x && d.nx < 2) throw Error(FDLB_EINVAL, "a bounded axis needs at least 2 cells");
    if (!d.periodic_y && d.ny < 2) throw Error(FDLB_EINVAL, "a bounded axis needs at least 2 cells");
    // The relaxation conserves momentum only if each rule integrates xi^2 exactly (sum w xi^2 = 1):
    // a Gauss rule of n nodes (per half-line) integrates degree 2n - 1, so n >= 2.  One node per
    // half-line gives sum w xi^2 = 2 / pi, and a one-node full-range rule has xi = 0 only.
    if (d.qx_n < 2 || d.qy_n < 2)
        throw Error(FDLB_EINVAL, "each velocity rule needs at least 2 nodes (per half-line for half-range) so that it "
                                 "integrates xi^2 exactly");
    if (d.precision != FDLB_FP32 && d.precision != FDLB_FP64 && d.precision != FDLB_MIXED)
        throw Error(FDLB_EINVAL, "precision must be FDLB_FP32, FDLB_FP64 or FDLB_MIXED");
    if (!(d.cfl > 0) || !std::isfinite(d.cfl)) throw Error(FDLB_EINVAL, "cfl must be positive and finite");
    if (!(d.kn > 0)) throw Error(FDLB_EINVAL, "kn must be positive (INFINITY allowed)");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(d.wall_u[i])) throw Error(FDLB_EINVAL, "wall speeds must be finite");
    if (!(d.lx >= 0) || !(d.ly >= 0) || !std::isfinite(d.lx) || !std::isfinite(d.ly))
        throw Error(FDLB_EINVAL, "domain lengths must be positive and finite (0 means 1)");
    p.d = d;
    if (p.d.lx == 0) p.d.lx = 1.0;
    if (p.d.ly == 0) p.d.ly = 1.0;
    std::vector<double> x, wx, y, wy;
    rule(d.qx_kind, d.qx_n, x, wx);
    rule(d.qy_kind, d.qy_n, y, wy);
    const int qx = (int)x.size(), qy = (int)y.size();
    p.q = qx * qy;
    if (p.q > 1024) throw Error(FDLB_EINVAL, "at most 1024 velocities");
    p.xi_x.resize(p.q);
    p.xi_y.resize(p.q);
    p.w.resize(p.q);
    for (int j = 0; j < qy; ++j)
        for (int i = 0; i < qx; ++i) {
            const int a = j * qx + i;
            p.xi_x[a] = x[i];
            p.xi_y[a] = y[j];
            p.w[a] = wy[j] * wx[i];
        }
    p.plane = (int64_t)d.nx * d.ny;
    p.L = std::max(d.nx, d.ny);
    // Time step of the unsplit donor cell: dt max_alpha(|xi_x| / dx + |xi_y| / dy) = CFL with
    // 1 / dx = N_x / l_x, counting only bounded axes (transport along a periodic single cell
    // vanishes).
    p.nux_scale = d.periodic_x ? 0.0 : (double)d.nx / p.d.lx;
    p.nuy_scale = d.periodic_y ? 0.0 : (double)d.ny / p.d.ly;
    double speed = 0;
    for (int a = 0; a < p.q; ++a)
        speed = std::max(speed, std::fabs(p.xi_x[a]) * p.nux_scale + std::fabs(p.xi_y[a]) * p.nuy_scale);
    if (!(speed > 0)) throw Error(FDLB_EINVAL, "no transport: both axes periodic");
    p.dt = d.cfl / speed;
    p.omega = std::isinf(d.kn) ? 0.0 : p.dt / d.kn;
    if (!d.allow_unstable && (d.cfl > 1.0 || p.omega > 1.0))
        throw Error(FDLB_EUNSTABLE, "explicit scheme unstable: need cfl <= 1 and dt/Kn <= 1 (dt/Kn = " +
                                        std::to_string(p.omega) + ")");
    // Pseudo-time stretch s of each velocity for steady iterations with local steps.  For one
    // velocity, with the equilibrium held fixed, the update h + s (S h - h) multiplies a Fourier
    // mode by 1 - s omega - s nu (1 - omega) z, z = 1 - e^{-i theta} (nu = nu_x + nu_y with a
    // z per axis), a circle that stays in the unit disk while s (omega + 2 nu (1 - omega)) <= 2.
    // s is taken as large as the problem's own margin allows, s (omega + 2 nu (1 - omega)) = 2 cfl
    // (the plain scheme has s = 1 and omega + 2 nu (1 - omega) <= 2 cfl for its fastest
    // velocity), with the stretched relaxation rate s omega <= 1 as in the plain scheme and
    // s <= FDLB_PSEUDO_MAX.
    p.pt.assign(p.q, 1.0);
    for (int a = 0; a < p.q; ++a) {
        const double nu = p.dt * (std::fabs(p.xi_x[a]) * p.nux_scale + std::fabs(p.xi_y[a]) * p.nuy_scale);
        double f = FDLB_PSEUDO_MAX;
        const double den = nu * (1.0 - p.omega) + 0.5 * p.omega;
        if (den > 0) f = std::min(f, d.cfl / den);
        if (p.omega > 0) f = std::min(f, 1.0 / p.omega);
        if (nu == 0 && p.omega == 0) f = 1.0;  // a population that never changes
        p.pt[a] = (double)(float)std::max(1.0, f);  // the kernels' table holds it as a float
    }
    // Wall constants of Eq. (9) in deviation form.  The wall density is the arriving flux over
    // the flux its emission (Eq. 8) carries per unit density, E = sum over leaving xi of
    // xi_n w: the wall is then impermeable for any rule.  A half-range rule integrates xi over
    // the half-line exactly, E = (2 pi)^(-1/2), and this is Eq. (9) as printed; a full-range
    // rule on a walled axis (the standard lattice) has its own E (0.444 for 4 nodes).
    for (int wl = 0; wl < 4; ++wl) {
        WallConst& W = p.wall[wl];
        W = WallConst{};
        W.active = (wl == BOTTOM || wl == TOP) ? !d.periodic_y : !d.periodic_x;
        W.u = d.wall_u[wl];
        long double A = 0, Bn = 0, Bt = 0, E = 0;
        for (int a = 0; a < p.q; ++a) {
            const double xn = wl == BOTTOM ? p.xi_y[a] : wl == TOP ? -p.xi_y[a] : wl == LEFT ? p.xi_x[a] : -p.xi_x[a];
            const double xt = (wl == BOTTOM || wl == TOP) ? p.xi_x[a] : p.xi_y[a];
            if (xn < 0) {
                A += (long double)(-xn) * p.w[a];
                Bn += (long double)(-xn) * p.w[a] * xn;
                Bt += (long double)(-xn) * p.w[a] * xt;
            } else if (xn > 0) {
                E += (long double)xn * p.w[a];
            }
        }
        const long double k = 1.0L / E;
        W.A = (double)A;
        W.Bn = (double)Bn;
        W.Bt = (double)Bt;
        W.k = (double)k;
        W.c0 = (double)(k * A - 1.0L);
    }
    // Velocity table grouped by quadrant: (+,+), (-,+), (+,-), (-,-); zero counts as +.
    p.quad_order.clear();
    for (int qd = 0; qd < 4; ++qd) {
        p.quad_begin[qd] = (int)p.quad_order.size();
        for (int a = 0; a < p.q; ++a) {
            const int sx = p.xi_x[a] < 0 ? 1 : 0, sy = p.xi_y[a] < 0 ? 1 : 0;
            if (sx + 2 * sy == qd) p.quad_order.push_back(a);
        }
    }
    p.quad_begin[4] = p.q;
    // Device layout.  A mixed-precision state starts in float inside buffers sized for double.
    p.prec = d.precision == FDLB_FP64 ? FDLB_FP64 : FDLB_FP32;
    p.elem = p.prec == FDLB_FP32 ? 4 : 8;
    const size_t store_elem = d.precision == FDLB_FP32 ? 4 : 8;
    p.pop_bytes = align256((size_t)p.q * p.plane * store_elem);
    p.state_bytes = 2 * p.pop_bytes;
    int maxb = 1;
    for (int prec : {FDLB_FP32, FDLB_FP64}) {
        if (d.precision != FDLB_MIXED && prec != p.prec) continue;
        for (const TileShape& t : tile_shapes(prec)) {
            const int64_t nb =
                (int64_t)((d.nx + t.tile_w() - 1) / t.tile_w()) * ((d.ny + t.tile_h() - 1) / t.tile_h());
            maxb = (int)std::max<int64_t>(maxb, nb);
        }
    }
    p.max_blocks = maxb;
    size_t off = 0;
    p.mom_bytes = align256(3 * (size_t)p.plane * sizeof(double));
    p.off_mom = off;
    off += 2 * p.mom_bytes;
    p.phi_bytes = align256(4 * (size_t)p.L * sizeof(double));
    p.off_phi = off;
    off += 2 * p.phi_bytes;
    p.off_part = off;  // residual partials, one region per buffer parity
    off += 2 * align256((size_t)maxb * 3 * sizeof(double));
    p.off_ctrl = off;
    off += align256(CTRL_DOUBLES * sizeof(double));
    p.off_vel = off;
    off += align256((size_t)p.q * (p.prec == FDLB_FP32 ? sizeof(VelEntry<float>) : sizeof(VelEntry<double>)));
    p.off_vel64 = off;
    off += align256((size_t)p.q * sizeof(VelEntry<double>));
    p.off_wall = off;
    off += align256(4 * sizeof(WallConst));
    p.off_wnat = off;
    off += align256((size_t)p.q * sizeof(double));
    p.io_bytes = align256(std::max<size_t>(4 * (size_t)p.plane * sizeof(double) + 64, 3 * (size_t)p.L * sizeof(double)));
    p.off_io = off;
    off += p.io_bytes;
    p.work_bytes = off;
    p.tile = heuristic_tile(p);
    p.tile_alt = d.precision == FDLB_MIXED ? heuristic_tile(p, FDLB_FP64) : -1;
    if (d.precision != FDLB_FP64) p.vel32 = vel_table<float>(p);
    p.vel64 = vel_table<double>(p);
}

// Switch the precision the kernels run in (FDLB_MIXED only changes it); the tile of the
// other precision is kept for the way back.
static void set_active(fdlb_problem& p, int prec) {
    if (p.prec == prec) return;
    p.prec = prec;
    p.elem = prec == FDLB_FP32 ? 4 : 8;
    std::swap(p.tile, p.tile_alt);
}

// A new state of a mixed-precision problem starts in float.
static void restart_precision(fdlb_problem& p) {
    if (p.d.precision == FDLB_MIXED) set_active(p, FDLB_FP32);
}

template <class T>
std::vector<VelEntry<T>> vel_table(const fdlb_problem& p) {
    std::vector<VelEntry<T>> v(p.q);
    for (int e = 0; e < p.q; ++e) {
        const int a = p.quad_order[e];
        VelEntry<T>& c = v[e];
        std::memset(&c, 0, sizeof(c));
        const double w = p.w[a], x = p.xi_x[a], y = p.xi_y[a];
        c.ow = (T)(p.omega * w);
        c.owx = (T)(p.omega * w * x);
        c.owy = (T)(p.omega * w * y);
        c.w = (T)w;
        c.wx = (T)(w * x);
        c.wy = (T)(w * y);
        c.xx = (T)x;
        c.xy = (T)y;
        c.nux = (T)(p.dt * std::fabs(x) * p.nux_scale);
        c.nuy = (T)(p.dt * std::fabs(y) * p.nuy_scale);
        c.alpha = a;
        c.pt = (float)p.pt[a];
        c.off = (int64_t)a * p.plane * (int64_t)sizeof(T);
    }
    return v;
}

// ---------------------------------------------------------------------------
// Binding and initial states.
// ---------------------------------------------------------------------------
static void require_bound(const fdlb_problem& p) {
    if (!p.bound) throw Error(FDLB_ESTATE, "problem is not bound to device memory (call fdlb_bind)");
}
static void require_seeded(const fdlb_problem& p) {
    require_bound(p);
    if (!p.seeded) throw Error(FDLB_ESTATE, "state not initialised (call an init or upload function)");
}

void bind(fdlb_problem& p, void* d_state, void* d_work, void* stream) {
    if (!d_state || !d_work) throw Error(FDLB_EINVAL, "device buffers must not be NULL");
    if (((uintptr_t)d_state & 255) || ((uintptr_t)d_work & 255))
        throw Error(FDLB_EINVAL, "device buffers must be 256-byte aligned");
    for (auto& kv : p.graphs) (void)hipGraphExecDestroy(kv.second);
    p.graphs.clear();
    p.d_state = (char*)d_state;
    p.d_work = (char*)d_work;
    p.stream = (hipStream_t)stream;
    if (!p.pinned) FDLB_HIP(hipHostMalloc((void**)&p.pinned, 64 * sizeof(double), hipHostMallocDefault));
    if (p.d.precision != FDLB_FP64)
        FDLB_HIP(hipMemcpyAsync(p.d_work + p.off_vel, p.vel32.data(), p.vel32.size() * sizeof(p.vel32[0]),
                                hipMemcpyHostToDevice, p.stream));
    FDLB_HIP(hipMemcpyAsync(p.d_work + p.off_vel64, p.vel64.data(), p.vel64.size() * sizeof(p.vel64[0]),
                            hipMemcpyHostToDevice, p.stream));
    if (p.d.precision == FDLB_FP64)
        FDLB_HIP(hipMemcpyAsync(p.d_work + p.off_vel, p.vel64.data(), p.vel64.size() * sizeof(p.vel64[0]),
                                hipMemcpyHostToDevice, p.stream));
    FDLB_HIP(hipMemcpyAsync(p.d_work + p.off_wall, p.wall, sizeof(p.wall), hipMemcpyHostToDevice, p.stream));
    FDLB_HIP(hipMemcpyAsync(p.d_work + p.off_wnat, p.w.data(), p.q * sizeof(double), hipMemcpyHostToDevice, p.stream));
    FDLB_HIP(hipStreamSynchronize(p.stream));
    p.bound = true;
    p.seeded = false;
}

static char* pop_buf(fdlb_problem& p, int parity) { return p.d_state + (size_t)parity * p.pop_bytes; }
static char* mom_buf(fdlb_problem& p, int parity) { return p.d_work + p.off_mom + (size_t)parity * p.mom_bytes; }
static double* phi_buf(fdlb_problem& p, int parity) {
    return (double*)(p.d_work + p.off_phi + (size_t)parity * p.phi_bytes);
}
static double* ctrl(fdlb_problem& p) { return (double*)(p.d_work + p.off_ctrl); }
// Residual partials of the step that reads population buffer `parity`.
double* partials_of(fdlb_problem& p, int parity) {
    return (double*)(p.d_work + p.off_part + (size_t)parity * align256((size_t)p.max_blocks * 3 * sizeof(double)));
}
static double* part_buf(fdlb_problem& p, int parity) { return partials_of(p, parity); }
static const VelEntry<double>* vel64(fdlb_problem& p) { return (const VelEntry<double>*)(p.d_work + p.off_vel64); }
static double* io(fdlb_problem& p) { return (double*)(p.d_work + p.off_io); }

// Reset the step counter and convergence records (host-to-device copy, never inside a graph).
// Without `sync` the copy from the problem's pinned slot may still be pending on return: the
// caller synchronizes the stream before that slot is written again.
static void reset_ctrl(fdlb_problem& p, double tol, bool sync = true) {
    double* h = p.pinned;
    std::fill(h, h + 8, 0.0);
    h[CTRL_FIRST_BELOW] = -1.0;
    h[CTRL_DIVERGED] = -1.0;
    h[CTRL_TOL] = tol;
    h[CTRL_FREEZE] = 0.0;
    p.freeze_on = false;
    FDLB_HIP(hipMemcpyAsync(ctrl(p), h, 8 * sizeof(double), hipMemcpyHostToDevice, p.stream));
    if (sync) FDLB_HIP(hipStreamSynchronize(p.stream));
}

// Recompute the moment and wall-flux buffers of the current state.
static void refresh_moments(fdlb_problem& p) {
    const int par = p.parity;
    if (p.prec == FDLB_FP32)
        launch_moments<float>((const float*)pop_buf(p, par), (double*)mom_buf(p, par), phi_buf(p, par),
                              (const VelEntry<float>*)(p.d_work + p.off_vel), p.q, p.d.nx, p.d.ny, p.L,
                              (const WallConst*)(p.d_work + p.off_wall), p.stream);
    else
        launch_moments<double>((const double*)pop_buf(p, par), (double*)mom_buf(p, par), phi_buf(p, par), vel64(p),
                               p.q, p.d.nx, p.d.ny, p.L, (const WallConst*)(p.d_work + p.off_wall), p.stream);
}

void init_equilibrium(fdlb_problem& p, const double* rho, const double* ux, const double* uy, int renorm) {
    require_bound(p);
    const int64_t n = p.plane;
    double* in = io(p);
    std::vector<double> r;
    const double *pr = nullptr, *pu = nullptr, *pv = nullptr;
    if (rho || renorm) {
        r.assign(n, 1.0);
        if (rho) std::copy(rho, rho + n, r.begin());
        if (renorm) {
            long double s = 0;
            for (double v : r) s += v;
            if (!(s > 0)) throw Error(FDLB_EINVAL, "total mass must be positive");
            const double scale = (double)((long double)n / s);
            for (double& v : r) v *= scale;
        }
        FDLB_HIP(hipMemcpyAsync(in, r.data(), n * sizeof(double), hipMemcpyHostToDevice, p.stream));
        pr = in;
    }
    if (ux) {
        FDLB_HIP(hipMemcpyAsync(in + n, ux, n * sizeof(double), hipMemcpyHostToDevice, p.stream));
        pu = in + n;
    }
    if (uy) {
        FDLB_HIP(hipMemcpyAsync(in + 2 * n, uy, n * sizeof(double), hipMemcpyHostToDevice, p.stream));
        pv = in + 2 * n;
    }
    p.parity = 0;
    restart_precision(p);
    if (p.prec == FDLB_FP32)
        launch_seed<float>((float*)pop_buf(p, 0), p.q, n, vel64(p), pr, pu, pv, nullptr, nullptr, nullptr, nullptr,
                           p.stream);
    else
        launch_seed<double>((double*)pop_buf(p, 0), p.q, n, vel64(p), pr, pu, pv, nullptr, nullptr, nullptr, nullptr,
                            p.stream);
    refresh_moments(p);
    FDLB_HIP(hipStreamSynchronize(p.stream));  // r is a host temporary
    p.seeded = true;
    reset_ctrl(p, 0.0);
}

// The state at rest (rho = 1, u = 0), as init_equilibrium with no fields, enqueued without
// waiting: the caller synchronizes the stream before the problem's pinned slot is reused (a batch
// re-seeds all its members and waits once).
void init_rest_async(fdlb_problem& p) {
    require_bound(p);
    p.parity = 0;
    restart_precision(p);
    if (p.prec == FDLB_FP32)
        launch_seed<float>((float*)pop_buf(p, 0), p.q, p.plane, vel64(p), nullptr, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr, p.stream);
    else
        launch_seed<double>((double*)pop_buf(p, 0), p.q, p.plane, vel64(p), nullptr, nullptr, nullptr, nullptr,
                            nullptr, nullptr, nullptr, p.stream);
    refresh_moments(p);
    p.seeded = true;
    reset_ctrl(p, 0.0, false);
}

void init_equilibrium_dev(fdlb_problem& p, const float* rho, const float* ux, const float* uy, int renorm) {
    require_bound(p);
    if (!rho || !ux || !uy) throw Error(FDLB_EINVAL, "device fields must not be NULL");
    double* scale = nullptr;
    if (renorm) {
        scale = io(p) + 4 * p.plane;
        launch_mass_scale(rho, p.plane, scale, p.stream);
    }
    p.parity = 0;
    restart_precision(p);
    if (p.prec == FDLB_FP32)
        launch_seed<float>((float*)pop_buf(p, 0), p.q, p.plane, vel64(p), nullptr, nullptr, nullptr, rho, ux, uy,
                           scale, p.stream);
    else
        launch_seed<double>((double*)pop_buf(p, 0), p.q, p.plane, vel64(p), nullptr, nullptr, nullptr, rho, ux, uy,
                            scale, p.stream);
    refresh_moments(p);
    p.seeded = true;
    reset_ctrl(p, 0.0);
}

void state_upload(fdlb_problem& p, const double* f) {
    require_bound(p);
    if (!f) throw Error(FDLB_EINVAL, "NULL host array");
    p.parity = 0;
    restart_precision(p);
    const int chunk = 4;
    for (int a0 = 0; a0 < p.q; a0 += chunk) {
        const int a1 = std::min(p.q, a0 + chunk);
        FDLB_HIP(hipMemcpyAsync(io(p), f + (size_t)a0 * p.plane, (size_t)(a1 - a0) * p.plane * sizeof(double),
                                hipMemcpyHostToDevice, p.stream));
        if (p.prec == FDLB_FP32)
            launch_from_raw<float>(io(p), (const double*)(p.d_work + p.off_wnat), a0, a1, p.plane,
                                   (float*)pop_buf(p, 0), p.stream);
        else
            launch_from_raw<double>(io(p), (const double*)(p.d_work + p.off_wnat), a0, a1, p.plane,
                                    (double*)pop_buf(p, 0), p.stream);
        FDLB_HIP(hipStreamSynchronize(p.stream));
    }
    refresh_moments(p);
    FDLB_HIP(hipStreamSynchronize(p.stream));
    p.seeded = true;
    reset_ctrl(p, 0.0);
}

void state_download(fdlb_problem& p, double* f) {
    require_seeded(p);
    if (!f) throw Error(FDLB_EINVAL, "NULL host array");
    const int chunk = 4;
    for (int a0 = 0; a0 < p.q; a0 += chunk) {
        const int a1 = std::min(p.q, a0 + chunk);
        if (p.prec == FDLB_FP32)
            launch_to_raw<float>((const float*)pop_buf(p, p.parity), (const double*)(p.d_work + p.off_wnat), a0, a1,
                                 p.plane, io(p), p.stream);
        else
            launch_to_raw<double>((const double*)pop_buf(p, p.parity), (const double*)(p.d_work + p.off_wnat), a0, a1,
                                  p.plane, io(p), p.stream);
        FDLB_HIP(hipMemcpyAsync(f + (size_t)a0 * p.plane, io(p), (size_t)(a1 - a0) * p.plane * sizeof(double),
                                hipMemcpyDeviceToHost, p.stream));
        FDLB_HIP(hipStreamSynchronize(p.stream));
    }
}

// Exact checkpoint: the current population buffer, its moment and wall-flux
// buffers and the step counter, as raw device bytes.
// A checkpoint opens with a header naming the problem it belongs to, checked before anything
// else is read: [magic, nx, ny, q, requested precision, precision of the stored state, x rule,
// y rule], a rule as 1000 kind + nodes (two sets with the same Q, such as a half-range rule and
// its transpose, order their populations differently).
constexpr double CKPT_MAGIC = 1178881090.0 + 2.0;  // "FDLB" as an integer, format 2
constexpr size_t CKPT_HEAD = 8 * sizeof(double);

static double rule_code(int kind, int n) { return 1000.0 * kind + n; }

size_t checkpoint_bytes(const fdlb_problem& p) {
    return CKPT_HEAD + p.pop_bytes + p.mom_bytes + p.phi_bytes + 8 * sizeof(double);
}

void checkpoint_save(fdlb_problem& p, void* host) {
    require_seeded(p);
    if (!host) throw Error(FDLB_EINVAL, "NULL host buffer");
    const double head[8] = {CKPT_MAGIC, (double)p.d.nx, (double)p.d.ny, (double)p.q, (double)p.d.precision,
                            (double)p.prec, rule_code(p.d.qx_kind, p.d.qx_n), rule_code(p.d.qy_kind, p.d.qy_n)};
    std::memcpy(host, head, CKPT_HEAD);
    char* h = (char*)host + CKPT_HEAD;
    FDLB_HIP(hipMemcpyAsync(h, pop_buf(p, p.parity), p.pop_bytes, hipMemcpyDeviceToHost, p.stream));
    FDLB_HIP(hipMemcpyAsync(h + p.pop_bytes, mom_buf(p, p.parity), p.mom_bytes, hipMemcpyDeviceToHost, p.stream));
    FDLB_HIP(hipMemcpyAsync(h + p.pop_bytes + p.mom_bytes, phi_buf(p, p.parity), p.phi_bytes, hipMemcpyDeviceToHost,
                            p.stream));
    FDLB_HIP(hipMemcpyAsync(h + p.pop_bytes + p.mom_bytes + p.phi_bytes, ctrl(p), 8 * sizeof(double),
                            hipMemcpyDeviceToHost, p.stream));
    FDLB_HIP(hipStreamSynchronize(p.stream));
}

void checkpoint_load(fdlb_problem& p, const void* host) {
    require_bound(p);
    if (!host) throw Error(FDLB_EINVAL, "NULL host buffer");
    double head[8];
    std::memcpy(head, host, CKPT_HEAD);
    if (head[0] != CKPT_MAGIC) throw Error(FDLB_EINVAL, "not a checkpoint of this library");
    if (head[1] != (double)p.d.nx || head[2] != (double)p.d.ny || head[3] != (double)p.q ||
        head[4] != (double)p.d.precision || head[6] != rule_code(p.d.qx_kind, p.d.qx_n) ||
        head[7] != rule_code(p.d.qy_kind, p.d.qy_n))
        throw Error(FDLB_EINVAL, "checkpoint of a different problem (grid, velocity set or precision)");
    const double prec = head[5];
    if (prec != (double)FDLB_FP32 && prec != (double)FDLB_FP64) throw Error(FDLB_EINVAL, "corrupt checkpoint header");
    if (p.d.precision != FDLB_MIXED && prec != (double)p.prec) throw Error(FDLB_EINVAL, "corrupt checkpoint header");
    const char* h = (const char*)host + CKPT_HEAD;
    // The saved control block, with the freeze request of a steady solve cleared: a restored
    // problem marches until a solve asks again.  The state goes to the buffer its step count
    // names (every path keeps the current buffer at step mod 2; a steady solve re-derives it).
    double c[8];
    std::memcpy(c, h + p.pop_bytes + p.mom_bytes + p.phi_bytes, 8 * sizeof(double));
    const double saved_step = c[CTRL_STEP];
    if (!(saved_step >= 0) || saved_step != std::floor(saved_step) || saved_step > 9.0e15)
        throw Error(FDLB_EINVAL, "corrupt checkpoint (step counter)");
    c[CTRL_FREEZE] = 0.0;
    if (p.d.precision == FDLB_MIXED) set_active(p, (int)prec);
    std::memcpy(p.pinned, c, sizeof(c));  // the control block is copied from pinned staging
    const int par = (int)((int64_t)saved_step & 1);
    FDLB_HIP(hipMemcpyAsync(pop_buf(p, par), h, p.pop_bytes, hipMemcpyHostToDevice, p.stream));
    FDLB_HIP(hipMemcpyAsync(mom_buf(p, par), h + p.pop_bytes, p.mom_bytes, hipMemcpyHostToDevice, p.stream));
    FDLB_HIP(hipMemcpyAsync(phi_buf(p, par), h + p.pop_bytes + p.mom_bytes, p.phi_bytes, hipMemcpyHostToDevice,
                            p.stream));
    FDLB_HIP(hipMemcpyAsync(ctrl(p), p.pinned, 8 * sizeof(double), hipMemcpyHostToDevice, p.stream));
    FDLB_HIP(hipStreamSynchronize(p.stream));
    p.parity = par;
    p.freeze_on = false;
    p.seeded = true;
}

// ---------------------------------------------------------------------------
// Time marching.
// ---------------------------------------------------------------------------
static int nblocks_of(const fdlb_problem& p, int tile);

// prev: this step reduces the previous step's residual partials inline.
template <class T>
static StepArgs<T> step_args(fdlb_problem& p, int parity, int tile, bool prev) {
    constexpr bool f32 = std::is_same<T, float>::value;
    const TileShape& t = tile_shapes(f32 ? FDLB_FP32 : FDLB_FP64)[tile];
    StepArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.src = (const T*)pop_buf(p, parity);
    a.dst = (T*)pop_buf(p, parity ^ 1);
    a.mom_in = (const double*)mom_buf(p, parity);
    a.mom_out = (double*)mom_buf(p, parity ^ 1);
    a.phi_in = phi_buf(p, parity);
    a.phi_out = phi_buf(p, parity ^ 1);
    a.partials = part_buf(p, parity);
    a.prev_partials = part_buf(p, parity ^ 1);
    a.prev_nb = prev ? nblocks_of(p, tile) : 0;
    a.pseudo = p.pseudo ? 1 : 0;
    a.ctrl = ctrl(p);
    a.vel = (const VelEntry<T>*)(p.d_work + (f32 ? p.off_vel : p.off_vel64));
    for (int i = 0; i < 5; ++i) a.quad_begin[i] = p.quad_begin[i];
    a.nx = p.d.nx;
    a.ny = p.d.ny;
    a.L = p.L;
    a.tiles_x = (p.d.nx + t.tile_w() - 1) / t.tile_w();
    a.tiles_y = (p.d.ny + t.tile_h() - 1) / t.tile_h();
    a.plane = p.plane;
    a.omega = (T)p.omega;
    a.omega_d = p.omega;
    for (int i = 0; i < 4; ++i) a.wall[i] = p.wall[i];
    return a;
}

static int nblocks_of(const fdlb_problem& p, int tile) {
    const TileShape& t = tile_shapes(p.prec)[tile];
    return ((p.d.nx + t.tile_w() - 1) / t.tile_w()) * ((p.d.ny + t.tile_h() - 1) / t.tile_h());
}

static bool inline_reduce(const fdlb_problem& p, int tile) { return nblocks_of(p, tile) <= INLINE_REDUCE_MAX_BLOCKS; }

// prev: the launch also reduces the previous step's partials, in one extra block.
static void launch_step_of(fdlb_problem& p, int parity, int tile, bool prev) {
    const int nb = nblocks_of(p, tile) + (prev ? 1 : 0);
    if (p.prec == FDLB_FP32)
        launch_step<float>(tile, step_args<float>(p, parity, tile, prev), nb, p.stream);
    else
        launch_step<double>(tile, step_args<double>(p, parity, tile, prev), nb, p.stream);
}

// Enqueue k steps from buffer `parity`: fused step kernels, and either a reduction kernel per
// step (large grids) or inline reductions closed by one single-wave reduction (small grids).
// Every chunk ends with its last step recorded, so the host may read the control block.
static void enqueue_chunk(fdlb_problem& p, int parity, int tile, int64_t k) {
    const int nb = nblocks_of(p, tile);
    const bool inl = inline_reduce(p, tile);
    int par = parity;
    for (int64_t i = 0; i < k; ++i) {
        launch_step_of(p, par, tile, inl && i > 0);
        if (!inl) launch_reduce(part_buf(p, par), nb, ctrl(p), 1, p.stream);
        par ^= 1;
    }
    if (inl && k > 0) launch_reduce_wave(part_buf(p, par ^ 1), nb, ctrl(p), p.stream);
}

static void enqueue_steps(fdlb_problem& p, int64_t n) {
    enqueue_chunk(p, p.parity, p.tile, n);
    if (n & 1) p.parity ^= 1;
}

// Plain stepping never freezes: clear the flag a previous steady solve left set.
static void unfreeze(fdlb_problem& p) {
    if (!p.freeze_on) return;
    p.pinned[CTRL_FREEZE] = 0.0;
    FDLB_HIP(hipMemcpyAsync(ctrl(p) + CTRL_FREEZE, p.pinned + CTRL_FREEZE, sizeof(double), hipMemcpyHostToDevice,
                            p.stream));
    FDLB_HIP(hipStreamSynchronize(p.stream));
    p.freeze_on = false;
}

// Mixed precision: carry the current float state over to double in place (the widened
// values are exact), then recompute its moments and wall fluxes with the double kernels so
// that the next step sees exactly what a double run from this state would.
// Widen a mixed-precision problem's state to double, enqueued on its stream.
void promote_async(fdlb_problem& p) {
    require_seeded(p);
    if (p.d.precision != FDLB_MIXED) throw Error(FDLB_EINVAL, "only a FDLB_MIXED problem changes precision");
    if (p.prec == FDLB_FP64) return;
    const int par = p.parity;
    const int64_t n = (int64_t)p.q * p.plane;
    launch_widen((const float*)pop_buf(p, par), (double*)pop_buf(p, par ^ 1), n, p.stream);
    launch_copy(pop_buf(p, par), pop_buf(p, par ^ 1), (size_t)n * sizeof(double), p.stream);
    set_active(p, FDLB_FP64);
    refresh_moments(p);
}

void promote(fdlb_problem& p) {
    promote_async(p);
    FDLB_HIP(hipStreamSynchronize(p.stream));
}

bool MixedSwitch::update(double r, int64_t step) {
    if (!on) return false;
    if (r < 0.9 * best) {
        best = r;
        best_step = step;
    }
    return r < FDLB_MIXED_SWITCH_R || step - best_step >= FDLB_MIXED_STALL_STEPS;
}

void step(fdlb_problem& p, int64_t n) {
    require_seeded(p);
    if (n < 0) throw Error(FDLB_EINVAL, "nsteps must be >= 0");
    unfreeze(p);
    enqueue_steps(p, n);
}

// fdlb_step on a caller's state buffer with the library's static device array as the workspace
// (for callers that cannot allocate).  The problem's binding, if any, is set aside for the call
// and restored afterwards; nothing is allocated, and no graph is captured or replayed.
void step_static(fdlb_problem& p, void* d_state, int64_t n, void* stream) {
    if (!d_state) throw Error(FDLB_EINVAL, "device state buffer must not be NULL");
    if ((uintptr_t)d_state & 255) throw Error(FDLB_EINVAL, "device state buffer must be 256-byte aligned");
    if (n < 0) throw Error(FDLB_EINVAL, "nsteps must be >= 0");
    if (p.d.precision == FDLB_MIXED) throw Error(FDLB_EINVAL, "fdlb_step_static takes FDLB_FP32 or FDLB_FP64 problems");
    if (p.off_io > (size_t)FDLB_STATIC_SCRATCH_BYTES)
        throw Error(FDLB_EINVAL, "problem needs " + std::to_string(p.off_io) + " bytes of workspace; the static scratch holds " +
                                     std::to_string((size_t)FDLB_STATIC_SCRATCH_BYTES));
    char* scratch = static_scratch();
    struct Saved {
        fdlb_problem& p;
        char *st, *wk;
        hipStream_t s;
        int parity;
        ~Saved() {
            p.d_state = st;
            p.d_work = wk;
            p.stream = s;
            p.parity = parity;
        }
    } saved{p, p.d_state, p.d_work, p.stream, p.parity};
    p.d_state = (char*)d_state;
    p.d_work = scratch;
    p.stream = (hipStream_t)stream;
    p.parity = 0;
    // Everything the kernels read is written here first: tables, a fresh control block (by a
    // kernel, not a memset), and the moments and wall fluxes of the given state.
    // (the float kernels read the float table, the double kernels the double one: the places
    // step_args and refresh_moments take them from)
    if (p.prec == FDLB_FP32)
        FDLB_HIP(hipMemcpyAsync(scratch + p.off_vel, p.vel32.data(), p.vel32.size() * sizeof(p.vel32[0]),
                                hipMemcpyHostToDevice, p.stream));
    else
        FDLB_HIP(hipMemcpyAsync(scratch + p.off_vel64, p.vel64.data(), p.vel64.size() * sizeof(p.vel64[0]),
                                hipMemcpyHostToDevice, p.stream));
    FDLB_HIP(hipMemcpyAsync(scratch + p.off_wall, p.wall, sizeof(p.wall), hipMemcpyHostToDevice, p.stream));
    launch_ctrl_reset(ctrl(p), p.stream);
    refresh_moments(p);
    enqueue_chunk(p, 0, p.tile, n);
}

void step_timed(fdlb_problem& p, int64_t n, double* ms_step, double* ms_reduce) {
    require_seeded(p);
    if (n < 1) throw Error(FDLB_EINVAL, "nsteps must be >= 1");
    unfreeze(p);
    std::vector<hipEvent_t> ev(2 * n + 1, nullptr);
    double a = 0, b = 0;
    try {
        for (auto& e : ev) FDLB_HIP(hipEventCreate(&e));
        const int nb = nblocks_of(p, p.tile);
        const bool inl = inline_reduce(p, p.tile);
        FDLB_HIP(hipEventRecord(ev[0], p.stream));
        for (int64_t i = 0; i < n; ++i) {  // every step closed by its own reduction kernel
            launch_step_of(p, p.parity, p.tile, false);
            FDLB_HIP(hipEventRecord(ev[2 * i + 1], p.stream));
            if (inl) launch_reduce_wave(part_buf(p, p.parity), nb, ctrl(p), p.stream);
            else launch_reduce(part_buf(p, p.parity), nb, ctrl(p), 1, p.stream);
            FDLB_HIP(hipEventRecord(ev[2 * i + 2], p.stream));
            p.parity ^= 1;
        }
        FDLB_HIP(hipEventSynchronize(ev[2 * n]));
        for (int64_t i = 0; i < n; ++i) {
            float t1 = 0, t2 = 0;
            FDLB_HIP(hipEventElapsedTime(&t1, ev[2 * i], ev[2 * i + 1]));
            FDLB_HIP(hipEventElapsedTime(&t2, ev[2 * i + 1], ev[2 * i + 2]));
            a += t1;
            b += t2;
        }
    } catch (...) {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        throw;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (ms_step) *ms_step = a;
    if (ms_reduce) *ms_reduce = b;
}

// Replay k steps as one captured graph (k even keeps the buffer parity).
static void enqueue_graph(fdlb_problem& p, int k) {
    auto key = std::make_tuple(k, p.prec, p.tile, p.parity);
    auto it = p.graphs.find(key);
    if (it == p.graphs.end()) {
        hipGraph_t g;
        FDLB_HIP(hipStreamBeginCapture(p.stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_chunk(p, p.parity, p.tile, k);
        } catch (...) {
            hipGraph_t dummy;
            (void)hipStreamEndCapture(p.stream, &dummy);
            throw;
        }
        FDLB_HIP(hipStreamEndCapture(p.stream, &g));
        hipGraphExec_t ge;
        FDLB_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        FDLB_HIP(hipGraphDestroy(g));
        it = p.graphs.emplace(key, ge).first;
    }
    FDLB_HIP(hipGraphLaunch(it->second, p.stream));
    if (k & 1) p.parity ^= 1;
}

static void read_ctrl(fdlb_problem& p) {
    FDLB_HIP(hipMemcpyAsync(p.pinned, ctrl(p), 8 * sizeof(double), hipMemcpyDeviceToHost, p.stream));
    FDLB_HIP(hipStreamSynchronize(p.stream));
}

void last_residual(fdlb_problem& p, double* r, int64_t* steps) {
    require_seeded(p);
    read_ctrl(p);
    if (r) *r = p.pinned[CTRL_LAST_R];
    if (steps) *steps = (int64_t)p.pinned[CTRL_STEP];
}

int solve_steady(fdlb_problem& p, double tol, int64_t max_steps, int32_t check_every, int32_t use_graph,
                 fdlb_report* rep) {
    require_seeded(p);
    if (!(tol >= 0) || max_steps < 0 || check_every < 1) throw Error(FDLB_EINVAL, "bad solve arguments");
    const bool graph = use_graph && p.stream != nullptr && check_every >= 2;
    // Keep the step counter; clear the convergence records, set the tolerance, and ask the
    // kernels to stop updating at the first step below it (the state then stays there).
    read_ctrl(p);
    const double base = p.pinned[CTRL_STEP];
    p.pinned[CTRL_FIRST_BELOW] = -1.0;
    p.pinned[CTRL_DIVERGED] = -1.0;
    p.pinned[CTRL_TOL] = tol;
    p.pinned[CTRL_FREEZE] = 1.0;
    FDLB_HIP(hipMemcpyAsync(ctrl(p) + CTRL_FIRST_BELOW, p.pinned + CTRL_FIRST_BELOW, 5 * sizeof(double),
                            hipMemcpyHostToDevice, p.stream));
    FDLB_HIP(hipStreamSynchronize(p.stream));
    p.freeze_on = true;
    MixedSwitch sw(p.d.precision == FDLB_MIXED && p.prec == FDLB_FP32 && tol < FDLB_MIXED_SWITCH_R, base);
    double fp32_until = p.prec == FDLB_FP32 ? -1.0 : base;  // step count where the float phase ended
    const auto t0 = std::chrono::steady_clock::now();
    int64_t launched = 0;
    int status = FDLB_ENOTCONVERGED;
    int32_t hlen = 0;
    while (launched < max_steps) {
        const int64_t k = std::min<int64_t>(check_every, max_steps - launched);
        if (graph && k == check_every) enqueue_graph(p, (int)k);
        else enqueue_steps(p, k);
        launched += k;
        read_ctrl(p);
        if (rep && rep->history && hlen < rep->history_cap) rep->history[hlen++] = p.pinned[CTRL_LAST_R];
        if (p.pinned[CTRL_DIVERGED] >= 0) {
            status = FDLB_EDIVERGED;
            break;
        }
        if (p.pinned[CTRL_FIRST_BELOW] >= 0) {
            status = FDLB_OK;
            break;
        }
        if (p.prec == FDLB_FP32 && sw.update(p.pinned[CTRL_LAST_R], (int64_t)p.pinned[CTRL_STEP])) {
            promote(p);
            fp32_until = p.pinned[CTRL_STEP];
        }
    }
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    // The device may have stopped inside the last chunk: its step counter says where.
    const int64_t done = (int64_t)(p.pinned[CTRL_STEP] - base);
    p.parity = (int)((int64_t)p.pinned[CTRL_STEP] & 1);
    const int64_t done32 = fp32_until < 0 ? done : (int64_t)(fp32_until - base);
    if (rep) {
        rep->steps = done;
        rep->first_below = status == FDLB_OK ? (int64_t)(p.pinned[CTRL_FIRST_BELOW] - base) : -1;
        rep->residual = p.pinned[CTRL_LAST_R];
        rep->wall_s = wall;
        const double upd = (double)done * (double)p.plane * p.q;
        rep->updates_per_s = wall > 0 ? upd / wall : 0;
        const double cell_q = (double)p.plane * p.q;
        const double bytes = cell_q * (8.0 * (double)done32 + 16.0 * (double)(done - done32));
        rep->bytes_per_s = wall > 0 ? bytes / wall : 0;
        rep->status = status;
        rep->history_len = hlen;
        rep->steps_fp32 = done32;
    }
    if (status == FDLB_EDIVERGED) {
        throw Error(FDLB_EDIVERGED, "solve diverged at step " + std::to_string((int64_t)(p.pinned[CTRL_DIVERGED] - base)) +
                                        " (non-finite residual or |u| > 0.5)");
    }
    return status;
}

// ---------------------------------------------------------------------------
// Outputs.
// ---------------------------------------------------------------------------
void moments(fdlb_problem& p, double* rho, double* ux, double* uy, double* pxy) {
    require_seeded(p);
    if (p.prec == FDLB_FP32)
        launch_post<float>((const float*)pop_buf(p, p.parity), vel64(p), p.q, p.d.nx, p.d.ny, p.omega, io(p), p.stream);
    else
        launch_post<double>((const double*)pop_buf(p, p.parity), vel64(p), p.q, p.d.nx, p.d.ny, p.omega, io(p),
                            p.stream);
    double* outs[4] = {rho, ux, uy, pxy};
    for (int i = 0; i < 4; ++i)
        if (outs[i])
            FDLB_HIP(hipMemcpyAsync(outs[i], io(p) + (size_t)i * p.plane, p.plane * sizeof(double),
                                    hipMemcpyDeviceToHost, p.stream));
    FDLB_HIP(hipStreamSynchronize(p.stream));
}

void wall_profile(fdlb_problem& p, int wall, double* rho, double* ut, double* pxy) {
    require_seeded(p);
    if (wall < 0 || wall > 3) throw Error(FDLB_EINVAL, "wall index must be 0..3");
    if (!p.wall[wall].active) throw Error(FDLB_EINVAL, "that wall is absent (periodic axis)");
    const int n = (wall == BOTTOM || wall == TOP) ? p.d.nx : p.d.ny;
    if (p.prec == FDLB_FP32)
        launch_wall_profile<float>((const float*)pop_buf(p, p.parity), vel64(p), p.q, p.d.nx, p.d.ny, wall,
                                   &p.wall[wall], p.omega, io(p), p.stream);
    else
        launch_wall_profile<double>((const double*)pop_buf(p, p.parity), vel64(p), p.q, p.d.nx, p.d.ny, wall,
                                    &p.wall[wall], p.omega, io(p), p.stream);
    double* outs[3] = {rho, ut, pxy};
    for (int i = 0; i < 3; ++i)
        if (outs[i])
            FDLB_HIP(hipMemcpyAsync(outs[i], io(p) + (size_t)i * n, n * sizeof(double), hipMemcpyDeviceToHost,
                                    p.stream));
    FDLB_HIP(hipStreamSynchronize(p.stream));
}

// Training samples of the warm-start network from the current state: per cell the encoded
// input (Kn, x, y) and the fields scaled by the fastest wall speed.  Asynchronous.
void field_samples(fdlb_problem& p, float* in, float* target) {
    require_seeded(p);
    if (!in || !target) throw Error(FDLB_EINVAL, "NULL output array");
    if (!std::isfinite(p.d.kn)) throw Error(FDLB_EINVAL, "samples need a finite Kn");
    double uw = 0;
    for (int w = 0; w < 4; ++w)
        if (p.wall[w].active) uw = std::max(uw, std::fabs(p.wall[w].u));
    if (!(uw > 0)) throw Error(FDLB_EINVAL, "samples need a moving wall (the fields are scaled by its speed)");
    if (p.prec == FDLB_FP32)
        launch_post<float>((const float*)pop_buf(p, p.parity), vel64(p), p.q, p.d.nx, p.d.ny, p.omega, io(p), p.stream);
    else
        launch_post<double>((const double*)pop_buf(p, p.parity), vel64(p), p.q, p.d.nx, p.d.ny, p.omega, io(p),
                            p.stream);
    launch_field_samples(io(p), p.d.nx, p.d.ny, mlp_kn_feature(p.d.kn), 1.0 / uw, in, target, p.stream);
}

// ---------------------------------------------------------------------------
// Tiles.
// ---------------------------------------------------------------------------
void set_pseudo_time(fdlb_problem& p, int on) {
    if (p.pseudo == (on != 0)) return;
    p.pseudo = on != 0;
    for (auto& kv : p.graphs) (void)hipGraphExecDestroy(kv.second);  // their launches carry the flag
    p.graphs.clear();
}

void set_tile(fdlb_problem& p, int tile) {
    if (tile < 0) {
        p.tile = heuristic_tile(p);
        return;
    }
    const auto& shapes = tile_shapes(p.prec);
    if (tile >= (int)shapes.size()) throw Error(FDLB_EINVAL, "tile index out of range");
    if (!tile_fits(shapes[tile], p.d.nx, p.d.ny, p.d.periodic_x, p.d.periodic_y))
        throw Error(FDLB_EINVAL, "tile shape does not fit this grid");
    if (nblocks_of(p, tile) > p.max_blocks) throw Error(FDLB_EINVAL, "tile needs more blocks than the workspace holds");
    p.tile = tile;
}

static std::string tune_key(const fdlb_problem& p) {
    return tune_key_prefix() + "/problem/prec" + std::to_string(p.d.precision) + "/" + std::to_string(p.d.nx) + "x" +
           std::to_string(p.d.ny) + "/q" + std::to_string(p.q) + "/per" + std::to_string(p.d.periodic_x) +
           std::to_string(p.d.periodic_y);
}

double autotune(fdlb_problem& p, int steps) {
    require_bound(p);
    if (steps < 1) throw Error(FDLB_EINVAL, "steps must be >= 1");
    restart_precision(p);  // a mixed-precision problem tunes its float phase
    const auto& shapes = tile_shapes(p.prec);
    std::string key;
    if (tune_cache_enabled()) {
        key = tune_key(p);
        int t = -1, ta = -1;
        double ms = 0;
        if (tune_cache_get(key, t, ta, ms) && t < (int)shapes.size() &&
            tile_fits(shapes[t], p.d.nx, p.d.ny, p.d.periodic_x, p.d.periodic_y) && nblocks_of(p, t) <= p.max_blocks) {
            p.tile = t;
            init_equilibrium(p, nullptr, nullptr, nullptr, 0);
            return ms;
        }
    }
    hipEvent_t e0, e1;
    FDLB_HIP(hipEventCreate(&e0));
    FDLB_HIP(hipEventCreate(&e1));
    double best = 1e300;
    int best_tile = p.tile;
    try {
        for (int t = 0; t < (int)shapes.size(); ++t) {
            if (!tile_fits(shapes[t], p.d.nx, p.d.ny, p.d.periodic_x, p.d.periodic_y)) continue;
            p.tile = t;
            init_equilibrium(p, nullptr, nullptr, nullptr, 0);
            step(p, 2);  // warm-up
            FDLB_HIP(hipEventRecord(e0, p.stream));
            step(p, steps);
            FDLB_HIP(hipEventRecord(e1, p.stream));
            FDLB_HIP(hipEventSynchronize(e1));
            float ms = 0;
            FDLB_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms / steps < best) {
                best = ms / steps;
                best_tile = t;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p.tile = best_tile;
    init_equilibrium(p, nullptr, nullptr, nullptr, 0);
    if (!key.empty()) tune_cache_put(key, best_tile, -1, best);
    return best;
}

}  // namespace fdlb
