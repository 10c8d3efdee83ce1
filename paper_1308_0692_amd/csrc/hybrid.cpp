// Host side of the hybrid half-range / full-range channel (fdlb_hybrid_*): validation, velocity
// sets, interface maps, device layout and the solve loop.  The kernels are in hybrid.hip.
//
// Interface maps (the coupling proposed in the paper's closing remarks, in this library's
// reading): a post-relaxation distribution g of one zone, for one x node, is expanded in
// probabilists' Hermite polynomials with the source rule, c_m = (1/m!) sum_a g_a He_m(xi_a),
// and evaluated at the target nodes, g'_k = w'_k sum_{m <= K} c_m He_m(xi'_k).  From bulk to
// layer K = n_full - 1 (the polynomial through the bulk values); from layer to bulk
// K = min(n_half, n_full) - 1 (the half-range rule integrates degree 2 n_half - 1 exactly, so
// it carries polynomials of degree <= n_half - 1 exactly through every coefficient up to K).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <vector>

#include "fdlb_internal.h"

struct fdlb_hybrid {
    std::vector<fdlb_hybrid_desc> desc;
    std::vector<fdlb::HybChan> ch;
    std::vector<double> tab;
    std::vector<int64_t> sdoubles;   // state doubles per channel
    std::vector<double> dt;
    std::vector<size_t> lds;         // LDS bytes per channel
    std::vector<int64_t> updates;    // cell-velocity updates per step per channel
    std::vector<fdlb::HybCtl> ctl_reset;  // host source of control-block resets (outlives the copies)
    size_t state_bytes = 0, work_bytes = 0;
    size_t off_chan = 0, off_tab = 0, off_ctl = 0, off_ring = 0, off_stage = 0;
    size_t lds_max = 0;
    char* d_state = nullptr;
    char* d_work = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
};

namespace fdlb {
namespace {

using ld = long double;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

ld hermite_e(int m, ld x) {
    if (m == 0) return 1;
    ld p0 = 1, p1 = x;
    for (int k = 1; k < m; ++k) {
        const ld p2 = x * p1 - (ld)k * p0;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

// T[k][a] carrying a weighted distribution on `src` nodes to `dst` nodes (weights wd) through
// its Hermite expansion truncated at `degree`.
std::vector<double> transfer(const std::vector<double>& src, const std::vector<double>& dst,
                             const std::vector<double>& wd, int degree) {
    std::vector<double> T(dst.size() * src.size());
    for (size_t k = 0; k < dst.size(); ++k)
        for (size_t a = 0; a < src.size(); ++a) {
            ld s = 0, fact = 1;
            for (int m = 0; m <= degree; ++m) {
                if (m > 0) fact *= m;
                s += hermite_e(m, dst[k]) * hermite_e(m, src[a]) / fact;
            }
            T[k * src.size() + a] = (double)((ld)wd[k] * s);
        }
    return T;
}

void rule(int kind, int n, std::vector<double>& x, std::vector<double>& w) {
    if (kind == FDLB_HALF) {
        if (n < 2 || n > 16) throw Error(FDLB_EINVAL, "half-range x rule needs 2..16 nodes per half-line");
        x.resize(2 * n);
        w.resize(2 * n);
        quad_half_range(n, x.data(), w.data());
    } else if (kind == FDLB_FULL) {
        if (n < 2 || n > 32) throw Error(FDLB_EINVAL, "full-range x rule needs 2..32 nodes");
        x.resize(n);
        w.resize(n);
        quad_full_range(n, x.data(), w.data());
    } else {
        throw Error(FDLB_EINVAL, "x rule kind must be FDLB_HALF or FDLB_FULL");
    }
}

void create(fdlb_hybrid& h, const fdlb_hybrid_desc* descs, int n) {
    if (!descs || n < 1 || n > 16384) throw Error(FDLB_EINVAL, "need 1..16384 channel descriptions");
    h.desc.assign(descs, descs + n);
    size_t tab_total = 0, state_total = 0, stage = 0;
    for (int c = 0; c < n; ++c) {
        const fdlb_hybrid_desc& d = descs[c];
        const std::string who = "channel " + std::to_string(c) + ": ";
        if (d.ny < 2 || d.ny > 4096) throw Error(FDLB_EINVAL, who + "ny must be 2..4096");
        if (d.layer < 1 || 2 * d.layer > d.ny) throw Error(FDLB_EINVAL, who + "layer must be 1..ny/2");
        if (!(d.kn > 0)) throw Error(FDLB_EINVAL, who + "Kn must be > 0 (INFINITY allowed)");
        if (!(d.cfl > 0) || !std::isfinite(d.cfl)) throw Error(FDLB_EINVAL, who + "cfl must be > 0");
        if (d.cfl > 1) throw Error(FDLB_EUNSTABLE, who + "cfl > 1");
        if (!std::isfinite(d.u_bottom) || !std::isfinite(d.u_top)) throw Error(FDLB_EINVAL, who + "plate speeds must be finite");
        if (d.n_half < 2 || d.n_half > 8) throw Error(FDLB_EINVAL, who + "n_half must be 2..8");
        if (d.n_full < 2 || d.n_full > 16) throw Error(FDLB_EINVAL, who + "n_full must be 2..16");
        std::vector<double> xx, wx, yh(2 * d.n_half), wh(2 * d.n_half), yf(d.n_full), wf(d.n_full);
        rule(d.qx_kind, d.qx_n, xx, wx);
        quad_half_range(d.n_half, yh.data(), wh.data());
        quad_full_range(d.n_full, yf.data(), wf.data());
        const int nx = (int)xx.size(), nh = (int)yh.size(), nf = (int)yf.size();
        if (nx * nh > 512) throw Error(FDLB_EINVAL, who + "more than 512 layer velocities");
        const bool bulk = 2 * d.layer < d.ny;
        double vmax = 0;
        for (double y : yh) vmax = std::max(vmax, std::fabs(y));
        if (bulk)
            for (double y : yf) vmax = std::max(vmax, std::fabs(y));
        const double dt = d.cfl / (vmax * d.ny);
        const double omega = std::isinf(d.kn) ? 0.0 : dt / d.kn;
        if (omega > 1) throw Error(FDLB_EUNSTABLE, who + "dt / Kn > 1: refine the grid or raise Kn");
        // table
        const size_t t0 = h.tab.size();
        auto put = [&](const std::vector<double>& v) { h.tab.insert(h.tab.end(), v.begin(), v.end()); };
        put(xx);
        put(wx);
        put(yh);
        put(wh);
        for (double y : yh) h.tab.push_back(dt * std::fabs(y) * d.ny);
        put(yf);
        put(wf);
        for (double y : yf) h.tab.push_back(dt * std::fabs(y) * d.ny);
        const int ka = std::min(d.n_half, d.n_full) - 1, kb = d.n_full - 1;
        put(transfer(yh, yf, wf, ka));
        put(transfer(yf, yh, wh, kb));
        // per-plane constants of the march kernel (layer planes, then bulk planes)
        for (int zone = 0; zone < 2; ++zone) {
            const std::vector<double>& yz = zone == 0 ? yh : yf;
            const std::vector<double>& wz = zone == 0 ? wh : wf;
            for (size_t a = 0; a < yz.size(); ++a)
                for (int i = 0; i < (int)xx.size(); ++i) {
                    const double W = wz[a] * wx[i], y = yz[a];
                    const double e[8] = {omega * W, omega * W * xx[i], omega * W * y, W, xx[i], y,
                                         dt * std::fabs(y) * d.ny, y > 0 ? 1.0 : (y < 0 ? -1.0 : 0.0)};
                    h.tab.insert(h.tab.end(), e, e + 8);
                }
        }
        double sx = 0, leave = 0;
        for (double w : wx) sx += w;
        for (int a = 0; a < nh; ++a)
            if (yh[a] > 0) leave += yh[a] * wh[a];
        HybChan C{};
        C.ny = d.ny;
        C.layer = d.layer;
        C.nx = nx;
        C.nh = nh;
        C.nf = nf;
        C.qh = nx * nh;
        C.qf = nx * nf;
        C.active = 1;
        C.tab_off = (int64_t)t0;
        C.ntab = (int32_t)(h.tab.size() - t0);
        C.omega = omega;
        C.e_inv = 1.0 / (leave * sx);
        C.u_bottom = d.u_bottom;
        C.u_top = d.u_top;
        double sxx = 0;
        for (int i = 0; i < nx; ++i) sxx += xx[i] * wx[i];
        for (int wall = 0; wall < 2; ++wall) {
            double A = 0, By = 0;
            for (int a = 0; a < nh; ++a) {
                const bool arriving = wall == 0 ? yh[a] < 0 : yh[a] > 0;
                if (!arriving) continue;
                A += std::fabs(yh[a]) * wh[a];
                By += std::fabs(yh[a]) * yh[a] * wh[a];
            }
            C.wA[wall] = A * sx;
            C.wBx[wall] = A * sxx;
            C.wBy[wall] = By * sx;
        }
        const int64_t S = 2 * (int64_t)d.layer * C.qh + (int64_t)(d.ny - 2 * d.layer) * C.qf;
        C.state_off = (int64_t)(state_total / sizeof(double));
        state_total += align256((size_t)S * sizeof(double));
        C.hist_off = (int64_t)c * HYB_RING;
        h.ch.push_back(C);
        h.sdoubles.push_back(S);
        h.dt.push_back(dt);
        h.lds.push_back(hybrid_lds_bytes(C));
        h.updates.push_back(S);
        h.lds_max = std::max(h.lds_max, h.lds.back());
        stage = std::max(stage, (size_t)(4 * d.ny + 8));
        tab_total = h.tab.size();
    }
    h.state_bytes = state_total;
    HybCtl z{};
    z.first_below = -1;
    z.residual = NAN;
    h.ctl_reset.assign(n, z);
    size_t off = 0;
    h.off_chan = off;
    off += align256(n * sizeof(HybChan));
    h.off_tab = off;
    off += align256(tab_total * sizeof(double));
    h.off_ctl = off;
    off += align256(n * sizeof(HybCtl));
    h.off_ring = off;
    off += align256((size_t)n * HYB_RING * sizeof(double));
    h.off_stage = off;
    off += align256(stage * sizeof(double));
    h.work_bytes = off;
}

fdlb_hybrid& hh(fdlb_hybrid* h) {
    if (!h) throw Error(FDLB_EINVAL, "NULL hybrid handle");
    return *h;
}

void need_bound(const fdlb_hybrid& h) {
    if (!h.bound) throw Error(FDLB_ESTATE, "hybrid batch is not bound");
}

void need_channel(const fdlb_hybrid& h, int i) {
    if (i < 0 || i >= (int)h.ch.size()) throw Error(FDLB_EINVAL, "channel index out of range");
}

HybChan* d_chans(fdlb_hybrid& h) { return (HybChan*)(h.d_work + h.off_chan); }
double* d_tab(fdlb_hybrid& h) { return (double*)(h.d_work + h.off_tab); }
HybCtl* d_ctl(fdlb_hybrid& h) { return (HybCtl*)(h.d_work + h.off_ctl); }
double* d_ring(fdlb_hybrid& h) { return (double*)(h.d_work + h.off_ring); }
double* d_stage(fdlb_hybrid& h) { return (double*)(h.d_work + h.off_stage); }

void upload_chans(fdlb_hybrid& h) {
    FDLB_HIP(hipMemcpyAsync(d_chans(h), h.ch.data(), h.ch.size() * sizeof(HybChan), hipMemcpyHostToDevice, h.stream));
}

void reset_ctl(fdlb_hybrid& h, int i) {
    FDLB_HIP(hipMemcpyAsync(d_ctl(h) + i, &h.ctl_reset[i], sizeof(HybCtl), hipMemcpyHostToDevice, h.stream));
}

void bind(fdlb_hybrid& h, void* d_state, void* d_work, void* stream) {
    if (!d_state || !d_work) throw Error(FDLB_EINVAL, "NULL device buffer");
    if (((uintptr_t)d_state & 255) || ((uintptr_t)d_work & 255)) throw Error(FDLB_EINVAL, "buffers must be 256-byte aligned");
    int dev = 0;
    FDLB_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    FDLB_HIP(hipGetDeviceProperties(&prop, dev));
    for (size_t c = 0; c < h.ch.size(); ++c)
        if (h.lds[c] > prop.sharedMemPerBlock)
            throw Error(FDLB_EINVAL, "channel " + std::to_string(c) + " needs " + std::to_string(h.lds[c]) +
                                         " bytes of LDS, more than the " + std::to_string(prop.sharedMemPerBlock) +
                                         " a workgroup may hold");
    hybrid_allow_lds(h.lds_max);
    h.d_state = (char*)d_state;
    h.d_work = (char*)d_work;
    h.stream = (hipStream_t)stream;
    upload_chans(h);
    FDLB_HIP(hipMemcpyAsync(d_tab(h), h.tab.data(), h.tab.size() * sizeof(double), hipMemcpyHostToDevice, h.stream));
    for (size_t c = 0; c < h.ch.size(); ++c) reset_ctl(h, (int)c);
    FDLB_HIP(hipStreamSynchronize(h.stream));
    h.bound = true;
}

void init_equilibrium(fdlb_hybrid& h, int i, const double* rho, const double* ux, const double* uy) {
    need_bound(h);
    need_channel(h, i);
    const int ny = h.ch[i].ny;
    std::vector<double> f(3 * (size_t)ny, 0.0);
    for (int j = 0; j < ny; ++j) {
        f[j] = rho ? rho[j] : 1.0;
        f[ny + j] = ux ? ux[j] : 0.0;
        f[2 * ny + j] = uy ? uy[j] : 0.0;
        if (!(f[j] > 0) || !std::isfinite(f[j]) || !std::isfinite(f[ny + j]) || !std::isfinite(f[2 * ny + j]))
            throw Error(FDLB_EINVAL, "seed fields must be finite with rho > 0");
    }
    FDLB_HIP(hipMemcpyAsync(d_stage(h), f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice, h.stream));
    launch_hybrid_seed(d_chans(h), i, ny, d_tab(h), (double*)h.d_state, d_stage(h), h.stream);
    reset_ctl(h, i);
    FDLB_HIP(hipStreamSynchronize(h.stream));
}

void set_state(fdlb_hybrid& h, int i, const double* host) {
    need_bound(h);
    need_channel(h, i);
    if (!host) throw Error(FDLB_EINVAL, "NULL state");
    FDLB_HIP(hipMemcpyAsync((double*)h.d_state + h.ch[i].state_off, host, h.sdoubles[i] * sizeof(double),
                            hipMemcpyHostToDevice, h.stream));
    reset_ctl(h, i);
    FDLB_HIP(hipStreamSynchronize(h.stream));
}

void get_state(fdlb_hybrid& h, int i, double* host) {
    need_bound(h);
    need_channel(h, i);
    if (!host) throw Error(FDLB_EINVAL, "NULL state");
    FDLB_HIP(hipMemcpyAsync(host, (double*)h.d_state + h.ch[i].state_off, h.sdoubles[i] * sizeof(double),
                            hipMemcpyDeviceToHost, h.stream));
    FDLB_HIP(hipStreamSynchronize(h.stream));
}

void step(fdlb_hybrid& h, int64_t nsteps) {
    need_bound(h);
    if (nsteps < 0) throw Error(FDLB_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return;
    bool changed = false;
    for (auto& c : h.ch)
        if (!c.active) {
            c.active = 1;
            changed = true;
        }
    if (changed) {
        upload_chans(h);
        FDLB_HIP(hipStreamSynchronize(h.stream));  // h.ch may change again before the copy would run
    }
    launch_hybrid_march(d_chans(h), (int)h.ch.size(), d_tab(h), (double*)h.d_state, d_ctl(h), d_ring(h), nsteps,
                        0.0, 0, h.lds_max, h.stream);
}

int solve(fdlb_hybrid& h, double tol, int64_t max_steps, int64_t chunk, fdlb_report* reps) {
    need_bound(h);
    if (!(tol >= 0) || max_steps < 0) throw Error(FDLB_EINVAL, "need tol >= 0 and max_steps >= 0");
    if (chunk <= 0) chunk = 100000;
    const int n = (int)h.ch.size();
    std::vector<HybCtl> ctl(n);
    FDLB_HIP(hipMemcpyAsync(ctl.data(), d_ctl(h), n * sizeof(HybCtl), hipMemcpyDeviceToHost, h.stream));
    FDLB_HIP(hipStreamSynchronize(h.stream));
    std::vector<int64_t> steps0(n);
    for (int c = 0; c < n; ++c) {
        steps0[c] = ctl[c].steps;
        ctl[c].status = 0;
        ctl[c].first_below = -1;
    }
    FDLB_HIP(hipMemcpyAsync(d_ctl(h), ctl.data(), n * sizeof(HybCtl), hipMemcpyHostToDevice, h.stream));
    const auto t0 = std::chrono::steady_clock::now();
    int64_t done = 0;
    while (done < max_steps) {
        const int64_t run = std::min(chunk, max_steps - done);
        int active = 0;
        for (int c = 0; c < n; ++c) {
            h.ch[c].active = ctl[c].status == 0 ? 1 : 0;
            active += h.ch[c].active;
        }
        if (!active) break;
        upload_chans(h);
        launch_hybrid_march(d_chans(h), n, d_tab(h), (double*)h.d_state, d_ctl(h), d_ring(h), run, tol, 1,
                            h.lds_max, h.stream);
        FDLB_HIP(hipMemcpyAsync(ctl.data(), d_ctl(h), n * sizeof(HybCtl), hipMemcpyDeviceToHost, h.stream));
        FDLB_HIP(hipStreamSynchronize(h.stream));
        done += run;
    }
    FDLB_HIP(hipStreamSynchronize(h.stream));
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int rc = FDLB_OK;
    for (int c = 0; c < n; ++c) {
        const int st = ctl[c].status == 1 ? FDLB_OK : ctl[c].status == 2 ? FDLB_EDIVERGED : FDLB_ENOTCONVERGED;
        if (st == FDLB_EDIVERGED) rc = FDLB_EDIVERGED;
        else if (st == FDLB_ENOTCONVERGED && rc == FDLB_OK) rc = FDLB_ENOTCONVERGED;
        if (!reps) continue;
        fdlb_report& r = reps[c];
        const int64_t taken = ctl[c].steps - steps0[c];
        r.steps = taken;
        r.first_below = ctl[c].first_below >= 0 ? ctl[c].first_below - steps0[c] : -1;
        r.residual = ctl[c].residual;
        r.wall_s = wall;
        r.updates_per_s = wall > 0 ? (double)h.updates[c] * (double)taken / wall : 0.0;
        r.bytes_per_s = r.updates_per_s * 2.0 * sizeof(double);
        r.status = st;
        r.steps_fp32 = 0;
        r.history_len = 0;
        if (r.history && r.history_cap > 0 && taken > 0) {
            const int64_t len = std::min<int64_t>({(int64_t)r.history_cap, taken, (int64_t)HYB_RING});
            std::vector<double> ring(HYB_RING);
            FDLB_HIP(hipMemcpyAsync(ring.data(), d_ring(h) + (size_t)c * HYB_RING, HYB_RING * sizeof(double),
                                    hipMemcpyDeviceToHost, h.stream));
            FDLB_HIP(hipStreamSynchronize(h.stream));
            const int64_t last = ctl[c].steps;  // step numbers last - len + 1 .. last
            for (int64_t s = 0; s < len; ++s) r.history[s] = ring[(last - len + s) % HYB_RING];
            r.history_len = (int32_t)len;
        }
    }
    return rc;
}

void post(fdlb_hybrid& h, int i, std::vector<double>& out) {
    need_bound(h);
    need_channel(h, i);
    const int ny = h.ch[i].ny;
    launch_hybrid_post(d_chans(h), i, d_tab(h), (const double*)h.d_state, d_stage(h), h.lds[i], h.stream);
    out.resize(4 * (size_t)ny + 8);
    FDLB_HIP(hipMemcpyAsync(out.data(), d_stage(h), out.size() * sizeof(double), hipMemcpyDeviceToHost, h.stream));
    FDLB_HIP(hipStreamSynchronize(h.stream));
}

}  // namespace

// partial moments of the march kernel: [G][3][ny] and [G][2]
static size_t hybrid_part_doubles(const HybChan& c) {
    const int nl = 2 * c.layer, nb = c.ny - 2 * c.layer;
    const int G = hyb_groups(((nl + 63) >> 6) + ((nb + 63) >> 6));
    return (size_t)G * (3 * (size_t)c.ny + 2);
}

size_t hybrid_lds_bytes(const HybChan& c) {
    const size_t S = 2 * (size_t)c.layer * c.qh + (size_t)(c.ny - 2 * c.layer) * c.qf;
    return sizeof(double) * ((size_t)c.ntab + 2 * S + 5 * (size_t)c.ny + 2 * (size_t)c.qh + 4 * (HYB_MARCH_THREADS / 64) + 2 +
                             2 * ((size_t)c.qh + c.qf) + 64 + hybrid_part_doubles(c));
}

int guard_call(const std::function<int()>& f);

}  // namespace fdlb

using namespace fdlb;

extern "C" {

int fdlb_hybrid_create(const fdlb_hybrid_desc* descs, int n, fdlb_hybrid** out) {
    return guard_call([&] {
        if (!out) throw Error(FDLB_EINVAL, "NULL output handle");
        *out = nullptr;
        auto h = std::make_unique<fdlb_hybrid>();
        create(*h, descs, n);
        *out = h.release();
        return FDLB_OK;
    });
}

void fdlb_hybrid_destroy(fdlb_hybrid* h) { delete h; }

size_t fdlb_hybrid_state_bytes(const fdlb_hybrid* h) { return h ? h->state_bytes : 0; }
size_t fdlb_hybrid_workspace_bytes(const fdlb_hybrid* h) { return h ? h->work_bytes : 0; }

int fdlb_hybrid_info(const fdlb_hybrid* h, int i, int32_t* q_layer, int32_t* q_bulk, int64_t* state_doubles,
                     double* dt, double* omega) {
    return guard_call([&] {
        if (!h) throw Error(FDLB_EINVAL, "NULL hybrid handle");
        need_channel(*h, i);
        if (q_layer) *q_layer = h->ch[i].qh;
        if (q_bulk) *q_bulk = h->ch[i].qf;
        if (state_doubles) *state_doubles = h->sdoubles[i];
        if (dt) *dt = h->dt[i];
        if (omega) *omega = h->ch[i].omega;
        return FDLB_OK;
    });
}

int fdlb_hybrid_bind(fdlb_hybrid* h, void* d_state, void* d_workspace, void* stream) {
    return guard_call([&] {
        bind(hh(h), d_state, d_workspace, stream);
        return FDLB_OK;
    });
}

int fdlb_hybrid_init_equilibrium(fdlb_hybrid* h, int i, const double* rho, const double* ux, const double* uy) {
    return guard_call([&] {
        init_equilibrium(hh(h), i, rho, ux, uy);
        return FDLB_OK;
    });
}

int fdlb_hybrid_set_state(fdlb_hybrid* h, int i, const double* host_state) {
    return guard_call([&] {
        set_state(hh(h), i, host_state);
        return FDLB_OK;
    });
}

int fdlb_hybrid_get_state(fdlb_hybrid* h, int i, double* host_state) {
    return guard_call([&] {
        get_state(hh(h), i, host_state);
        return FDLB_OK;
    });
}

int fdlb_hybrid_step(fdlb_hybrid* h, int64_t nsteps) {
    return guard_call([&] {
        step(hh(h), nsteps);
        return FDLB_OK;
    });
}

int fdlb_hybrid_solve(fdlb_hybrid* h, double tol, int64_t max_steps, int64_t chunk, fdlb_report* reps) {
    return guard_call([&] { return solve(hh(h), tol, max_steps, chunk, reps); });
}

int fdlb_hybrid_moments(fdlb_hybrid* h, int i, double* rho, double* ux, double* uy, double* pxy) {
    return guard_call([&] {
        std::vector<double> out;
        post(hh(h), i, out);
        const int ny = h->ch[i].ny;
        double* dst[4] = {rho, ux, uy, pxy};
        for (int q = 0; q < 4; ++q)
            if (dst[q]) std::memcpy(dst[q], out.data() + (size_t)q * ny, ny * sizeof(double));
        return FDLB_OK;
    });
}

int fdlb_hybrid_faces(fdlb_hybrid* h, int i, double* out8) {
    return guard_call([&] {
        if (!out8) throw Error(FDLB_EINVAL, "NULL output");
        std::vector<double> out;
        post(hh(h), i, out);
        std::memcpy(out8, out.data() + 4 * (size_t)h->ch[i].ny, 8 * sizeof(double));
        return FDLB_OK;
    });
}

}  // extern "C"
