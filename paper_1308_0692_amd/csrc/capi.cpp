// extern "C" entry points of libfdlb (declared in include/fdlb.h).  Each one
// converts exceptions into status codes and a thread-local message.
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <string>

#include "fdlb_internal.h"

namespace fdlb {
void build_problem(fdlb_problem& p, const fdlb_problem_desc& d);
void bind(fdlb_problem& p, void* d_state, void* d_work, void* stream);
void init_equilibrium(fdlb_problem& p, const double* rho, const double* ux, const double* uy, int renorm);
void init_equilibrium_dev(fdlb_problem& p, const float* rho, const float* ux, const float* uy, int renorm);
void state_upload(fdlb_problem& p, const double* f);
void state_download(fdlb_problem& p, double* f);
size_t checkpoint_bytes(const fdlb_problem& p);
void checkpoint_save(fdlb_problem& p, void* host);
void checkpoint_load(fdlb_problem& p, const void* host);
void step(fdlb_problem& p, int64_t n);
void step_static(fdlb_problem& p, void* d_state, int64_t n, void* stream);
void step_timed(fdlb_problem& p, int64_t n, double* ms_step, double* ms_reduce);
void last_residual(fdlb_problem& p, double* r, int64_t* steps);
int solve_steady(fdlb_problem& p, double tol, int64_t max_steps, int32_t check_every, int32_t use_graph,
                 fdlb_report* rep);
void moments(fdlb_problem& p, double* rho, double* ux, double* uy, double* pxy);
void wall_profile(fdlb_problem& p, int wall, double* rho, double* ut, double* pxy);
void set_tile(fdlb_problem& p, int tile);
void set_pseudo_time(fdlb_problem& p, int on);
double autotune(fdlb_problem& p, int steps);
void promote(fdlb_problem& p);
void field_samples(fdlb_problem& p, float* in, float* target);

static thread_local std::string g_last_error;

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw Error(FDLB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
static int guard(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return FDLB_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return FDLB_EINVAL;
    } catch (...) {
        g_last_error = "unknown error";
        return FDLB_EINVAL;
    }
}

int guard_call(const std::function<int()>& f) { return guard(f); }

static fdlb_problem& handle(fdlb_problem* p) {
    if (!p) throw Error(FDLB_EINVAL, "NULL problem handle");
    return *p;
}

}  // namespace fdlb

using namespace fdlb;

extern "C" {

int fdlb_quad_half_range(int n, double* nodes, double* weights) {
    return guard([&] {
        if (!nodes || !weights) throw Error(FDLB_EINVAL, "NULL output array");
        quad_half_range(n, nodes, weights);
        return FDLB_OK;
    });
}

int fdlb_quad_full_range(int n, double* nodes, double* weights) {
    return guard([&] {
        if (!nodes || !weights) throw Error(FDLB_EINVAL, "NULL output array");
        quad_full_range(n, nodes, weights);
        return FDLB_OK;
    });
}

int fdlb_problem_create(const fdlb_problem_desc* desc, fdlb_problem** out) {
    return guard([&] {
        if (!desc || !out) throw Error(FDLB_EINVAL, "NULL argument");
        *out = nullptr;
        fdlb_problem* p = new fdlb_problem();
        try {
            build_problem(*p, *desc);
        } catch (...) {
            delete p;
            throw;
        }
        *out = p;
        return FDLB_OK;
    });
}

void fdlb_problem_destroy(fdlb_problem* p) { delete p; }

int fdlb_problem_q(const fdlb_problem* p) { return p ? p->q : FDLB_EINVAL; }
double fdlb_problem_dt(const fdlb_problem* p) { return p ? p->dt : std::nan(""); }
double fdlb_problem_omega(const fdlb_problem* p) { return p ? p->omega : std::nan(""); }

int fdlb_problem_velocities(const fdlb_problem* p, double* xi_x, double* xi_y, double* w) {
    return guard([&] {
        if (!p) throw Error(FDLB_EINVAL, "NULL problem handle");
        if (xi_x) std::memcpy(xi_x, p->xi_x.data(), p->q * sizeof(double));
        if (xi_y) std::memcpy(xi_y, p->xi_y.data(), p->q * sizeof(double));
        if (w) std::memcpy(w, p->w.data(), p->q * sizeof(double));
        return FDLB_OK;
    });
}

size_t fdlb_state_bytes(const fdlb_problem* p) { return p ? p->state_bytes : 0; }
size_t fdlb_workspace_bytes(const fdlb_problem* p) { return p ? p->work_bytes : 0; }

int fdlb_bind(fdlb_problem* p, void* d_state, void* d_workspace, void* stream) {
    return guard([&] {
        bind(handle(p), d_state, d_workspace, stream);
        return FDLB_OK;
    });
}

int fdlb_init_equilibrium(fdlb_problem* p, const double* rho, const double* ux, const double* uy,
                          int renormalize_mass) {
    return guard([&] {
        init_equilibrium(handle(p), rho, ux, uy, renormalize_mass);
        return FDLB_OK;
    });
}

int fdlb_init_equilibrium_dev(fdlb_problem* p, const float* d_rho, const float* d_ux, const float* d_uy,
                              int renormalize_mass) {
    return guard([&] {
        init_equilibrium_dev(handle(p), d_rho, d_ux, d_uy, renormalize_mass);
        return FDLB_OK;
    });
}

int fdlb_state_upload(fdlb_problem* p, const double* f_host) {
    return guard([&] {
        state_upload(handle(p), f_host);
        return FDLB_OK;
    });
}

int fdlb_state_download(fdlb_problem* p, double* f_host) {
    return guard([&] {
        state_download(handle(p), f_host);
        return FDLB_OK;
    });
}

size_t fdlb_checkpoint_bytes(const fdlb_problem* p) { return p ? checkpoint_bytes(*p) : 0; }

int fdlb_checkpoint_save(fdlb_problem* p, void* host_buf) {
    return guard([&] {
        checkpoint_save(handle(p), host_buf);
        return FDLB_OK;
    });
}

int fdlb_checkpoint_load(fdlb_problem* p, const void* host_buf) {
    return guard([&] {
        checkpoint_load(handle(p), host_buf);
        return FDLB_OK;
    });
}

int fdlb_step(fdlb_problem* p, int64_t nsteps) {
    return guard([&] {
        step(handle(p), nsteps);
        return FDLB_OK;
    });
}

int fdlb_step_static(fdlb_problem* p, void* d_state, int64_t nsteps, void* stream) {
    return guard([&] {
        step_static(handle(p), d_state, nsteps, stream);
        return FDLB_OK;
    });
}

int fdlb_step_timed(fdlb_problem* p, int64_t nsteps, double* ms_step_kernels, double* ms_reduce_kernels) {
    return guard([&] {
        step_timed(handle(p), nsteps, ms_step_kernels, ms_reduce_kernels);
        return FDLB_OK;
    });
}

int fdlb_last_residual(fdlb_problem* p, double* residual, int64_t* steps) {
    return guard([&] {
        last_residual(handle(p), residual, steps);
        return FDLB_OK;
    });
}

int fdlb_solve_steady(fdlb_problem* p, double tol, int64_t max_steps, int32_t check_every, int32_t use_graph,
                      fdlb_report* report) {
    return guard([&] { return solve_steady(handle(p), tol, max_steps, check_every, use_graph, report); });
}

int fdlb_moments(fdlb_problem* p, double* rho, double* ux, double* uy, double* pxy) {
    return guard([&] {
        moments(handle(p), rho, ux, uy, pxy);
        return FDLB_OK;
    });
}

int fdlb_wall_profile(fdlb_problem* p, int wall, double* rho, double* u_t, double* pxy) {
    return guard([&] {
        wall_profile(handle(p), wall, rho, u_t, pxy);
        return FDLB_OK;
    });
}

int fdlb_tile_count(int precision) {
    if (precision != FDLB_FP32 && precision != FDLB_FP64) return FDLB_EINVAL;
    return (int)tile_shapes(precision).size();
}

int fdlb_tile_describe(int precision, int tile, char* buf, size_t len) {
    return guard([&] {
        if (precision != FDLB_FP32 && precision != FDLB_FP64) throw Error(FDLB_EINVAL, "bad precision");
        const auto& s = tile_shapes(precision);
        if (tile < 0 || tile >= (int)s.size()) throw Error(FDLB_EINVAL, "tile index out of range");
        if (!buf || len == 0) throw Error(FDLB_EINVAL, "NULL buffer");
        const TileShape& t = s[tile];
        std::string d = "vx" + std::to_string(t.vx) + " lx" + std::to_string(t.lx) + " k" + std::to_string(t.k) +
                        " w" + std::to_string(t.wpb) + (t.wa > 1 ? " a" + std::to_string(t.wa) : std::string()) +
                        (t.wx > 1 ? " x" + std::to_string(t.wx) : std::string()) + (t.nt ? " nt" : "") + (t.pd > 1 ? " p" + std::to_string(t.pd) : std::string()) + " (" +
                        std::to_string(t.tile_w()) + "x" + std::to_string(t.tile_h()) + ")";
        std::strncpy(buf, d.c_str(), len - 1);
        buf[len - 1] = 0;
        return FDLB_OK;
    });
}

int fdlb_problem_set_tile(fdlb_problem* p, int tile) {
    return guard([&] {
        set_tile(handle(p), tile);
        return FDLB_OK;
    });
}

int fdlb_problem_get_tile(const fdlb_problem* p) { return p ? p->tile : FDLB_EINVAL; }

int fdlb_set_pseudo_time(fdlb_problem* p, int on) {
    return guard([&] {
        set_pseudo_time(handle(p), on);
        return FDLB_OK;
    });
}

int fdlb_problem_pseudo_weights(const fdlb_problem* p, double* stretch) {
    return guard([&] {
        if (!p) throw Error(FDLB_EINVAL, "NULL problem handle");
        if (!stretch) throw Error(FDLB_EINVAL, "NULL output array");
        for (int a = 0; a < p->q; ++a) stretch[a] = p->pt[a];
        return FDLB_OK;
    });
}

int fdlb_problem_active_precision(const fdlb_problem* p) { return p ? p->prec : FDLB_EINVAL; }

int fdlb_promote(fdlb_problem* p) {
    return guard([&] {
        promote(handle(p));
        return FDLB_OK;
    });
}

int fdlb_autotune(fdlb_problem* p, int steps, double* best_ms_per_step) {
    return guard([&] {
        const double ms = autotune(handle(p), steps);
        if (best_ms_per_step) *best_ms_per_step = ms;
        return FDLB_OK;
    });
}

int fdlb_set_tune_cache(const char* path) {
    return guard([&] {
        set_tune_cache_path(path);
        return FDLB_OK;
    });
}

int fdlb_field_samples(fdlb_problem* p, float* d_in, float* d_target) {
    return guard([&] {
        field_samples(handle(p), d_in, d_target);
        return FDLB_OK;
    });
}

int fdlb_stream_copy(void* d_dst, const void* d_src, size_t bytes, void* stream) {
    return guard([&] {
        if (!d_dst || !d_src) throw Error(FDLB_EINVAL, "NULL buffer");
        launch_copy(d_dst, d_src, bytes, (hipStream_t)stream);
        return FDLB_OK;
    });
}

int fdlb_stream_probe(void* d_dst, const void* d_src, size_t bytes, int mode, void* stream) {
    return guard([&] {
        if (mode < FDLB_COPY_PLAIN || mode > FDLB_COPY_WRITE) throw Error(FDLB_EINVAL, "unknown probe mode");
        if (!d_dst || (mode != FDLB_COPY_WRITE && !d_src)) throw Error(FDLB_EINVAL, "NULL device buffer");
        launch_copy(d_dst, d_src, bytes, (hipStream_t)stream, mode);
        return FDLB_OK;
    });
}

const char* fdlb_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
