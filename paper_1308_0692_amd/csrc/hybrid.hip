// Hybrid half-range / full-range channel: one workgroup per channel, the whole state resident
// in LDS for a launch.
//
// A channel is a 1-D column of ny cells between two plates (x periodic with one cell, so only
// y transport acts).  The first and last `layer` cells use the x rule times a half-range y
// rule (the paper's method, where the Knudsen layers live); the cells between use the x rule
// times a full-range y rule, the cheaper set that the paper's closing remarks propose for the
// bulk.  The march kernel keeps the populations and each cell's moments in LDS; a step is one
// pass with a wave per chunk of 64 cells of one zone and group of planes (a lane relaxes its
// cell's population and its donor from the moments of their cells, transports by the donor
// cell, sees a donor in the other zone through the interface map and the plate emission at a
// wall, and keeps its cell's partial moments in registers) and one pass with a thread per cell
// (moments of the new state from the partials, the residual terms, the next emission density),
// two barriers in all and no global memory traffic inside the loop but a write-back of the
// residuals every 64 steps.  A small channel's step is a few microseconds of one CU instead of
// a kernel launch, and a batch of channels (a Kn sweep) fills the chip with one workgroup each.
#include "fdlb_internal.h"

namespace fdlb {
namespace {

struct HybView {
    int ny, L, nl, nb, nx, nh, nf, qh, qf;
    const double *xx, *wx, *yh, *wh, *nuh, *yf, *wf, *nuf, *A, *B;
};

__device__ inline HybView hyb_view(const HybChan& C, const double* tb) {
    HybView v;
    v.ny = C.ny;
    v.L = C.layer;
    v.nl = 2 * C.layer;
    v.nb = C.ny - 2 * C.layer;
    v.nx = C.nx;
    v.nh = C.nh;
    v.nf = C.nf;
    v.qh = C.qh;
    v.qf = C.qf;
    v.xx = tb;
    v.wx = v.xx + v.nx;
    v.yh = v.wx + v.nx;
    v.wh = v.yh + v.nh;
    v.nuh = v.wh + v.nh;
    v.yf = v.nuh + v.nh;
    v.wf = v.yf + v.nf;
    v.nuf = v.wf + v.nf;
    v.A = v.nuf + v.nf;
    v.B = v.A + v.nf * v.nh;
    return v;
}

__device__ inline bool in_layer(const HybView& v, int j) { return j < v.L || j >= v.ny - v.L; }
// index of a layer cell among the layer cells (bottom layer, then top layer)
__device__ inline int lcell(const HybView& v, int j) { return j < v.L ? j : j - v.nb; }
// LDS index of layer velocity alpha (= a nx + i) in layer cell j, of bulk velocity kappa in bulk cell j
__device__ inline int lidx(const HybView& v, int alpha, int j) { return alpha * v.nl + lcell(v, j); }
__device__ inline int bidx(const HybView& v, int kappa, int j) { return v.nl * v.qh + kappa * v.nb + (j - v.L); }

__device__ inline void cell_moments(const HybView& v, const double* f, int j, double& r, double& jx, double& jy) {
    r = 0.0;
    jx = 0.0;
    jy = 0.0;
    if (in_layer(v, j)) {
        for (int a = 0; a < v.nh; ++a) {
            double s = 0.0, sx = 0.0;
            for (int i = 0; i < v.nx; ++i) {
                const double p = f[lidx(v, a * v.nx + i, j)];
                s += p;
                sx += v.xx[i] * p;
            }
            r += s;
            jx += sx;
            jy += v.yh[a] * s;
        }
    } else {
        for (int k = 0; k < v.nf; ++k) {
            double s = 0.0, sx = 0.0;
            for (int i = 0; i < v.nx; ++i) {
                const double p = f[bidx(v, k * v.nx + i, j)];
                s += p;
                sx += v.xx[i] * p;
            }
            r += s;
            jx += sx;
            jy += v.yf[k] * s;
        }
    }
}

// Relax cell j in place; a wall cell also writes its plate's emission into ghost[wall][alpha].
__device__ inline void cell_relax(const HybView& v, double* f, int j, double r, double jx, double jy,
                                  const HybChan& C, double* ghost) {
    const double om = C.omega;
    if (in_layer(v, j)) {
        double flux_down = 0.0, flux_up = 0.0;
        for (int a = 0; a < v.nh; ++a) {
            const double y = v.yh[a];
            for (int i = 0; i < v.nx; ++i) {
                const int idx = lidx(v, a * v.nx + i, j);
                const double W = v.wh[a] * v.wx[i];
                const double feq = W * (r + v.xx[i] * jx + y * jy);
                const double g = f[idx] + om * (feq - f[idx]);
                f[idx] = g;
                if (y < 0.0) flux_down -= y * g;
                else flux_up += y * g;
            }
        }
        if (j == 0) {  // bottom plate: arriving xi_y < 0, emission into xi_y > 0
            const double rho_w = flux_down * C.e_inv;
            for (int a = 0; a < v.nh; ++a)
                if (v.yh[a] > 0.0)
                    for (int i = 0; i < v.nx; ++i)
                        ghost[a * v.nx + i] = v.wh[a] * v.wx[i] * rho_w * (1.0 + v.xx[i] * C.u_bottom);
        }
        if (j == v.ny - 1) {  // top plate: arriving xi_y > 0, emission into xi_y < 0
            const double rho_w = flux_up * C.e_inv;
            for (int a = 0; a < v.nh; ++a)
                if (v.yh[a] < 0.0)
                    for (int i = 0; i < v.nx; ++i)
                        ghost[v.qh + a * v.nx + i] = v.wh[a] * v.wx[i] * rho_w * (1.0 + v.xx[i] * C.u_top);
        }
    } else {
        for (int k = 0; k < v.nf; ++k) {
            const double y = v.yf[k];
            for (int i = 0; i < v.nx; ++i) {
                const int idx = bidx(v, k * v.nx + i, j);
                const double W = v.wf[k] * v.wx[i];
                const double feq = W * (r + v.xx[i] * jx + y * jy);
                f[idx] = f[idx] + om * (feq - f[idx]);
            }
        }
    }
}

// A double moved across lanes by a DPP control (both 32-bit halves); lanes without a source
// get 0.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double x) {
    const int lo = __double2loint(x), hi = __double2hiint(x);
    const int l = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xf, false);
    const int h = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xf, false);
    return __hiloint2double(h, l);
}

__device__ inline double lane_value(double x, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}

// Sum over the 64 lanes of a wave, the same value in every lane: a scan within each row of 16
// lanes (row_shr 1, 2, 4, 8), then the row totals carried across rows (row_bcast 15 and 31),
// read from the last lane.  DPP moves are register operations: no LDS round trip.
__device__ inline double wave_sum(double x) {
    x += dpp_move<0x111, 0xf>(x);  // row_shr:1
    x += dpp_move<0x112, 0xf>(x);  // row_shr:2
    x += dpp_move<0x114, 0xf>(x);  // row_shr:4
    x += dpp_move<0x118, 0xf>(x);  // row_shr:8
    x += dpp_move<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_move<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return lane_value(x, 63);
}

// Sum of the first 16 lanes' values, the same in every lane (row 0's scan).
__device__ inline double row0_sum(double x) {
    x += dpp_move<0x111, 0xf>(x);
    x += dpp_move<0x112, 0xf>(x);
    x += dpp_move<0x114, 0xf>(x);
    x += dpp_move<0x118, 0xf>(x);
    return lane_value(x, 15);
}

// LDS carve shared by the march and post kernels (doubles).
struct Carve {
    double *tb, *fa, *fb, *mom, *uo, *ghost, *red, *rw, *ifc, *lring, *part;
};

__device__ inline Carve carve(double* lds, const HybChan& C, int S) {
    Carve c;
    c.tb = lds;
    c.fa = c.tb + C.ntab;
    c.fb = c.fa + S;
    c.mom = c.fb + S;
    c.uo = c.mom + 3 * C.ny;
    c.ghost = c.uo + 2 * C.ny;
    c.red = c.ghost + 2 * C.qh;
    c.rw = c.red + 4 * (HYB_MARCH_THREADS / 64);  // two slots of wave partials
    c.ifc = c.rw + 2;                             // [bulk from layer L-1, layer from bulk L, bulk from
                                                  //  layer ny-L, layer from bulk ny-L-1]
    c.lring = c.ifc + 2 * (C.qh + C.qf);          // the current 64-step block of the residual ring
    c.part = c.lring + 64;                        // the march kernel's partial moments
    return c;
}

__device__ inline int state_doubles(const HybChan& C) {
    return 2 * C.layer * C.qh + (C.ny - 2 * C.layer) * C.qf;
}

// The interface cells' populations carried to the other zone's nodes, raw (before relaxation):
// the maps reproduce the equilibrium exactly, so the map of a relaxed distribution is the
// relaxation, with the donor cell's moments, of the mapped raw one.  ifc holds, in order, the
// bulk nodes seen from layer cell L - 1, the layer nodes seen from bulk cell L, the bulk nodes
// seen from layer cell ny - L and the layer nodes seen from bulk cell ny - L - 1.  Items are
// taken from `first` by `stride`.
__device__ inline void interface_pass(const HybView& v, const double* f, double* ifc, int first, int stride) {
    if (v.nb == 0) return;
    const int per_side = v.qf + v.qh;
    for (int w = first; w < 2 * per_side; w += stride) {
        const int side = w < per_side ? 0 : 1;  // 0: lower interface, 1: upper
        int r = w - side * per_side;
        const int lay = side == 0 ? v.L - 1 : v.ny - v.L, blk = side == 0 ? v.L : v.ny - v.L - 1;
        double acc = 0.0;
        if (r < v.qf) {  // bulk node (k, i) from the layer cell
            const int k = r / v.nx, i = r - k * v.nx;
            const double* arow = v.A + k * v.nh;
            for (int a = 0; a < v.nh; ++a) acc += arow[a] * f[lidx(v, a * v.nx + i, lay)];
        } else {         // layer node (a, i) from the bulk cell
            const int q = r - v.qf;
            const int a = q / v.nx, i = q - a * v.nx;
            const double* brow = v.B + a * v.nf;
            for (int k = 0; k < v.nf; ++k) acc += brow[k] * f[bidx(v, k * v.nx + i, blk)];
        }
        ifc[side * per_side + r] = acc;
    }
}

// relaxed value of one population from its stored value and its cell's moments (Eqs. 1, 5)
__device__ inline double relaxed(double f, double W, double xx, double y, double r, double jx, double jy, double om) {
    return f + om * (W * (r + xx * jx + y * jy) - f);
}

// March every active channel: at most nsteps steps; with solve, stop at the first step whose
// residual is below tol or not finite.  Per step:
//   move     a wave per chunk of 64 cells of one zone, a lane per cell walking every plane of its
//            zone's set: the relaxed value of the population and of its donor (relaxed on the fly
//            from the donor cell's moments; the interface value when the donor is in the other
//            zone; the plate emission at a wall) give the new value, whose moments, residual
//            terms and (at a wall cell) arriving flux accumulate in the lane's registers
//   barrier
//   the interface cells' new populations carried to the other zone's nodes
//   barrier  (the residual of the step is formed from the wave partials during the next moves,
//            by every thread in the same order, so that all threads take the same decision and
//            leave the loop together)
__global__ void __launch_bounds__(HYB_MARCH_THREADS) hybrid_march_kernel(const HybChan* __restrict__ chans,
                                                                         const double* __restrict__ tab,
                                                                         double* __restrict__ state,
                                                                         HybCtl* __restrict__ ctl,
                                                                         double* __restrict__ ring, int64_t nsteps,
                                                                         double tol, int solve) {
    constexpr int NT = HYB_MARCH_THREADS;
    extern __shared__ double lds[];
    const HybChan C = chans[blockIdx.x];
    if (!C.active) return;
    HybCtl ct = ctl[blockIdx.x];
    if (solve && ct.status != 0) return;
    const int tid = threadIdx.x;
    const int S = state_doubles(C);
    const Carve m = carve(lds, C, S);
    for (int i = tid; i < C.ntab; i += NT) m.tb[i] = tab[C.tab_off + i];
    double* gs = state + C.state_off;
    for (int i = tid; i < S; i += NT) m.fa[i] = gs[i];
    // Residuals go to an LDS copy of the ring's current 64-step block, written back every 64 steps
    // and at the end: a global store inside the loop would hold its wave at every barrier until
    // the store completed.
    const int64_t blk0 = ct.steps & ~(int64_t)63;
    if (tid < 64) m.lring[tid] = ring[C.hist_off + (blk0 + tid) % HYB_RING];
    __syncthreads();
    const HybView v = hyb_view(C, m.tb);
    const int ny = v.ny, nl = v.nl, nb = v.nb, nx = v.nx, L = v.L;
    const double om = C.omega;
    // per-plane constants (after the maps in the channel's table), 8 doubles a plane: omega W,
    // omega W xi_x, omega W xi_y, W, xi_x, xi_y, the Courant number and the sign of xi_y, layer
    // planes then bulk planes
    const double* __restrict__ ptab = tab + C.tab_off + (v.B + v.nh * v.nf - m.tb);
    double* mc = m.mom;  // [3][ny]: rho, j_x, j_y of the current state's cells

    // The density of the emission a wall will see when this state relaxes: the arriving flux of
    // the relaxed populations, (1 - omega) Phi(f) + omega (rho A + j_x Bx + j_y By) with Phi(f)
    // the arriving flux of f, over the flux one unit of emitted density carries (Eq. 9 read as
    // impermeability).
    auto wall_density = [&](int wall, double phi, double r, double jx, double jy) {
        return C.e_inv * ((1.0 - om) * phi + om * (r * C.wA[wall] + jx * C.wBx[wall] + jy * C.wBy[wall]));
    };
    // moments of the loaded state, a thread per cell
    for (int j = tid; j < ny; j += NT) {
        double r = 0.0, jx = 0.0, jy = 0.0, phi_dn = 0.0, phi_up = 0.0;
        if (in_layer(v, j)) {
            const int c = lcell(v, j);
            for (int a = 0; a < v.nh; ++a) {
                double sa = 0.0, sx = 0.0;
                for (int i = 0; i < nx; ++i) {
                    const double p = m.fa[(a * nx + i) * nl + c];
                    sa += p;
                    sx += v.xx[i] * p;
                }
                const double y = v.yh[a];
                r += sa;
                jx += sx;
                jy += y * sa;
                if (y < 0.0) phi_dn -= y * sa;
                else phi_up += y * sa;
            }
        } else {
            cell_moments(v, m.fa, j, r, jx, jy);
        }
        mc[j] = r;
        mc[ny + j] = jx;
        mc[2 * ny + j] = jy;
        m.uo[j] = jx / r;
        m.uo[ny + j] = jy / r;
        if (j == 0) m.rw[0] = wall_density(0, phi_dn, r, jx, jy);
        if (j == ny - 1) m.rw[1] = wall_density(1, phi_up, r, jx, jy);
    }
    double* ifc_bl = m.ifc;                 // bulk nodes seen from layer cell L - 1
    double* ifc_lb = ifc_bl + v.qf;         // layer nodes seen from bulk cell L
    double* ifc_bt = ifc_lb + v.qh;         // bulk nodes seen from layer cell ny - L
    double* ifc_lt = ifc_bt + v.qf;         // layer nodes seen from bulk cell ny - L - 1
    interface_pass(v, m.fa, m.ifc, NT - 1 - tid, NT);
    __syncthreads();

    // Work items: a chunk of 64 consecutive cells of one zone (the layer cells in their list
    // order, then the bulk cells) and one of G groups of its planes (every G-th plane).  A lane
    // owns one cell and walks the group's planes: the plane index is the same across the wave,
    // so the tables are read at uniform addresses, and the cell's partial moments accumulate in
    // registers; the partials of the G groups are summed after the barrier.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int ncl = (nl + 63) >> 6, ncb = (nb + 63) >> 6;
    const int G = hyb_groups(ncl + ncb);
    const int nitems = (ncl + ncb) * G;
    double* part = m.part;                  // [G][3][ny] partial moments, then [G][2] plate fluxes
    double* pphi = part + 3 * G * ny;
    double* cur = m.fa;
    double* nxt = m.fb;
    int64_t taken = 0;
    int stop = 0;
    double R = ct.residual;
    bool pending = false;  // the residual of step `taken` is still to be formed from its wave partials
    // The moves of step taken + 1 start before the residual of step `taken` is formed (its wave
    // partials were complete at the barrier that ended it): the reduction overlaps the moves, and
    // a converged step leaves the loop with the tentative new state discarded.
    while (true) {
        const bool more = taken < nsteps;
        if (more) {
            const double rw0 = m.rw[0], rw1 = m.rw[1];
            for (int item = wave; item < nitems; item += NT / 64) {
                const int chunk = item / G, g = item - chunk * G;
                const bool layer = chunk < ncl;
                const int ci = (layer ? chunk : chunk - ncl) * 64 + lane;  // index in the zone's cell list
                const int ncell = layer ? nl : nb;
                const bool act = ci < ncell;
                const int cc = act ? ci : ncell - 1;                        // idle lanes shadow the last cell
                const int j = layer ? (cc < L ? cc : cc + nb) : L + cc;
                const int jm = j > 0 ? j - 1 : j, jp = j < ny - 1 ? j + 1 : j;
                const double r0 = mc[j], x0 = mc[ny + j], y0m = mc[2 * ny + j];
                const double rm = mc[jm], xm = mc[ny + jm], ym = mc[2 * ny + jm];
                const double rp = mc[jp], xp = mc[ny + jp], yp = mc[2 * ny + jp];
                const int qz = layer ? v.qh : v.qf;
                // this zone's plane constants, read from the global table at addresses uniform across
                // the wave (scalar loads, off the LDS queue)
                const double* __restrict__ pz = ptab + (layer ? 0 : 8 * v.qh);
                // a donor across the zone boundary is seen through the interface values
                const bool lo_other = (j - 1 >= 0) && (in_layer(v, j - 1) != layer);
                const bool hi_other = (j + 1 < ny) && (in_layer(v, j + 1) != layer);
                const double* ifc_lo = layer ? ifc_lt : ifc_bl;  // donor j - 1 in the other zone
                const double* ifc_hi = layer ? ifc_lb : ifc_bt;  // donor j + 1 in the other zone
                const int cm = layer ? lcell(v, jm) : jm - L, cp = layer ? lcell(v, jp) : jp - L;
                const int base = layer ? 0 : nl * v.qh;
                double nr = 0.0, njx = 0.0, njy = 0.0, phi_dn = 0.0, phi_up = 0.0;
                for (int alpha = g; alpha < qz; alpha += G) {
                    const double* __restrict__ pe = pz + 8 * alpha;
                    const double ow = pe[0], owx = pe[1], owy = pe[2], W = pe[3], xx = pe[4], y = pe[5];
                    const double nu = pe[6];
                    const int dir = (int)pe[7];  // sign of xi_y
                    const int pl = base + alpha * ncell;
                    const double f0 = cur[pl + cc];
                    const double gsf = f0 + ((ow * r0 + owx * x0 + owy * y0m) - om * f0);
                    double fnew = gsf;
                    if (dir > 0) {          // donor below
                        const double fd = lo_other ? ifc_lo[alpha] : cur[pl + cm];
                        double gu = fd + ((ow * rm + owx * xm + owy * ym) - om * fd);
                        if (j == 0) gu = W * rw0 * (1.0 + xx * C.u_bottom);
                        fnew = gsf - nu * (gsf - gu);
                    } else if (dir < 0) {   // donor above
                        const double fd = hi_other ? ifc_hi[alpha] : cur[pl + cp];
                        double gu = fd + ((ow * rp + owx * xp + owy * yp) - om * fd);
                        if (j == ny - 1) gu = W * rw1 * (1.0 + xx * C.u_top);
                        fnew = gsf - nu * (gsf - gu);
                    }
                    if (act) nxt[pl + cc] = fnew;
                    nr += fnew;
                    njx += xx * fnew;
                    njy += y * fnew;
                    if (dir < 0) phi_dn -= y * fnew;
                    else phi_up += y * fnew;
                }
                if (act) {
                    double* pg = part + 3 * g * ny;
                    pg[j] = nr;
                    pg[ny + j] = njx;
                    pg[2 * ny + j] = njy;
                    if (j == 0) pphi[2 * g] = phi_dn;
                    if (j == ny - 1) pphi[2 * g + 1] = phi_up;
                }
            }
        }
        if (pending) {
            // lane w < NT / 64 of every wave reads wave w's partials; a row scan adds them
            static_assert(NT / 64 <= 16, "the residual's wave partials must fit one row of lanes");
            const double* rd = m.red + (taken & 1) * 2 * (NT / 64);
            const bool has = lane < NT / 64;
            const double sdu = row0_sum(has ? rd[2 * lane] : 0.0);
            const double suu = row0_sum(has ? rd[2 * lane + 1] : 0.0);
            R = suu > 0.0 ? sqrt(sdu) / sqrt(suu) : (sdu == 0.0 ? 0.0 : INFINITY);
            const int64_t sn = ct.steps + taken;  // step number of this residual (from 1)
            if (tid == 0) m.lring[(sn - 1) & 63] = R;
            if ((sn & 63) == 0 && tid < 64)       // a full block: written back by wave 0
                ring[C.hist_off + (sn - 64 + tid) % HYB_RING] = m.lring[tid];
            pending = false;
            if (solve) {  // every thread holds the same R: the exit is block-uniform
                if (!isfinite(R)) {
                    stop = 2;
                    break;
                }
                if (R < tol) {
                    stop = 1;
                    break;
                }
            }
        }
        if (!more) break;
        __syncthreads();
        // the new state's moments from the groups' partials (a thread per cell), its residual
        // terms and the plates' next emission densities; the interface values of the new state
        double du = 0.0, uu = 0.0;
        for (int j = tid; j < ny; j += NT) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int g = 0; g < G; ++g) {
                const double* pg = part + 3 * g * ny;
                r += pg[j];
                jx += pg[ny + j];
                jy += pg[2 * ny + j];
            }
            mc[j] = r;
            mc[ny + j] = jx;
            mc[2 * ny + j] = jy;
            const double ux = jx / r, uy = jy / r;
            const double dx = ux - m.uo[j], dy = uy - m.uo[ny + j];
            du += dx * dx + dy * dy;
            uu += ux * ux + uy * uy;
            m.uo[j] = ux;
            m.uo[ny + j] = uy;
            if (j == 0 || j == ny - 1) {
                for (int wall = 0; wall < 2; ++wall) {
                    if (j != (wall == 0 ? 0 : ny - 1)) continue;
                    double phi = 0.0;
                    for (int g = 0; g < G; ++g) phi += pphi[2 * g + wall];
                    m.rw[wall] = wall_density(wall, phi, r, jx, jy);
                }
            }
        }
        interface_pass(v, nxt, m.ifc, NT - 1 - tid, NT);
        du = wave_sum(du);
        uu = wave_sum(uu);
        ++taken;
        if (lane == 0) {
            double* rd = m.red + (taken & 1) * 2 * (NT / 64);
            rd[2 * wave] = du;
            rd[2 * wave + 1] = uu;
        }
        __syncthreads();
        double* t = cur;
        cur = nxt;
        nxt = t;
        pending = true;
    }
    // every write to `cur` happened before the last barrier (or the load's); the ring's last
    // block holds every residual recorded (wave 0 wrote them, in order)
    for (int i = tid; i < S; i += NT) gs[i] = cur[i];
    {
        const int64_t sn = ct.steps + taken - (pending ? 1 : 0);  // last residual recorded
        if (tid < 64 && (sn & 63) != 0 && sn > blk0 && tid < (int)(sn & 63))
            ring[C.hist_off + ((sn & ~(int64_t)63) + tid) % HYB_RING] = m.lring[tid];
    }
    if (tid == 0) {
        ct.steps += taken;
        if (taken > 0) ct.residual = R;
        if (solve) {
            ct.status = stop;
            if (stop == 1 && ct.first_below < 0) ct.first_below = ct.steps;
        } else {
            ct.status = 0;
            ct.first_below = -1;
        }
        ctl[blockIdx.x] = ct;
    }
}

// f = w (rho + xi_x rho u_x + xi_y rho u_y) on each cell's own set, from fields [3][ny].
__global__ void __launch_bounds__(HYB_THREADS) hybrid_seed_kernel(const HybChan* __restrict__ chans, int ch,
                                                                  const double* __restrict__ tab,
                                                                  double* __restrict__ state,
                                                                  const double* __restrict__ fields) {
    const HybChan C = chans[ch];
    const HybView v = hyb_view(C, tab + C.tab_off);
    double* f = state + C.state_off;
    for (int j = threadIdx.x; j < v.ny; j += HYB_THREADS) {
        const double r = fields[j], jx = r * fields[v.ny + j], jy = r * fields[2 * v.ny + j];
        if (in_layer(v, j)) {
            for (int a = 0; a < v.nh; ++a)
                for (int i = 0; i < v.nx; ++i)
                    f[lidx(v, a * v.nx + i, j)] = v.wh[a] * v.wx[i] * (r + v.xx[i] * jx + v.yh[a] * jy);
        } else {
            for (int k = 0; k < v.nf; ++k)
                for (int i = 0; i < v.nx; ++i)
                    f[bidx(v, k * v.nx + i, j)] = v.wf[k] * v.wx[i] * (r + v.xx[i] * jx + v.yf[k] * jy);
        }
    }
}

// Outputs of one channel into out: rho, u_x, u_y, p_xy per cell ([4][ny]) and the eight face
// values (bottom plate u_x, p_xy; top plate u_x, p_xy; lower interface flux from the layer cell,
// from the bulk cell; upper interface flux from the bulk cell, from the layer cell).
__global__ void __launch_bounds__(HYB_THREADS) hybrid_post_kernel(const HybChan* __restrict__ chans, int ch,
                                                                  const double* __restrict__ tab,
                                                                  const double* __restrict__ state,
                                                                  double* __restrict__ out) {
    extern __shared__ double lds[];
    const HybChan C = chans[ch];
    const int tid = threadIdx.x;
    const int S = state_doubles(C);
    const Carve m = carve(lds, C, S);
    for (int i = tid; i < C.ntab; i += HYB_THREADS) m.tb[i] = tab[C.tab_off + i];
    const double* gs = state + C.state_off;
    for (int i = tid; i < S; i += HYB_THREADS) m.fa[i] = gs[i];
    __syncthreads();
    const HybView v = hyb_view(C, m.tb);
    const int ny = v.ny;
    for (int j = tid; j < ny; j += HYB_THREADS) {
        double r, jx, jy;
        cell_moments(v, m.fa, j, r, jx, jy);
        out[j] = r;
        out[ny + j] = jx / r;
        out[2 * ny + j] = jy / r;
        cell_relax(v, m.fa, j, r, jx, jy, C, m.ghost);
        double p = 0.0;
        if (in_layer(v, j)) {
            for (int a = 0; a < v.nh; ++a)
                for (int i = 0; i < v.nx; ++i) p += v.xx[i] * v.yh[a] * m.fa[lidx(v, a * v.nx + i, j)];
        } else {
            for (int k = 0; k < v.nf; ++k)
                for (int i = 0; i < v.nx; ++i) p += v.xx[i] * v.yf[k] * m.fa[bidx(v, k * v.nx + i, j)];
        }
        out[3 * ny + j] = p;
    }
    __syncthreads();
    if (tid != 0) return;
    double* face = out + 4 * ny;
    const double* g = m.fa;
    for (int wall = 0; wall < 2; ++wall) {
        const int j = wall == 0 ? 0 : ny - 1;
        double r = 0.0, jx = 0.0, p = 0.0;
        for (int a = 0; a < v.nh; ++a) {
            const double y = v.yh[a];
            const bool arriving = wall == 0 ? y < 0.0 : y > 0.0;
            for (int i = 0; i < v.nx; ++i) {
                const double val = arriving ? g[lidx(v, a * v.nx + i, j)] : m.ghost[wall * v.qh + a * v.nx + i];
                r += val;
                jx += v.xx[i] * val;
                p += v.xx[i] * y * val;
            }
        }
        face[2 * wall] = jx / r;
        face[2 * wall + 1] = p;
    }
    if (v.nb == 0) {
        for (int q = 4; q < 8; ++q) face[q] = NAN;
        return;
    }
    // y-flux of x-momentum through the face between cells lo and lo + 1 as the update of the
    // cell on `side` (0: lo, 1: lo + 1) transports it
    for (int q = 0; q < 4; ++q) {
        const int lo = q < 2 ? v.L - 1 : ny - v.L - 1;
        const int side = (q == 0 || q == 2) ? 0 : 1;
        const int own = lo + side;
        double flux = 0.0;
        if (in_layer(v, own)) {
            for (int a = 0; a < v.nh; ++a) {
                const double y = v.yh[a];
                const int src = y > 0.0 ? lo : lo + 1;
                for (int i = 0; i < v.nx; ++i) {
                    double val;
                    if (in_layer(v, src)) {
                        val = g[lidx(v, a * v.nx + i, src)];
                    } else {
                        val = 0.0;
                        for (int k = 0; k < v.nf; ++k) val += v.B[a * v.nf + k] * g[bidx(v, k * v.nx + i, src)];
                    }
                    flux += v.xx[i] * y * val;
                }
            }
        } else {
            for (int k = 0; k < v.nf; ++k) {
                const double y = v.yf[k];
                if (y == 0.0) continue;
                const int src = y > 0.0 ? lo : lo + 1;
                for (int i = 0; i < v.nx; ++i) {
                    double val;
                    if (!in_layer(v, src)) {
                        val = g[bidx(v, k * v.nx + i, src)];
                    } else {
                        val = 0.0;
                        for (int a = 0; a < v.nh; ++a) val += v.A[k * v.nh + a] * g[lidx(v, a * v.nx + i, src)];
                    }
                    flux += v.xx[i] * y * val;
                }
            }
        }
        face[4 + q] = flux;
    }
}

}  // namespace

void hybrid_allow_lds(size_t bytes) {
    FDLB_HIP(hipFuncSetAttribute((const void*)hybrid_march_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)bytes));
    FDLB_HIP(hipFuncSetAttribute((const void*)hybrid_post_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)bytes));
}

void launch_hybrid_march(const HybChan* d_chans, int n, const double* d_tab, double* d_state, HybCtl* d_ctl,
                         double* d_ring, int64_t nsteps, double tol, int solve, size_t lds, hipStream_t stream) {
    hipLaunchKernelGGL(hybrid_march_kernel, dim3(n), dim3(HYB_MARCH_THREADS), lds, stream, d_chans, d_tab, d_state, d_ctl,
                       d_ring, nsteps, tol, solve);
    FDLB_HIP(hipGetLastError());
}

void launch_hybrid_seed(const HybChan* d_chans, int ch, int ny, const double* d_tab, double* d_state,
                        const double* d_fields, hipStream_t stream) {
    (void)ny;
    hipLaunchKernelGGL(hybrid_seed_kernel, dim3(1), dim3(HYB_THREADS), 0, stream, d_chans, ch, d_tab, d_state,
                       d_fields);
    FDLB_HIP(hipGetLastError());
}

void launch_hybrid_post(const HybChan* d_chans, int ch, const double* d_tab, const double* d_state, double* d_out,
                        size_t lds, hipStream_t stream) {
    hipLaunchKernelGGL(hybrid_post_kernel, dim3(1), dim3(HYB_THREADS), lds, stream, d_chans, ch, d_tab, d_state,
                       d_out);
    FDLB_HIP(hipGetLastError());
}

}  // namespace fdlb
