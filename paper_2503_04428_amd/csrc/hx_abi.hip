// C ABI of the gfx950 hydrodynamics step (see include/hydro.h for the contract).
//
// Host side only: validates the configuration, derives the per-axis geometry tables
// (Sect. 3.1.1: cell centres, widths, dV and dS factors, computed in FP64 on the host),
// lays out the caller's workspace and enqueues the kernels on the caller's stream.
#include "hydro.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

#include "hx_launch.h"
#include "hx_arith.h"
#include "hx_run1d.h"

namespace {

thread_local std::string g_err;

hx_status fail(hx_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHECK(call)                                                                          \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(HX_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));               \
    } while (0)

constexpr size_t ALIGN = 256;
constexpr int MAX_RED_BLOCKS = 2048;
constexpr int MAX_SHELL_CHUNKS = 64;

size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// image of index i on an axis of n cells (periodic / transmissive / reflective)
int bc_map(int i, int n, int lo, int hi, bool& flip)
{
    flip = false;
    if (i < 0) {
        if (lo == HX_BOUNDARY_PERIODIC)
            return i + n;
        if (lo == HX_BOUNDARY_TRANSMISSIVE)
            return 0;
        flip = true;
        return -1 - i;
    }
    if (i >= n) {
        if (hi == HX_BOUNDARY_PERIODIC)
            return i - n;
        if (hi == HX_BOUNDARY_TRANSMISSIVE)
            return n - 1;
        flip = true;
        return 2 * n - 1 - i;
    }
    return i;
}

struct Layout {
    size_t state[2];
    size_t tab[3][4];  // cm, cp, w, kap per axis
    size_t rabs, sabs, rf, vr, hr, ct, sf;
    size_t gr, menc, shell, partial, dtpart, dt, flag, tot, mlp, time, xfaces, run;
    size_t total;
    int ntab[3];
    int nchunk, nred;
};

int nvar_of(const hx_config* c) { return 5 + c->nscalar + (c->dual_energy ? 1 : 0); }

long long ncells_of(const hx_config* c) { return (long long)c->n[0] * c->n[1] * c->n[2]; }

hx_status validate(const hx_config* c)
{
    if (!c)
        return fail(HX_EINVAL, "null configuration");
    if (c->ndim < 1 || c->ndim > 3)
        return fail(HX_EINVAL, "ndim must be 1, 2 or 3 (got %d)", c->ndim);
    if (c->geom != HX_GEOM_CART && c->geom != HX_GEOM_SPH)
        return fail(HX_EINVAL, "unknown geometry %d", c->geom);
    if (c->nscalar < 0 || c->nscalar > 4)
        return fail(HX_EINVAL, "nscalar must be 0..4 (got %d)", c->nscalar);
    if (c->nghost != 2 && c->nghost != 3)
        return fail(HX_EINVAL, "nghost must be 2 or 3 (got %d)", c->nghost);
    if (c->limiter < HX_LIMITER_NONE || c->limiter > HX_LIMITER_MLP)
        return fail(HX_EINVAL, "unknown limiter %d", c->limiter);
    if (c->limiter == HX_LIMITER_MLP) {
        if (c->precision != HX_PRECISION_FP32)
            return fail(HX_EINVAL, "the learned limiter runs in the FP32 form");
        if (c->nghost != 3)
            return fail(HX_EINVAL, "the learned limiter needs nghost = 3");
        if (c->riemann != HX_RIEMANN_HLLC)
            return fail(HX_EINVAL, "the learned limiter is built with HLLC");
        if (c->nscalar > 2)
            return fail(HX_EINVAL, "the learned limiter supports at most 2 passive scalars");
    }
    if (c->riemann != HX_RIEMANN_HLL && c->riemann != HX_RIEMANN_HLLC)
        return fail(HX_EINVAL, "unknown Riemann solver %d", c->riemann);
    if (c->dual_energy != 0 && c->dual_energy != 1)
        return fail(HX_EINVAL, "dual_energy must be 0 or 1 (got %d)", c->dual_energy);
    if (c->dual_energy) {
        if (c->precision != HX_PRECISION_FP64)
            return fail(HX_EINVAL, "the internal-energy monitor is built for the FP64 form");
        if (c->riemann != HX_RIEMANN_HLLC)
            return fail(HX_EINVAL, "the internal-energy monitor needs HLLC (its interface velocity)");
        if (c->limiter == HX_LIMITER_MLP)
            return fail(HX_EINVAL, "the internal-energy monitor is not built with the learned limiter");
        if (c->nscalar > 3)
            return fail(HX_EINVAL, "with the internal-energy monitor at most 3 passive scalars");
        if (!(c->de_eps >= 0.0))
            return fail(HX_EINVAL, "de_eps must be >= 0");
    }
    if (c->eos != HX_EOS_GAS && c->eos != HX_EOS_GAS_RAD)
        return fail(HX_EINVAL, "unknown EoS %d", c->eos);
    if (c->eos == HX_EOS_GAS_RAD) {
        if (c->precision != HX_PRECISION_FP64)
            return fail(HX_EINVAL, "the gas + radiation EoS is built for the FP64 form");
        if (c->limiter == HX_LIMITER_MLP)
            return fail(HX_EINVAL, "the gas + radiation EoS is not built with the learned limiter");
        if (!(c->eos_R > 0.0) || !(c->eos_arad >= 0.0) || !std::isfinite(c->eos_R) || !std::isfinite(c->eos_arad))
            return fail(HX_EINVAL, "the gas + radiation EoS needs eos_R > 0 and eos_arad >= 0");
    }
    if (c->ni_heating != 0 && c->ni_heating != 1)
        return fail(HX_EINVAL, "ni_heating must be 0 or 1 (got %d)", c->ni_heating);
    if (c->ni_heating) {
        if (c->precision != HX_PRECISION_FP64)
            return fail(HX_EINVAL, "the 56Ni heating is built for the FP64 form");
        if (c->ni_scalar < 0 || c->ni_scalar >= c->nscalar)
            return fail(HX_EINVAL, "ni_scalar %d is not one of the %d passive scalars", c->ni_scalar, c->nscalar);
        if (!(c->ni_tau[0] > 0.0) || !(c->ni_tau[1] > c->ni_tau[0]) || !std::isfinite(c->ni_tau[1]))
            return fail(HX_EINVAL, "the 56Ni heating needs 0 < tau_Ni < tau_Co");
        if (!(c->ni_m > 0.0) || !std::isfinite(c->ni_m) || !(c->ni_Q[0] >= 0.0) || !(c->ni_Q[1] >= 0.0) ||
            !std::isfinite(c->ni_Q[0]) || !std::isfinite(c->ni_Q[1]))
            return fail(HX_EINVAL, "the 56Ni heating needs ni_m > 0 and finite Q >= 0");
    }
    if (c->centroid != 0 && c->centroid != 1)
        return fail(HX_EINVAL, "centroid must be 0 or 1 (got %d)", c->centroid);
    if (c->centroid && c->limiter == HX_LIMITER_MLP)
        return fail(HX_EINVAL, "reconstruction about volume centroids is not built with the learned limiter");
    if (c->precision != HX_PRECISION_FP64 && c->precision != HX_PRECISION_FP32)
        return fail(HX_EINVAL, "unknown precision %d", c->precision);
    if (!(c->gamma > 1.0) || !(c->cfl > 0.0))
        return fail(HX_EINVAL, "need gamma > 1 and cfl > 0");
    for (int d = 0; d < 3; d++) {
        const bool act = d < c->ndim;
        if (act && c->n[d] < c->nghost)
            return fail(HX_EINVAL, "axis %d: %d cells, need at least nghost = %d", d, c->n[d], c->nghost);
        // ndim 1 (Cartesian) may carry a batch of independent rows on axis 1
        const bool batch_axis = c->ndim == 1 && d == 1 && c->geom == HX_GEOM_CART;
        if (!act && c->n[d] != 1 && !(batch_axis && c->n[d] >= 1))
            return fail(HX_EINVAL, "inactive axis %d must have n = 1 (a batch of 1D rows needs Cartesian ndim 1)", d);
        if (!c->faces[d])
            return fail(HX_EINVAL, "faces of axis %d missing", d);
        const int nf = act ? c->n[d] + 1 + 2 * c->nghost : 2;
        for (int f = 1; f < nf; f++)
            if (!(c->faces[d][f] > c->faces[d][f - 1]))
                return fail(HX_EINVAL, "faces of axis %d must increase (index %d)", d, f);
        for (int s = 0; s < 2; s++)
            if (c->bc[d][s] < 0 || c->bc[d][s] > 2)
                return fail(HX_EINVAL, "unknown boundary %d on axis %d", c->bc[d][s], d);
        if (act && ((c->bc[d][0] == HX_BOUNDARY_PERIODIC) != (c->bc[d][1] == HX_BOUNDARY_PERIODIC)))
            return fail(HX_EINVAL, "axis %d: periodic boundaries must be periodic on both sides", d);
    }
    if (c->ndim == 3 && c->n[0] > 1 << 20)
        return fail(HX_EINVAL, "axis 0 too long");
    if (c->gravity < HX_GRAVITY_NONE || c->gravity > HX_GRAVITY_POINT_MONOPOLE)
        return fail(HX_EINVAL, "unknown gravity %d", c->gravity);
    if (c->gravity == HX_GRAVITY_UNIFORM && c->geom != HX_GEOM_CART)
        return fail(HX_EINVAL, "uniform gravity needs Cartesian geometry");
    if ((c->gravity == HX_GRAVITY_POINT || c->gravity == HX_GRAVITY_POINT_MONOPOLE) && c->geom != HX_GEOM_SPH)
        return fail(HX_EINVAL, "point-mass gravity needs spherical geometry");
    if (c->gravity == HX_GRAVITY_POINT_MONOPOLE && c->n[0] > HX_MAX_NR)
        return fail(HX_EINVAL, "enclosed-mass gravity supports at most %d radial cells", HX_MAX_NR);
    if (c->geom == HX_GEOM_SPH) {
        const double r0 = c->faces[0][c->nghost];
        if (r0 < 0.0 || (r0 == 0.0 && c->bc[0][0] != HX_BOUNDARY_REFLECTIVE))
            return fail(HX_EINVAL, "spherical grid: r must be positive (r = 0 needs a reflective centre)");
        const double* th = c->faces[1];
        const int o = c->ndim >= 2 ? c->nghost : 0;
        const double t0 = th[o], t1 = th[o + c->n[1]];
        if (t0 < 0.0 || t1 > M_PI + 1e-12)
            return fail(HX_EINVAL, "spherical grid: theta must lie in [0, pi]");
    }
    return HX_OK;
}

Layout layout(const hx_config* c)
{
    Layout L;
    const int nv = nvar_of(c);
    const long long nc = ncells_of(c);
    const size_t rb = c->precision == HX_PRECISION_FP32 ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += up(bytes);
        return o;
    };
    L.state[0] = take(rb * nv * nc);
    L.state[1] = take(rb * nv * nc);
    for (int d = 0; d < 3; d++) {
        L.ntab[d] = d < c->ndim ? c->n[d] + 2 * c->nghost : 1;
        for (int t = 0; t < 4; t++)
            L.tab[d][t] = take(sizeof(double) * L.ntab[d]);
    }
    L.rabs = take(sizeof(double) * L.ntab[0]);
    L.sabs = take(sizeof(double) * L.ntab[1]);
    L.rf = take(sizeof(double) * (c->n[0] + 1));
    L.vr = take(sizeof(double) * c->n[0]);
    L.hr = take(sizeof(double) * c->n[0]);
    L.ct = take(sizeof(double) * c->n[1]);
    L.sf = take(sizeof(double) * (c->n[1] + 1));
    L.gr = take(sizeof(double) * c->n[0]);
    L.menc = take(sizeof(double) * c->n[0]);
    long long rows = (long long)c->n[1] * c->n[2];
    L.nchunk = (int)(rows < MAX_SHELL_CHUNKS ? rows : MAX_SHELL_CHUNKS);
    L.shell = take(sizeof(double) * (size_t)L.nchunk * c->n[0]);
    long long nb = (nc + 255) / 256;
    L.nred = (int)(nb < MAX_RED_BLOCKS ? nb : MAX_RED_BLOCKS);
    L.partial = take(sizeof(double) * (size_t)L.nred * (nv > 1 ? nv : 1));
    // per-workgroup CFL maxima written by the sweep, sized for the smallest z chunk
    L.dtpart = take(sizeof(double) * (size_t)hx::sweep_nblocks(c->ndim, c->n, 1));
    L.dt = take(sizeof(double));
    L.flag = take(sizeof(int));
    L.tot = take(sizeof(double) * nv);
    L.mlp = take(sizeof(float) * HX_MLP_NPARAM);
    L.time = take(sizeof(double));  // the decay clock of the 56Ni heating
    L.run = take(2 * sizeof(double));  // final time and step count of hx_run_1d
    L.xfaces = take(sizeof(double) * (c->n[0] + 1 + 2 * c->nghost));  // axis-0 faces (grid shift)
    L.total = off;
    return L;
}

__global__ void clear_flag_kernel(int* f) { f[0] = 0; }

__global__ void set_time_kernel(double* t, double v) { t[0] = v; }

// t += dt after a heated step, dt from the host or from the device
__global__ void advance_time_kernel(double* t, double dt, const double* d_dt) { t[0] = t[0] + (d_dt ? d_dt[0] : dt); }

}  // namespace

struct hx_ctx {
    hx_config cfg;
    std::vector<double> faces[3];
    std::vector<double> host_tabs;  // staging of the geometry upload (kept alive for the async copy)
    int nvar = 0, ng = 0;
    long long ncells = 0;
    bool fp32 = false;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout L;
    void* state[2] = {nullptr, nullptr};
    int cur = 0;
    bool have_state = false;
    bool have_mlp = false;
    hx::Geo geo;
    int kz = 0;       // z planes per workgroup set by hx_set_zchunk (0: automatic)
    int kz_auto = 0;  // the automatic choice, made at the first 3D step
    double scale = 0.0;  // 4 pi / Omega_w
    bool dtpart_valid = false;  // the sweep's CFL maxima describe the current state
    long long dtpart_nb = 0;
};

namespace {

template <typename T>
T* at(hx_ctx* c, size_t off)
{
    return reinterpret_cast<T*>(c->ws + off);
}

// geometry of the oracle's definitions, computed once on the host in FP64
void build_geometry(hx_ctx* x, std::vector<double>& h, std::vector<std::pair<size_t, size_t>>& spans)
{
    const hx_config& c = x->cfg;
    const int ng = c.nghost;
    auto xf = [&](int d, int i) { return d < c.ndim ? x->faces[d][i + ng] : x->faces[d][i]; };
    auto xcen = [&](int d, int i) { return 0.5 * (xf(d, i) + xf(d, i + 1)); };
    auto dxc = [&](int d, int i) { return xf(d, i + 1) - xf(d, i); };
    auto push = [&](size_t off, const std::vector<double>& v) {
        spans.push_back({off, h.size()});
        h.insert(h.end(), v.begin(), v.end());
    };
    // reconstruction position of cell i on axis d: the face midpoint, or with the centroid option
    // the volume centroid of a spherical cell along r (measure r^2 dr) and theta (sin theta dtheta);
    // a ghost cell's is its image's, mirrored about the boundary face or moved across a periodic axis
    const bool cen = c.centroid && c.geom == HX_GEOM_SPH;
    std::function<double(int, int)> xrec = [&](int d, int i) -> double {
        if (!cen || d == 2)
            return xcen(d, i);
        const int n = c.n[d];
        if (i < 0)
            return c.bc[d][0] == HX_BOUNDARY_PERIODIC ? xrec(d, i + n) - (xf(d, n) - xf(d, 0))
                                                      : 2.0 * xf(d, 0) - xrec(d, -1 - i);
        if (i >= n)
            return c.bc[d][1] == HX_BOUNDARY_PERIODIC ? xrec(d, i - n) + (xf(d, n) - xf(d, 0))
                                                      : 2.0 * xf(d, n) - xrec(d, 2 * n - 1 - i);
        const double a = xf(d, i), b = xf(d, i + 1);
        if (d == 0)
            return 0.75 * ((b + a) * (b * b + a * a)) / (b * b + b * a + a * a);
        return ((std::sin(b) - b * std::cos(b)) - (std::sin(a) - a * std::cos(a))) / (std::cos(a) - std::cos(b));
    };
    for (int d = 0; d < 3; d++) {
        const bool act = d < c.ndim;
        const int nt = x->L.ntab[d];
        std::vector<double> cm(nt, 0.5), cp(nt, 0.5), w(nt, 0.0), kap(nt, 1.0);
        for (int t = 0; t < nt; t++) {
            const int i = act ? t - ng : 0;
            bool fl;
            const int im = act ? bc_map(i, c.n[d], c.bc[d][0], c.bc[d][1], fl) : 0;
            w[t] = dxc(d, im);
            if (act && i - 1 >= -ng && i + 1 <= c.n[d] + ng - 1) {
                if (cen && d < 2) {
                    // increments (x_+ - x_c) sigma and (x_c - x_-) sigma about the centroid x_c
                    const double xc = xrec(d, i);
                    const double hp = xf(d, i + 1) - xc;
                    cm[t] = hp / (xc - xrec(d, i - 1));
                    cp[t] = hp / (xrec(d, i + 1) - xc);
                    kap[t] = (xc - xf(d, i)) / hp;
                } else {
                    const double half = 0.5 * dxc(d, i);
                    cm[t] = half / (xcen(d, i) - xcen(d, i - 1));
                    cp[t] = half / (xcen(d, i + 1) - xcen(d, i));
                }
            }
        }
        push(x->L.tab[d][0], cm);
        push(x->L.tab[d][1], cp);
        push(x->L.tab[d][2], w);
        push(x->L.tab[d][3], kap);
    }
    {
        const int nt = x->L.ntab[0];
        std::vector<double> rabs(nt);
        for (int t = 0; t < nt; t++) {
            bool fl;
            const int im = bc_map(t - ng, c.n[0], c.bc[0][0], c.bc[0][1], fl);
            rabs[t] = std::fabs(xcen(0, im));
        }
        push(x->L.rabs, rabs);
    }
    {
        const int nt = x->L.ntab[1];
        const bool act = c.ndim >= 2;
        std::vector<double> sabs(nt);
        for (int t = 0; t < nt; t++) {
            bool fl;
            const int im = act ? bc_map(t - ng, c.n[1], c.bc[1][0], c.bc[1][1], fl) : 0;
            sabs[t] = std::fabs(std::sin(xcen(1, im)));
        }
        push(x->L.sabs, sabs);
    }
    const int n0 = c.n[0], n1 = c.n[1];
    std::vector<double> rf(n0 + 1), vr(n0), hr(n0), ct(n1), sf(n1 + 1);
    for (int i = 0; i <= n0; i++)
        rf[i] = xf(0, i);
    for (int i = 0; i < n0; i++) {
        const double rm = xf(0, i), rp = xf(0, i + 1);
        vr[i] = (rp * rp * rp - rm * rm * rm) / 3.0;
        hr[i] = 0.5 * (rp * rp - rm * rm);
    }
    // a batch of 1D rows has one theta cell's worth of faces; the remaining entries stay 0
    const int nth = c.ndim >= 2 ? n1 : 1;
    for (int j = 0; j < n1; j++)
        ct[j] = j < nth ? std::cos(xf(1, j)) - std::cos(xf(1, j + 1)) : 0.0;
    for (int j = 0; j <= n1; j++)
        sf[j] = j <= nth ? std::sin(xf(1, j)) : 0.0;
    push(x->L.rf, rf);
    push(x->L.vr, vr);
    push(x->L.hr, hr);
    push(x->L.ct, ct);
    push(x->L.sf, sf);
    // solid angle of the wedge and point-mass gravity (the monopole part is recomputed per step)
    double om_t = 0.0, om_p = 0.0;
    for (int j = 0; j < nth; j++)
        om_t += ct[j];
    for (int k = 0; k < c.n[2]; k++)
        om_p += dxc(2, k);
    x->scale = 4.0 * M_PI / (om_t * om_p);
    std::vector<double> gr(n0, 0.0);
    if (c.gravity == HX_GRAVITY_POINT || c.gravity == HX_GRAVITY_POINT_MONOPOLE) {
        for (int i = 0; i < n0; i++) {
            const double rc = xcen(0, i);
            gr[i] = -(c.G * (c.Mc + 0.0)) / (rc * rc);
        }
    }
    push(x->L.gr, gr);
    push(x->L.xfaces, x->faces[0]);
}

// Build the geometry tables and queue their upload on the context's stream.  Tables whose slots
// follow each other in the workspace (only alignment padding between them) go up in one copy,
// the padding as zeros: two copies in all (the tables, the axis-0 faces).  The staging vector
// stays alive in the context for the asynchronous copies.
hipError_t upload_geometry(hx_ctx* x)
{
    std::vector<double> h;
    std::vector<std::pair<size_t, size_t>> spans;  // (workspace byte offset, first element in h)
    build_geometry(x, h, spans);
    std::vector<double>& img = x->host_tabs;
    img.clear();
    std::vector<std::pair<size_t, size_t>> runs;  // (workspace byte offset, first element in img)
    size_t run_end = 0;
    for (size_t s = 0; s < spans.size(); s++) {
        const size_t beg = spans[s].second;
        const size_t end = s + 1 < spans.size() ? spans[s + 1].second : h.size();
        const size_t off = spans[s].first;
        if (runs.empty() || off < run_end || off - run_end >= ALIGN)
            runs.push_back({off, img.size()});
        else
            img.insert(img.end(), (off - run_end) / sizeof(double), 0.0);
        img.insert(img.end(), h.begin() + beg, h.begin() + end);
        run_end = off + sizeof(double) * (end - beg);
    }
    for (size_t r = 0; r < runs.size(); r++) {
        const size_t beg = runs[r].second;
        const size_t end = r + 1 < runs.size() ? runs[r + 1].second : img.size();
        const hipError_t e = hipMemcpyAsync(x->ws + runs[r].first, img.data() + beg, sizeof(double) * (end - beg),
                                            hipMemcpyHostToDevice, x->stream);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hx::Geo geo_of(hx_ctx* x)
{
    hx::Geo g;
    for (int d = 0; d < 3; d++) {
        g.cm[d] = at<double>(x, x->L.tab[d][0]);
        g.cp[d] = at<double>(x, x->L.tab[d][1]);
        g.w[d] = at<double>(x, x->L.tab[d][2]);
        g.kap[d] = at<double>(x, x->L.tab[d][3]);
    }
    g.rabs = at<double>(x, x->L.rabs);
    g.sabs = at<double>(x, x->L.sabs);
    g.rf = at<double>(x, x->L.rf);
    g.vr = at<double>(x, x->L.vr);
    g.hr = at<double>(x, x->L.hr);
    g.ct = at<double>(x, x->L.ct);
    g.sf = at<double>(x, x->L.sf);
    return g;
}

hx::DtParams dt_params(hx_ctx* x)
{
    hx::DtParams p;
    p.U = x->state[x->cur];
    for (int d = 0; d < 3; d++)
        p.n[d] = x->cfg.n[d];
    p.ng = x->ng;
    p.ndim = x->cfg.ndim;
    p.geom = x->cfg.geom;
    p.nvar = x->nvar;
    p.plane = x->ncells;
    p.gamma = x->cfg.gamma;
    p.gm1 = x->cfg.gamma - 1.0;
    p.eos = x->cfg.eos;
    p.eos_R = x->cfg.eos_R;
    p.eos_arad = x->cfg.eos_arad;
    p.geo = x->geo;
    p.partial = at<double>(x, x->L.partial);
    p.flag = at<int>(x, x->L.flag);
    return p;
}

hx_status enqueue_step(hx_ctx* x, double dt, const double* d_dt)
{
    if (!x->have_state)
        return fail(HX_ESTATE, "step before set_state");
    const hx_config& c = x->cfg;
    if (c.gravity == HX_GRAVITY_POINT_MONOPOLE) {
        hx::ShellParams s;
        s.U = x->state[x->cur];
        for (int d = 0; d < 3; d++)
            s.n[d] = c.n[d];
        s.ng = x->ng;
        s.ndim = c.ndim;
        s.geo = x->geo;
        s.partial = at<double>(x, x->L.shell);
        s.gr = at<double>(x, x->L.gr);
        s.menc = at<double>(x, x->L.menc);
        s.scale = x->scale;
        s.G = c.G;
        s.Mc = c.Mc;
        HIPCHECK(hx::launch_shell(s, x->fp32, x->L.nchunk, x->stream));
    }
    hx::SweepParams p;
    p.U = x->state[x->cur];
    p.Unew = x->state[1 - x->cur];
    for (int d = 0; d < 3; d++) {
        p.n[d] = c.n[d];
        p.bc[d][0] = c.bc[d][0];
        p.bc[d][1] = c.bc[d][1];
        p.g0[d] = c.g0[d];
    }
    p.ng = x->ng;
    p.plane = x->ncells;
    p.gamma = c.gamma;
    p.dt_host = dt;
    p.dt_dev = d_dt;
    p.limiter = c.limiter;
    p.riemann = c.riemann;
    p.gravity = c.gravity;
    p.gr = at<double>(x, x->L.gr);
    p.geo = x->geo;
    p.flag = at<int>(x, x->L.flag);
    p.dtpart = at<double>(x, x->L.dtpart);
    p.mlp = at<float>(x, x->L.mlp);
    p.de_eps = c.de_eps;
    p.eos_R = c.eos_R;
    p.eos_arad = c.eos_arad;
    p.ni = c.ni_heating ? 5 + c.ni_scalar : -1;
    for (int i = 0; i < 2; i++) {
        p.ni_Q[i] = c.ni_Q[i];
        p.ni_tau[i] = c.ni_tau[i];
    }
    p.ni_m = c.ni_m;
    p.t_in = at<double>(x, x->L.time);
    p.centroid = c.centroid && c.geom == HX_GEOM_SPH ? 1 : 0;
    // the fixed HLLC + van Leer sweeps are built without the 56Ni heating and with face-midpoint
    // reconstruction
    const bool spec = c.limiter == HX_LIMITER_VANLEER && c.riemann == HX_RIEMANN_HLLC && !c.ni_heating && !p.centroid;
    if (c.limiter == HX_LIMITER_MLP && !x->have_mlp)
        return fail(HX_ESTATE, "the learned limiter needs hx_set_mlp before stepping");
    // the instantiation for this configuration; with occ, only its workgroups per compute unit
    auto sweep = [&](int* occ) -> hipError_t {
        if (c.dual_energy)
            return c.eos == HX_EOS_GAS_RAD ? hx::launch_sweep_fp64_de_rad(p, c.ndim, x->nvar, c.geom, x->stream, occ)
                                           : hx::launch_sweep_fp64_de(p, c.ndim, x->nvar, c.geom, x->stream, occ);
        if (c.eos == HX_EOS_GAS_RAD)
            return c.ndim == 3 ? hx::launch_sweep_fp64_3d_ilp(p, 4, x->nvar, c.geom, x->stream, occ)
                               : hx::launch_sweep_fp64_rad(p, c.ndim, x->nvar, c.geom, x->stream, occ);
        if (c.limiter == HX_LIMITER_MLP)
            return hx::launch_sweep_fp32_mlp(p, c.ndim, x->nvar, c.geom, x->stream, occ);
        if (x->fp32)
            return spec ? hx::launch_sweep_fp32_hllc_vl(p, c.ndim, x->nvar, c.geom, x->stream, occ)
                        : hx::launch_sweep_fp32_generic(p, c.ndim, x->nvar, c.geom, x->stream, occ);
        if (spec && c.ndim == 3 && x->nvar >= 6)
            return hx::launch_sweep_fp64_3d_ilp(p, 1, x->nvar, c.geom, x->stream, occ);
        return spec ? hx::launch_sweep_fp64_hllc_vl(p, c.ndim, x->nvar, c.geom, x->stream, occ)
                    : hx::launch_sweep_fp64_generic(p, c.ndim, x->nvar, c.geom, x->stream, occ);
    };
    if (c.ndim == 3 && x->kz == 0 && x->kz_auto == 0) {
        int occ = 0, dev = 0, cus = 0;
        p.kz = 1;
        HIPCHECK(sweep(&occ));
        HIPCHECK(hipGetDevice(&dev));
        HIPCHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        if (occ < 1 || cus < 1)
            return fail(HX_EHIP, "the sweep does not fit on a compute unit (occupancy %d)", occ);
        const dim3 g = hx::sweep_grid(3, c.n, 1);
        x->kz_auto = hx::choose_zchunk(c.n[2], (long long)g.x * g.y, (long long)occ * cus,
                                       c.limiter == HX_LIMITER_MLP ? 8 : 4);
    }
    const int kz = x->kz > 0 ? x->kz : x->kz_auto;
    p.kz = c.ndim == 3 ? (kz < c.n[2] ? kz : c.n[2]) : 1;
    hipError_t e = sweep(nullptr);
    if (e != hipSuccess)
        return fail(HX_EHIP, "sweep launch failed: %s", hipGetErrorString(e));
    x->cur = 1 - x->cur;
    if (c.ni_heating) {
        advance_time_kernel<<<1, 1, 0, x->stream>>>(at<double>(x, x->L.time), dt, d_dt);
        HIPCHECK(hipGetLastError());
    }
    x->dtpart_valid = true;
    x->dtpart_nb = hx::sweep_nblocks(c.ndim, c.n, p.kz);
    return HX_OK;
}

hx_status sync_check(hx_ctx* x)
{
    int flag = 0;
    HIPCHECK(hipMemcpyAsync(&flag, at<int>(x, x->L.flag), sizeof(int), hipMemcpyDeviceToHost, x->stream));
    HIPCHECK(hipStreamSynchronize(x->stream));
    if (flag)
        return fail(HX_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or non-finite) met");
    return HX_OK;
}

}  // namespace

extern "C" {

size_t hx_workspace_bytes(const hx_config* cfg)
{
    if (validate(cfg) != HX_OK)
        return 0;
    return layout(cfg).total;
}

hx_status hx_create(const hx_config* cfg, void* d_workspace, size_t workspace_bytes, void* hip_stream,
                    hx_ctx** out)
{
    if (!out)
        return fail(HX_EINVAL, "null output pointer");
    *out = nullptr;
    hx_status st = validate(cfg);
    if (st != HX_OK)
        return st;
    Layout L = layout(cfg);
    if (!d_workspace || workspace_bytes < L.total)
        return fail(HX_ENOSPACE, "workspace of %zu bytes, need %zu", workspace_bytes, L.total);
    if (reinterpret_cast<uintptr_t>(d_workspace) % ALIGN)
        return fail(HX_EINVAL, "workspace must be %zu-byte aligned", ALIGN);
    hx_ctx* x = new (std::nothrow) hx_ctx();
    if (!x)
        return fail(HX_EINVAL, "out of host memory");
    x->cfg = *cfg;
    x->ng = cfg->nghost;
    x->nvar = nvar_of(cfg);
    x->ncells = ncells_of(cfg);
    x->fp32 = cfg->precision == HX_PRECISION_FP32;
    x->stream = (hipStream_t)hip_stream;
    x->ws = (char*)d_workspace;
    x->L = L;
    for (int d = 0; d < 3; d++) {
        const int nf = d < cfg->ndim ? cfg->n[d] + 1 + 2 * cfg->nghost : 2;
        x->faces[d].assign(cfg->faces[d], cfg->faces[d] + nf);
        x->cfg.faces[d] = nullptr;
    }
    x->state[0] = x->ws + L.state[0];
    x->state[1] = x->ws + L.state[1];
    x->geo = geo_of(x);
    {
        const hipError_t e = upload_geometry(x);
        if (e != hipSuccess) {
            delete x;
            return fail(HX_EHIP, "geometry upload failed: %s", hipGetErrorString(e));
        }
    }
    clear_flag_kernel<<<1, 1, 0, x->stream>>>(at<int>(x, L.flag));
    set_time_kernel<<<1, 1, 0, x->stream>>>(at<double>(x, L.time), 0.0);
    hipError_t e = hipStreamSynchronize(x->stream);
    if (e != hipSuccess) {
        delete x;
        return fail(HX_EHIP, "create: %s", hipGetErrorString(e));
    }
    *out = x;
    return HX_OK;
}

hx_status hx_shift_grid(hx_ctx* x, double delta)
{
    if (!x)
        return fail(HX_EINVAL, "null context");
    if (!x->have_state)
        return fail(HX_ESTATE, "grid shift before set_state");
    const hx_config& c = x->cfg;
    const int ng = c.nghost, n0 = c.n[0];
    std::vector<double>& f = x->faces[0];
    if (!std::isfinite(delta))
        return fail(HX_EINVAL, "non-finite shift");
    for (int i = ng - 2; i < n0 + ng + 2; i++)
        if (!(std::fabs(delta) <= f[i + 1] - f[i]))
            return fail(HX_EINVAL, "shift %g wider than cell %d of axis 0 (%g)", delta, i - ng, f[i + 1] - f[i]);
    if (c.geom == HX_GEOM_SPH) {
        const double r0 = f[ng] + delta;
        if (r0 < 0.0 || (r0 == 0.0 && c.bc[0][0] != HX_BOUNDARY_REFLECTIVE))
            return fail(HX_EINVAL, "the shift would move the inner radius to %g", r0);
    }
    hx::ShiftParams p;
    p.U = x->state[x->cur];
    p.Unew = x->state[1 - x->cur];
    p.n0 = n0;
    p.ng = ng;
    p.plane = x->ncells;
    p.nvar = x->nvar;
    p.sph = c.geom == HX_GEOM_SPH;
    p.de = c.dual_energy ? 1 : 0;
    p.bc0[0] = c.bc[0][0];
    p.bc0[1] = c.bc[0][1];
    p.xf = at<double>(x, x->L.xfaces);
    p.delta = delta;
    HIPCHECK(hx::launch_shift(p, x->fp32, x->stream));
    x->cur = 1 - x->cur;
    x->dtpart_valid = false;
    // the staging of the last geometry upload is reused: wait for the queued work first
    HIPCHECK(hipStreamSynchronize(x->stream));
    for (double& v : f)
        v += delta;
    HIPCHECK(upload_geometry(x));
    return HX_OK;
}

hx_status hx_set_time(hx_ctx* x, double t)
{
    if (!x || !std::isfinite(t))
        return fail(HX_EINVAL, "null context or non-finite time");
    set_time_kernel<<<1, 1, 0, x->stream>>>(at<double>(x, x->L.time), t);
    HIPCHECK(hipGetLastError());
    return HX_OK;
}

hx_status hx_get_time(hx_ctx* x, double* t)
{
    if (!x || !t)
        return fail(HX_EINVAL, "null argument");
    double h = 0.0;
    HIPCHECK(hipMemcpyAsync(&h, at<double>(x, x->L.time), sizeof(double), hipMemcpyDeviceToHost, x->stream));
    HIPCHECK(hipStreamSynchronize(x->stream));
    *t = h;
    return HX_OK;
}

hx_status hx_set_state(hx_ctx* x, const double* d_U)
{
    if (!x || !d_U)
        return fail(HX_EINVAL, "null argument");
    const long long n = (long long)x->nvar * x->ncells;
    if (x->fp32) {
        HIPCHECK(hx::launch_convert(d_U, x->state[0], n, true, x->stream));
    } else {
        HIPCHECK(hipMemcpyAsync(x->state[0], d_U, sizeof(double) * n, hipMemcpyDeviceToDevice, x->stream));
    }
    x->cur = 0;
    x->have_state = true;
    x->dtpart_valid = false;
    clear_flag_kernel<<<1, 1, 0, x->stream>>>(at<int>(x, x->L.flag));
    HIPCHECK(hipGetLastError());
    return HX_OK;
}

hx_status hx_get_state(hx_ctx* x, double* d_U)
{
    if (!x || !d_U)
        return fail(HX_EINVAL, "null argument");
    if (!x->have_state)
        return fail(HX_ESTATE, "no state loaded");
    const long long n = (long long)x->nvar * x->ncells;
    if (x->fp32) {
        HIPCHECK(hx::launch_convert(x->state[x->cur], d_U, n, false, x->stream));
    } else {
        HIPCHECK(hipMemcpyAsync(d_U, x->state[x->cur], sizeof(double) * n, hipMemcpyDeviceToDevice, x->stream));
    }
    return HX_OK;
}

hx_status hx_compute_dt_device(hx_ctx* x, double* d_dt)
{
    if (!x || !d_dt)
        return fail(HX_EINVAL, "null argument");
    if (!x->have_state)
        return fail(HX_ESTATE, "no state loaded");
    if (x->dtpart_valid) {
        // the last sweep already reduced the CFL rate of the state it wrote, per workgroup
        HIPCHECK(hx::launch_dt_final(at<double>(x, x->L.dtpart), (int)x->dtpart_nb, x->cfg.cfl, d_dt, x->stream));
        return HX_OK;
    }
    hx::DtParams p = dt_params(x);
    HIPCHECK(hx::launch_dt(p, x->fp32, x->L.nred, x->cfg.cfl, d_dt, x->stream));
    return HX_OK;
}

hx_status hx_compute_dt(hx_ctx* x, double* h_dt)
{
    if (!x || !h_dt)
        return fail(HX_EINVAL, "null argument");
    hx_status st = hx_compute_dt_device(x, at<double>(x, x->L.dt));
    if (st != HX_OK)
        return st;
    HIPCHECK(hipMemcpyAsync(h_dt, at<double>(x, x->L.dt), sizeof(double), hipMemcpyDeviceToHost, x->stream));
    return sync_check(x);
}

hx_status hx_step(hx_ctx* x, double dt)
{
    if (!x)
        return fail(HX_EINVAL, "null context");
    if (!(dt > 0.0) || !std::isfinite(dt))
        return fail(HX_EINVAL, "dt must be positive and finite");
    return enqueue_step(x, dt, nullptr);
}

hx_status hx_step_device(hx_ctx* x, const double* d_dt)
{
    if (!x || !d_dt)
        return fail(HX_EINVAL, "null argument");
    return enqueue_step(x, 0.0, d_dt);
}

hx_status hx_run_1d(hx_ctx* x, double t0, double t_end, int max_steps, double* h_t, int* h_steps)
{
    if (!x || !h_t || !h_steps)
        return fail(HX_EINVAL, "null argument");
    if (!x->have_state)
        return fail(HX_ESTATE, "run before set_state");
    const hx_config& c = x->cfg;
    if (c.ndim != 1 || c.geom != HX_GEOM_CART || c.n[1] != 1)
        return fail(HX_EINVAL, "hx_run_1d runs one Cartesian 1D row (ndim 1, n[1] = 1)");
    if (c.n[0] > hx::RUN1D_MAX_CELLS)
        return fail(HX_EINVAL, "hx_run_1d holds at most %d cells (got %d)", hx::RUN1D_MAX_CELLS, c.n[0]);
    if (c.gravity != HX_GRAVITY_NONE || c.dual_energy || c.eos != HX_EOS_GAS || c.ni_heating ||
        c.limiter == HX_LIMITER_MLP)
        return fail(HX_EINVAL, "hx_run_1d supports the ideal gas without gravity, heating, the internal-energy "
                               "monitor or the learned limiter");
    if (!std::isfinite(t0) || !std::isfinite(t_end) || max_steps < 1)
        return fail(HX_EINVAL, "need finite t0, t_end and max_steps >= 1");
    int dev = 0, maxlds = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t lds = hx::run1d_lds_bytes(c.n[0], x->nvar, x->fp32) + 512;
    if (lds > (size_t)maxlds)
        return fail(HX_EINVAL, "hx_run_1d needs %zu bytes of LDS for %d cells and %d fields, the device has %d",
                    lds, c.n[0], x->nvar, maxlds);
    hx::Run1dParams p;
    p.U = x->state[x->cur];
    p.n = c.n[0];
    p.ng = x->ng;
    p.plane = x->ncells;
    p.gamma = c.gamma;
    p.cfl = c.cfl;
    p.limiter = c.limiter;
    p.riemann = c.riemann;
    p.bc0[0] = c.bc[0][0];
    p.bc0[1] = c.bc[0][1];
    p.geo = x->geo;
    p.flag = at<int>(x, x->L.flag);
    p.out = at<double>(x, x->L.run);
    p.t0 = t0;
    p.t_end = t_end;
    p.max_steps = max_steps;
    HIPCHECK(hx::launch_run1d(p, x->nvar, x->fp32, x->stream));
    x->dtpart_valid = false;  // the sweep's CFL maxima no longer describe the state
    double out[2];
    HIPCHECK(hipMemcpyAsync(out, p.out, sizeof out, hipMemcpyDeviceToHost, x->stream));
    const hx_status st = sync_check(x);
    *h_t = out[0];
    *h_steps = (int)out[1];
    return st;
}

hx_status hx_totals(hx_ctx* x, double* h_tot)
{
    if (!x || !h_tot)
        return fail(HX_EINVAL, "null argument");
    if (!x->have_state)
        return fail(HX_ESTATE, "no state loaded");
    hx::DtParams p = dt_params(x);
    HIPCHECK(hx::launch_totals(p, x->fp32, x->L.nred, at<double>(x, x->L.tot), x->stream));
    HIPCHECK(hipMemcpyAsync(h_tot, at<double>(x, x->L.tot), sizeof(double) * x->nvar, hipMemcpyDeviceToHost,
                            x->stream));
    return sync_check(x);
}

hx_status hx_check(hx_ctx* x)
{
    if (!x)
        return fail(HX_EINVAL, "null context");
    return sync_check(x);
}

hx_status hx_set_mlp(hx_ctx* x, const float* h_w, size_t n)
{
    if (!x || !h_w)
        return fail(HX_EINVAL, "null argument");
    if (n != HX_MLP_NPARAM)
        return fail(HX_EINVAL, "expected %d weights, got %zu", HX_MLP_NPARAM, n);
    HIPCHECK(hipMemcpyAsync(at<float>(x, x->L.mlp), h_w, sizeof(float) * n, hipMemcpyHostToDevice, x->stream));
    HIPCHECK(hipStreamSynchronize(x->stream));
    x->have_mlp = true;
    return HX_OK;
}

hx_status hx_set_zchunk(hx_ctx* x, int kz)
{
    if (!x || kz < 0)
        return fail(HX_EINVAL, "z chunk must be >= 0");
    x->kz = kz;
    return HX_OK;
}

hx_status hx_get_zchunk(hx_ctx* x, int* kz)
{
    if (!x || !kz)
        return fail(HX_EINVAL, "null argument");
    *kz = x->kz > 0 ? x->kz : x->kz_auto;
    return HX_OK;
}

hx_status hx_enclosed_mass(hx_ctx* x, double* h_menc)
{
    if (!x || !h_menc)
        return fail(HX_EINVAL, "null argument");
    if (x->cfg.gravity != HX_GRAVITY_POINT_MONOPOLE)
        return fail(HX_ESTATE, "no enclosed-mass gravity in this configuration");
    HIPCHECK(hipMemcpyAsync(h_menc, at<double>(x, x->L.menc), sizeof(double) * x->cfg.n[0], hipMemcpyDeviceToHost,
                            x->stream));
    HIPCHECK(hipStreamSynchronize(x->stream));
    return HX_OK;
}

hx_status hx_arith_check(const double* d_a, const double* d_b, long long n, double* d_q, double* d_s, void* hip_stream)
{
    if (!d_a || !d_b || !d_q || !d_s || n < 0)
        return fail(HX_EINVAL, "invalid argument");
    if (n == 0)
        return HX_OK;
    HIPCHECK(hx::launch_arith_check(d_a, d_b, n, d_q, d_s, (hipStream_t)hip_stream));
    return HX_OK;
}

hx_status hx_mlp_eval(const float* d_w, const float* d_x, long long n, float* d_phi, void* hip_stream)
{
    if (!d_w || !d_x || !d_phi || n < 0)
        return fail(HX_EINVAL, "invalid argument");
    if (n == 0)
        return HX_OK;
    HIPCHECK(hx::launch_mlp_eval(d_w, d_x, n, d_phi, (hipStream_t)hip_stream));
    return HX_OK;
}

hx_status hx_mlp_features(const double* d_fine, int nrows, int nfine, int ratio, double gamma, float* d_x,
                          float* d_a, float* d_t, float* d_wt, void* hip_stream)
{
    if (!d_fine || !d_x || !d_a || !d_t || !d_wt || nrows < 1 || ratio < 2 || nfine < 5 * ratio ||
        nfine % ratio != 0 || !(gamma > 1.0))
        return fail(HX_EINVAL, "invalid argument");
    HIPCHECK(hx::launch_mlp_features(d_fine, nrows, nfine, ratio, gamma, d_x, d_a, d_t, d_wt,
                                     (hipStream_t)hip_stream));
    return HX_OK;
}

size_t hx_mlp_grad_workspace_bytes(long long n)
{
    if (n < 1)
        return 0;
    return sizeof(float) * (size_t)hx::mlp_grad_blocks(n) * (HX_MLP_NPARAM + 2);
}

hx_status hx_mlp_grad(const float* d_w, const float* d_x, const float* d_a, const float* d_t, const float* d_wt,
                      long long n, float* d_grad, float* d_loss, void* d_work, size_t work_bytes, void* hip_stream)
{
    if (!d_w || !d_x || !d_a || !d_t || !d_wt || !d_grad || !d_loss || !d_work || n < 1)
        return fail(HX_EINVAL, "invalid argument");
    if (work_bytes < hx_mlp_grad_workspace_bytes(n))
        return fail(HX_ENOSPACE, "scratch of %zu bytes, need %zu", work_bytes, hx_mlp_grad_workspace_bytes(n));
    HIPCHECK(hx::launch_mlp_grad(d_w, d_x, d_a, d_t, d_wt, n, d_grad, d_loss, (float*)d_work,
                                 (hipStream_t)hip_stream));
    return HX_OK;
}

hx_status hx_mlp_grad_noalloc(const float* d_w, const float* d_x, const float* d_a, const float* d_t,
                              const float* d_wt, long long n, float* d_grad, float* d_loss, void* hip_stream)
{
    if (!d_w || !d_x || !d_a || !d_t || !d_wt || !d_grad || !d_loss || n < 1)
        return fail(HX_EINVAL, "invalid argument");
    const size_t need = hx_mlp_grad_workspace_bytes(n);
    if (need > hx::mlp_grad_scratch_bytes())
        return fail(HX_ENOSPACE, "%lld samples need %zu bytes of scratch, the static scratch holds %zu", n, need,
                    hx::mlp_grad_scratch_bytes());
    HIPCHECK(hx::launch_mlp_grad_noalloc(d_w, d_x, d_a, d_t, d_wt, n, d_grad, d_loss, (hipStream_t)hip_stream));
    return HX_OK;
}

hx_status hx_mlp_adam(float* d_w, const float* d_grad, float* d_m, float* d_v, int step, float lr, float beta1,
                      float beta2, float eps, void* hip_stream)
{
    if (!d_w || !d_grad || !d_m || !d_v || step < 1)
        return fail(HX_EINVAL, "invalid argument");
    HIPCHECK(hx::launch_mlp_adam(d_w, d_grad, d_m, d_v, step, lr, beta1, beta2, eps, (hipStream_t)hip_stream));
    return HX_OK;
}

const char* hx_last_error(void) { return g_err.c_str(); }

void hx_destroy(hx_ctx* x) { delete x; }

}  // extern "C"
