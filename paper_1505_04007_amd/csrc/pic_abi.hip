// Host side of the gfx950 FDTD-PIC library: the C ABI declared in pic.h.
//
// pic_init validates the problem, precomputes every coefficient in FP64
// (Drude ca/cb of Eq. 6 in increment form, CPML b/c/kappa, particle
// constants), rounds them once to FP32, uploads state, and sorts the
// particles by cell.  pic_step enqueues, per step, on one stream:
//   [sort every sort_every steps] -> H update -> push + deposit ->
//   Drude J + E update -> probe DFT
// and polls a device non-finite flag every check_every steps.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_internal.hpp"

namespace {

constexpr double kC = 299792458.0;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kEps0 = 1.0 / (kMu0 * kC * kC);
constexpr double kEta0 = kMu0 * kC;
constexpr int kFamilies = 5;  // h_update, push_deposit, e_update, probe, sort

thread_local std::string g_init_error;

}  // namespace

struct pic_ctx {
    int n[3] = {0, 0, 0};
    int bc[3] = {0, 0, 0};
    int per[3] = {0, 0, 0};
    int npml = 0;
    double dx = 0, dt = 0, S = 0;
    hipStream_t stream = nullptr;
    bool poisoned = false;
    std::string err;
    std::vector<void *> allocs;

    float *E[3] = {nullptr, nullptr, nullptr};
    float *H[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    int hcur = 0;  // host mirror of DevState.parity after the last step
    pic::PmlAxis pml[3];
    pic::DevState *dstate = nullptr;  // step clock advanced by the kernels
    // argument blocks, fixed after pic_init (the step clock lives in dstate)
    pic::FieldArgs fa{};
    pic::PartArgs pa{};
    pic::SortArgs sa{};
    pic::ProbeArgs pr{};

    int mlo[3] = {0, 0, 0}, mhi[3] = {0, 0, 0};
    bool has_metal = false;
    size_t nbox = 0;                     // cells of the metal box
    std::vector<double> wp_box, g_box;  // wp, gamma of its cells (x fastest)
    float *Jp[3] = {nullptr, nullptr, nullptr};
    float2 *coef = nullptr;

    float *Jb[3] = {nullptr, nullptr, nullptr};
    float *Havg[3] = {nullptr, nullptr, nullptr};  // B^n for the gather (particle box only)

    int np = 0;
    float *P[2][6] = {};
    int *pid[2] = {nullptr, nullptr};
    int pcur = 0;
    int *key = nullptr, *rank = nullptr, *counts = nullptr, *box = nullptr, *scan_tmp = nullptr;
    int *boxpart = nullptr;  // per-workgroup partial boxes of the sort's count kernel
    int scan_len = 0;
    float ah = 0.f, qd = 0.f;
    double q = 0, m = 0, w = 0;
    unsigned long long *d_pushes = nullptr;  // per-wavefront push counters
    size_t n_wave_slots = 0;
    int *d_nan = nullptr;
    int deposit_mode = 0;

    int nprobe = 0, nfreq = 0;
    int *pidx = nullptr;
    double *omega = nullptr, *fre = nullptr, *fim = nullptr;
    float *series = nullptr;
    long long series_len = 0;

    bool diag = false;
    double *rho = nullptr, *rho0 = nullptr, *acc = nullptr;
    int *d_live = nullptr;

    long long step = 0;
    int tile = 0;  // field-kernel tile shape (pic_tune)
    int sort_every = 0, check_every = 0;
    long long since_sort = 0;

    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[kFamilies];
};

namespace {

pic_status fail(pic_ctx *c, pic_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) {
        c->err = buf;
        if (st == PIC_EDEVICE || st == PIC_EUNSTABLE) c->poisoned = true;
    } else {
        g_init_error = buf;
    }
    return st;
}

#define HIP_TRY(ctx, call)                                                                         \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((ctx), PIC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));        \
    } while (0)

template <typename T>
pic_status dalloc(pic_ctx *c, T **p, size_t count)
{
    void *q = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, e == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EDEVICE,
                    "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    c->allocs.push_back(q);
    *p = (T *)q;
    return PIC_OK;
}

#define TRY(x)                                                                                     \
    do {                                                                                           \
        pic_status s_ = (x);                                                                       \
        if (s_ != PIC_OK) return s_;                                                               \
    } while (0)

// CPML coefficients at position `pos` (cells) along an axis of n cells.
void cpml_coeff(const pic_grid &g, int npml, int n, double pos, double dx, double dt, float &b,
                float &c, float &ik)
{
    const double L = (double)npml;
    double rho = 0.0;
    if (pos < L) rho = L - pos;
    if (pos > (double)n - L) rho = pos - ((double)n - L);
    if (rho <= 0.0) {
        b = 1.f;
        c = 0.f;
        ik = 1.f;
        return;
    }
    const double m = g.pml_m;
    const double r = rho / L;
    const double smax = g.pml_sigma_scale * 0.8 * (m + 1.0) / (kEta0 * dx);
    const double sig = smax * std::pow(r, m);
    const double kap = 1.0 + (g.pml_kappa_max - 1.0) * std::pow(r, m);
    const double alp = g.pml_alpha_max * (1.0 - r);
    const double bb = std::exp(-(sig / kap + alp) * dt / kEps0);
    const double cc = sig > 0.0 ? sig * (bb - 1.0) / (sig * kap + kap * kap * alp) : 0.0;
    b = (float)bb;
    c = (float)cc;
    ik = (float)(1.0 / kap);
}

// Fill the argument blocks once; nothing in them changes from step to step.
void build_args(pic_ctx *c)
{
    pic::FieldArgs &a = c->fa;
    a = pic::FieldArgs{};
    a.nx = c->n[0];
    a.ny = c->n[1];
    a.nz = c->n[2];
    a.tile = c->tile;
    a.gx = (c->n[0] + pic::TILE_FX[c->tile] - 1) / pic::TILE_FX[c->tile];
    a.gy = (c->n[1] + pic::TILE_FY[c->tile] - 1) / pic::TILE_FY[c->tile];
    a.S = (float)c->S;
    for (int d = 0; d < 3; ++d) {
        a.per[d] = c->per[d];
        a.pml[d] = c->pml[d];
        a.mlo[d] = c->has_metal ? c->mlo[d] : 0;
        a.mhi[d] = c->has_metal ? c->mhi[d] : 0;
        a.E[d] = c->E[d];
        a.H[0][d] = c->H[0][d];
        a.H[1][d] = c->H[1][d];
        a.Havg[d] = c->Havg[d];
        a.Jp[d] = c->Jp[d];
        a.Jb[d] = c->Jb[d];
    }
    a.coef = c->coef;
    a.pbox = c->np > 0 ? c->box : nullptr;
    a.nan_flag = c->d_nan;
    a.st = c->dstate;

    pic::PartArgs &pa = c->pa;
    pa = pic::PartArgs{};
    pa.n = c->np;
    for (int s2 = 0; s2 < 2; ++s2)
        for (int q = 0; q < 6; ++q) pa.P[s2][q] = c->P[s2][q];
    pa.nx = c->n[0];
    pa.ny = c->n[1];
    pa.nz = c->n[2];
    for (int d = 0; d < 3; ++d) {
        pa.per[d] = c->per[d];
        pa.E[d] = c->E[d];
        pa.B[d] = c->Havg[d];
        pa.Jb[d] = c->Jb[d];
    }
    pa.S = (float)c->S;
    pa.ah = c->ah;
    pa.qd = c->qd;
    pa.pushes = c->d_pushes;
    pa.st = c->dstate;

    pic::SortArgs &sa = c->sa;
    sa = pic::SortArgs{};
    sa.n = c->np;
    sa.nx = c->n[0];
    sa.ny = c->n[1];
    sa.nz = c->n[2];
    sa.ncell = c->n[0] * c->n[1] * c->n[2];
    for (int s2 = 0; s2 < 2; ++s2) {
        for (int q = 0; q < 6; ++q) sa.P[s2][q] = c->P[s2][q];
        sa.id[s2] = c->pid[s2];
    }
    sa.key = c->key;
    sa.rank = c->rank;
    sa.counts = c->counts;
    sa.box = c->box;
    sa.boxpart = c->boxpart;
    sa.st = c->dstate;

    pic::ProbeArgs &pr = c->pr;
    pr = pic::ProbeArgs{};
    pr.nprobe = c->nprobe;
    pr.nfreq = c->nfreq;
    pr.pidx = c->pidx;
    pr.omega = c->omega;
    pr.fre = c->fre;
    pr.fim = c->fim;
    pr.series = c->series;
    pr.series_len = c->series_len;
    pr.dt = c->dt;
    pr.Ez = c->E[2];
    pr.st = c->dstate;
}

void tstart(pic_ctx *c, int fam)
{
    if (!c->timing) return;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    (void)hipEventRecord(a, c->stream);
    c->ev[fam].push_back({a, b});
}

void tstop(pic_ctx *c, int fam)
{
    if (!c->timing) return;
    (void)hipEventRecord(c->ev[fam].back().second, c->stream);
}

pic_status do_sort(pic_ctx *c)
{
    if (c->np <= 0) return PIC_OK;
    tstart(c, 4);
    pic::launch_sort(c->sa, c->scan_tmp, c->stream);
    tstop(c, 4);
    HIP_TRY(c, hipGetLastError());
    c->pcur = 1 - c->pcur;  // mirrors the device-side flip in the sort's last kernel
    c->since_sort = 0;
    return PIC_OK;
}

// One step after the sort check, on the context's stream (no
// synchronisation); host mirrors of the device step clock advance with it.
// `rec`, when given, copies the bunch current deposited in this step out
// before the E update consumes it.
pic_status step_body(pic_ctx *c, const pic::BoxCopyArgs *rec)
{
    // 1. H^{n+1/2}
    tstart(c, 0);
    pic::launch_h_update(c->fa, c->stream);
    tstop(c, 0);
    // 2. gather E^n, B^n; Boris; move; deposit J_b^{n+1/2}
    if (c->np > 0) {
        tstart(c, 1);
        pic::launch_push_deposit(c->pa, c->deposit_mode, c->stream);
        tstop(c, 1);
        if (rec) pic::launch_box_copy(*rec, c->stream);
    }
    // 3-4. Drude J^{n+1/2} (Eq. 6), E^{n+1} (Eq. 8 with the bunch current)
    tstart(c, 2);
    pic::launch_e_update(c->fa, c->stream);
    tstop(c, 2);
    // 5. probes; advances the device step clock
    tstart(c, 3);
    pic::launch_probe(c->pr, c->stream);
    tstop(c, 3);
    c->hcur = 1 - c->hcur;
    c->step++;
    c->since_sort++;
    HIP_TRY(c, hipGetLastError());
    return PIC_OK;
}

pic_status step_once(pic_ctx *c)
{
    if (c->np > 0 && c->sort_every > 0 && c->since_sort >= c->sort_every) TRY(do_sort(c));
    return step_body(c, nullptr);
}

pic::DiagArgs diag_args(pic_ctx *c)
{
    pic::DiagArgs a{};
    a.nx = c->n[0];
    a.ny = c->n[1];
    a.nz = c->n[2];
    for (int d = 0; d < 3; ++d) {
        a.per[d] = c->per[d];
        a.npml[d] = c->bc[d] == PIC_BC_CPML ? c->npml : 0;
        a.mlo[d] = c->has_metal ? c->mlo[d] : 0;
        a.mhi[d] = c->has_metal ? c->mhi[d] : -2;
    }
    for (int d = 0; d < 3; ++d) {
        a.E[d] = c->E[d];
        a.H[d] = c->H[c->hcur][d];
    }
    a.np = c->np;
    if (c->np > 0) {
        a.x = c->P[c->pcur][0];
        a.y = c->P[c->pcur][1];
        a.z = c->P[c->pcur][2];
        a.ux = c->P[c->pcur][3];
        a.uy = c->P[c->pcur][4];
        a.uz = c->P[c->pcur][5];
    }
    a.qw_over_vol = c->q * c->w / (c->dx * c->dx * c->dx);
    a.eps0_over_dx = kEps0 / c->dx;
    a.acc = c->acc;
    return a;
}

bool finite_nonneg(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!(std::isfinite(p[i]) && p[i] >= 0.0)) return false;
    return true;
}

}  // namespace

extern "C" {

int pic_abi_version(void) { return PIC_ABI_VERSION; }

const char *pic_last_error(const pic_ctx *ctx)
{
    if (!ctx) return g_init_error.c_str();
    return ctx->err.c_str();
}

void pic_destroy(pic_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (void *p : ctx->allocs) (void)hipFree(p);
    for (int f = 0; f < kFamilies; ++f)
        for (auto &e : ctx->ev[f]) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    delete ctx;
}

static pic_status init_impl(pic_ctx *c, const pic_grid *grid, double dx, double dt,
                            const double *wp_map, const double *gamma_map,
                            const pic_particles *parts, const pic_opts *opts)
{
    const pic_grid &g = *grid;
    const int nn[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
        if (g.bc[d] < PIC_BC_PEC || g.bc[d] > PIC_BC_CPML)
            return fail(c, PIC_EINVAL, "bc[%d] = %d is not a pic_bc code", d, g.bc[d]);
        const int nmin = g.bc[d] == PIC_BC_PERIODIC ? 1 : 2;
        if (nn[d] < nmin) return fail(c, PIC_EINVAL, "axis %d has %d cells (minimum %d)", d, nn[d], nmin);
        c->n[d] = nn[d];
        c->bc[d] = g.bc[d];
        c->per[d] = g.bc[d] == PIC_BC_PERIODIC;
    }
    const long long ncell = (long long)nn[0] * nn[1] * nn[2];
    if (ncell > 0x7fffffffLL) return fail(c, PIC_EINVAL, "grid of %lld cells exceeds 2^31-1", ncell);
    bool any_cpml = false;
    for (int d = 0; d < 3; ++d) any_cpml = any_cpml || g.bc[d] == PIC_BC_CPML;
    if (any_cpml) {
        if (g.npml < 1) return fail(c, PIC_EINVAL, "npml = %d must be >= 1 on a CPML axis", g.npml);
        for (int d = 0; d < 3; ++d)
            if (g.bc[d] == PIC_BC_CPML && 2 * g.npml >= nn[d])
                return fail(c, PIC_EINVAL, "2*npml = %d must be < n = %d on axis %d", 2 * g.npml, nn[d], d);
        if (!(g.pml_m >= 0.0) || !(g.pml_sigma_scale >= 0.0) || !(g.pml_kappa_max >= 1.0) ||
            !(g.pml_alpha_max >= 0.0))
            return fail(c, PIC_EINVAL, "CPML parameters out of range (m, sigma scale >= 0, kappa_max >= 1, alpha_max >= 0)");
    }
    c->npml = any_cpml ? g.npml : 0;
    if (!(dx > 0.0) || !(dt > 0.0) || !std::isfinite(dx) || !std::isfinite(dt))
        return fail(c, PIC_EINVAL, "dx and dt must be positive and finite");
    if (!wp_map || !gamma_map) return fail(c, PIC_EINVAL, "wp_map and gamma_map are required");
    if (!finite_nonneg(wp_map, (size_t)ncell) || !finite_nonneg(gamma_map, (size_t)ncell))
        return fail(c, PIC_EINVAL, "wp_map / gamma_map must be finite and >= 0");
    c->dx = dx;
    c->dt = dt;
    c->S = kC * dt / dx;
    double wpmax = 0.0;
    for (long long q = 0; q < ncell; ++q) wpmax = std::max(wpmax, wp_map[q]);
    const double cfl = 3.0 * c->S * c->S + 0.25 * (wpmax * dt) * (wpmax * dt);
    if (cfl > 1.0 + 1e-12)
        return fail(c, PIC_EINVAL, "time step violates 3 (c dt/dx)^2 + (wp dt/2)^2 <= 1 (value %.6g)", cfl);

    pic_opts o{};
    if (opts) o = *opts;
    c->stream = (hipStream_t)o.stream;
    c->sort_every = o.sort_every > 0 ? o.sort_every : 0;
    c->check_every = o.check_every > 0 ? o.check_every : 0;
    c->timing = o.timing != 0;
    c->diag = o.diag != 0;
    c->deposit_mode = o.deposit_mode == 1 ? 1 : 0;
    if (o.nprobe < 0 || o.nfreq < 0 || o.series_len < 0)
        return fail(c, PIC_EINVAL, "nprobe, nfreq and series_len must be >= 0");
    if (o.nprobe > 256) return fail(c, PIC_EINVAL, "at most 256 probes");
    if (o.nprobe > 0 && !o.probe_xyz) return fail(c, PIC_EINVAL, "probe_xyz is NULL");
    if (o.nfreq > 0 && !o.omega) return fail(c, PIC_EINVAL, "omega is NULL");

    // particles: validate on the host
    const bool with_p = parts && parts->n > 0;
    if (with_p) {
        const pic_particles &P = *parts;
        if (P.n > 0x7fffffffLL) return fail(c, PIC_EINVAL, "at most 2^31-1 particles");
        if (!P.x || !P.y || !P.z || !P.ux || !P.uy || !P.uz)
            return fail(c, PIC_EINVAL, "particle arrays must be non-NULL");
        if (!(P.m > 0.0) || !std::isfinite(P.q) || !std::isfinite(P.weight))
            return fail(c, PIC_EINVAL, "particle mass must be > 0, charge and weight finite");
        const double *X[3] = {P.x, P.y, P.z};
        for (long long i = 0; i < P.n; ++i)
            for (int d = 0; d < 3; ++d) {
                const double v = X[d][i] / dx;
                if (!(v >= 0.0 && v < (double)nn[d]))
                    return fail(c, PIC_EINVAL, "particle %lld lies outside the box on axis %d", i, d);
            }
    }

    // ---- device allocations (E and H may come from the caller) ----
    const size_t N = (size_t)ncell;
    if (o.bufs) {
        const float *given[9];
        int ng = 0;
        for (int d = 0; d < 3; ++d) {
            given[ng++] = o.bufs->E[d];
            given[ng++] = o.bufs->H[0][d];
            given[ng++] = o.bufs->H[1][d];
        }
        for (int q = 0; q < ng; ++q) {
            if (!given[q]) continue;
            if ((uintptr_t)given[q] % 4 != 0) return fail(c, PIC_EINVAL, "bufs: field pointer %d is not 4-byte aligned", q);
            for (int r = 0; r < q; ++r)
                if (given[r] && given[r] < given[q] + N && given[q] < given[r] + N)
                    return fail(c, PIC_EINVAL, "bufs: field arrays %d and %d overlap", r, q);
        }
    }
    for (int d = 0; d < 3; ++d) {
        float *gE = o.bufs ? o.bufs->E[d] : nullptr;
        float *gH0 = o.bufs ? o.bufs->H[0][d] : nullptr;
        float *gH1 = o.bufs ? o.bufs->H[1][d] : nullptr;
        if (gE) c->E[d] = gE;
        else TRY(dalloc(c, &c->E[d], N));
        if (gH0) c->H[0][d] = gH0;
        else TRY(dalloc(c, &c->H[0][d], N));
        if (gH1) c->H[1][d] = gH1;
        else TRY(dalloc(c, &c->H[1][d], N));
        HIP_TRY(c, hipMemsetAsync(c->E[d], 0, N * 4, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->H[0][d], 0, N * 4, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->H[1][d], 0, N * 4, c->stream));
    }
    TRY(dalloc(c, &c->d_nan, 1));
    HIP_TRY(c, hipMemsetAsync(c->d_nan, 0, 4, c->stream));
    TRY(dalloc(c, &c->acc, 16));
    TRY(dalloc(c, &c->d_live, 1));
    TRY(dalloc(c, &c->dstate, 1));
    HIP_TRY(c, hipMemsetAsync(c->dstate, 0, sizeof(pic::DevState), c->stream));

    // host staging kept alive until the final synchronisation
    std::vector<std::vector<float>> stage;
    auto upload = [&](void *dst, const void *src, size_t bytes) -> pic_status {
        HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
        return PIC_OK;
    };

    // optional initial fields (compact Yee layout, SI).  On a PEC wall (also
    // behind a CPML) tangential E and normal H vanish: the stored lower-wall
    // planes are zeroed, as the upper-wall planes are implicitly.
    auto on_wall = [&](size_t q, int comp, bool electric) {
        const int id[3] = {(int)(q % nn[0]), (int)((q / nn[0]) % nn[1]), (int)(q / ((size_t)nn[0] * nn[1]))};
        for (int a = 0; a < 3; ++a) {
            if (c->per[a] || id[a] != 0) continue;
            if (electric ? a != comp : a == comp) return true;
        }
        return false;
    };
    for (int d = 0; d < 3; ++d) {
        if (o.init_E[d]) {
            stage.emplace_back(N);
            for (size_t q = 0; q < N; ++q) stage.back()[q] = on_wall(q, d, true) ? 0.f : (float)o.init_E[d][q];
            TRY(upload(c->E[d], stage.back().data(), N * 4));
        }
        if (o.init_H[d]) {
            stage.emplace_back(N);
            for (size_t q = 0; q < N; ++q)
                stage.back()[q] = on_wall(q, d, false) ? 0.f : (float)(o.init_H[d][q] * kEta0);
            TRY(upload(c->H[0][d], stage.back().data(), N * 4));
        }
    }

    // Drude coefficients on the metal bounding box (cell owns its three edges)
    int lo[3] = {nn[0], nn[1], nn[2]}, hi[3] = {-1, -1, -1};
    for (int k = 0; k < nn[2]; ++k)
        for (int j = 0; j < nn[1]; ++j)
            for (int i = 0; i < nn[0]; ++i) {
                const size_t q = (size_t)i + (size_t)nn[0] * ((size_t)j + (size_t)nn[1] * k);
                if (wp_map[q] > 0.0) {
                    const int id[3] = {i, j, k};
                    for (int d = 0; d < 3; ++d) {
                        lo[d] = std::min(lo[d], id[d]);
                        hi[d] = std::max(hi[d], id[d]);
                    }
                }
            }
    c->has_metal = hi[0] >= 0;
    if (c->has_metal) {
        for (int d = 0; d < 3; ++d) {
            c->mlo[d] = lo[d];
            c->mhi[d] = hi[d] + 1;
        }
        const int wx = c->mhi[0] - c->mlo[0], wy = c->mhi[1] - c->mlo[1], wz = c->mhi[2] - c->mlo[2];
        const size_t nb = (size_t)wx * wy * wz;
        c->nbox = nb;
        c->wp_box.assign(nb, 0.0);
        c->g_box.assign(nb, 0.0);
        std::vector<float> cf(2 * nb);
        for (int k = 0; k < wz; ++k)
            for (int j = 0; j < wy; ++j)
                for (int i = 0; i < wx; ++i) {
                    const size_t q = (size_t)(i + c->mlo[0]) +
                                     (size_t)nn[0] * ((size_t)(j + c->mlo[1]) + (size_t)nn[1] * (k + c->mlo[2]));
                    const double wp = wp_map[q], gm = gamma_map[q];
                    // Eq. 6 rescaled by dt/eps0: Jt += cbt E - d Jt
                    const double cbt = 2.0 * (wp * dt) * (wp * dt) / (2.0 + gm * dt);
                    const double dd = 2.0 * gm * dt / (2.0 + gm * dt);
                    const size_t b = (size_t)i + (size_t)wx * ((size_t)j + (size_t)wy * k);
                    c->wp_box[b] = wp;
                    c->g_box[b] = gm;
                    cf[2 * b] = wp > 0.0 ? (float)cbt : 0.f;
                    cf[2 * b + 1] = wp > 0.0 ? (float)dd : 0.f;
                }
        TRY(dalloc(c, &c->coef, nb));
        stage.emplace_back(std::move(cf));
        TRY(upload(c->coef, stage.back().data(), 2 * nb * 4));
        for (int d = 0; d < 3; ++d) {
            TRY(dalloc(c, &c->Jp[d], nb));
            HIP_TRY(c, hipMemsetAsync(c->Jp[d], 0, nb * 4, c->stream));
        }
    }

    // CPML tables and psi slabs
    for (int d = 0; d < 3; ++d) {
        pic::PmlAxis &P = c->pml[d];
        P = pic::PmlAxis{};
        if (g.bc[d] != PIC_BC_CPML) continue;
        P.on = 1;
        P.npml = g.npml;
        const int n = nn[d];
        std::vector<float> tab(6 * (size_t)n);
        for (int i = 0; i < n; ++i) {
            cpml_coeff(g, g.npml, n, (double)i, dx, dt, tab[0 * n + i], tab[1 * n + i], tab[2 * n + i]);
            cpml_coeff(g, g.npml, n, i + 0.5, dx, dt, tab[3 * n + i], tab[4 * n + i], tab[5 * n + i]);
        }
        float *dtab = nullptr;
        TRY(dalloc(c, &dtab, tab.size()));
        stage.emplace_back(std::move(tab));
        TRY(upload(dtab, stage.back().data(), stage.back().size() * 4));
        P.bE = dtab;
        P.cE = dtab + n;
        P.kE = dtab + 2 * n;
        P.bH = dtab + 3 * n;
        P.cH = dtab + 4 * n;
        P.kH = dtab + 5 * n;
        const size_t slab = (size_t)2 * g.npml * (N / (size_t)n);
        for (int q = 0; q < 2; ++q) {
            TRY(dalloc(c, &P.psiE[q], slab));
            TRY(dalloc(c, &P.psiH[q], slab));
            HIP_TRY(c, hipMemsetAsync(P.psiE[q], 0, slab * 4, c->stream));
            HIP_TRY(c, hipMemsetAsync(P.psiH[q], 0, slab * 4, c->stream));
        }
    }

    // probes: nearest Ez node, i, j rounded half up, k = floor(z/dx)
    c->nprobe = o.nprobe;
    c->nfreq = o.nfreq;
    c->series_len = o.series_len;
    if (c->nprobe > 0) {
        std::vector<int> pidx(c->nprobe);
        for (int p = 0; p < c->nprobe; ++p) {
            const int i = (int)std::floor(o.probe_xyz[3 * p] / dx + 0.5);
            const int j = (int)std::floor(o.probe_xyz[3 * p + 1] / dx + 0.5);
            const int k = (int)std::floor(o.probe_xyz[3 * p + 2] / dx);
            if (i < 0 || i >= nn[0] || j < 0 || j >= nn[1] || k < 0 || k >= nn[2])
                return fail(c, PIC_EINVAL, "probe %d maps to Ez node (%d,%d,%d) outside the stored grid", p, i, j, k);
            pidx[p] = i + nn[0] * (j + nn[1] * k);
        }
        TRY(dalloc(c, &c->pidx, c->nprobe));
        HIP_TRY(c, hipMemcpyAsync(c->pidx, pidx.data(), 4 * pidx.size(), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const size_t nf = (size_t)c->nprobe * c->nfreq;
        TRY(dalloc(c, &c->omega, c->nfreq > 0 ? c->nfreq : 1));
        TRY(dalloc(c, &c->fre, nf ? nf : 1));
        TRY(dalloc(c, &c->fim, nf ? nf : 1));
        if (c->nfreq > 0)
            HIP_TRY(c, hipMemcpyAsync(c->omega, o.omega, 8 * (size_t)c->nfreq, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->fre, 0, 8 * (nf ? nf : 1), c->stream));
        HIP_TRY(c, hipMemsetAsync(c->fim, 0, 8 * (nf ? nf : 1), c->stream));
        if (c->series_len > 0) TRY(dalloc(c, &c->series, (size_t)c->series_len * c->nprobe));
    }

    // particles: FP32 cell-unit positions, u/c
    if (with_p) {
        const pic_particles &P = *parts;
        c->np = (int)P.n;
        c->q = P.q;
        c->m = P.m;
        c->w = P.weight;
        c->ah = (float)(P.q * dt / (2.0 * P.m * kC));
        c->qd = (float)(-P.q * P.weight / (kEps0 * dx * dx));
        const double *src[6] = {P.x, P.y, P.z, P.ux, P.uy, P.uz};
        for (int s = 0; s < 2; ++s) {
            for (int q = 0; q < 6; ++q) TRY(dalloc(c, &c->P[s][q], (size_t)c->np));
            TRY(dalloc(c, &c->pid[s], (size_t)c->np));
        }
        for (int q = 0; q < 6; ++q) {
            stage.emplace_back((size_t)c->np);
            const double sc = q < 3 ? 1.0 / dx : 1.0 / kC;
            for (int i = 0; i < c->np; ++i) stage.back()[i] = (float)(src[q][i] * sc);
            if (q < 3) {
                // keep the FP32 cell coordinate inside [0, n) after rounding
                for (int i = 0; i < c->np; ++i)
                    if (stage.back()[i] >= (float)nn[q]) stage.back()[i] = std::nextafter((float)nn[q], 0.f);
            }
            TRY(upload(c->P[0][q], stage.back().data(), (size_t)c->np * 4));
        }
        std::vector<int> ids(c->np);
        for (int i = 0; i < c->np; ++i) ids[i] = i;
        HIP_TRY(c, hipMemcpyAsync(c->pid[0], ids.data(), 4 * (size_t)c->np, hipMemcpyHostToDevice, c->stream));
        // one push counter per wavefront of the push launch
        c->n_wave_slots = ((size_t)c->np + pic::PBLOCK - 1) / pic::PBLOCK * (pic::PBLOCK / 64);
        TRY(dalloc(c, &c->d_pushes, c->n_wave_slots));
        HIP_TRY(c, hipMemsetAsync(c->d_pushes, 0, 8 * c->n_wave_slots, c->stream));
        TRY(dalloc(c, &c->key, (size_t)c->np));
        TRY(dalloc(c, &c->rank, (size_t)c->np));
        TRY(dalloc(c, &c->counts, (size_t)ncell + 1));
        TRY(dalloc(c, &c->box, 6));
        TRY(dalloc(c, &c->boxpart, 6 * (((size_t)c->np + pic::PBLOCK - 1) / pic::PBLOCK)));
        c->scan_len = pic::scan_tmp_size((int)ncell + 1);
        TRY(dalloc(c, &c->scan_tmp, (size_t)c->scan_len));
        for (int d = 0; d < 3; ++d) {
            TRY(dalloc(c, &c->Jb[d], N));
            HIP_TRY(c, hipMemsetAsync(c->Jb[d], 0, N * 4, c->stream));
            TRY(dalloc(c, &c->Havg[d], N));
            HIP_TRY(c, hipMemsetAsync(c->Havg[d], 0, N * 4, c->stream));
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        build_args(c);
        TRY(do_sort(c));
        if (c->diag) {
            const size_t nodes = (size_t)(nn[0] + 1) * (nn[1] + 1) * (nn[2] + 1);
            TRY(dalloc(c, &c->rho, nodes));
            TRY(dalloc(c, &c->rho0, nodes));
            HIP_TRY(c, hipMemsetAsync(c->rho0, 0, nodes * 8, c->stream));
            pic::DiagArgs a = diag_args(c);
            a.rho = c->rho0;
            pic::launch_rho(a, c->stream);
            HIP_TRY(c, hipGetLastError());
        }
    }
    build_args(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipGetLastError());
    c->since_sort = 0;
    return PIC_OK;
}

pic_status pic_init(pic_ctx **ctx, const pic_grid *grid, double dx, double dt, const double *wp_map,
                    const double *gamma_map, const pic_particles *particles, const pic_opts *opts)
{
    if (!ctx) return fail(nullptr, PIC_EINVAL, "ctx is NULL");
    *ctx = nullptr;
    if (!grid) return fail(nullptr, PIC_EINVAL, "grid is NULL");
    pic_ctx *c = new (std::nothrow) pic_ctx();
    if (!c) return fail(nullptr, PIC_ENOMEM, "out of host memory");
    pic_status st = init_impl(c, grid, dx, dt, wp_map, gamma_map, particles, opts);
    if (st != PIC_OK) {
        g_init_error = c->err;
        pic_destroy(c);
        return st;
    }
    *ctx = c;
    return PIC_OK;
}

#define CHECK_CTX(c)                                                                               \
    do {                                                                                           \
        if (!(c)) return fail(nullptr, PIC_EINVAL, "ctx is NULL");                                 \
        if ((c)->poisoned) return PIC_ESTATE;                                                      \
    } while (0)

pic_status pic_step(pic_ctx *c, int64_t nsteps)
{
    CHECK_CTX(c);
    if (nsteps < 0) return fail(c, PIC_EINVAL, "nsteps must be >= 0");
    for (int64_t it = 0; it < nsteps; ++it) {
        TRY(step_once(c));
        if (c->check_every > 0 && c->step % c->check_every == 0) {
            int flag = 0;
            HIP_TRY(c, hipMemcpyAsync(&flag, c->d_nan, 4, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (flag) return fail(c, PIC_EUNSTABLE, "non-finite field value detected by step %lld", c->step);
        }
    }
    return PIC_OK;
}

pic_status pic_probe(pic_ctx *c, double *re, double *im, double *series)
{
    CHECK_CTX(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const size_t nf = (size_t)c->nprobe * c->nfreq;
    if (nf && re) HIP_TRY(c, hipMemcpy(re, c->fre, nf * 8, hipMemcpyDeviceToHost));
    if (nf && im) HIP_TRY(c, hipMemcpy(im, c->fim, nf * 8, hipMemcpyDeviceToHost));
    if (series && c->series) {
        const long long ns = std::min<long long>(c->step, c->series_len);
        std::vector<float> tmp((size_t)ns * c->nprobe);
        if (!tmp.empty())
            HIP_TRY(c, hipMemcpy(tmp.data(), c->series, tmp.size() * 4, hipMemcpyDeviceToHost));
        for (size_t q = 0; q < tmp.size(); ++q) series[q] = tmp[q];
    }
    return PIC_OK;
}

}  // extern "C"

namespace {

// Device memory of one pic_grad call, released on every exit path once the
// stream has drained.
struct GradScratch {
    hipStream_t s = nullptr;
    std::vector<void *> p;
    ~GradScratch()
    {
        if (p.empty()) return;
        (void)hipStreamSynchronize(s);
        for (void *q : p) (void)hipFree(q);
    }
};

template <typename T>
pic_status galloc(pic_ctx *c, GradScratch &g, T **out, size_t count)
{
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, e == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EDEVICE,
                    "pic_grad: hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    g.p.push_back(q);
    *out = (T *)q;
    return PIC_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t slab_cells(const pic_ctx *c, int a)
{
    const size_t N = (size_t)c->n[0] * c->n[1] * c->n[2];
    return (size_t)2 * c->npml * (N / (size_t)c->n[a]);
}

// Everything a fields-only step reads and writes: the state one checkpoint holds.
struct StateArr {
    void *p;
    size_t bytes;
};

std::vector<StateArr> field_state(pic_ctx *c, int h)
{
    const size_t N = (size_t)c->n[0] * c->n[1] * c->n[2];
    std::vector<StateArr> v;
    for (int d = 0; d < 3; ++d) v.push_back({c->E[d], N * 4});
    for (int d = 0; d < 3; ++d) v.push_back({c->H[h][d], N * 4});
    if (c->has_metal)
        for (int d = 0; d < 3; ++d) v.push_back({c->Jp[d], c->nbox * 4});
    for (int a = 0; a < 3; ++a)
        if (c->pml[a].on)
            for (int q = 0; q < 2; ++q) {
                v.push_back({c->pml[a].psiE[q], slab_cells(c, a) * 4});
                v.push_back({c->pml[a].psiH[q], slab_cells(c, a) * 4});
            }
    v.push_back({c->dstate, sizeof(pic::DevState)});
    return v;
}

size_t state_bytes(pic_ctx *c)
{
    size_t b = 0;
    for (const StateArr &a : field_state(c, 0)) b += align256(a.bytes);
    return b;
}

struct Mirror {
    int hcur;
    long long step, since_sort;
};

pic_status ckpt_save(pic_ctx *c, char *dst, Mirror &m)
{
    size_t off = 0;
    for (const StateArr &a : field_state(c, c->hcur)) {
        HIP_TRY(c, hipMemcpyAsync(dst + off, a.p, a.bytes, hipMemcpyDeviceToDevice, c->stream));
        off += align256(a.bytes);
    }
    m = {c->hcur, c->step, c->since_sort};
    return PIC_OK;
}

pic_status ckpt_load(pic_ctx *c, const char *src, const Mirror &m)
{
    size_t off = 0;
    for (const StateArr &a : field_state(c, m.hcur)) {
        HIP_TRY(c, hipMemcpyAsync(a.p, src + off, a.bytes, hipMemcpyDeviceToDevice, c->stream));
        off += align256(a.bytes);
    }
    c->hcur = m.hcur;
    c->step = m.step;
    c->since_sort = m.since_sort;
    return PIC_OK;
}

// The cells the E update of a step reads the bunch current from: the particle
// box of the last sort widened by the step's margin (as the kernel computes
// it, in FP32), clipped to the grid; whole axes where periodic.
void jb_region(const pic_ctx *c, const int box[6], long long since_sort, int lo[3], int w[3])
{
    const int m = 3 + (int)std::ceil((float)(since_sort + 1) * (float)c->S);
    for (int d = 0; d < 3; ++d) {
        long long l = 0, h = c->n[d] - 1;
        if (!c->per[d]) {
            l = std::max<long long>(0, (long long)box[d] - m);
            h = std::min<long long>(c->n[d] - 1, (long long)box[3 + d] + m);
        }
        lo[d] = (int)std::min<long long>(l, c->n[d]);
        w[d] = h >= l ? (int)(h - l + 1) : 0;
    }
    if (w[0] == 0 || w[1] == 0 || w[2] == 0) w[0] = w[1] = w[2] = 0;
}

// Per-step record of the bunch current: packed boxes in a growing set of chunks.
struct JbRecord {
    int lo[3], w[3];
    float *p;
};

struct Arena {
    float *cur = nullptr;
    size_t used = 0, cap = 0;
};

pic_status arena_take(pic_ctx *c, GradScratch &g, Arena &ar, size_t count, float **out)
{
    const size_t need = (count + 63) & ~(size_t)63;
    if (ar.used + need > ar.cap) {
        const size_t cap = std::max<size_t>(need, (size_t)16 << 20);
        TRY(galloc(c, g, &ar.cur, cap));
        ar.cap = cap;
        ar.used = 0;
    }
    *out = ar.cur + ar.used;
    ar.used += need;
    return PIC_OK;
}

// The adjoint reads, for every step, E^n and J^{n-1/2} on the metal box
// (the Drude gradient's factors).  store_all: the forward run keeps that
// snapshot for every step and the reverse pass needs no replay; otherwise
// it keeps a field checkpoint every K steps and the bunch current of every
// step, and the reverse pass replays each segment to regenerate them.
pic_status grad_impl(pic_ctx *c, double omega0, long long N, long long K, bool store_all, double *L,
                     double *dL_dwp, double *dL_dgamma)
{
    const size_t ncell = (size_t)c->n[0] * c->n[1] * c->n[2];
    const int npr = c->nprobe;
    const double dt = c->dt;
    if (store_all) K = N;
    const long long nseg = (N + K - 1) / K;
    const long long s0 = c->step;
    GradScratch g;
    g.s = c->stream;

    pic::TrajArgs ta{};
    for (int d = 0; d < 3; ++d) {
        ta.E[d] = c->E[d];
        ta.Jp[d] = c->Jp[d];
        ta.mlo[d] = c->mlo[d];
        ta.w[d] = c->mhi[d] - c->mlo[d];
    }
    ta.nx = c->n[0];
    ta.ny = c->n[1];
    float *traj = nullptr;  // metal-box snapshots: one per step of a segment, or of the run
    TRY(galloc(c, g, &traj, (size_t)K * 6 * c->nbox));

    // ---- forward run: snapshots or checkpoints + bunch current, probe Ez ----
    const size_t ckb = state_bytes(c);
    char *ck = nullptr;
    if (!store_all) TRY(galloc(c, g, &ck, ckb * (size_t)(nseg + 1)));
    std::vector<Mirror> mir((size_t)nseg + 1);
    double *gser = nullptr;
    TRY(galloc(c, g, &gser, (size_t)N * npr));
    std::vector<JbRecord> rec((size_t)N);
    Arena ar;
    pic::ProbeArgs prs = c->pr;
    c->pr.gser = gser;
    c->pr.g0 = s0;
    c->pr.gn = N;
    int hbox[6] = {0, 0, 0, -1, -1, -1};
    bool have_box = false;
    pic_status st = PIC_OK;
    for (long long r = 0; r < N && st == PIC_OK; ++r) {
        if (store_all) {
            if (c->has_metal) {
                ta.out = traj + (size_t)r * 6 * c->nbox;
                pic::launch_traj_store(ta, c->stream);
            }
            st = step_once(c);
            continue;
        }
        if (r % K == 0) st = ckpt_save(c, ck + (size_t)(r / K) * ckb, mir[(size_t)(r / K)]);
        if (st != PIC_OK) break;
        if (c->np <= 0) {
            st = step_body(c, nullptr);
            continue;
        }
        if (c->sort_every > 0 && c->since_sort >= c->sort_every) {
            st = do_sort(c);
            have_box = false;
            if (st != PIC_OK) break;
        }
        if (!have_box) {
            hipError_t e = hipMemcpyAsync(hbox, c->box, sizeof hbox, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) {
                st = fail(c, PIC_EDEVICE, "pic_grad: reading the particle box failed: %s", hipGetErrorString(e));
                break;
            }
            have_box = true;
        }
        JbRecord &R = rec[(size_t)r];
        jb_region(c, hbox, c->since_sort, R.lo, R.w);
        const size_t cnt = (size_t)3 * R.w[0] * R.w[1] * R.w[2];
        R.p = nullptr;
        if (cnt) {
            st = arena_take(c, g, ar, cnt, &R.p);
            if (st != PIC_OK) break;
        }
        pic::BoxCopyArgs ra{};
        for (int d = 0; d < 3; ++d) {
            ra.grid[d] = c->Jb[d];
            ra.lo[d] = R.lo[d];
            ra.w[d] = R.w[d];
        }
        ra.packed = R.p;
        ra.nx = c->n[0];
        ra.ny = c->n[1];
        ra.to_grid = 0;
        st = step_body(c, cnt ? &ra : nullptr);
    }
    c->pr = prs;
    TRY(st);
    {
        int flag = 0;
        HIP_TRY(c, hipMemcpyAsync(&flag, c->d_nan, 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (flag) return fail(c, PIC_EUNSTABLE, "non-finite field value detected by step %lld", c->step);
    }

    // ---- objective and its seeds dL/dEz_p^n ----
    std::vector<double> ez((size_t)N * npr);
    HIP_TRY(c, hipMemcpy(ez.data(), gser, ez.size() * 8, hipMemcpyDeviceToHost));
    std::vector<double> Fr(npr, 0.0), Fi(npr, 0.0);
    for (long long r = 0; r < N; ++r) {
        const double th = omega0 * (double)(s0 + 1 + r) * dt;
        const double cs = std::cos(th), sn = std::sin(th);
        for (int p = 0; p < npr; ++p) {
            Fr[p] += dt * ez[(size_t)r * npr + p] * cs;
            Fi[p] -= dt * ez[(size_t)r * npr + p] * sn;
        }
    }
    double l = 0.0;
    for (int p = 0; p < npr; ++p) l += Fr[p] * Fr[p] + Fi[p] * Fi[p];
    *L = l;
    std::vector<double> seed((size_t)N * npr);
    double sigma = 0.0;
    for (long long r = 0; r < N; ++r) {
        const double th = omega0 * (double)(s0 + 1 + r) * dt;
        for (int p = 0; p < npr; ++p) {
            const double v = 2.0 * dt * (Fr[p] * std::cos(th) - Fi[p] * std::sin(th));
            seed[(size_t)r * npr + p] = v;
            sigma = std::max(sigma, std::fabs(v));
        }
    }
    if (dL_dwp) std::fill(dL_dwp, dL_dwp + ncell, 0.0);
    if (dL_dgamma) std::fill(dL_dgamma, dL_dgamma + ncell, 0.0);
    if (!c->has_metal || sigma == 0.0 || (!dL_dwp && !dL_dgamma)) return PIC_OK;

    // ---- adjoint state (seeds scaled by 1/sigma, so the adjoint is O(1) in FP32) ----
    Mirror endm{};
    char *endck = store_all ? nullptr : ck + (size_t)nseg * ckb;
    if (!store_all) TRY(ckpt_save(c, endck, endm));
    std::vector<float> seedf(seed.size());
    for (size_t q = 0; q < seed.size(); ++q) seedf[q] = (float)(seed[q] / sigma);
    float *dseed = nullptr;
    TRY(galloc(c, g, &dseed, seedf.size()));
    HIP_TRY(c, hipMemcpyAsync(dseed, seedf.data(), seedf.size() * 4, hipMemcpyHostToDevice, c->stream));

    pic::AdjArgs aa{};
    aa.nx = c->n[0];
    aa.ny = c->n[1];
    aa.nz = c->n[2];
    aa.gx = (c->n[0] + pic::FX - 1) / pic::FX;  // the adjoint kernels use the default tile
    aa.gy = (c->n[1] + pic::FY - 1) / pic::FY;
    aa.S = (float)c->S;
    for (int d = 0; d < 3; ++d) {
        aa.per[d] = c->per[d];
        aa.pml[d] = c->pml[d];
        aa.mlo[d] = c->mlo[d];
        aa.mhi[d] = c->mhi[d];
        TRY(galloc(c, g, &aa.Ea[d], ncell));
        TRY(galloc(c, g, &aa.Ha[d], ncell));
        TRY(galloc(c, g, &aa.Ja[d], c->nbox));
        HIP_TRY(c, hipMemsetAsync(aa.Ea[d], 0, ncell * 4, c->stream));
        HIP_TRY(c, hipMemsetAsync(aa.Ha[d], 0, ncell * 4, c->stream));
        HIP_TRY(c, hipMemsetAsync(aa.Ja[d], 0, c->nbox * 4, c->stream));
        if (c->pml[d].on)
            for (int q = 0; q < 2; ++q) {
                const size_t sc = slab_cells(c, d);
                TRY(galloc(c, g, &aa.psiEa[d][q], sc));
                TRY(galloc(c, g, &aa.psiHa[d][q], sc));
                TRY(galloc(c, g, &aa.DE[d][q], sc));
                TRY(galloc(c, g, &aa.DH[d][q], sc));
                HIP_TRY(c, hipMemsetAsync(aa.psiEa[d][q], 0, sc * 4, c->stream));
                HIP_TRY(c, hipMemsetAsync(aa.psiHa[d][q], 0, sc * 4, c->stream));
                HIP_TRY(c, hipMemsetAsync(aa.DE[d][q], 0, sc * 4, c->stream));
                HIP_TRY(c, hipMemsetAsync(aa.DH[d][q], 0, sc * 4, c->stream));
            }
    }
    aa.coef = c->coef;
    TRY(galloc(c, g, &aa.gcb, c->nbox));
    TRY(galloc(c, g, &aa.gd, c->nbox));
    HIP_TRY(c, hipMemsetAsync(aa.gcb, 0, c->nbox * 8, c->stream));
    HIP_TRY(c, hipMemsetAsync(aa.gd, 0, c->nbox * 8, c->stream));
    aa.nprobe = npr;
    aa.pidx = c->pidx;

    // replay: fields only, bunch current from the record, E update reading
    // and clearing it over the whole grid, probes not accumulated
    int *dfull = nullptr;
    pic::FieldArgs fr = c->fa;
    for (int d = 0; d < 3; ++d) fr.Havg[d] = nullptr;
    if (c->np > 0) {
        const int full[6] = {0, 0, 0, c->n[0] - 1, c->n[1] - 1, c->n[2] - 1};
        TRY(galloc(c, g, &dfull, 6));
        HIP_TRY(c, hipMemcpyAsync(dfull, full, sizeof full, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        fr.pbox = dfull;
    }
    pic::ProbeArgs pq = c->pr;
    pq.nprobe = 0;
    pq.nfreq = 0;
    pq.series = nullptr;
    pq.gser = nullptr;

    // dL/dE^{s0+N} and the CPML weights of the last step's E update
    aa.mode = 2;
    aa.seed = dseed + (size_t)(N - 1) * npr;
    aa.traj = nullptr;
    pic::launch_adj_edge(aa, c->stream);
    for (long long j = nseg - 1; j >= 0; --j) {
        const long long a0 = j * K, b0 = std::min(N, a0 + K);
        if (!store_all) TRY(ckpt_load(c, ck + (size_t)j * ckb, mir[(size_t)j]));
        for (long long r = a0; r < b0 && !store_all; ++r) {
            ta.out = traj + (size_t)(r - a0) * 6 * c->nbox;
            pic::launch_traj_store(ta, c->stream);
            pic::launch_h_update(fr, c->stream);
            const JbRecord &R = rec[(size_t)r];
            if (c->np > 0 && R.p) {
                pic::BoxCopyArgs sa{};
                for (int d = 0; d < 3; ++d) {
                    sa.grid[d] = c->Jb[d];
                    sa.lo[d] = R.lo[d];
                    sa.w[d] = R.w[d];
                }
                sa.packed = R.p;
                sa.nx = c->n[0];
                sa.ny = c->n[1];
                sa.to_grid = 1;
                pic::launch_box_copy(sa, c->stream);
            }
            pic::launch_e_update(fr, c->stream);
            pic::launch_probe(pq, c->stream);
            c->hcur = 1 - c->hcur;
            c->step++;
            c->since_sort++;
        }
        // reverse steps s0 + r, r = b0-1 .. a0
        for (long long r = b0 - 1; r >= a0; --r) {
            pic::launch_adj_face(aa, c->stream);
            aa.mode = 1 | (r > 0 ? 2 : 0);
            aa.traj = traj + (size_t)(r - a0) * 6 * c->nbox;
            aa.seed = r > 0 ? dseed + (size_t)(r - 1) * npr : nullptr;
            pic::launch_adj_edge(aa, c->stream);
        }
        HIP_TRY(c, hipGetLastError());
    }
    if (!store_all) TRY(ckpt_load(c, endck, endm));

    // ---- chain rule to (wp, gamma) per cell, FP64 on the host ----
    std::vector<double> gcb(c->nbox), gd(c->nbox);
    HIP_TRY(c, hipMemcpyAsync(gcb.data(), aa.gcb, c->nbox * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(gd.data(), aa.gd, c->nbox * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int wx = c->mhi[0] - c->mlo[0], wy = c->mhi[1] - c->mlo[1], wz = c->mhi[2] - c->mlo[2];
    for (int k = 0; k < wz; ++k)
        for (int j = 0; j < wy; ++j)
            for (int i = 0; i < wx; ++i) {
                const size_t b = (size_t)i + (size_t)wx * ((size_t)j + (size_t)wy * k);
                const size_t q = (size_t)(i + c->mlo[0]) +
                                 (size_t)c->n[0] * ((size_t)(j + c->mlo[1]) + (size_t)c->n[1] * (k + c->mlo[2]));
                const double wp = c->wp_box[b], gm = c->g_box[b];
                if (!(wp > 0.0)) continue;  // cbt = 2 (wp dt)^2 / (2 + g dt): flat at wp = 0; J = 0 there
                const double den = 2.0 + gm * dt;
                const double dcb_dwp = 4.0 * wp * dt * dt / den;
                const double dcb_dg = -2.0 * wp * wp * dt * dt * dt / (den * den);
                const double dd_dg = 4.0 * dt / (den * den);
                if (dL_dwp) dL_dwp[q] = sigma * gcb[b] * dcb_dwp;
                if (dL_dgamma) dL_dgamma[q] = sigma * (gcb[b] * dcb_dg + gd[b] * dd_dg);
            }
    return PIC_OK;
}

// The fastest shape; the default one unless another beats it by more than
// 3 % (isolated H + E timings do not see the particle kernels' cache traffic
// between them, so small margins do not carry over to whole steps).
int pick_shape(const double *ms)
{
    int best = 0;
    for (int v = 1; v < pic::N_TILE_SHAPES; ++v)
        if (ms[v] < ms[best]) best = v;
    return ms[best] < 0.97 * ms[0] ? best : 0;
}

// Average milliseconds of one H + E launch pair for every tile shape, timed
// on the context's stream from its current field state; the state (fields,
// CPML memories, Drude current, step clock, non-finite flag) is restored
// afterwards.
pic_status tune_fields(pic_ctx *c, int reps, double *ms)
{
    GradScratch g;
    g.s = c->stream;
    char *ck = nullptr;
    TRY(galloc(c, g, &ck, state_bytes(c)));
    Mirror m{};
    TRY(ckpt_save(c, ck, m));
    int nan0 = 0;
    HIP_TRY(c, hipMemcpyAsync(&nan0, c->d_nan, 4, hipMemcpyDeviceToHost, c->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(c, hipEventCreate(&e0));
    hipError_t er = hipEventCreate(&e1);
    if (er != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, PIC_EDEVICE, "hipEventCreate failed: %s", hipGetErrorString(er));
    }
    pic_status st = PIC_OK;
    for (int v = 0; v < pic::N_TILE_SHAPES && st == PIC_OK; ++v) {
        pic::FieldArgs f = c->fa;
        f.tile = v;
        f.gx = (c->n[0] + pic::TILE_FX[v] - 1) / pic::TILE_FX[v];
        f.gy = (c->n[1] + pic::TILE_FY[v] - 1) / pic::TILE_FY[v];
        pic::launch_h_update(f, c->stream);
        pic::launch_e_update(f, c->stream);
        (void)hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps; ++r) {
            pic::launch_h_update(f, c->stream);
            pic::launch_e_update(f, c->stream);
        }
        (void)hipEventRecord(e1, c->stream);
        hipError_t e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) st = fail(c, PIC_EDEVICE, "timing a tile shape failed: %s", hipGetErrorString(e));
        ms[v] = (double)t / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TRY(st);
    TRY(ckpt_load(c, ck, m));
    HIP_TRY(c, hipMemcpyAsync(c->d_nan, &nan0, 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

}  // namespace

extern "C" {

pic_status pic_grad(pic_ctx *c, double omega0, int64_t nsteps, int64_t ckpt_every, double *L,
                    double *dL_dwp, double *dL_dgamma)
{
    CHECK_CTX(c);
    if (nsteps < 1) return fail(c, PIC_EINVAL, "nsteps must be >= 1");
    if (ckpt_every < 0) return fail(c, PIC_EINVAL, "ckpt_every must be >= 0");
    if (!L) return fail(c, PIC_EINVAL, "L is NULL");
    if (!std::isfinite(omega0)) return fail(c, PIC_EINVAL, "omega0 must be finite");
    if (c->nprobe < 1) return fail(c, PIC_EINVAL, "pic_grad needs at least one probe");
    long long K = ckpt_every > 0 ? (long long)ckpt_every : (long long)std::ceil(std::sqrt((double)nsteps));
    K = std::max(1LL, std::min<long long>(K, nsteps));
    // automatic interval: keep every step's metal-box snapshot (no replay)
    // when they fit in half the free device memory
    bool store_all = false;
    if (ckpt_every == 0) {
        size_t freeb = 0, totalb = 0;
        HIP_TRY(c, hipMemGetInfo(&freeb, &totalb));
        const double need = (double)nsteps * 6.0 * (double)c->nbox * 4.0;
        store_all = need <= 0.5 * (double)freeb;
    }
    return grad_impl(c, omega0, (long long)nsteps, K, store_all, L, dL_dwp, dL_dgamma);
}

// Field-kernel tile autotuner: time H + E launches of every tile shape on
// the context's own grid, from a saved field state that is restored
// afterwards, and keep the fastest.
pic_status pic_tune(pic_ctx *c, int32_t reps, int32_t force, pic_tune_out *out)
{
    CHECK_CTX(c);
    if (force < -1 || force >= pic::N_TILE_SHAPES)
        return fail(c, PIC_EINVAL, "force must be -1 or a tile shape index below %d", pic::N_TILE_SHAPES);
    if (force < 0 && reps < 1) return fail(c, PIC_EINVAL, "reps must be >= 1");
    pic_tune_out res{};
    res.nshapes = pic::N_TILE_SHAPES;
    if (force >= 0) {
        c->tile = force;
    } else {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        pic_status st = tune_fields(c, reps, res.ms);
        if (st != PIC_OK) return st;
        c->tile = pick_shape(res.ms);
    }
    build_args(c);
    res.tile = c->tile;
    res.fx = pic::TILE_FX[c->tile];
    res.fy = pic::TILE_FY[c->tile];
    res.order = pic::TILE_ZO[c->tile];
    if (out) *out = res;
    return PIC_OK;
}

pic_status pic_read_fields(pic_ctx *c, int which, double *out)
{
    CHECK_CTX(c);
    if (!out) return fail(c, PIC_EINVAL, "host_out is NULL");
    const size_t N = (size_t)c->n[0] * c->n[1] * c->n[2];
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<float> tmp(N);
    for (int d = 0; d < 3; ++d) {
        double *dst = out + d * N;
        if (which == PIC_FIELD_E || which == PIC_FIELD_H || which == PIC_FIELD_JB) {
            const float *src = which == PIC_FIELD_E ? c->E[d] : which == PIC_FIELD_H ? c->H[c->hcur][d] : c->Jb[d];
            const double sc = which == PIC_FIELD_H ? 1.0 / kEta0 : which == PIC_FIELD_JB ? kEps0 / c->dt : 1.0;
            if (!src) {
                for (size_t q = 0; q < N; ++q) dst[q] = 0.0;
                continue;
            }
            HIP_TRY(c, hipMemcpy(tmp.data(), src, N * 4, hipMemcpyDeviceToHost));
            for (size_t q = 0; q < N; ++q) dst[q] = tmp[q] * sc;
        } else if (which == PIC_FIELD_JPOL) {
            for (size_t q = 0; q < N; ++q) dst[q] = 0.0;
            if (!c->has_metal) continue;
            const int wx = c->mhi[0] - c->mlo[0], wy = c->mhi[1] - c->mlo[1], wz = c->mhi[2] - c->mlo[2];
            std::vector<float> box((size_t)wx * wy * wz);
            HIP_TRY(c, hipMemcpy(box.data(), c->Jp[d], box.size() * 4, hipMemcpyDeviceToHost));
            const double sc = kEps0 / c->dt;
            for (int k = 0; k < wz; ++k)
                for (int j = 0; j < wy; ++j)
                    for (int i = 0; i < wx; ++i)
                        dst[(size_t)(i + c->mlo[0]) + (size_t)c->n[0] * ((size_t)(j + c->mlo[1]) + (size_t)c->n[1] * (k + c->mlo[2]))] =
                            box[(size_t)i + (size_t)wx * ((size_t)j + (size_t)wy * k)] * sc;
        } else {
            return fail(c, PIC_EINVAL, "unknown field %d", which);
        }
    }
    return PIC_OK;
}

pic_status pic_read_particles(pic_ctx *c, double *out)
{
    CHECK_CTX(c);
    if (c->np == 0) return PIC_OK;
    if (!out) return fail(c, PIC_EINVAL, "host_out is NULL");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const size_t n = (size_t)c->np;
    std::vector<float> tmp(6 * n);
    std::vector<int> ids(n);
    for (int q = 0; q < 6; ++q)
        HIP_TRY(c, hipMemcpy(tmp.data() + q * n, c->P[c->pcur][q], n * 4, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(ids.data(), c->pid[c->pcur], n * 4, hipMemcpyDeviceToHost));
    for (size_t p = 0; p < n; ++p) {
        const int id = ids[p];
        if (id < 0 || (size_t)id >= n) return fail(c, PIC_EDEVICE, "particle id table corrupted");
        const bool dead = !(tmp[p] >= 0.f && tmp[n + p] >= 0.f && tmp[2 * n + p] >= 0.f &&
                            tmp[p] < (float)c->n[0] && tmp[n + p] < (float)c->n[1] &&
                            tmp[2 * n + p] < (float)c->n[2]);
        for (int q = 0; q < 6; ++q) {
            const double sc = q < 3 ? c->dx : kC;
            out[q * n + id] = (dead && q < 3) ? NAN : tmp[q * n + p] * sc;
        }
    }
    return PIC_OK;
}

pic_status pic_diag(pic_ctx *c, pic_diag_out *out)
{
    CHECK_CTX(c);
    if (!out) return fail(c, PIC_EINVAL, "out is NULL");
    HIP_TRY(c, hipMemsetAsync(c->acc, 0, 16 * 8, c->stream));
    pic::DiagArgs a = diag_args(c);
    if (c->diag && c->np > 0) {
        const size_t nodes = (size_t)(c->n[0] + 1) * (c->n[1] + 1) * (c->n[2] + 1);
        HIP_TRY(c, hipMemsetAsync(c->rho, 0, nodes * 8, c->stream));
        a.rho = c->rho;
        pic::launch_rho(a, c->stream);
        a.rho0 = c->rho0;
    }
    pic::launch_diag_reduce(a, c->stream);
    HIP_TRY(c, hipGetLastError());
    double acc[16];
    HIP_TRY(c, hipMemcpyAsync(acc, c->acc, sizeof acc, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::memset(out, 0, sizeof *out);
    out->field_energy = 0.5 * kEps0 * acc[0] * c->dx * c->dx * c->dx;
    const double cnt = acc[1];
    out->count = cnt;
    for (int d = 0; d < 3; ++d) {
        const double mean = cnt > 0 ? acc[2 + d] / cnt : 0.0;
        const double var = cnt > 0 ? acc[5 + d] / cnt - mean * mean : 0.0;
        out->mean[d] = mean * c->dx;
        out->rms[d] = (var > 0 ? std::sqrt(var) : 0.0) * c->dx;
        out->umean[d] = (cnt > 0 ? acc[8 + d] / cnt : 0.0) * kC;
    }
    out->gauss_max = acc[11];
    out->rho0_max = acc[12];
    out->checked_nodes = (int64_t)acc[13];
    return PIC_OK;
}

pic_status pic_stats(pic_ctx *c, pic_stats_out *out)
{
    CHECK_CTX(c);
    if (!out) return fail(c, PIC_EINVAL, "out is NULL");
    unsigned long long pushes = 0;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->n_wave_slots) {
        std::vector<unsigned long long> slots(c->n_wave_slots);
        HIP_TRY(c, hipMemcpy(slots.data(), c->d_pushes, 8 * slots.size(), hipMemcpyDeviceToHost));
        for (unsigned long long v : slots) pushes += v;
    }
    out->steps = c->step;
    out->pushes = (int64_t)pushes;
    out->hcur = c->hcur;
    out->live = 0;
    for (int d = 0; d < 3; ++d) {
        out->pbox[d] = 0;
        out->pbox[3 + d] = -1;
    }
    if (c->np > 0) {
        HIP_TRY(c, hipMemcpy(out->pbox, c->box, sizeof out->pbox, hipMemcpyDeviceToHost));
        pic_diag_out d;
        pic_status st = pic_diag(c, &d);
        if (st != PIC_OK) return st;
        out->live = (int64_t)d.count;
    }
    return PIC_OK;
}

pic_status pic_timing(pic_ctx *c, double *ms_total, int64_t *launches, int reset)
{
    CHECK_CTX(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int f = 0; f < kFamilies; ++f) {
        double tot = 0.0;
        for (auto &e : c->ev[f]) {
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, e.first, e.second));
            tot += ms;
        }
        if (ms_total) ms_total[f] = tot;
        if (launches) launches[f] = (int64_t)c->ev[f].size();
        if (reset) {
            for (auto &e : c->ev[f]) {
                (void)hipEventDestroy(e.first);
                (void)hipEventDestroy(e.second);
            }
            c->ev[f].clear();
        }
    }
    return PIC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched simulations: one launch per kernel family for all members, and a
// whole sort period captured once as a HIP graph.
// ---------------------------------------------------------------------------
struct pic_batch {
    std::vector<pic_ctx *> ctx;
    hipStream_t stream = nullptr;  // the batch's own stream (capturable)
    hipStream_t ext = nullptr;     // the members' stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    pic::FieldArgs *d_fa = nullptr;
    pic::PartArgs *d_pa = nullptr;
    pic::ProbeArgs *d_pr = nullptr;
    int *d_tiles = nullptr, *d_pblocks = nullptr;
    int total_tiles = 0, total_pblocks = 0;
    int push_mode = 0;  // bit 0: per-lane atomics, bit 1: some member has a periodic x axis
    int sort_every = 0;
    int tile = 0;       // field-kernel tile shape shared by all members (pic_batch_tune)
    bool particles = false;
    bool use_graph = false;
    int graph_steps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

pic_status bfail(pic_batch *b, pic_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    else g_init_error = buf;
    return st;
}

#define BHIP(b, call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return bfail((b), PIC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

void batch_free(pic_batch *b)
{
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    void *ptrs[5] = {b->d_fa, b->d_pa, b->d_pr, b->d_tiles, b->d_pblocks};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
}

// The four batched launches of one step (sorts are issued separately).
void batch_launches(pic_batch *b)
{
    const int n = (int)b->ctx.size();
    pic::launch_h_update_batch(b->d_fa, b->d_tiles, n, b->total_tiles, b->tile, b->stream);
    if (b->particles)
        pic::launch_push_deposit_batch(b->d_pa, b->d_pblocks, n, b->total_pblocks, b->push_mode, b->stream);
    pic::launch_e_update_batch(b->d_fa, b->d_tiles, n, b->total_tiles, b->tile, b->stream);
    pic::launch_probe_batch(b->d_pr, n, b->stream);
}

void batch_mirror_step(pic_batch *b)
{
    for (pic_ctx *c : b->ctx) {
        c->hcur = 1 - c->hcur;
        c->step++;
        c->since_sort++;
    }
}

pic_status batch_sorts(pic_batch *b, bool only_due)
{
    for (pic_ctx *c : b->ctx) {
        if (c->np <= 0 || c->sort_every <= 0) continue;
        if (only_due && c->since_sort < c->sort_every) continue;
        pic::launch_sort(c->sa, c->scan_tmp, b->stream);
        c->pcur = 1 - c->pcur;
        c->since_sort = 0;
    }
    BHIP(b, hipGetLastError());
    return PIC_OK;
}

}  // namespace

extern "C" {

// Field argument blocks of every member for tile shape `shape`, and the
// prefix table of tiles per member.
pic_status batch_upload_fields(pic_batch *b, int shape)
{
    const int n = (int)b->ctx.size();
    std::vector<pic::FieldArgs> fa(n);
    std::vector<int> tiles(n + 1, 0);
    for (int q = 0; q < n; ++q) {
        const pic_ctx *c = b->ctx[q];
        fa[q] = c->fa;
        fa[q].tile = shape;
        fa[q].gx = (c->n[0] + pic::TILE_FX[shape] - 1) / pic::TILE_FX[shape];
        fa[q].gy = (c->n[1] + pic::TILE_FY[shape] - 1) / pic::TILE_FY[shape];
        tiles[q + 1] = tiles[q] + pic::field_tiles(c->n[0], c->n[1], c->n[2], shape);
    }
    BHIP(b, hipMemcpy(b->d_fa, fa.data(), sizeof(pic::FieldArgs) * n, hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->d_tiles, tiles.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
    b->tile = shape;
    b->total_tiles = tiles[n];
    return PIC_OK;
}

// Capture one sort period (sort_every steps, then the sorts; since_sort is 0
// at the start of every replay); fields-only batches capture 10 steps.
pic_status batch_capture(pic_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_steps = (b->particles && b->sort_every > 0) ? b->sort_every : 10;
    BHIP(b, hipStreamSynchronize(b->ext));
    BHIP(b, hipStreamSynchronize(b->stream));
    BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    for (int s2 = 0; s2 < b->graph_steps; ++s2) batch_launches(b);
    if (b->particles && b->sort_every > 0)
        for (pic_ctx *c : b->ctx)
            if (c->np > 0) pic::launch_sort(c->sa, c->scan_tmp, b->stream);
    hipError_t e = hipStreamEndCapture(b->stream, &b->graph);  // always leave capture mode
    if (e != hipSuccess) return bfail(b, PIC_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return PIC_OK;
}

static pic_status batch_create_impl(pic_batch *b, pic_ctx *const *ctxs, int32_t n, int32_t use_graph)
{
    std::vector<pic::PartArgs> pa(n);
    std::vector<pic::ProbeArgs> pr(n);
    std::vector<int> pblk(n + 1, 0);
    for (int q = 0; q < n; ++q) {
        pic_ctx *c = ctxs[q];
        if (!c || c->poisoned) return bfail(b, PIC_EINVAL, "context %d is NULL or poisoned", q);
        for (int r = 0; r < q; ++r)
            if (ctxs[r] == c) return bfail(b, PIC_EINVAL, "context %d appears twice", q);
        if (q > 0 && c->stream != ctxs[0]->stream)
            return bfail(b, PIC_EINVAL, "all contexts must share one stream");
        if (c->np > 0) {
            if (b->particles && (c->sort_every != b->sort_every || (b->push_mode & 1) != c->deposit_mode))
                return bfail(b, PIC_EINVAL, "contexts with particles must share sort_every and deposit_mode");
            b->particles = true;
            b->sort_every = c->sort_every;
            b->push_mode = (b->push_mode & 2) | c->deposit_mode;
            if (c->per[0]) b->push_mode |= 2;
        }
        b->ctx.push_back(c);
        pa[q] = c->pa;
        pr[q] = c->pr;
        pblk[q + 1] = pblk[q] + (c->np + pic::PBLOCK - 1) / pic::PBLOCK;
    }
    b->ext = ctxs[0]->stream;
    // an own stream: the members' stream may be the null stream, which cannot be captured
    BHIP(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    BHIP(b, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    BHIP(b, hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    b->total_pblocks = pblk[n];
    BHIP(b, hipMalloc(&b->d_fa, sizeof(pic::FieldArgs) * n));
    BHIP(b, hipMalloc(&b->d_pa, sizeof(pic::PartArgs) * n));
    BHIP(b, hipMalloc(&b->d_pr, sizeof(pic::ProbeArgs) * n));
    BHIP(b, hipMalloc(&b->d_tiles, sizeof(int) * (n + 1)));
    BHIP(b, hipMalloc(&b->d_pblocks, sizeof(int) * (n + 1)));
    pic_status st = batch_upload_fields(b, 0);
    if (st != PIC_OK) return st;
    BHIP(b, hipMemcpy(b->d_pa, pa.data(), sizeof(pic::PartArgs) * n, hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->d_pr, pr.data(), sizeof(pic::ProbeArgs) * n, hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->d_pblocks, pblk.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
    b->use_graph = use_graph != 0;
    if (b->use_graph) return batch_capture(b);
    return PIC_OK;
}

pic_status pic_batch_create(pic_batch **out, pic_ctx *const *ctxs, int32_t n, int32_t use_graph)
{
    if (!out) return bfail(nullptr, PIC_EINVAL, "batch is NULL");
    *out = nullptr;
    if (!ctxs || n < 1 || n > 64) return bfail(nullptr, PIC_EINVAL, "need 1..64 contexts");
    pic_batch *b = new (std::nothrow) pic_batch();
    if (!b) return bfail(nullptr, PIC_ENOMEM, "out of host memory");
    pic_status st = batch_create_impl(b, ctxs, n, use_graph);
    if (st != PIC_OK) {
        g_init_error = b->err;
        batch_free(b);
        delete b;
        return st;
    }
    *out = b;
    return PIC_OK;
}

pic_status pic_batch_step(pic_batch *b, int64_t nsteps)
{
    if (!b) return bfail(nullptr, PIC_EINVAL, "batch is NULL");
    if (nsteps < 0) return bfail(b, PIC_EINVAL, "nsteps must be >= 0");
    for (pic_ctx *c : b->ctx)
        if (c->poisoned) return bfail(b, PIC_ESTATE, "a member context is poisoned");
    // order the batch's stream after, and the members' stream behind, this work
    BHIP(b, hipEventRecord(b->ev_in, b->ext));
    BHIP(b, hipStreamWaitEvent(b->stream, b->ev_in, 0));
    while (nsteps > 0) {
        bool aligned = true;
        for (pic_ctx *c : b->ctx)
            aligned = aligned && (c->np == 0 || c->sort_every == 0 || c->since_sort == 0);
        if (b->use_graph && aligned && nsteps >= b->graph_steps) {
            BHIP(b, hipGraphLaunch(b->exec, b->stream));
            for (int s2 = 0; s2 < b->graph_steps; ++s2) batch_mirror_step(b);
            if (b->particles && b->sort_every > 0)
                for (pic_ctx *c : b->ctx)
                    if (c->np > 0) {
                        c->pcur = 1 - c->pcur;
                        c->since_sort = 0;
                    }
            nsteps -= b->graph_steps;
            continue;
        }
        pic_status st = batch_sorts(b, true);
        if (st != PIC_OK) return st;
        batch_launches(b);
        BHIP(b, hipGetLastError());
        batch_mirror_step(b);
        --nsteps;
    }
    BHIP(b, hipEventRecord(b->ev_out, b->stream));
    BHIP(b, hipStreamWaitEvent(b->ext, b->ev_out, 0));
    return PIC_OK;
}

pic_status pic_batch_tune(pic_batch *b, int32_t reps, int32_t force, pic_tune_out *out)
{
    if (!b) return bfail(nullptr, PIC_EINVAL, "batch is NULL");
    if (force < -1 || force >= pic::N_TILE_SHAPES)
        return bfail(b, PIC_EINVAL, "force must be -1 or a tile shape index below %d", pic::N_TILE_SHAPES);
    if (force < 0 && reps < 1) return bfail(b, PIC_EINVAL, "reps must be >= 1");
    for (pic_ctx *c : b->ctx)
        if (c->poisoned) return bfail(b, PIC_ESTATE, "a member context is poisoned");
    pic_tune_out res{};
    res.nshapes = pic::N_TILE_SHAPES;
    int best = force;
    if (force < 0) {
        BHIP(b, hipStreamSynchronize(b->ext));
        BHIP(b, hipStreamSynchronize(b->stream));
        // save every member's field state; the timed launches advance it
        std::vector<void *> saved;
        std::vector<Mirror> mir(b->ctx.size());
        pic_status st = PIC_OK;
        for (size_t q = 0; q < b->ctx.size() && st == PIC_OK; ++q) {
            void *p = nullptr;
            if (hipMalloc(&p, state_bytes(b->ctx[q])) != hipSuccess) {
                (void)hipGetLastError();
                st = bfail(b, PIC_ENOMEM, "no device memory to save member %zu", q);
                break;
            }
            saved.push_back(p);
            if (ckpt_save(b->ctx[q], (char *)p, mir[q]) != PIC_OK) st = bfail(b, PIC_EDEVICE, "saving member %zu failed", q);
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (st == PIC_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
            st = bfail(b, PIC_EDEVICE, "hipEventCreate failed");
        if (st == PIC_OK && hipStreamSynchronize(b->ext) != hipSuccess) st = bfail(b, PIC_EDEVICE, "sync failed");
        const int n = (int)b->ctx.size();
        for (int v = 0; v < pic::N_TILE_SHAPES && st == PIC_OK; ++v) {
            st = batch_upload_fields(b, v);
            if (st != PIC_OK) break;
            pic::launch_h_update_batch(b->d_fa, b->d_tiles, n, b->total_tiles, v, b->stream);
            pic::launch_e_update_batch(b->d_fa, b->d_tiles, n, b->total_tiles, v, b->stream);
            (void)hipEventRecord(e0, b->stream);
            for (int r = 0; r < reps; ++r) {
                pic::launch_h_update_batch(b->d_fa, b->d_tiles, n, b->total_tiles, v, b->stream);
                pic::launch_e_update_batch(b->d_fa, b->d_tiles, n, b->total_tiles, v, b->stream);
            }
            (void)hipEventRecord(e1, b->stream);
            float t = 0.f;
            hipError_t e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) st = bfail(b, PIC_EDEVICE, "timing a tile shape failed: %s", hipGetErrorString(e));
            res.ms[v] = (double)t / reps;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (size_t q = 0; q < saved.size(); ++q) {
            if (ckpt_load(b->ctx[q], (char *)saved[q], mir[q]) != PIC_OK && st == PIC_OK)
                st = bfail(b, PIC_EDEVICE, "restoring member %zu failed", q);
        }
        (void)hipStreamSynchronize(b->ext);
        for (void *p : saved) (void)hipFree(p);
        if (st != PIC_OK) return st;
        best = pick_shape(res.ms);
    }
    pic_status st = batch_upload_fields(b, best);
    if (st != PIC_OK) return st;
    if (b->use_graph) {
        st = batch_capture(b);
        if (st != PIC_OK) return st;
    }
    res.tile = best;
    res.fx = pic::TILE_FX[best];
    res.fy = pic::TILE_FY[best];
    res.order = pic::TILE_ZO[best];
    if (out) *out = res;
    return PIC_OK;
}

void pic_batch_destroy(pic_batch *b)
{
    if (!b) return;
    batch_free(b);
    delete b;
}

const char *pic_batch_last_error(const pic_batch *b)
{
    if (!b) return g_init_error.c_str();
    return b->err.c_str();
}

}  // extern "C"
