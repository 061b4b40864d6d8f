// Host side of the gfx950 FDTD-PIC library: the C ABI declared in pic.h
// (context, init, stepping, probes, read-back, diagnostics, timing; the
// gradient and tuner are in pic_grad.hip, batches in pic_batch.hip).
//
// pic_init validates the problem, precomputes every coefficient in FP64
// (Drude ca/cb of Eq. 6 in increment form, CPML b/c/kappa, particle
// constants), rounds them once to FP32, uploads state, and sorts the
// particles by cell.  pic_step enqueues, per step, on one stream:
//   [sort every sort_every steps] -> H update -> push + deposit ->
//   Drude J + E update -> probe DFT
// and polls a device non-finite flag every check_every steps.
#include "pic_host.hpp"

namespace {

thread_local std::string g_init_error;

}  // namespace

namespace pich {

std::string &init_error() { return g_init_error; }

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

}  // namespace pich

using namespace pich;

namespace {

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

bool finite_nonneg(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!(std::isfinite(p[i]) && p[i] >= 0.0)) return false;
    return true;
}

}  // namespace

namespace pich {

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
        a.Jq[d] = c->Jq[d];
    }
    a.qinv = c->qinv;
    a.coef = c->coef;
    a.pbox = c->np > 0 ? c->box : nullptr;
    a.nan_flag = c->d_nan;
    a.st = c->dstate;

    pic::PartArgs &pa = c->pa;
    pa = pic::PartArgs{};
    pa.n = c->np;
    pa.nx = c->n[0];
    pa.ny = c->n[1];
    pa.nz = c->n[2];
    for (int d = 0; d < 3; ++d) {
        pa.per[d] = c->per[d];
        pa.E[d] = c->E[d];
        pa.B[d] = c->Havg[d];
        pa.Jb[d] = c->Jb[d];
        pa.Jq[d] = c->Jq[d];
    }
    pa.qscale = (float)c->qscale;
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
    sa.runs = c->runs;
    sa.first = c->first;
    sa.box = c->box;
    sa.boxpart = c->boxpart;
    sa.scan_tmp = c->scan_tmp;
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

// Launch timing (opts.timing): a pair of events around each launch of the
// sampled steps (every step, or every timing_every-th) and around every sort.
// A pair that cannot be created is skipped (that launch goes untimed) rather
// than recorded with invalid handles.
void tstart(pic_ctx *c, int fam)
{
    c->timed_now = false;
    if (!c->timing) return;
    if (fam != 4 && c->timing_every > 1 && c->step % c->timing_every != 0) return;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(a);
        return;
    }
    (void)hipEventRecord(a, c->stream);
    c->ev[fam].push_back({a, b});
    c->timed_now = true;
}

void tstop(pic_ctx *c, int fam)
{
    if (!c->timing || !c->timed_now) return;
    (void)hipEventRecord(c->ev[fam].back().second, c->stream);
    c->timed_now = false;
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

// ---- one-pass field sweep ----

// Point the context's E-side arrays at block e and rebuild the argument blocks.
static void set_e_side(pic_ctx *c, int e)
{
    c->ecur = e;
    for (int d = 0; d < 3; ++d) {
        c->E[d] = c->Eb[e] + d * c->fs;
        if (c->Jpb[e]) c->Jp[d] = c->Jpb[e] + d * c->nbox;
    }
    for (int a = 0; a < 3; ++a)
        if (c->psiEb[a][e])
            for (int q = 0; q < 2; ++q) c->pml[a].psiE[q] = c->psiEb[a][e] + q * c->slab[a];
    build_args(c);
}

static pic::FusedArgs fused_args(const pic_ctx *c)
{
    pic::FusedArgs a{};
    a.nx = c->n[0];
    a.ny = c->n[1];
    a.nz = c->n[2];
    a.S = (float)c->S;
    a.N = (int)c->fs;
    const int e = c->ecur;
    a.Ein = c->Eb[e];
    a.Eout = c->Eb[e ^ 1];
    a.Hin = c->H[c->hcur ^ 1][0];  // H^{n+1/2}, from this step's H update
    a.Hout = c->H[c->hcur][0];     // over H^{n-1/2}
    a.Havg = c->np > 0 ? c->Havg[0] : nullptr;
    for (int d = 0; d < 3; ++d) {
        a.per[d] = c->per[d];
        a.pon[d] = c->pml[d].on;
        a.npml[d] = c->pml[d].npml;
        a.tab[d] = c->pml[d].bE;  // bE cE kE bH cH kH, n apart
        a.slab[d] = (int)c->slab[d];
        a.psiEin[d] = c->psiEb[d][e];
        a.psiEout[d] = c->psiEb[d][e ^ 1];
        a.psiH[d] = c->pml[d].psiH[0];
        a.mlo[d] = c->has_metal ? c->mlo[d] : 0;
        a.mhi[d] = c->has_metal ? c->mhi[d] : 0;
    }
    a.nbox = (int)c->nbox;
    a.Jpin = c->Jpb[e];
    a.Jpout = c->Jpb[e ^ 1];
    a.coef = c->coef;
    a.Jb = c->np > 0 ? c->Jb[0] : nullptr;
    a.pbox = c->np > 0 ? c->box : nullptr;
    a.nan_flag = c->d_nan;
    a.st = c->dstate;
    a.gy = (c->n[1] + pic::FUSED_ROWS - 1) / pic::FUSED_ROWS;
    return a;
}

// A step whose H update the previous sweep (or the chain's start) made:
// the sort when due (not for the chain's first step, sorted before its H
// update), the push, then either the sweep (this step's E update and the
// next step's H update) or this step's E update alone, then the probes.
static pic_status chain_step(pic_ctx *c, bool sweep, bool first)
{
    if (!first && c->np > 0 && c->sort_every > 0 && c->since_sort >= c->sort_every) TRY(do_sort(c));
    if (c->np > 0) {
        tstart(c, 1);
        pic::launch_push_deposit(c->pa, c->deposit_mode, c->stream);
        tstop(c, 1);
    }
    if (sweep) {
        tstart(c, 5);
        pic::launch_fused(fused_args(c), c->stream);
        if (c->np > 0)
            pic::launch_jb_clear(c->Jb[0], (int)c->fs, c->n[0], c->n[1], c->n[2], c->per, c->box, (float)c->S,
                                 c->dstate, c->stream);
        tstop(c, 5);
        set_e_side(c, c->ecur ^ 1);  // the probes read the new E
    } else {
        tstart(c, 2);
        pic::launch_e_update(c->fa, c->stream);
        tstop(c, 2);
    }
    tstart(c, 3);
    pic::launch_probe(c->pr, c->stream);
    tstop(c, 3);
    c->hcur = 1 - c->hcur;
    c->step++;
    c->since_sort++;
    HIP_TRY(c, hipGetLastError());
    return PIC_OK;
}

// The non-finite poll of pic_step.
static pic_status poll_nan(pic_ctx *c)
{
    if (c->check_every > 0 && c->step % c->check_every == 0) {
        int flag = 0;
        HIP_TRY(c, hipMemcpyAsync(&flag, c->d_nan, 4, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (flag) return fail(c, PIC_EUNSTABLE, "non-finite field value detected by step %lld", c->step);
    }
    return PIC_OK;
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

}  // namespace pich

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

// Component stride of the field blocks the library allocates: the cell
// count plus 1 MiB + 256 B, so that a field's three components do not sit a
// power of two apart (on a grid of 2^k cells that maps them onto the same
// HBM channels and slows the streaming kernels by a few per cent).
constexpr size_t kFieldPad = 262208;
static size_t field_stride(size_t N) { return N + kFieldPad; }

// The component stride shared by the fields the caller gives: 0 when it gives
// none, -1 when a given field is not three equally spaced arrays (at least N
// apart) or two fields differ.
static long long given_stride(const pic_opts &o, size_t N)
{
    if (!o.bufs) return 0;
    long long st = 0;
    for (int f = 0; f < 3; ++f) {
        float *const *p = f == 0 ? o.bufs->E : o.bufs->H[f - 1];
        const int given = (p[0] != nullptr) + (p[1] != nullptr) + (p[2] != nullptr);
        if (given == 0) continue;
        if (given != 3) return -1;
        const long long s1 = p[1] - p[0], s2 = p[2] - p[1];
        if (s1 != s2 || s1 < (long long)N || (st && st != s1)) return -1;
        st = s1;
    }
    return st;
}

// The component stride of the library's own field blocks: the caller's, when
// it gives fields, so that the one-pass sweep can address them all alike.
static size_t block_stride(const pic_opts &o, size_t N)
{
    const long long g = given_stride(o, N);
    return g > 0 ? (size_t)g : field_stride(N);
}

// The one-pass field sweep (asked for with field_sweep = 1) needs a
// workgroup to span x, the FP32 bunch
// current, and each of E, H[0], H[1] as one block with components N apart
// (any the caller gives must already be laid out so).
static bool fused_eligible(const pic_grid &g, const pic_opts &o)
{
    if (o.field_sweep != 1 || o.deposit_mode == 2 || g.nx > 1024) return false;
    return given_stride(o, (size_t)g.nx * g.ny * g.nz) >= 0;
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
    bind_static_scratch(c);
    c->sort_every = o.sort_every > 0 ? o.sort_every : 0;
    c->check_every = o.check_every > 0 ? o.check_every : 0;
    if (o.timing < 0) return fail(c, PIC_EINVAL, "timing = %d must be >= 0", o.timing);
    c->timing = o.timing != 0;
    c->timing_every = o.timing > 1 ? o.timing : 1;
    c->diag = o.diag != 0;
    if (o.deposit_mode < 0 || o.deposit_mode > 2)
        return fail(c, PIC_EINVAL, "deposit_mode = %d is not 0, 1 or 2", o.deposit_mode);
    c->deposit_mode = o.deposit_mode;
    if (o.field_sweep < 0 || o.field_sweep > 1)
        return fail(c, PIC_EINVAL, "field_sweep = %d is not 0 or 1", o.field_sweep);
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
    // for the one-pass sweep each field the library allocates is one block,
    // its components c->fs apart (the sweep addresses them from one base);
    // otherwise every component is an allocation of its own
    const bool blocks = fused_eligible(g, o);
    c->fs = blocks ? block_stride(o, N) : N;
    {
        float *blk[3] = {nullptr, nullptr, nullptr};  // E, H[0], H[1]
        for (int f = 0; blocks && f < 3; ++f) {
            bool any = false;
            for (int d = 0; d < 3; ++d) {
                float *gv = o.bufs ? (f == 0 ? o.bufs->E[d] : o.bufs->H[f - 1][d]) : nullptr;
                any = any || gv;
            }
            if (!any) TRY(dalloc(c, &blk[f], 2 * c->fs + N));
        }
        for (int d = 0; d < 3; ++d) {
            float *gE = o.bufs ? o.bufs->E[d] : nullptr;
            float *gH0 = o.bufs ? o.bufs->H[0][d] : nullptr;
            float *gH1 = o.bufs ? o.bufs->H[1][d] : nullptr;
            if (gE) c->E[d] = gE;
            else if (blk[0]) c->E[d] = blk[0] + d * c->fs;
            else TRY(dalloc(c, &c->E[d], N));
            if (gH0) c->H[0][d] = gH0;
            else if (blk[1]) c->H[0][d] = blk[1] + d * c->fs;
            else TRY(dalloc(c, &c->H[0][d], N));
            if (gH1) c->H[1][d] = gH1;
            else if (blk[2]) c->H[1][d] = blk[2] + d * c->fs;
            else TRY(dalloc(c, &c->H[1][d], N));
            HIP_TRY(c, hipMemsetAsync(c->E[d], 0, N * 4, c->stream));
            HIP_TRY(c, hipMemsetAsync(c->H[0][d], 0, N * 4, c->stream));
            HIP_TRY(c, hipMemsetAsync(c->H[1][d], 0, N * 4, c->stream));
        }
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
        if (blocks) {
            float *jblk = nullptr;
            TRY(dalloc(c, &jblk, 3 * nb));
            HIP_TRY(c, hipMemsetAsync(jblk, 0, 3 * nb * 4, c->stream));
            for (int d = 0; d < 3; ++d) c->Jp[d] = jblk + d * nb;
        } else {
            for (int d = 0; d < 3; ++d) {
                TRY(dalloc(c, &c->Jp[d], nb));
                HIP_TRY(c, hipMemsetAsync(c->Jp[d], 0, nb * 4, c->stream));
            }
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
        if (blocks) {
            float *pe = nullptr, *ph = nullptr;
            TRY(dalloc(c, &pe, 2 * slab));
            TRY(dalloc(c, &ph, 2 * slab));
            HIP_TRY(c, hipMemsetAsync(pe, 0, 2 * slab * 4, c->stream));
            HIP_TRY(c, hipMemsetAsync(ph, 0, 2 * slab * 4, c->stream));
            for (int q = 0; q < 2; ++q) {
                P.psiE[q] = pe + q * slab;
                P.psiH[q] = ph + q * slab;
            }
        } else {
            for (int q = 0; q < 2; ++q) {
                TRY(dalloc(c, &P.psiE[q], slab));
                TRY(dalloc(c, &P.psiH[q], slab));
                HIP_TRY(c, hipMemsetAsync(P.psiE[q], 0, slab * 4, c->stream));
                HIP_TRY(c, hipMemsetAsync(P.psiH[q], 0, slab * 4, c->stream));
            }
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
        std::vector<std::vector<float>> cellpos(3, std::vector<float>((size_t)c->np));
        for (int q = 0; q < 3; ++q)
            for (int i = 0; i < c->np; ++i) {
                float v = (float)(src[q][i] / dx);
                // keep the FP32 cell coordinate inside [0, n) after rounding
                if (v >= (float)nn[q]) v = std::nextafter((float)nn[q], 0.f);
                cellpos[q][i] = v;
            }
        // load order: by cell, and by x inside a cell.  The device's sorts keep
        // the order of every cell whose particles stay contiguous, so under a
        // near-uniform drift the particles of a wavefront stay ordered by their
        // deposit windows (pic_read_particles returns the original order).
        std::vector<std::pair<uint64_t, int>> order((size_t)c->np);
        for (int i = 0; i < c->np; ++i) {
            const uint64_t cell = (uint64_t)std::min((int)cellpos[0][i], nn[0] - 1) +
                                  (uint64_t)nn[0] * ((uint64_t)std::min((int)cellpos[1][i], nn[1] - 1) +
                                                     (uint64_t)nn[1] * (uint64_t)std::min((int)cellpos[2][i], nn[2] - 1));
            uint32_t xb;
            std::memcpy(&xb, &cellpos[0][i], 4);  // x >= 0: the bits order like the values
            order[i] = {(cell << 32) | xb, i};
        }
        std::sort(order.begin(), order.end());
        std::vector<int> ids(c->np);
        for (int i = 0; i < c->np; ++i) ids[i] = order[i].second;
        for (int q = 0; q < 6; ++q) {
            stage.emplace_back((size_t)c->np);
            const double sc = 1.0 / kC;
            for (int i = 0; i < c->np; ++i)
                stage.back()[i] = q < 3 ? cellpos[q][ids[i]] : (float)(src[q][ids[i]] * sc);
            TRY(upload(c->P[0][q], stage.back().data(), (size_t)c->np * 4));
        }
        HIP_TRY(c, hipMemcpyAsync(c->pid[0], ids.data(), 4 * (size_t)c->np, hipMemcpyHostToDevice, c->stream));
        // one push counter per wavefront of the push launch
        c->n_wave_slots = ((size_t)c->np + 63) / 64;
        TRY(dalloc(c, &c->d_pushes, c->n_wave_slots));
        HIP_TRY(c, hipMemsetAsync(c->d_pushes, 0, 8 * c->n_wave_slots, c->stream));
        TRY(dalloc(c, &c->key, (size_t)c->np));
        TRY(dalloc(c, &c->rank, (size_t)c->np));
        TRY(dalloc(c, &c->counts, (size_t)ncell + 1));
        TRY(dalloc(c, &c->runs, (size_t)ncell + 1));
        TRY(dalloc(c, &c->first, (size_t)ncell + 1));
        // 0 at every key from here on: each sort clears the keys it used
        HIP_TRY(c, hipMemsetAsync(c->counts, 0, ((size_t)ncell + 1) * 4, c->stream));
        HIP_TRY(c, hipMemsetAsync(c->runs, 0, ((size_t)ncell + 1) * 4, c->stream));
        TRY(dalloc(c, &c->box, 6));
        TRY(dalloc(c, &c->boxpart, 6 * (((size_t)c->np + pic::PBLOCK - 1) / pic::PBLOCK)));
        c->scan_len = pic::scan_tmp_size(ncell + 1);
        TRY(dalloc(c, &c->scan_tmp, (size_t)c->scan_len));
        if (c->deposit_mode == 2) {
            // fixed point: 2^24 units per the largest current one particle can
            // put on an edge (|qd|), so a wavefront's sum fits in 31 bits and
            // 2^39 such contributions in an edge's 64-bit total
            const double unit = std::fabs((double)c->qd);
            c->qscale = (double)(float)(unit > 0.0 ? 16777216.0 / unit : 1.0);
            c->qinv = 1.0 / c->qscale;
        }
        for (int d = 0; d < 3; ++d) {
            if (c->deposit_mode == 2) {
                TRY(dalloc(c, &c->Jq[d], N));
                HIP_TRY(c, hipMemsetAsync(c->Jq[d], 0, N * 8, c->stream));
            }
        }
        if (blocks) {
            float *jb = nullptr, *hv = nullptr;
            TRY(dalloc(c, &jb, 2 * c->fs + N));
            HIP_TRY(c, hipMemsetAsync(jb, 0, (2 * c->fs + N) * 4, c->stream));
            TRY(dalloc(c, &hv, 2 * c->fs + N));
            HIP_TRY(c, hipMemsetAsync(hv, 0, (2 * c->fs + N) * 4, c->stream));
            for (int d = 0; d < 3; ++d) {
                c->Jb[d] = jb + d * c->fs;
                c->Havg[d] = hv + d * c->fs;
            }
        } else {
            for (int d = 0; d < 3; ++d) {
                if (c->deposit_mode != 2) {
                    TRY(dalloc(c, &c->Jb[d], N));
                    HIP_TRY(c, hipMemsetAsync(c->Jb[d], 0, N * 4, c->stream));
                }
                TRY(dalloc(c, &c->Havg[d], N));
                HIP_TRY(c, hipMemsetAsync(c->Havg[d], 0, N * 4, c->stream));
            }
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
    if (blocks) {
        // second blocks of the E-side state for the one-pass sweep
        c->fused = true;
        c->Eb[0] = c->E[0];
        TRY(dalloc(c, &c->Eb[1], 2 * c->fs + N));
        HIP_TRY(c, hipMemsetAsync(c->Eb[1], 0, (2 * c->fs + N) * 4, c->stream));
        if (c->has_metal) {
            c->Jpb[0] = c->Jp[0];
            TRY(dalloc(c, &c->Jpb[1], 3 * c->nbox));
            HIP_TRY(c, hipMemsetAsync(c->Jpb[1], 0, 3 * c->nbox * 4, c->stream));
        }
        for (int d = 0; d < 3; ++d) {
            if (!c->pml[d].on) continue;
            c->slab[d] = (size_t)2 * g.npml * (N / (size_t)nn[d]);
            c->psiEb[d][0] = c->pml[d].psiE[0];
            TRY(dalloc(c, &c->psiEb[d][1], 2 * c->slab[d]));
            HIP_TRY(c, hipMemsetAsync(c->psiEb[d][1], 0, 2 * c->slab[d] * 4, c->stream));
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

pic_status pic_query_sizes(const pic_grid *grid, int64_t nparticles, const pic_opts *opts,
                           pic_buffer_sizes *out)
{
    if (!grid || !out) return fail(nullptr, PIC_EINVAL, "pic_query_sizes: grid and out are required");
    const pic_grid &g = *grid;
    const long long n[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1) return fail(nullptr, PIC_EINVAL, "axis %d has %lld cells", d, n[d]);
        if (g.bc[d] == PIC_BC_CPML && (g.npml < 1 || 2LL * g.npml >= n[d]))
            return fail(nullptr, PIC_EINVAL, "npml = %d does not fit axis %d", g.npml, d);
    }
    const long long N = n[0] * n[1] * n[2];
    if (N > 0x7fffffffLL) return fail(nullptr, PIC_EINVAL, "grid of %lld cells exceeds 2^31-1", N);
    if (nparticles < 0 || nparticles > 0x7fffffffLL)
        return fail(nullptr, PIC_EINVAL, "nparticles = %lld out of range", (long long)nparticles);
    pic_opts o{};
    if (opts) o = *opts;
    if (o.nprobe < 0 || o.nfreq < 0 || o.series_len < 0)
        return fail(nullptr, PIC_EINVAL, "nprobe, nfreq and series_len must be >= 0");
    // what pic_init allocates, in its order (dalloc of at least one element each)
    auto bytes = [](long long count, long long size) { return (count > 0 ? count : 1) * size; };
    long long total = 0;
    const bool fused = fused_eligible(g, o);                 // field blocks (the sweep) or arrays
    const long long FS = (long long)block_stride(o, (size_t)N);
    for (int f = 0; f < 3; ++f) {                             // E, H ping-pong
        const int gf = o.bufs ? (f == 0 ? (o.bufs->E[0] != nullptr) + (o.bufs->E[1] != nullptr) +
                                              (o.bufs->E[2] != nullptr)
                                        : (o.bufs->H[f - 1][0] != nullptr) + (o.bufs->H[f - 1][1] != nullptr) +
                                              (o.bufs->H[f - 1][2] != nullptr))
                              : 0;
        total += gf == 0 && fused ? bytes(2 * FS + N, 4) : (3 - gf) * bytes(N, 4);
    }
    total += bytes(1, 4) + bytes(16, 8) + bytes(1, 4) + bytes(1, sizeof(pic::DevState));
    for (int d = 0; d < 3; ++d) {                             // CPML tables and memories
        if (g.bc[d] != PIC_BC_CPML) continue;
        total += bytes(6 * n[d], 4) + 4 * bytes(2LL * g.npml * (N / n[d]), 4);
    }
    if (o.nprobe > 0) {
        const long long nf = (long long)o.nprobe * o.nfreq;
        total += bytes(o.nprobe, 4) + bytes(o.nfreq, 8) + 2 * bytes(nf, 8);
        if (o.series_len > 0) total += bytes(o.series_len * o.nprobe, 4);
    }
    const long long np = nparticles;
    if (np > 0) {
        total += 2 * 6 * bytes(np, 4) + 2 * bytes(np, 4);    // particle state, ids
        total += bytes((np + 63) / 64, 8);                    // push counters
        total += 2 * bytes(np, 4);                            // sort keys, ranks
        total += 3 * bytes(N + 1, 4) + bytes(6, 4);           // cell counts, runs, run starts; box
        total += bytes(6 * ((np + pic::PBLOCK - 1) / pic::PBLOCK), 4);
        total += bytes(pic::scan_tmp_size(N + 1), 4);
        const long long fblk = fused ? bytes(2 * FS + N, 4) : 3 * bytes(N, 4);
        total += o.deposit_mode == 2 ? 3 * bytes(N, 8) : fblk;  // J_b (fixed point: 64-bit)
        total += fblk;                                          // time-centred H
        if (o.diag) total += 2 * bytes((n[0] + 1) * (n[1] + 1) * (n[2] + 1), 8);
    }
    if (fused) {                                              // the sweep's second E-side blocks
        total += bytes(2 * FS + N, 4);
        for (int d = 0; d < 3; ++d)
            if (g.bc[d] == PIC_BC_CPML) total += bytes(2 * 2LL * g.npml * (N / n[d]), 4);
    }
    out->field_elems = N;
    out->field_bytes = 4 * N;
    out->device_bytes = total;
    // (cbt, d) + J_pol, and the sweep's second J_pol block
    out->bytes_per_metal_box_cell = sizeof(float2) + (fused ? 6 : 3) * sizeof(float);
    return PIC_OK;
}

pic_status pic_step(pic_ctx *c, int64_t nsteps)
{
    CHECK_CTX(c);
    if (nsteps < 0) return fail(c, PIC_EINVAL, "nsteps must be >= 0");
    if (c->fused && nsteps >= 3) {
        // an even number of sweeps, so the E-side blocks end where they began;
        // the steps before them and the last E update use the separate kernels
        const int64_t sweeps = (nsteps - 1) & ~1LL;
        for (int64_t it = 0; it < nsteps - 1 - sweeps; ++it) {
            TRY(step_once(c));
            TRY(poll_nan(c));
        }
        if (c->np > 0 && c->sort_every > 0 && c->since_sort >= c->sort_every) TRY(do_sort(c));
        tstart(c, 0);
        pic::launch_h_update(c->fa, c->stream);
        tstop(c, 0);
        for (int64_t m = 0; m < sweeps; ++m) {
            TRY(chain_step(c, true, m == 0));
            TRY(poll_nan(c));
        }
        TRY(chain_step(c, false, false));
        return poll_nan(c);
    }
    for (int64_t it = 0; it < nsteps; ++it) {
        TRY(step_once(c));
        TRY(poll_nan(c));
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
            if (which == PIC_FIELD_JB && c->Jq[d]) {
                std::vector<long long> q(N);
                HIP_TRY(c, hipMemcpy(q.data(), c->Jq[d], N * 8, hipMemcpyDeviceToHost));
                for (size_t i = 0; i < N; ++i) dst[i] = (double)q[i] * c->qinv * sc;
                continue;
            }
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
    out->device_bytes = (int64_t)c->dev_bytes;
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
