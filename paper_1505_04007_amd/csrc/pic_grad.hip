// Host side of the gradient (pic_grad) and of the field-kernel tuner
// (pic_tune): field-state checkpoints, the recorded bunch current, the
// reverse pass over the adjoint kernels, and the timed choice of tile shape.
#include "pic_host.hpp"

#include <mutex>

using namespace pich;

namespace {

// Device scratch of pic_grad_noalloc: every buffer of that call is carved
// from this array instead of being allocated.  Each device the library runs
// on holds its own copy until the process ends; all calls on one device share
// it.  Host code never passes the array's name to a kernel or a copy (on the
// host it is only a stand-in for the symbol): it uses the device address
// bound per device below.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kMaxDevices] = {};

}  // namespace

namespace pich {

void bind_static_scratch(pic_ctx *c)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        c->sscratch_err = "pic_grad_noalloc: no usable current device at pic_init";
        return;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            c->sscratch_err = std::string("pic_grad_noalloc: hipGetSymbolAddress of the static scratch failed: ") +
                              hipGetErrorString(e);
            return;
        }
        g_scratch_addr[dev] = (char *)p;
    }
    c->sscratch = g_scratch_addr[dev];
}

size_t slab_cells(const pic_ctx *c, int a)
{
    const size_t N = (size_t)c->n[0] * c->n[1] * c->n[2];
    return (size_t)2 * c->npml * (N / (size_t)c->n[a]);
}

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

}  // namespace pich

namespace {

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
pic_status grad_impl(pic_ctx *c, GradScratch &g, double omega0, long long N, long long K, bool store_all,
                     double *L, double *dL_dwp, double *dL_dgamma)
{
    const size_t ncell = (size_t)c->n[0] * c->n[1] * c->n[2];
    const int npr = c->nprobe;
    const double dt = c->dt;
    if (store_all) K = N;
    const long long nseg = (N + K - 1) / K;
    const long long s0 = c->step;

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
            // this step's E update writes the snapshot as it reads E^n and J_pol
            if (c->has_metal) c->fa.snap = traj + (size_t)r * 6 * c->nbox;
            st = step_once(c);
            c->fa.snap = nullptr;
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
            fr.snap = c->has_metal ? traj + (size_t)(r - a0) * 6 * c->nbox : nullptr;
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

// Device bytes grad_impl takes from its scratch in store-all mode: every
// galloc of that path (snapshots, probe record, seeds, adjoint state,
// gradient accumulators, the full-grid box), each rounded as galloc rounds.
size_t store_all_bytes(const pic_ctx *c, long long N)
{
    auto r = [](size_t b) { return align256(std::max<size_t>(b, 256)); };
    const size_t ncell = (size_t)c->n[0] * c->n[1] * c->n[2];
    const size_t npr = (size_t)c->nprobe;
    size_t t = r((size_t)N * 6 * c->nbox * 4) + r((size_t)N * npr * 8) + r((size_t)N * npr * 4);
    for (int d = 0; d < 3; ++d) {
        t += 2 * r(ncell * 4) + r(c->nbox * 4);
        if (c->pml[d].on) t += 8 * r(slab_cells(c, d) * 4);
    }
    t += 2 * r(c->nbox * 8);
    if (c->np > 0) t += r(6 * sizeof(int));
    return t;
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
    if (!store_all && c->np > 0 && c->deposit_mode == 2)
        return fail(c, PIC_ENOTSUP,
                    "pic_grad with checkpoints records the FP32 bunch current: not available with the "
                    "fixed-point deposit (deposit_mode 2); use ckpt_every = 0 with enough device memory");
    GradScratch g;
    g.s = c->stream;
    return grad_impl(c, g, omega0, (long long)nsteps, K, store_all, L, dL_dwp, dL_dgamma);
}

// pic_grad in its store-all form with every device buffer carved from the
// static scratch: no device memory is allocated or freed.
pic_status pic_grad_noalloc(pic_ctx *c, double omega0, int64_t nsteps, double *L, double *dL_dwp,
                            double *dL_dgamma)
{
    CHECK_CTX(c);
    if (nsteps < 1) return fail(c, PIC_EINVAL, "nsteps must be >= 1");
    if (!L) return fail(c, PIC_EINVAL, "L is NULL");
    if (!std::isfinite(omega0)) return fail(c, PIC_EINVAL, "omega0 must be finite");
    if (c->nprobe < 1) return fail(c, PIC_EINVAL, "pic_grad_noalloc needs at least one probe");
    if (!c->sscratch) return fail(c, PIC_EDEVICE, "%s", c->sscratch_err.c_str());
    if (nsteps > ((long long)1 << 40)) return fail(c, PIC_EINVAL, "nsteps = %lld is too large", (long long)nsteps);
    const size_t need = store_all_bytes(c, (long long)nsteps);
    if (need > kStaticScratchBytes)
        return fail(c, PIC_EINVAL,
                    "pic_grad_noalloc: %lld steps need %zu bytes of device scratch, more than the static "
                    "scratch's %zu (use pic_grad)",
                    (long long)nsteps, need, kStaticScratchBytes);
    GradScratch g;
    g.s = c->stream;
    g.fixed = c->sscratch;
    g.cap = kStaticScratchBytes;
    // per-launch timing creates HIP events; this path creates nothing
    const bool timing = c->timing;
    c->timing = false;
    const pic_status st = grad_impl(c, g, omega0, (long long)nsteps, (long long)nsteps, true, L, dL_dwp, dL_dgamma);
    c->timing = timing;
    return st;
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

}  // extern "C"
