// Host side of batched simulations (pic_batch_*): one launch per kernel
// family for all members, and a whole sort period captured once as a HIP
// graph.
#include "pic_host.hpp"

#include <climits>

using namespace pich;

struct pic_batch {
    std::vector<pic_ctx *> ctx;
    hipStream_t stream = nullptr;  // the batch's own stream (capturable)
    hipStream_t ext = nullptr;     // the members' stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    pic::FieldArgs *d_fa = nullptr;
    pic::PartArgs *d_pa = nullptr;
    pic::ProbeArgs *d_pr = nullptr;
    int *d_tiles = nullptr, *d_pblocks = nullptr;  // per work unit: member << 24 | its own unit
    pic::SortArgs *d_sa = nullptr;                 // the sort arguments of the members with particles
    int *d_sblocks = nullptr;                      // their sort workgroups (index into d_sa << 24 | unit)
    int n_sorted = 0, total_sblocks = 0;
    size_t tiles_cap = 0;                          // entries d_tiles holds (the largest tile shape's count)
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
    else pich::init_error() = buf;
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
    void *ptrs[7] = {b->d_fa, b->d_pa, b->d_pr, b->d_tiles, b->d_pblocks, b->d_sa, b->d_sblocks};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
}

// The four batched launches of one step (sorts are issued separately).
void batch_launches(pic_batch *b)
{
    const int n = (int)b->ctx.size();
    pic::launch_h_update_batch(b->d_fa, b->d_tiles, b->total_tiles, b->tile, b->stream);
    if (b->particles)
        pic::launch_push_deposit_batch(b->d_pa, b->d_pblocks, b->total_pblocks, b->push_mode, b->stream);
    pic::launch_e_update_batch(b->d_fa, b->d_tiles, b->total_tiles, b->tile, b->stream);
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

// Work-unit table of a batched launch: counts[q] units of member q, in member
// order; entry = q << 24 | the unit's index within member q.
std::vector<int> unit_table(const std::vector<long long> &counts)
{
    std::vector<int> t;
    for (size_t q = 0; q < counts.size(); ++q)
        for (long long u = 0; u < counts[q]; ++u) t.push_back((int)(q << 24) | (int)u);
    return t;
}

// Field argument blocks of every member for tile shape `shape`, and the
// field launches' work-unit table (re-made when the tuner changes the shape).
pic_status batch_upload_fields(pic_batch *b, int shape)
{
    const int n = (int)b->ctx.size();
    std::vector<pic::FieldArgs> fa(n);
    std::vector<long long> tiles(n);
    for (int q = 0; q < n; ++q) {
        const pic_ctx *c = b->ctx[q];
        fa[q] = c->fa;
        fa[q].tile = shape;
        fa[q].gx = (c->n[0] + pic::TILE_FX[shape] - 1) / pic::TILE_FX[shape];
        fa[q].gy = (c->n[1] + pic::TILE_FY[shape] - 1) / pic::TILE_FY[shape];
        tiles[q] = pic::batch_field_units(c->n[0], c->n[1], c->n[2], shape);
        if (tiles[q] >= (1LL << 24)) return bfail(b, PIC_EINVAL, "member %d has too many field tiles for a batch", q);
    }
    const std::vector<int> tab = unit_table(tiles);
    if (tab.size() > b->tiles_cap) return bfail(b, PIC_EINVAL, "field tile table larger than allocated");
    BHIP(b, hipMemcpy(b->d_fa, fa.data(), sizeof(pic::FieldArgs) * n, hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->d_tiles, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice));
    b->tile = shape;
    b->total_tiles = (int)tab.size();
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
    // every member with particles is due at the end of the period: all their
    // sorts in one launch per kernel
    if (b->particles && b->sort_every > 0)
        pic::launch_sort_batch(b->d_sa, b->d_sblocks, b->total_sblocks, b->n_sorted, b->stream);
    hipError_t e = hipStreamEndCapture(b->stream, &b->graph);  // always leave capture mode
    if (e != hipSuccess) return bfail(b, PIC_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return PIC_OK;
}

}  // namespace

extern "C" {

static pic_status batch_create_impl(pic_batch *b, pic_ctx *const *ctxs, int32_t n, int32_t use_graph)
{
    std::vector<pic::PartArgs> pa(n);
    std::vector<pic::ProbeArgs> pr(n);
    std::vector<long long> pblk(n, 0);
    std::vector<pic::SortArgs> sa;
    std::vector<long long> sblk;
    for (int q = 0; q < n; ++q) {
        pic_ctx *c = ctxs[q];
        if (!c || c->poisoned) return bfail(b, PIC_EINVAL, "context %d is NULL or poisoned", q);
        for (int r = 0; r < q; ++r)
            if (ctxs[r] == c) return bfail(b, PIC_EINVAL, "context %d appears twice", q);
        if (q > 0 && c->stream != ctxs[0]->stream)
            return bfail(b, PIC_EINVAL, "all contexts must share one stream");
        if (c->np > 0) {
            if (c->deposit_mode == 2)
                return bfail(b, PIC_ENOTSUP, "context %d uses the fixed-point deposit, which batches do not run", q);
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
        pblk[q] = ((long long)c->np + pic::PUSH_BLOCK - 1) / pic::PUSH_BLOCK;
        if (c->np > 0) {
            sa.push_back(c->sa);
            sblk.push_back(((long long)c->np + pic::PBLOCK - 1) / pic::PBLOCK);
        }
    }
    long long total_pb = 0;
    for (long long v : pblk) total_pb += v;
    if (total_pb > INT_MAX) return bfail(b, PIC_EINVAL, "too many particles in the batch for one launch");
    const std::vector<int> ptab = unit_table(pblk);
    long long total_sb = 0;
    for (long long v : sblk) total_sb += v;
    if (total_sb > INT_MAX) return bfail(b, PIC_EINVAL, "too many particles in the batch for one launch");
    const std::vector<int> stab = unit_table(sblk);
    b->ext = ctxs[0]->stream;
    // an own stream: the members' stream may be the null stream, which cannot be captured
    BHIP(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    BHIP(b, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
    BHIP(b, hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    b->total_pblocks = (int)ptab.size();
    BHIP(b, hipMalloc(&b->d_fa, sizeof(pic::FieldArgs) * n));
    BHIP(b, hipMalloc(&b->d_pa, sizeof(pic::PartArgs) * n));
    BHIP(b, hipMalloc(&b->d_pr, sizeof(pic::ProbeArgs) * n));
    BHIP(b, hipMalloc(&b->d_pblocks, sizeof(int) * std::max<size_t>(ptab.size(), 1)));
    b->n_sorted = (int)sa.size();
    b->total_sblocks = (int)stab.size();
    BHIP(b, hipMalloc(&b->d_sa, sizeof(pic::SortArgs) * std::max<size_t>(sa.size(), 1)));
    BHIP(b, hipMalloc(&b->d_sblocks, sizeof(int) * std::max<size_t>(stab.size(), 1)));
    // the field tile table for the shape with the most tiles, so the tuner
    // rewrites it in place
    for (int v = 0; v < pic::N_TILE_SHAPES; ++v) {
        long long t = 0;
        for (pic_ctx *c : b->ctx) t += pic::batch_field_units(c->n[0], c->n[1], c->n[2], v);
        if (t > INT_MAX) return bfail(b, PIC_EINVAL, "too many field tiles in the batch for one launch");
        b->tiles_cap = std::max(b->tiles_cap, (size_t)t);
    }
    BHIP(b, hipMalloc(&b->d_tiles, sizeof(int) * std::max<size_t>(b->tiles_cap, 1)));
    pic_status st = batch_upload_fields(b, 0);
    if (st != PIC_OK) return st;
    BHIP(b, hipMemcpy(b->d_pa, pa.data(), sizeof(pic::PartArgs) * n, hipMemcpyHostToDevice));
    BHIP(b, hipMemcpy(b->d_pr, pr.data(), sizeof(pic::ProbeArgs) * n, hipMemcpyHostToDevice));
    if (!ptab.empty())
        BHIP(b, hipMemcpy(b->d_pblocks, ptab.data(), sizeof(int) * ptab.size(), hipMemcpyHostToDevice));
    if (!sa.empty()) {
        BHIP(b, hipMemcpy(b->d_sa, sa.data(), sizeof(pic::SortArgs) * sa.size(), hipMemcpyHostToDevice));
        BHIP(b, hipMemcpy(b->d_sblocks, stab.data(), sizeof(int) * stab.size(), hipMemcpyHostToDevice));
    }
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
        pich::init_error() = b->err;
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
        for (int v = 0; v < pic::N_TILE_SHAPES && st == PIC_OK; ++v) {
            st = batch_upload_fields(b, v);
            if (st != PIC_OK) break;
            pic::launch_h_update_batch(b->d_fa, b->d_tiles, b->total_tiles, v, b->stream);
            pic::launch_e_update_batch(b->d_fa, b->d_tiles, b->total_tiles, v, b->stream);
            (void)hipEventRecord(e0, b->stream);
            for (int r = 0; r < reps; ++r) {
                pic::launch_h_update_batch(b->d_fa, b->d_tiles, b->total_tiles, v, b->stream);
                pic::launch_e_update_batch(b->d_fa, b->d_tiles, b->total_tiles, v, b->stream);
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
    if (!b) return pich::init_error().c_str();
    return b->err.c_str();
}

}  // extern "C"

