// Host-side internals shared by the library's host sources (pic_abi.hip:
// context, init, stepping, read-back; pic_grad.hip: checkpoints, gradient,
// tuner; pic_batch.hip: batches).  Not part of the ABI: nothing here is
// exported from libpic.so.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pic.h"
#include "pic_internal.hpp"

namespace pich {

constexpr double kC = 299792458.0;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kEps0 = 1.0 / (kMu0 * kC * kC);
constexpr double kEta0 = kMu0 * kC;
constexpr int kFamilies = 6;  // h_update, push_deposit, e_update, probe, sort, field_sweep

}  // namespace pich

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
    int *runs = nullptr, *first = nullptr;  // the sort's per-key run counts and run starts
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
    // deposit_mode 2: the bunch current in fixed point (units per V/m and back)
    unsigned long long *Jq[3] = {nullptr, nullptr, nullptr};
    double qscale = 0.0, qinv = 0.0;
    size_t dev_bytes = 0;  // device memory allocated through dalloc at pic_init
    bool timed_now = false;  // the launch being issued has a start event

    long long step = 0;
    int tile = 0;  // field-kernel tile shape (pic_tune)
    int sort_every = 0, check_every = 0;
    long long since_sort = 0;

    bool timing = false;
    int timing_every = 1;  // time the launches of every this many steps (and every sort)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[pich::kFamilies];

    // one-pass field sweep: the E-side state (E, J_pol, E-side CPML
    // memories) in two blocks each, ecur the one holding the current values;
    // every pic_step call ends with ecur = 0, the blocks pic_init set up
    bool fused = false;
    size_t fs = 0;                              // component stride of the field blocks (floats)
    float *Eb[2] = {nullptr, nullptr};          // [3N]
    float *Jpb[2] = {nullptr, nullptr};         // [3 nbox]
    float *psiEb[3][2] = {};                    // per CPML axis [2 slab]
    size_t slab[3] = {0, 0, 0};                 // psi cells per component of an axis
    int ecur = 0;

    // this device's address of the library's static gradient scratch (bound at
    // pic_init), or null with the reason in sscratch_err
    char *sscratch = nullptr;
    std::string sscratch_err;
};

namespace pich {

// Record an error on the context (or, with c == NULL, as the init error);
// a device error or a non-finite field poisons the context.
pic_status fail(pic_ctx *c, pic_status st, const char *fmt, ...);

// This thread's message of the last failed pic_init / pic_batch_create.
std::string &init_error();

#define HIP_TRY(ctx, call)                                                                         \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return pich::fail((ctx), PIC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));        \
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
    c->dev_bytes += bytes;
    *p = (T *)q;
    return PIC_OK;
}

#define TRY(x)                                                                                     \
    do {                                                                                           \
        pic_status s_ = (x);                                                                       \
        if (s_ != PIC_OK) return s_;                                                               \
    } while (0)

#define CHECK_CTX(c)                                                                               \
    do {                                                                                           \
        if (!(c)) return pich::fail(nullptr, PIC_EINVAL, "ctx is NULL");                          \
        if ((c)->poisoned) return PIC_ESTATE;                                                      \
    } while (0)

// The step sequence (pic_abi.hip).
void build_args(pic_ctx *c);
void tstart(pic_ctx *c, int fam);
void tstop(pic_ctx *c, int fam);
pic_status do_sort(pic_ctx *c);
pic_status step_body(pic_ctx *c, const pic::BoxCopyArgs *rec);
pic_status step_once(pic_ctx *c);
pic::DiagArgs diag_args(pic_ctx *c);

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Field-state checkpoints (pic_grad.hip), used by the gradient and the tuners.
// Device memory of one pic_grad call, released on every exit path once the
// stream has drained.  With `fixed` set, the buffers are carved instead from
// that region of `cap` bytes (the static scratch of pic_grad_noalloc) and
// nothing is allocated or freed.
struct GradScratch {
    hipStream_t s = nullptr;
    std::vector<void *> p;
    char *fixed = nullptr;
    size_t cap = 0, used = 0;
    ~GradScratch()
    {
        if (p.empty() && used == 0) return;
        (void)hipStreamSynchronize(s);
        for (void *q : p) (void)hipFree(q);
    }
};

template <typename T>
pic_status galloc(pic_ctx *c, GradScratch &g, T **out, size_t count)
{
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
    if (g.fixed) {
        const size_t b = align256(bytes);
        if (b > g.cap - g.used)
            return fail(c, PIC_EINVAL, "pic_grad_noalloc: the %zu-byte static scratch is exhausted", g.cap);
        *out = (T *)(g.fixed + g.used);
        g.used += b;
        return PIC_OK;
    }
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

// Everything a fields-only step reads and writes: the state one checkpoint holds.
struct StateArr {
    void *p;
    size_t bytes;
};

struct Mirror {
    int hcur;
    long long step, since_sort;
};

size_t slab_cells(const pic_ctx *c, int a);
std::vector<StateArr> field_state(pic_ctx *c, int h);
size_t state_bytes(pic_ctx *c);
pic_status ckpt_save(pic_ctx *c, char *dst, Mirror &m);
pic_status ckpt_load(pic_ctx *c, const char *src, const Mirror &m);

// The tuners' choice among timed shapes (pic_grad.hip).
int pick_shape(const double *ms);

// Bind this device's address of the static gradient scratch to the context
// (pic_grad.hip; called by pic_init with the context's device current).  A
// failure is recorded in c->sscratch_err for pic_grad_noalloc to report.
void bind_static_scratch(pic_ctx *c);

}  // namespace pich
