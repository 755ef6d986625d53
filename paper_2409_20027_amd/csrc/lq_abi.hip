// lq_abi.hip -- host side: the plan (sizes, offsets, segment decomposition,
// device descriptor tables, workspace layout) and the C entry points of
// include/lqscan.h.  Solve calls only enqueue kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lq_kernels.hpp"
#include "lqscan.h"

using lqk::InstDesc;
using lqk::TILE;

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

// Automatic segment length: about 16 segments at short horizons, at most 16
// stages per segment at long ones.
int auto_seg_len(int T)
{
    int L = T / 16;
    if (L < 1) L = 1;
    if (L > 16) L = 16;
    return L;
}

}  // namespace

// Scratch of lq_solve_static: the scan buffers of an allocation-free solve.
// In host code `scratch` names a host-side stand-in, not device memory: only
// the address hipGetSymbolAddress returns for the current device is passed
// to kernels.
static __device__ __align__(256) unsigned char scratch[LQ_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// The current device's copy of `scratch`, looked up once per device.
bool static_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return false;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return false;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return true;
}

}  // namespace

struct lq_plan {
    int batch = 0, prec = 0, mode = 0, seg_len_req = 0;
    int device = 0;
    std::vector<InstDesc> h_inst;
    InstDesc *d_inst = nullptr;
    int32_t *d_seg_start = nullptr;
    int32_t *d_x_start = nullptr;
    int64_t *d_elem_start = nullptr;
    int64_t total_seg = 0, total_x = 0, total_elem = 0, total_stages = 0;
    int max_nseg = 0;
    int seg_len_used = 0;
    int nk = 1;   // contraction slices of (n_max + 1)-long products
    int aff_radix = 4;   // radix of the affine-map scan levels
    // workspace layout (bytes)
    size_t off_Xa = 0, off_Xb = 0, off_Ya = 0, off_Yb = 0, off_st = 0, off_gt = 0, ws_bytes = 0, el_bytes = 0;
    // per-lane path: every instance has n = sn <= SMALL_NMAX and m = sm
    bool small = false;
    int sn = 0, sm = 0;
    // a plan over several size classes delegates to one sub-plan per class
    // (descriptors with this plan's array offsets and instance indices); each
    // sub-plan's scan buffers start at sub_off[c] in the workspace
    std::vector<lq_plan *> subs;
    std::vector<size_t> sub_off;
    const lq_plan *owner = nullptr;   // plan holding the timing events (subs: the parent)
    // diagnostic phase timing (events created by lq_plan_set_timing)
    mutable uint32_t tmask = 0;
    mutable std::vector<hipEvent_t> ev;
    mutable std::vector<int> ev_phase;
    mutable size_t ev_used = 0;
};

// Records events around one phase if its bit is enabled; `fn` enqueues it.
template <class F>
static void timed(const lq_plan *q, int phase, hipStream_t st, F fn)
{
    const lq_plan *p = q->owner ? q->owner : q;
    const bool on = (p->tmask >> phase) & 1u;
    size_t slot = p->ev_used;
    if (on && 2 * (slot + 1) <= p->ev.size()) {
        (void)hipEventRecord(p->ev[2 * slot], st);
        fn();
        (void)hipEventRecord(p->ev[2 * slot + 1], st);
        p->ev_phase[slot] = phase;
        p->ev_used = slot + 1;
    } else {
        fn();
    }
}

static lq_status hip_ok(hipError_t e) { return e == hipSuccess ? LQ_OK : LQ_ERR_HIP; }

static lq_status launched()
{
    return hipGetLastError() == hipSuccess ? LQ_OK : LQ_ERR_HIP;
}

// Radix of the affine-map scan levels.  A level costs a fixed launch-and-load
// latency plus, per entry, up to r - 1 dependent tile products.  When the
// entries fit one wave per SIMD the level is latency-bound and radix 8 saves
// levels; with more entries than SIMDs the products and the tile traffic
// dominate and radix 4 does least work per level that still halves the levels
// of radix 2.  With entries stored as n1 x n1 blocks the two radices measure
// within noise of each other on both kinds of workload (T = 16384, L = 16,
// n = 12, 1025 entries: 18.4 us per rollout scan at radix 4, 18.7 at radix 8;
// 256 x 4096 stages: 9.23 ms per differentiated solve at radix 4, 9.42 at
// radix 8), and radix 2 is slower on both.
// LQSCAN_AFFINE_RADIX (2, 4, 8, 16 or 32) overrides the choice.
static int choose_affine_radix(int64_t entries, int device)
{
    if (const char *e = getenv("LQSCAN_AFFINE_RADIX")) {
        const int r = atoi(e);
        if (r == 2 || r == 4 || r == 8 || r == 16 || r == 32) return r;
    }
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) cus = 256;
    return entries <= 4 * (int64_t)cus ? 8 : 4;
}

// Affine-map scan over the plan's entries, from `in` with `o` as the other
// buffer (prefix when suffix = 0, suffix otherwise); returns the buffer that
// holds the result.
static double *affine_scan(const lq_plan *p, hipStream_t st, int suffix, double *in, double *o)
{
    // a small class with few entries: every level in one workgroup, in place
    if (p->small && p->max_nseg > 1 &&
        lqk::launch_small_affine_scan1(p->sn, p->aff_radix, p->total_x, st, p->d_inst, p->d_x_start, p->batch,
                                       p->max_nseg, suffix, in))
        return in;
    for (int64_t dd = 1; dd < p->max_nseg; dd *= p->aff_radix) {
        if (p->small)
            lqk::launch_small_affine_ks(p->sn, p->aff_radix, p->total_x, st, p->d_inst, p->d_x_start, p->batch, (int)dd,
                                        suffix, in, o);
        else
            lqk::launch_affine_ks(p->nk, p->prec, p->aff_radix, (unsigned)p->total_x, st, p->d_inst, p->d_x_start,
                                  p->batch, (int)dd, suffix, in, o);
        std::swap(in, o);
    }
    return in;
}

// Largest state dimension served by the per-lane kernels (lq_small.hip).
// LQSCAN_SMALL=0 sends every instance through the matrix-core tile kernels.
constexpr int SMALL_NMAX = 4;
static bool small_path_enabled()
{
    const char *e = getenv("LQSCAN_SMALL");
    return !(e && e[0] == '0' && e[1] == 0);
}

extern "C" {

const char *lq_version(void) { return "lqscan 0.1 (gfx950, fp64 tiles)"; }

static lq_status plan_build(int32_t batch, const int32_t *nx, const int32_t *nu, const int32_t *T,
                            int32_t precision, int32_t mode, int32_t seg_len, const int32_t *seg_lens,
                            lq_plan **out)
{
    if (!out || batch <= 0 || !nx || !nu || !T) return LQ_ERR_ARG;
    if (precision != LQ_FP64 && precision != LQ_MIXED) return LQ_ERR_ARG;
    if (mode != LQ_SCAN && mode != LQ_SEQUENTIAL) return LQ_ERR_ARG;
    if (seg_len < 0) return LQ_ERR_ARG;
    *out = nullptr;
    if (seg_lens)
        for (int i = 0; i < batch; ++i)
            if (seg_lens[i] < 0) return LQ_ERR_ARG;
    for (int i = 0; i < batch; ++i) {
        if (T[i] < 1 || nx[i] < 1 || nu[i] < 1) return LQ_ERR_ARG;
        if (nx[i] > 15 || nu[i] > lqk::MMAX) return LQ_ERR_UNSUPPORTED;
        // the status word (-code) | (k << 8) holds stages k <= T below 2^23
        if (T[i] >= lqk::TMAX_STATUS) return LQ_ERR_UNSUPPORTED;
        // the kernels address stage k of an instance's array with a 32-bit
        // element offset
        if (((int64_t)T[i] + 1) * nx[i] * nx[i] >= ((int64_t)1 << 31)) return LQ_ERR_UNSUPPORTED;
    }
    lq_plan *p = new (std::nothrow) lq_plan();
    if (!p) return LQ_ERR_ARG;
    p->batch = batch;
    p->prec = precision;
    p->mode = mode;
    p->seg_len_req = seg_len;
    (void)hipGetDevice(&p->device);
    p->h_inst.resize(batch);
    std::vector<int32_t> seg_start(batch + 1), x_start(batch + 1);
    std::vector<int64_t> elem_start(batch + 1);
    int64_t oA = 0, oB = 0, oR = 0, oc = 0, oQT = 0, on = 0, oS = 0, os = 0, oG = 0, og = 0;
    int64_t seg = 0, el = 0, stages = 0;
    int max_nseg = 0, lmax = 0, nmax = 0;
    for (int i = 0; i < batch; ++i) {
        InstDesc &d = p->h_inst[i];
        const int64_t n = nx[i], m = nu[i], t = T[i];
        d.n = (int)n;
        d.m = (int)m;
        d.T = (int)t;
        const int req = seg_lens ? seg_lens[i] : seg_len;
        d.L = (mode == LQ_SEQUENTIAL) ? (int)t : (req > 0 ? std::min<int>(req, (int)t) : auto_seg_len((int)t));
        d.nseg = (int)((t + d.L - 1) / d.L);
        d.seg0 = (int)seg;
        d.xbase = (int)(seg + i);
        d.orig = i;
        d.elem0 = el;
        d.oA = oA; d.oB = oB; d.oR = oR; d.oc = oc; d.oQT = oQT; d.on = on;
        d.oS = oS; d.os = os; d.oG = oG; d.og = og;
        seg_start[i] = (int32_t)seg;
        x_start[i] = (int32_t)(seg + i);
        elem_start[i] = el;
        seg += d.nseg;
        el += t + 1;
        stages += t;
        oA += t * n * n; oB += t * n * m; oR += t * m * m; oc += t * n;
        oQT += n * n; on += n;
        oS += (t + 1) * n * n; os += (t + 1) * n; oG += t * m * n; og += t * m;
        max_nseg = std::max(max_nseg, d.nseg);
        lmax = std::max(lmax, d.L);
        nmax = std::max(nmax, d.n);
    }
    if (seg > INT32_MAX / 2) {
        delete p;
        return LQ_ERR_UNSUPPORTED;
    }
    seg_start[batch] = (int32_t)seg;
    x_start[batch] = (int32_t)(seg + batch);
    elem_start[batch] = el;
    p->total_seg = seg;
    p->total_x = seg + batch;
    p->total_elem = el;
    p->total_stages = stages;
    p->max_nseg = max_nseg;
    p->seg_len_used = lmax;
    p->nk = (nmax + 1 + 3) / 4;
    p->aff_radix = choose_affine_radix(p->total_x, p->device);
    // workspace: value scan ping-pong (3 tiles / entry), affine scan ping-pong (1 tile / entry)
    size_t off = 0;
    p->off_Xa = off; off = align_up(off + (size_t)p->total_x * 3 * TILE * sizeof(double));
    p->off_Xb = off; off = align_up(off + (size_t)p->total_x * 3 * TILE * sizeof(double));
    p->off_Ya = off; off = align_up(off + (size_t)p->total_x * TILE * sizeof(double));
    p->off_Yb = off; off = align_up(off + (size_t)p->total_x * TILE * sizeof(double));
    p->off_st = off; off = align_up(off + (size_t)os * sizeof(double));     // adjoint s~
    p->off_gt = off; off = align_up(off + (size_t)og * sizeof(double));     // adjoint gamma~
    p->ws_bytes = off;
    p->el_bytes = align_up((size_t)el * 4 * TILE * sizeof(double));

    lq_status st = LQ_OK;
    if (hipMalloc(&p->d_inst, sizeof(InstDesc) * batch) != hipSuccess ||
        hipMalloc(&p->d_seg_start, sizeof(int32_t) * (batch + 1)) != hipSuccess ||
        hipMalloc(&p->d_x_start, sizeof(int32_t) * (batch + 1)) != hipSuccess ||
        hipMalloc(&p->d_elem_start, sizeof(int64_t) * (batch + 1)) != hipSuccess)
        st = LQ_ERR_HIP;
    if (st == LQ_OK)
        st = hip_ok(hipMemcpy(p->d_inst, p->h_inst.data(), sizeof(InstDesc) * batch, hipMemcpyHostToDevice));
    if (st == LQ_OK)
        st = hip_ok(hipMemcpy(p->d_seg_start, seg_start.data(), sizeof(int32_t) * (batch + 1), hipMemcpyHostToDevice));
    if (st == LQ_OK)
        st = hip_ok(hipMemcpy(p->d_x_start, x_start.data(), sizeof(int32_t) * (batch + 1), hipMemcpyHostToDevice));
    if (st == LQ_OK)
        st = hip_ok(hipMemcpy(p->d_elem_start, elem_start.data(), sizeof(int64_t) * (batch + 1), hipMemcpyHostToDevice));
    if (st != LQ_OK) {
        lq_plan_destroy(p);
        return st;
    }
    *out = p;
    return LQ_OK;
}

// A plan over the given instances; when they fall into several size classes
// (each (n, m) with n <= SMALL_NMAX served by the per-lane kernels, every
// larger n by the tile kernels) it delegates to one sub-plan per class, whose
// descriptors keep this plan's array offsets and instance indices, so the
// packed arrays, outputs and status words are shared.  Workspace of such a
// plan: each sub-plan's scan buffers in turn, then the adjoint's s~ and
// gamma~ vectors in this plan's packing.
static lq_status plan_create(int32_t batch, const int32_t *nx, const int32_t *nu, const int32_t *T,
                             int32_t precision, int32_t mode, int32_t seg_len, const int32_t *seg_lens,
                             lq_plan **out)
{
    const bool sm = small_path_enabled();
    auto key = [&](int i) { return (sm && nx[i] <= SMALL_NMAX) ? nx[i] * 8 + nu[i] : 0; };
    // Automatic segment length of a per-lane class with fewer than
    // SMALL_SHORT_STAGES stages in all: at most SMALL_SHORT_L stages per
    // segment.  Such a class fills few waves, each lane's sweep is a
    // dependent chain of a few microseconds per stage, and the extra scan
    // level costs less (n = 4, T = 1024 Newton loop: 0.38 ms per step at
    // L = 4 against 0.41 at L = 16).
    constexpr int64_t SMALL_SHORT_STAGES = 16384;
    constexpr int SMALL_SHORT_L = 4;
    std::vector<int32_t> auto_lens;
    if (seg_len <= 0 && !seg_lens && mode != LQ_SEQUENTIAL && batch > 0) {
        std::vector<std::pair<int, int64_t>> cls;   // (class key, stages)
        for (int i = 0; i < batch; ++i) {
            auto it = std::find_if(cls.begin(), cls.end(), [&](const auto &c) { return c.first == key(i); });
            if (it == cls.end()) cls.push_back({key(i), (int64_t)T[i]});
            else it->second += T[i];
        }
        bool any = false;
        auto_lens.resize(batch);
        for (int i = 0; i < batch; ++i) {
            int L = auto_seg_len(T[i]);
            const int k = key(i);
            const auto it = std::find_if(cls.begin(), cls.end(), [&](const auto &c) { return c.first == k; });
            if (k && it->second < SMALL_SHORT_STAGES && L > SMALL_SHORT_L) {
                L = SMALL_SHORT_L;
                any = true;
            }
            auto_lens[i] = L;
        }
        if (any) seg_lens = auto_lens.data();
    }
    lq_plan *p = nullptr;
    lq_status st = plan_build(batch, nx, nu, T, precision, mode, seg_len, seg_lens, &p);
    if (st != LQ_OK) return st;
    std::vector<int> keys;
    for (int i = 0; i < batch; ++i)
        if (std::find(keys.begin(), keys.end(), key(i)) == keys.end()) keys.push_back(key(i));
    if (keys.size() == 1) {
        if (keys[0]) {
            p->small = true;
            p->sn = nx[0];
            p->sm = nu[0];
        }
        *out = p;
        return LQ_OK;
    }
    size_t off = 0;
    for (int kc : keys) {
        std::vector<int32_t> idx, cn, cm, cT, cL;
        for (int i = 0; i < batch; ++i)
            if (key(i) == kc) {
                idx.push_back(i);
                cn.push_back(nx[i]);
                cm.push_back(nu[i]);
                cT.push_back(T[i]);
                cL.push_back(seg_lens ? seg_lens[i] : 0);
            }
        lq_plan *q = nullptr;
        st = plan_build((int32_t)idx.size(), cn.data(), cm.data(), cT.data(), precision, mode, seg_len,
                        seg_lens ? cL.data() : nullptr, &q);
        if (st != LQ_OK) {
            lq_plan_destroy(p);
            return st;
        }
        p->subs.push_back(q);
        q->owner = p;
        if (kc) {
            q->small = true;
            q->sn = cn[0];
            q->sm = cm[0];
        }
        for (size_t j = 0; j < idx.size(); ++j) {
            InstDesc &dq = q->h_inst[j];
            const InstDesc &dp = p->h_inst[idx[j]];
            dq.orig = dp.orig;
            dq.elem0 = dp.elem0;
            dq.oA = dp.oA; dq.oB = dp.oB; dq.oR = dp.oR; dq.oc = dp.oc; dq.oQT = dp.oQT; dq.on = dp.on;
            dq.oS = dp.oS; dq.os = dp.os; dq.oG = dp.oG; dq.og = dp.og;
        }
        if (hipMemcpy(q->d_inst, q->h_inst.data(), sizeof(InstDesc) * q->h_inst.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
            lq_plan_destroy(p);
            return LQ_ERR_HIP;
        }
        p->sub_off.push_back(off);
        off = align_up(off + q->off_st);
    }
    int64_t ns = 0, ng = 0;
    for (const InstDesc &d : p->h_inst) {
        ns += (int64_t)(d.T + 1) * d.n;
        ng += (int64_t)d.T * d.m;
    }
    p->off_Xa = p->off_Xb = p->off_Ya = p->off_Yb = 0;   // unused: the sub-plans hold the scan buffers
    p->off_st = off; off = align_up(off + (size_t)ns * sizeof(double));
    p->off_gt = off; off = align_up(off + (size_t)ng * sizeof(double));
    p->ws_bytes = off;
    *out = p;
    return LQ_OK;
}

// The plans that run a call's work: a mixed plan's size-class sub-plans, or
// the plan itself; class c's scan buffers start at class_ws(p, c).
static int nclass(const lq_plan *p) { return p->subs.empty() ? 1 : (int)p->subs.size(); }
static const lq_plan *class_plan(const lq_plan *p, int c) { return p->subs.empty() ? p : p->subs[c]; }
static size_t class_ws(const lq_plan *p, int c) { return p->subs.empty() ? 0 : p->sub_off[c]; }

lq_status lq_plan_create(int32_t batch, const int32_t *nx, const int32_t *nu, const int32_t *T,
                         int32_t precision, int32_t mode, int32_t seg_len, lq_plan **out)
{
    return plan_create(batch, nx, nu, T, precision, mode, seg_len, nullptr, out);
}

lq_status lq_plan_create_seg(int32_t batch, const int32_t *nx, const int32_t *nu, const int32_t *T,
                             int32_t precision, const int32_t *seg_len, lq_plan **out)
{
    if (!seg_len) return LQ_ERR_ARG;
    return plan_create(batch, nx, nu, T, precision, LQ_SCAN, 0, seg_len, out);
}

lq_status lq_plan_create_tuned(int32_t batch, const int32_t *nx, const int32_t *nu, const int32_t *T,
                               int32_t precision, const char *cache_path, lq_plan **out)
{
    if (!out || batch <= 0 || !nx || !nu || !T) return LQ_ERR_ARG;
    if (precision != LQ_FP64 && precision != LQ_MIXED) return LQ_ERR_ARG;
    std::string text;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "rb");
        if (!f) return LQ_ERR_ARG;
        char buf[4096];
        size_t k;
        while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
        std::fclose(f);
    }
    // the tuner's classes: (n, m, T rounded up to a power of two), sized by
    // how many instances of the batch fall into them (rounded up likewise)
    auto bucket = [](int64_t v) {
        int64_t b = 1;
        while (b < v) b <<= 1;
        return b;
    };
    std::vector<int64_t> tb(batch);
    for (int i = 0; i < batch; ++i) tb[i] = bucket(T[i] > 0 ? T[i] : 1);
    std::vector<int32_t> lens(batch, 0);
    for (int i = 0; i < batch && !text.empty(); ++i) {
        int64_t count = 0;
        for (int j = 0; j < batch; ++j) count += (nx[j] == nx[i] && nu[j] == nu[i] && tb[j] == tb[i]);
        char key[128];
        std::snprintf(key, sizeof key, "\"n%d_m%d_T%lld_B%lld_%s\"", nx[i], nu[i], (long long)tb[i],
                      (long long)bucket(count), precision == LQ_MIXED ? "mixed" : "fp64");
        const size_t at = text.find(key);
        if (at == std::string::npos) continue;   // class not tuned: automatic
        const size_t l = text.find("\"L\"", at);
        const size_t close = text.find('}', at);
        if (l == std::string::npos || l > close) return LQ_ERR_ARG;
        const size_t colon = text.find(':', l);
        if (colon == std::string::npos) return LQ_ERR_ARG;
        char *end = nullptr;
        const long L = std::strtol(text.c_str() + colon + 1, &end, 10);
        if (end == text.c_str() + colon + 1 || L < -1 || L > INT32_MAX) return LQ_ERR_ARG;
        lens[i] = (L < 0) ? T[i] : (int32_t)L;   // -1: the sequential recursion
    }
    return plan_create(batch, nx, nu, T, precision, LQ_SCAN, 0, lens.data(), out);
}

void lq_plan_destroy(lq_plan *p)
{
    if (!p) return;
    for (lq_plan *q : p->subs) lq_plan_destroy(q);
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    if (p->d_inst) (void)hipFree(p->d_inst);
    if (p->d_seg_start) (void)hipFree(p->d_seg_start);
    if (p->d_x_start) (void)hipFree(p->d_x_start);
    if (p->d_elem_start) (void)hipFree(p->d_elem_start);
    delete p;
}

size_t lq_plan_workspace_bytes(const lq_plan *p) { return p ? p->ws_bytes : 0; }
size_t lq_plan_elements_bytes(const lq_plan *p) { return p ? p->el_bytes : 0; }
int32_t lq_plan_seg_len(const lq_plan *p) { return p ? p->seg_len_used : 0; }
int64_t lq_plan_total_stages(const lq_plan *p) { return p ? p->total_stages : 0; }

static bool aligned(const void *p) { return ((uintptr_t)p & (ALIGN - 1)) == 0; }

static lqk::ProbPtrs probptrs(const lq_problem *q)
{
    lqk::ProbPtrs P;
    P.A = q->A; P.B = q->B; P.c = q->c; P.Q = q->Q; P.R = q->R; P.M = q->M;
    P.q = q->q; P.r = q->r; P.QT = q->QT; P.qT = q->qT; P.x0 = q->x0;
    return P;
}

static bool prob_ok(const lq_problem *q)
{
    return q && q->A && q->B && q->Q && q->R && q->QT && q->x0;
}

lq_status lq_build_elements(const lq_plan *p, const lq_problem *prob, double *elements, int32_t *status,
                            void *stream)
{
    if (!p || !prob_ok(prob)) return LQ_ERR_ARG;
    if (!elements || !aligned(elements)) return LQ_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    timed(p, LQ_PH_BUILD, st, [&] {
        lqk::launch_build_elements(p->prec, (unsigned)p->total_elem, st, probptrs(prob), p->d_inst, p->d_elem_start,
                                   p->batch, elements, status);
    });
    return launched();
}

// Value pass: fold, log-depth scan, Bellman sweep.  With Yroll the sweep also
// writes the rollout scan's entries (its segment fold fused in).
static void value_pass(const lq_plan *p, const lqk::ProbPtrs &P, const double *elements, const lqk::ValPtrs &V,
                       char *ws, double *Yroll, int32_t *status, hipStream_t st, double *ckpt = nullptr,
                       int stride = 1)
{
    double *Xa = (double *)(ws + p->off_Xa), *Xb = (double *)(ws + p->off_Xb);
    timed(p, LQ_PH_VALUE_FOLD, st, [&] {
        if (p->small && !elements)
            lqk::launch_small_value_fold(p->sn, p->sm, p->total_seg, st, P, p->d_inst, p->d_seg_start, p->batch, Xa,
                                         status);
        else
            lqk::launch_value_fold(p->nk, p->prec, (unsigned)p->total_seg, st, P, p->d_inst, p->d_seg_start, p->batch,
                                   elements, Xa, 0, status);
    });
    double *in = Xa, *o = Xb;
    // entries 1 .. nseg-1 of each instance (the last holds the terminal)
    if (p->max_nseg > 2)
        timed(p, LQ_PH_VALUE_SCAN, st, [&] {
            // a small class with few entries: every level in one workgroup
            if (p->small && lqk::launch_small_value_scan1(p->sn, p->total_x, st, p->d_inst, p->d_x_start, p->batch,
                                                          p->max_nseg, Xa, status))
                return;
            for (int dd = 1; dd < p->max_nseg - 1; dd *= 2) {
                if (p->small)
                    lqk::launch_small_value_ks(p->sn, p->total_x, st, p->d_inst, p->d_x_start, p->batch, dd, in, o,
                                               status);
                else
                    lqk::launch_value_ks(p->nk, p->prec, (unsigned)p->total_x, st, p->d_inst, p->d_x_start, p->batch,
                                         dd, 0, in, o, status);
                std::swap(in, o);
            }
        });
    double *fin = in;
    timed(p, LQ_PH_VALUE_BELLMAN, st, [&] {
        if (p->small)
            lqk::launch_small_value_riccati(p->sn, p->sm, p->total_seg, st, P, p->d_inst, p->d_seg_start, p->batch,
                                            fin, V, Yroll, ckpt, stride, status);
        else
            lqk::launch_value_riccati(p->nk, p->prec, (unsigned)p->total_seg, st, P, p->d_inst, p->d_seg_start,
                                      p->batch, fin, V, Yroll, ckpt, stride, status);
    });
}

// States, controls and co-states from the scanned segment-start states.
static void roll_apply(const lq_plan *p, const lqk::ProbPtrs &P, const lqk::ValPtrs &V, const double *fin, double *x,
                       double *u, double *lambda, hipStream_t st)
{
    timed(p, LQ_PH_ROLL_APPLY, st, [&] {
        if (p->small)
            lqk::launch_small_roll_apply(p->sn, p->sm, p->total_seg, st, P, V, p->d_inst, p->d_seg_start, p->batch,
                                         fin, x, u, lambda);
        else
            lqk::launch_roll_apply(p->nk, p->prec, (unsigned)p->total_seg, st, P, V, p->d_inst, p->d_seg_start,
                                   p->batch, fin, x, u, lambda);
    });
}

// Rollout from its scan entries in Ya (Yb: ping-pong): prefix scan, then states.
static void rollout_scan_apply(const lq_plan *p, const lqk::ProbPtrs &P, const lqk::ValPtrs &V, double *Ya, double *Yb,
                               double *x, double *u, double *lambda, hipStream_t st)
{
    double *fin = Ya;
    if (p->max_nseg > 1) timed(p, LQ_PH_ROLL_SCAN, st, [&] { fin = affine_scan(p, st, 0, Ya, Yb); });
    roll_apply(p, P, V, fin, x, u, lambda, st);
}

static bool value_ok(const lq_value *v) { return v && v->S && v->s && v->Gamma && v->gamma; }

lq_status lq_scan_solve(const lq_plan *p, const lq_problem *prob, const double *elements, const lq_value *out,
                        void *workspace, int32_t *status, void *stream)
{
    if (!p || !prob_ok(prob) || !value_ok(out)) return LQ_ERR_ARG;
    if (!workspace || !aligned(workspace)) return LQ_ERR_WORKSPACE;
    if (elements && !aligned(elements)) return LQ_ERR_WORKSPACE;
    lqk::ValPtrs V{out->S, out->s, out->Gamma, out->gamma};
    for (int c = 0; c < nclass(p); ++c)
        value_pass(class_plan(p, c), probptrs(prob), elements, V, (char *)workspace + class_ws(p, c), nullptr, status,
                   (hipStream_t)stream);
    return launched();
}

lq_status lq_rollout(const lq_plan *p, const lq_problem *prob, const lq_value *val, double *x, double *u,
                     double *lambda, void *workspace, int32_t *status, void *stream)
{
    (void)status;
    if (!p || !prob_ok(prob) || !value_ok(val) || !x || !u) return LQ_ERR_ARG;
    if (!workspace || !aligned(workspace)) return LQ_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const lqk::ProbPtrs P = probptrs(prob);
    lqk::ValPtrs V{val->S, val->s, val->Gamma, val->gamma};
    for (int c = 0; c < nclass(p); ++c) {
        const lq_plan *q = class_plan(p, c);
        char *ws = (char *)workspace + class_ws(p, c);
        double *Ya = (double *)(ws + q->off_Ya), *Yb = (double *)(ws + q->off_Yb);
        timed(q, LQ_PH_ROLL_FOLD, st, [&] {
            lqk::launch_roll_fold(q->nk, q->prec, (unsigned)q->total_seg, st, P, V, q->d_inst, q->d_seg_start, q->batch,
                                  Ya);
        });
        rollout_scan_apply(q, P, V, Ya, Yb, x, u, lambda, st);
    }
    return launched();
}

// Conditional-value states: fold of every segment but the last (the unit at
// entry 0), prefix scan, the segment-start states from the prefix elements and
// S~_k0, then the closed-loop sweep inside each segment.
lq_status lq_rollout_cv(const lq_plan *p, const lq_problem *prob, const lq_value *val, double *x, double *u,
                        double *lambda, void *workspace, int32_t *status, void *stream)
{
    if (!p || !prob_ok(prob) || !value_ok(val) || !x || !u) return LQ_ERR_ARG;
    if (!workspace || !aligned(workspace)) return LQ_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const lqk::ProbPtrs P = probptrs(prob);
    lqk::ValPtrs V{val->S, val->s, val->Gamma, val->gamma};
    for (int c = 0; c < nclass(p); ++c) {
        const lq_plan *q = class_plan(p, c);
        char *ws = (char *)workspace + class_ws(p, c);
        double *Xa = (double *)(ws + q->off_Xa), *Xb = (double *)(ws + q->off_Xb);
        double *Ya = (double *)(ws + q->off_Ya);
        timed(q, LQ_PH_CV_FOLD, st, [&] {
            lqk::launch_value_fold(q->nk, q->prec, (unsigned)q->total_seg, st, P, q->d_inst, q->d_seg_start, q->batch,
                                   nullptr, Xa, 1, status);
        });
        double *in = Xa, *o = Xb;
        if (q->max_nseg > 1)
            timed(q, LQ_PH_CV_SCAN, st, [&] {
                for (int dd = 1; dd < q->max_nseg; dd *= 2) {
                    lqk::launch_value_ks(q->nk, q->prec, (unsigned)q->total_x, st, q->d_inst, q->d_x_start, q->batch,
                                         dd, 1, in, o, status);
                    std::swap(in, o);
                }
            });
        timed(q, LQ_PH_CV_START, st, [&] {
            lqk::launch_cv_start(q->nk, q->prec, (unsigned)q->total_seg, st, P, V, q->d_inst, q->d_seg_start, q->batch,
                                 in, Ya, status);
        });
        roll_apply(q, P, V, Ya, x, u, lambda, st);
    }
    return launched();
}

// Value pass and rollout of every size class, class c's scan buffers at
// ws + class_ws(p, c) (only each class plan's scan regions [0, off_st) are
// used); with ckpt the Bellman sweep also writes the checkpoint of the
// differentiated solve (class c's slots after those of the classes before it).
static lq_status solve_with(const lq_plan *p, const lq_problem *prob, const double *elements, const lq_value *out,
                            double *x, double *u, double *lambda, char *ws0, int32_t *status, hipStream_t st,
                            double *ckpt = nullptr, int stride = 1);

lq_status lq_solve(const lq_plan *p, const lq_problem *prob, const double *elements, const lq_value *out, double *x,
                   double *u, double *lambda, void *workspace, int32_t *status, void *stream)
{
    if (!p || !prob_ok(prob) || !value_ok(out) || !x || !u) return LQ_ERR_ARG;
    if (!workspace || !aligned(workspace)) return LQ_ERR_WORKSPACE;
    if (elements && !aligned(elements)) return LQ_ERR_WORKSPACE;
    return solve_with(p, prob, elements, out, x, u, lambda, (char *)workspace, status, (hipStream_t)stream);
}

size_t lq_plan_static_bytes(const lq_plan *p) { return p ? p->off_st : 0; }

// Checkpoint slots of one class plan for a stride: total_seg / stride + batch
// tiles (ckpt_slot); a mixed plan keeps its classes' slots one after another.
static int64_t ckpt_slots(const lq_plan *q, int stride) { return q->total_seg / stride + q->batch; }
static size_t class_ckpt_bytes(const lq_plan *q, int stride)
{
    return align_up((size_t)ckpt_slots(q, stride) * TILE * sizeof(double));
}

size_t lq_plan_checkpoint_bytes(const lq_plan *p, int32_t stride)
{
    if (!p || stride < 1) return 0;
    size_t b = 0;
    for (int c = 0; c < nclass(p); ++c) b += class_ckpt_bytes(class_plan(p, c), stride);
    return b;
}

static lq_status solve_with(const lq_plan *p, const lq_problem *prob, const double *elements, const lq_value *out,
                            double *x, double *u, double *lambda, char *ws0, int32_t *status, hipStream_t st,
                            double *ckpt, int stride)
{
    const lqk::ProbPtrs P = probptrs(prob);
    lqk::ValPtrs V{out->S, out->s, out->Gamma, out->gamma};
    for (int c = 0; c < nclass(p); ++c) {
        const lq_plan *q = class_plan(p, c);
        char *ws = ws0 + class_ws(p, c);
        double *Ya = (double *)(ws + q->off_Ya), *Yb = (double *)(ws + q->off_Yb);
        value_pass(q, P, elements, V, ws, Ya, status, st, ckpt, stride);
        rollout_scan_apply(q, P, V, Ya, Yb, x, u, lambda, st);
        if (ckpt) ckpt += class_ckpt_bytes(q, stride) / sizeof(double);
    }
    return launched();
}

// The checkpointed adjoint's workspace: the plan's workspace, then room for
// the recomputed S, s, Gamma, gamma.
struct RecomputeLayout {
    size_t S, s, G, g, total;
};
static RecomputeLayout recompute_layout(const lq_plan *p)
{
    RecomputeLayout L{};
    int64_t nS = 0, ns = 0, nG = 0, ng = 0;
    for (const InstDesc &d : p->h_inst) {
        nS += (int64_t)(d.T + 1) * d.n * d.n;
        ns += (int64_t)(d.T + 1) * d.n;
        nG += (int64_t)d.T * d.m * d.n;
        ng += (int64_t)d.T * d.m;
    }
    size_t off = align_up(p->ws_bytes);
    L.S = off; off = align_up(off + (size_t)nS * sizeof(double));
    L.s = off; off = align_up(off + (size_t)ns * sizeof(double));
    L.G = off; off = align_up(off + (size_t)nG * sizeof(double));
    L.g = off; off = align_up(off + (size_t)ng * sizeof(double));
    L.total = off;
    return L;
}

size_t lq_plan_adjoint_ckpt_workspace_bytes(const lq_plan *p) { return p ? recompute_layout(p).total : 0; }

lq_status lq_solve_ckpt(const lq_plan *p, const lq_problem *prob, const double *elements, const lq_value *out,
                        double *x, double *u, double *lambda, double *ckpt, int32_t stride, void *workspace,
                        int32_t *status, void *stream)
{
    if (!p || !prob_ok(prob) || !value_ok(out) || !x || !u || stride < 1) return LQ_ERR_ARG;
    if (!workspace || !aligned(workspace)) return LQ_ERR_WORKSPACE;
    if (elements && !aligned(elements)) return LQ_ERR_WORKSPACE;
    if (!ckpt || !aligned(ckpt)) return LQ_ERR_WORKSPACE;
    return solve_with(p, prob, elements, out, x, u, lambda, (char *)workspace, status, (hipStream_t)stream, ckpt,
                      stride);
}

lq_status lq_solve_static(const lq_plan *p, const lq_problem *prob, const double *elements, const lq_value *out,
                          double *x, double *u, double *lambda, int32_t *status, void *stream)
{
    if (!p || !prob_ok(prob) || !value_ok(out) || !x || !u) return LQ_ERR_ARG;
    if (elements && !aligned(elements)) return LQ_ERR_WORKSPACE;
    if (p->off_st > LQ_STATIC_SCRATCH_BYTES) return LQ_ERR_WORKSPACE;
    void *ws = nullptr;
    if (!static_scratch(&ws)) return LQ_ERR_HIP;
    return solve_with(p, prob, elements, out, x, u, lambda, (char *)ws, status, (hipStream_t)stream);
}

// The adjoint's scans and sweeps of one class plan q from the value functions
// and gains in val; its scan buffers at ws, the s~ and gamma~ vectors (in the
// caller's packing) at st_v and gt_v.
static void adjoint_class(const lq_plan *q, const lqk::ProbPtrs &P, const lqk::ValPtrs &val, const double *x,
                          const double *u, const double *lambda, const double *gx, const double *gu,
                          const lqk::GradPtrs &G, char *ws, double *st_v, double *gt_v, int32_t *status,
                          hipStream_t st)
{
    double *Ya = (double *)(ws + q->off_Ya), *Yb = (double *)(ws + q->off_Yb);
    lqk::AdjPtrs J{val.S, val.s, val.G, val.g, x, u, lambda, gx, gu, st_v, gt_v};
    const unsigned nseg = (unsigned)q->total_seg;
    // backward linear-term scan
    timed(q, LQ_PH_ADJ_BACK_FOLD, st, [&] {
        lqk::launch_adj_back_fold(q->nk, q->prec, nseg, st, P, J, q->d_inst, q->d_seg_start, q->batch, Ya);
    });
    double *fin = Ya;
    if (q->max_nseg > 1) timed(q, LQ_PH_ADJ_BACK_SCAN, st, [&] { fin = affine_scan(q, st, 1, Ya, Yb); });
    // the backward sweep also writes the forward scan's entries (its segment fold fused in)
    double *fwd = (fin == Ya) ? Yb : Ya, *fwd2 = fin;
    timed(q, LQ_PH_ADJ_BACK_APPLY, st, [&] {
        lqk::launch_adj_back_apply(q->nk, q->prec, nseg, st, P, J, q->d_inst, q->d_seg_start, q->batch, fin, fwd,
                                   status);
    });
    // forward derivative scan + gradients
    double *ffin = fwd;
    if (q->max_nseg > 1) timed(q, LQ_PH_ADJ_FWD_SCAN, st, [&] { ffin = affine_scan(q, st, 0, fwd, fwd2); });
    timed(q, LQ_PH_ADJ_FWD_APPLY, st, [&] {
        lqk::launch_adj_fwd_apply(q->nk, q->prec, nseg, st, P, J, G, q->d_inst, q->d_seg_start, q->batch, ffin);
    });
}

static lq_status adjoint_with(const lq_plan *p, const lq_problem *prob, const lqk::ValPtrs &val, const double *x,
                              const double *u, const double *lambda, const double *gx, const double *gu,
                              const lq_grads *grads, char *ws, int32_t *status, hipStream_t st)
{
    const lqk::ProbPtrs P = probptrs(prob);
    lqk::GradPtrs G{grads->A, grads->B, grads->c, grads->Q, grads->R, grads->M,
                    grads->q, grads->r, grads->QT, grads->qT, grads->x0};
    double *st_v = (double *)(ws + p->off_st), *gt_v = (double *)(ws + p->off_gt);
    for (int c = 0; c < nclass(p); ++c)
        adjoint_class(class_plan(p, c), P, val, x, u, lambda, gx, gu, G, ws + class_ws(p, c), st_v, gt_v, status, st);
    return launched();
}

lq_status lq_adjoint(const lq_plan *p, const lq_problem *prob, const lq_value *val, const double *x,
                     const double *u, const double *lambda, const double *gx, const double *gu,
                     const lq_grads *grads, void *workspace, int32_t *status, void *stream)
{
    // without the value functions: rerun the value pass (lq_adjoint_ckpt without a checkpoint)
    if (!val)
        return lq_adjoint_ckpt(p, prob, nullptr, 1, x, u, lambda, gx, gu, grads, workspace, status, stream);
    if (!p || !prob_ok(prob) || !value_ok(val)) return LQ_ERR_ARG;
    if (!x || !u || !lambda || !gx || !gu || !grads) return LQ_ERR_ARG;
    if (!workspace || !aligned(workspace)) return LQ_ERR_WORKSPACE;
    const lqk::ValPtrs V{val->S, val->s, val->Gamma, val->gamma};
    return adjoint_with(p, prob, V, x, u, lambda, gx, gu, grads, (char *)workspace, status, (hipStream_t)stream);
}

lq_status lq_adjoint_ckpt(const lq_plan *p, const lq_problem *prob, const double *ckpt, int32_t stride,
                          const double *x, const double *u, const double *lambda, const double *gx, const double *gu,
                          const lq_grads *grads, void *workspace, int32_t *status, void *stream)
{
    if (!p || !prob_ok(prob) || (ckpt && stride < 1)) return LQ_ERR_ARG;
    if (!x || !u || !lambda || !gx || !gu || !grads) return LQ_ERR_ARG;
    if (!workspace || !aligned(workspace)) return LQ_ERR_WORKSPACE;
    if (ckpt && !aligned(ckpt)) return LQ_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    const RecomputeLayout L = recompute_layout(p);
    const lqk::ValPtrs V{(double *)(ws + L.S), (double *)(ws + L.s), (double *)(ws + L.G), (double *)(ws + L.g)};
    const lqk::ProbPtrs P = probptrs(prob);
    const double *ck = ckpt;
    for (int c = 0; c < nclass(p); ++c) {
        const lq_plan *q = class_plan(p, c);
        if (ck) {
            timed(q, LQ_PH_ADJ_RECOMPUTE, st, [&] {
                lqk::launch_value_recompute(q->nk, q->prec, (unsigned)ckpt_slots(q, stride), st, P, q->d_inst,
                                            q->d_seg_start, q->batch, stride, ck, V, status);
            });
            ck += class_ckpt_bytes(q, stride) / sizeof(double);
        } else {
            value_pass(q, P, nullptr, V, ws + class_ws(p, c), nullptr, status, st);
        }
    }
    return adjoint_with(p, prob, V, x, u, lambda, gx, gu, grads, ws, status, st);
}

// ---------------------------------------------------------------------------
// Newton / interior point
// ---------------------------------------------------------------------------

// Layout of the Newton workspace after the plan's LQ workspace.
struct NmpcLayout {
    size_t QTb, A, B, P, M, Rt, Rh, d, th, g, lam, lamT, S, s, G, gm, dx, du, xc, uc, zero, status, total;
};

// Newton workspace after the LQ workspace: every array holds the plan's
// `batch` instances packed like the LQ arrays (all instances of equal sizes).
static NmpcLayout nmpc_layout(const lq_plan *p)
{
    const InstDesc &d = p->h_inst[0];
    const size_t n = d.n, m = d.m, T = d.T, D = sizeof(double), Bn = (size_t)p->batch;
    NmpcLayout L{};
    size_t off = align_up(p->ws_bytes);
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + Bn * bytes);
        return o;
    };
    L.QTb = take(n * n * D);
    L.A = take(T * n * n * D); L.B = take(T * n * m * D); L.P = take(T * n * n * D); L.M = take(T * n * m * D);
    L.Rt = take(T * m * m * D); L.Rh = take(T * m * m * D); L.d = take(T * m * D);
    L.th = take(T * n * D); L.g = take(T * n * D); L.lam = take((T + 1) * n * D); L.lamT = take(n * D);
    L.S = take((T + 1) * n * n * D); L.s = take((T + 1) * n * D); L.G = take(T * m * n * D);
    L.gm = take(T * m * D); L.dx = take((T + 1) * n * D); L.du = take(T * m * D);
    L.xc = take((T + 1) * n * D); L.uc = take(T * m * D); L.zero = take(n * D); L.status = take(sizeof(int32_t));
    L.total = off;
    return L;
}

static bool nmpc_matches(const lq_plan *p, const nmpc_problem *q)
{
    if (!p || !q || p->batch < 1) return false;
    for (const InstDesc &d : p->h_inst)
        if (d.n != q->nx || d.m != q->nu || d.T != q->T) return false;
    bool model_ok = false;
    switch (q->model) {
    case NMPC_TANH: model_ok = q->W && q->Bm; break;
    case NMPC_PENDULUM: model_ok = q->nx == 2 && q->nu == 1; break;
    case NMPC_CARTPOLE: model_ok = q->nx == 4 && q->nu == 1; break;
    default: break;
    }
    const bool aug_ok = !(q->admm_rho > 0.0) || (q->admm_z && q->admm_v);
    return model_ok && aug_ok && q->Q && q->R && q->QT && q->xref && q->x0 && q->umin < q->umax;
}

static lqk::NmpcPtrs nmpc_ptrs(const lq_plan *p, const nmpc_problem *q)
{
    lqk::NmpcPtrs N;
    N.nx = q->nx; N.nu = q->nu; N.T = q->T; N.batch = p->batch; N.h = q->h;
    N.W = q->W; N.Bm = q->Bm; N.Q = q->Q; N.R = q->R; N.QT = q->QT; N.xref = q->xref; N.x0 = q->x0;
    N.umin = q->umin; N.umax = q->umax;
    N.model = q->model;
    for (int i = 0; i < 4; ++i) N.prm[i] = q->param[i];
    N.rho = (q->admm_rho > 0.0) ? q->admm_rho : 0.0;
    N.z = q->admm_z;
    N.v = q->admm_v;
    return N;
}

static lqk::NmpcWork nmpc_work(const lq_plan *p, void *workspace)
{
    const NmpcLayout L = nmpc_layout(p);
    char *w = (char *)workspace;
    auto D = [&](size_t o) { return (double *)(w + o); };
    lqk::NmpcWork Wk;
    Wk.QTb = D(L.QTb);
    Wk.A = D(L.A); Wk.B = D(L.B); Wk.P = D(L.P); Wk.M = D(L.M); Wk.Rt = D(L.Rt); Wk.Rh = D(L.Rh); Wk.d = D(L.d);
    Wk.th = D(L.th); Wk.g = D(L.g); Wk.lam = D(L.lam); Wk.lamT = D(L.lamT); Wk.S = D(L.S); Wk.s = D(L.s);
    Wk.G = D(L.G); Wk.gm = D(L.gm); Wk.dx = D(L.dx); Wk.du = D(L.du); Wk.xc = D(L.xc); Wk.uc = D(L.uc);
    Wk.zero = D(L.zero);
    Wk.status = (int32_t *)(w + L.status);
    Wk.scal = nullptr;
    return Wk;
}

size_t nmpc_workspace_bytes(const lq_plan *p)
{
    if (!p || p->batch < 1) return 0;
    return nmpc_layout(p).total;
}

lq_status nmpc_init(const lq_plan *p, const nmpc_problem *prob, const nmpc_state *state, void *workspace,
                    void *stream)
{
    if (!nmpc_matches(p, prob) || !state || !state->x || !state->u || !state->scal) return LQ_ERR_ARG;
    if (prob->nx > 15 || prob->nu > lqk::MMAX) return LQ_ERR_UNSUPPORTED;
    (void)workspace;
    lqk::launch_nmpc_init((hipStream_t)stream, nmpc_ptrs(p, prob), state->x, state->u);
    return launched();
}

lq_status newton_step(const lq_plan *p, const nmpc_problem *prob, const nmpc_state *state, void *workspace,
                      int32_t *status, void *stream)
{
    (void)status;
    if (!nmpc_matches(p, prob) || !state || !state->x || !state->u || !state->scal) return LQ_ERR_ARG;
    if (!workspace || !aligned(workspace)) return LQ_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const lqk::NmpcPtrs N = nmpc_ptrs(p, prob);
    lqk::NmpcWork Wk = nmpc_work(p, workspace);
    Wk.scal = state->scal;
    char *ws = (char *)workspace;
    double *Ya = (double *)(ws + p->off_Ya), *Yb = (double *)(ws + p->off_Yb);
    // linearisation (with the step's clears) and the co-state pass (suffix
    // scan of [[A', g], [0, 1]])
    lqk::launch_nmpc_linearise(p->prec, st, N, Wk, state->x, state->u);
    // (n <= 4: the per-lane kernels, in FP64 whatever the plan's precision)
    if (p->small)
        lqk::launch_small_costate_fold(p->sn, p->total_seg, st, Wk, p->d_inst, p->d_seg_start, p->batch, Ya);
    else
        lqk::launch_costate_fold(p->nk, p->prec, (unsigned)p->total_seg, st, Wk, p->d_inst, p->d_seg_start, p->batch,
                                 Ya);
    double *in = affine_scan(p, st, 1, Ya, Yb);
    if (p->small)
        lqk::launch_small_costate_apply(p->sn, p->total_seg, st, Wk, p->d_inst, p->d_seg_start, p->batch, in);
    else
        lqk::launch_costate_apply(p->nk, p->prec, (unsigned)p->total_seg, st, Wk, p->d_inst, p->d_seg_start, p->batch,
                                  in);
    lqk::launch_nmpc_quadraticise(p->prec, st, N, Wk, state->x, state->u, state->scal);
    // the LQ step (all instances in one batched solve)
    lq_problem lp{};
    lp.A = Wk.A; lp.B = Wk.B; lp.c = nullptr; lp.Q = Wk.P; lp.R = Wk.Rt;
    lp.M = (prob->model == NMPC_TANH) ? nullptr : Wk.M;   // the tanh model has no mixed second derivative
    lp.q = nullptr; lp.r = Wk.d; lp.QT = Wk.QTb; lp.qT = nullptr; lp.x0 = Wk.zero;
    lq_value val{Wk.S, Wk.s, Wk.G, Wk.gm};
    const lq_status r = lq_solve(p, &lp, nullptr, &val, Wk.dx, Wk.du, nullptr, workspace, Wk.status, stream);
    if (r != LQ_OK) return r;
    // candidate, decision and commit
    lqk::launch_nmpc_candidate(st, N, Wk, state->x, state->u, state->scal);
    return launched();
}

lq_status nmpc_admm_update(const lq_plan *p, const nmpc_problem *prob, const nmpc_state *state, int32_t init,
                           void *stream)
{
    if (!nmpc_matches(p, prob) || !state || !state->u || !state->scal || !(prob->admm_rho > 0.0)) return LQ_ERR_ARG;
    lqk::launch_admm_update((hipStream_t)stream, nmpc_ptrs(p, prob), state->u, state->scal, init);
    return launched();
}

lq_status nmpc_shift(const lq_plan *p, const nmpc_problem *prob, const nmpc_state *state, double *x0,
                     double *u_applied, void *stream)
{
    if (!nmpc_matches(p, prob) || !state || !state->u || !x0 || !u_applied) return LQ_ERR_ARG;
    if (prob->nx > 15 || prob->nu > lqk::MMAX) return LQ_ERR_UNSUPPORTED;
    lqk::launch_nmpc_shift((hipStream_t)stream, nmpc_ptrs(p, prob), x0, state->u, u_applied);
    return launched();
}

lq_status lq_plan_set_timing(lq_plan *p, uint32_t mask, int32_t capacity)
{
    if (!p || capacity < 0) return LQ_ERR_ARG;
    for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
    p->ev.clear();
    p->ev_phase.clear();
    p->ev_used = 0;
    p->tmask = 0;
    if (mask == 0 || capacity == 0) return LQ_OK;
    p->ev.resize(2 * (size_t)capacity);
    p->ev_phase.resize((size_t)capacity);
    for (auto &e : p->ev)
        if (hipEventCreate(&e) != hipSuccess) return LQ_ERR_HIP;
    p->tmask = mask;
    return LQ_OK;
}

lq_status lq_plan_phase_times(lq_plan *p, double *ms, int64_t *count)
{
    if (!p) return LQ_ERR_ARG;
    double acc[LQ_NPHASE] = {0};
    int64_t cnt[LQ_NPHASE] = {0};
    for (size_t i = 0; i < p->ev_used; ++i) {
        if (hipEventSynchronize(p->ev[2 * i + 1]) != hipSuccess) return LQ_ERR_HIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, p->ev[2 * i], p->ev[2 * i + 1]) != hipSuccess) return LQ_ERR_HIP;
        acc[p->ev_phase[i]] += t;
        cnt[p->ev_phase[i]] += 1;
    }
    p->ev_used = 0;
    for (int i = 0; i < LQ_NPHASE; ++i) {
        if (ms) ms[i] = acc[i];
        if (count) count[i] = cnt[i];
    }
    return LQ_OK;
}

lq_status lq_selftest_tile_mm(const double *X, const double *Y, const double *Z, double *D, int32_t tx,
                              int32_t ty, int32_t precision, void *stream)
{
    if (!X || !Y || !D || (precision != LQ_FP64 && precision != LQ_MIXED)) return LQ_ERR_ARG;
    lqk::launch_selftest_mm(precision, (hipStream_t)stream, X, Y, Z, D, tx, ty);
    return launched();
}

lq_status lq_selftest_tile_inverse(const double *X, double *Xinv, int32_t n1, int32_t homog, int32_t *ok,
                                   void *stream)
{
    if (!X || !Xinv || !ok || n1 < 1 || n1 > 16 || (homog && n1 < 2)) return LQ_ERR_ARG;
    lqk::launch_selftest_inv((hipStream_t)stream, X, Xinv, n1, homog, ok);
    return launched();
}

}  // extern "C"
