// Host side of the reduced quasi-neutral model: validation, buffer layout,
// initialisation, graph capture and the pic_hyb_* entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hyb_internal.hpp"

using namespace hyb;

struct pic_hyb {
    pic_hyb_desc desc;
    Params hp;
    Params *dp = nullptr;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int device = 0;
    std::string err;
};

namespace {

thread_local std::string g_hyb_error;

int fail(std::string *err, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (err) *err = buf;
    g_hyb_error = buf;
    return code;
}

int hip_fail(std::string *err, hipError_t e, const char *what)
{
    return fail(err, PIC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HCHK(errp, expr)                                        \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return hip_fail(errp, e_, #expr); \
    } while (0)

int log2_pow2(int v)
{
    if (v <= 0 || (v & (v - 1))) return -1;
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t part_bytes = 0, grid_bytes = 0;
    size_t px[2], py[2], pux[2], puy[2], ppz[2], pid[2];
    size_t a1, a2, psi, it[2], rhsR, rhsC, dep[2][4], W, twx, twy, lapx, lapy, count, start, tstart[2], bins, scan, pdiag, gdiag,
        state, params, ring;
};

struct Carver {
    size_t off = 0;
    size_t take(size_t b)
    {
        const size_t o = off;
        off = align256(off + b);
        return o;
    }
};

int validate(const pic_hyb_desc *d, Layout *L, std::string *err)
{
    if (!d) return fail(err, PIC_E_INVALID_ARG, "null descriptor");
    const int lx = log2_pow2(d->nx), ly = log2_pow2(d->ny);
    if (lx < 3 || ly < 3 || d->nx > kMaxNodes || d->ny > kMaxNodes)
        return fail(err, PIC_E_UNSUPPORTED, "nodes %d x %d: each must be a power of two in 8..%d", d->nx, d->ny,
                    kMaxNodes);
    if (!(d->dx > 0.0 && std::isfinite(d->dx) && d->dy > 0.0 && std::isfinite(d->dy)))
        return fail(err, PIC_E_INVALID_ARG, "dx, dy must be positive");
    if (!(d->dt > 0.0 && std::isfinite(d->dt))) return fail(err, PIC_E_INVALID_ARG, "dt must be positive");
    if (!(d->nu >= 0.0 && std::isfinite(d->nu))) return fail(err, PIC_E_INVALID_ARG, "nu must be >= 0");
    if (!(d->n0 > 0.0 && std::isfinite(d->n0))) return fail(err, PIC_E_INVALID_ARG, "n0 must be positive");
    if (!(d->weight >= 0.0 && std::isfinite(d->weight))) return fail(err, PIC_E_INVALID_ARG, "weight must be >= 0");
    if (d->nparticles < 0 || d->nparticles > 0x7FFFFFFFll)
        return fail(err, PIC_E_INVALID_ARG, "nparticles %lld out of 0..2^31-1", (long long)d->nparticles);
    if (d->iters < 1 || d->iters > 64) return fail(err, PIC_E_INVALID_ARG, "iters %d out of 1..64", d->iters);
    if (d->diag_every < 0 || d->sort_every < 0) return fail(err, PIC_E_INVALID_ARG, "diag_every, sort_every >= 0");
    if (d->flags & ~(uint32_t)PIC_FLAG_NO_GRAPH) return fail(err, PIC_E_INVALID_ARG, "flags %u", d->flags);
    const double cells = (double)d->nx * d->ny;
    const double c0 = d->n0 - d->weight * (double)d->nparticles / cells;
    if (!(c0 > 0.0))
        return fail(err, PIC_E_UNSUPPORTED, "mean beam density %.6g >= n0: no quasi-neutral plasma left",
                    d->weight * (double)d->nparticles / cells);
    if (!L) return PIC_OK;
    const size_t N = (size_t)d->nparticles, C = (size_t)d->nx * d->ny;
    Carver p;
    for (int s = 0; s < 2; ++s) {
        L->px[s] = p.take(N * 8);
        L->py[s] = p.take(N * 8);
        L->pux[s] = p.take(N * 8);
        L->puy[s] = p.take(N * 8);
        L->ppz[s] = p.take(N * 8);
        L->pid[s] = p.take(N * 4);
    }
    L->part_bytes = std::max<size_t>(p.off, 256);
    Carver g;
    L->a1 = g.take(C * 8);
    L->a2 = g.take(C * 8);
    L->psi = g.take(C * 8);
    L->it[0] = g.take(C * 8);
    L->it[1] = g.take(C * 8);
    L->rhsR = g.take(C * 8);
    L->rhsC = g.take(C * 8);
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < 4; ++k) L->dep[s][k] = g.take(C * 8);
    L->W = g.take(C * 16);
    L->twx = g.take((size_t)d->nx / 2 * 16);
    L->twy = g.take((size_t)d->ny / 2 * 16);
    L->lapx = g.take((size_t)d->nx * 8);
    L->lapy = g.take((size_t)d->ny * 8);
    L->count = g.take(C * 4);
    L->start = g.take(C * 4);
    const int T = std::min(kMaxTile, std::min(d->nx, d->ny));
    const size_t ntiles = C / ((size_t)T * T);
    L->tstart[0] = g.take((ntiles + 1) * 4);
    L->tstart[1] = g.take((ntiles + 1) * 4);
    L->bins = g.take(ntiles * kWinC * kWinC * 4);
    L->scan = g.take(((C + kScanChunk - 1) / kScanChunk) * 4);
    L->pdiag = g.take(ntiles * kPDiag * 8);
    L->gdiag = g.take((size_t)kGridBlocks * kGDiag * 8);
    L->state = g.take(sizeof(State));
    L->params = g.take(sizeof(Params));
    L->ring = g.take((size_t)kRing * sizeof(pic_hyb_diag));
    L->grid_bytes = g.off;
    return PIC_OK;
}

template <typename T>
T *at(void *base, size_t off)
{
    return (T *)((char *)base + off);
}

int capture(pic_hyb *h)
{
    if (h->desc.flags & PIC_FLAG_NO_GRAPH) return PIC_OK;
    hipStream_t cs;
    HCHK(&h->err, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        hipError_t le = launch_step(h->hp, h->dp, cs, nullptr, nullptr, nullptr);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        if (le != hipSuccess) e = le;
        if (e == hipSuccess) {
            e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
            if (e == hipSuccess) h->graph = g;
            else (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(&h->err, e, "graph capture of the step");
    return PIC_OK;
}

int check_state(pic_hyb *h)
{
    State st;
    HCHK(&h->err, hipMemcpy(&st, h->hp.state, sizeof(st), hipMemcpyDeviceToHost));
    if (st.fatal & 1) return fail(&h->err, PIC_E_HIP, "a particle position became non-finite");
    return PIC_OK;
}

}  // namespace

extern "C" {

int pic_hyb_query(const pic_hyb_desc *desc, size_t *particle_bytes, size_t *grid_bytes)
{
    Layout L;
    const int rc = validate(desc, &L, nullptr);
    if (rc != PIC_OK) return rc;
    if (particle_bytes) *particle_bytes = L.part_bytes;
    if (grid_bytes) *grid_bytes = L.grid_bytes;
    return PIC_OK;
}

int pic_hyb_init(const pic_hyb_desc *desc, void *particles, size_t particle_bytes, void *grid, size_t grid_bytes,
                 void *hip_stream, const double *x, const double *y, const double *ux, const double *uy,
                 const double *uz, pic_hyb **out)
{
    if (!out) return fail(nullptr, PIC_E_INVALID_ARG, "null output handle");
    *out = nullptr;
    Layout L;
    int rc = validate(desc, &L, nullptr);
    if (rc != PIC_OK) return rc;
    if (!particles || !grid) return fail(nullptr, PIC_E_INVALID_ARG, "null device buffer");
    if (particle_bytes < L.part_bytes || grid_bytes < L.grid_bytes)
        return fail(nullptr, PIC_E_BUFFER_TOO_SMALL, "buffers of %zu / %zu bytes, need %zu / %zu", particle_bytes,
                    grid_bytes, L.part_bytes, L.grid_bytes);
    const int64_t N = desc->nparticles;
    if (N > 0 && (!x || !y || !ux || !uy || !uz)) return fail(nullptr, PIC_E_INVALID_ARG, "null particle array");
    const double Lx = desc->nx * desc->dx, Ly = desc->ny * desc->dy;
    for (int64_t i = 0; i < N; ++i) {
        if (!(x[i] >= 0.0 && x[i] < Lx && y[i] >= 0.0 && y[i] < Ly))
            return fail(nullptr, PIC_E_INVALID_ARG, "particle %lld at (%g, %g) outside the box", (long long)i, x[i],
                        y[i]);
        if (!(std::isfinite(ux[i]) && std::isfinite(uy[i]) && std::isfinite(uz[i])))
            return fail(nullptr, PIC_E_INVALID_ARG, "particle %lld: non-finite momentum", (long long)i);
    }
    pic_hyb *h = new pic_hyb();
    h->desc = *desc;
    h->stream = (hipStream_t)hip_stream;
    hipError_t he = hipGetDevice(&h->device);
    if (he != hipSuccess) {
        delete h;
        return hip_fail(nullptr, he, "hipGetDevice");
    }
    Params &P = h->hp;
    memset(&P, 0, sizeof(P));
    P.nx = desc->nx;
    P.ny = desc->ny;
    P.lx = log2_pow2(desc->nx);
    P.ly = log2_pow2(desc->ny);
    P.iters = desc->iters;
    P.diag_every = desc->diag_every;
    P.sort_every = desc->sort_every;
    P.cols_per_block = std::min(desc->nx, kFftLds / desc->ny);
    P.tile = std::min(kMaxTile, std::min(desc->nx, desc->ny));
    P.ltile = log2_pow2(P.tile);
    P.tiles_x = desc->nx / P.tile;
    P.ntiles = (desc->nx / P.tile) * (desc->ny / P.tile);
    P.np = N;
    P.cells = (int64_t)desc->nx * desc->ny;
    P.dx = desc->dx;
    P.dy = desc->dy;
    P.dt = desc->dt;
    P.nu = desc->nu;
    P.n0 = desc->n0;
    P.w = desc->weight;
    P.c0 = desc->n0 - desc->weight * (double)N / (double)P.cells;
    P.dA = desc->dx * desc->dy;
    P.inv_dx = 1.0 / desc->dx;
    P.inv_dy = 1.0 / desc->dy;
    P.Lx = Lx;
    P.Ly = Ly;
    for (int s = 0; s < 2; ++s) {
        P.x[s] = at<double>(particles, L.px[s]);
        P.y[s] = at<double>(particles, L.py[s]);
        P.ux[s] = at<double>(particles, L.pux[s]);
        P.uy[s] = at<double>(particles, L.puy[s]);
        P.pz[s] = at<double>(particles, L.ppz[s]);
        P.id[s] = at<uint32_t>(particles, L.pid[s]);
    }
    P.a1 = at<double>(grid, L.a1);
    P.a2 = at<double>(grid, L.a2);
    P.psi = at<double>(grid, L.psi);
    for (int s = 0; s < 2; ++s) P.it[s] = at<double>(grid, L.it[s]);
    P.rhsR = at<double>(grid, L.rhsR);
    P.rhsC = at<double>(grid, L.rhsC);
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < 4; ++k) P.dep[s][k] = at<Fix>(grid, L.dep[s][k]);
    P.W = at<double2>(grid, L.W);
    P.twx = at<double2>(grid, L.twx);
    P.twy = at<double2>(grid, L.twy);
    P.lapx = at<double>(grid, L.lapx);
    P.lapy = at<double>(grid, L.lapy);
    P.cell_count = at<int32_t>(grid, L.count);
    P.cell_start = at<int32_t>(grid, L.start);
    P.tile_start[0] = at<int32_t>(grid, L.tstart[0]);
    P.tile_start[1] = at<int32_t>(grid, L.tstart[1]);
    P.bins = at<int32_t>(grid, L.bins);
    P.scan_part = at<int32_t>(grid, L.scan);
    P.pdiag = at<double>(grid, L.pdiag);
    P.gdiag = at<double>(grid, L.gdiag);
    P.state = at<State>(grid, L.state);
    P.ring = at<pic_hyb_diag>(grid, L.ring);
    h->dp = at<Params>(grid, L.params);

    // twiddles exp(-2 pi i t / n) and the 5-point Laplacian's symbol per axis
    std::vector<double2> twx(desc->nx / 2), twy(desc->ny / 2);
    for (int t = 0; t < desc->nx / 2; ++t)
        twx[t] = make_double2(std::cos(2.0 * M_PI * t / desc->nx), -std::sin(2.0 * M_PI * t / desc->nx));
    for (int t = 0; t < desc->ny / 2; ++t)
        twy[t] = make_double2(std::cos(2.0 * M_PI * t / desc->ny), -std::sin(2.0 * M_PI * t / desc->ny));
    std::vector<double> lapx(desc->nx), lapy(desc->ny);
    for (int k = 0; k < desc->nx; ++k) {
        const double s = std::sin(M_PI * k / desc->nx);
        lapx[k] = 4.0 / (desc->dx * desc->dx) * s * s;
    }
    for (int k = 0; k < desc->ny; ++k) {
        const double s = std::sin(M_PI * k / desc->ny);
        lapy[k] = 4.0 / (desc->dy * desc->dy) * s * s;
    }
    std::vector<uint32_t> ids((size_t)N);
    for (int64_t i = 0; i < N; ++i) ids[(size_t)i] = (uint32_t)i;
    hipStream_t st = h->stream;
    std::string *e = &h->err;
#define ICHK(expr)                                   \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) {                      \
            const int c_ = hip_fail(e, e_, #expr);   \
            (void)hipStreamSynchronize(st);          \
            delete h;                                \
            return c_;                               \
        }                                            \
    } while (0)
    ICHK(hipMemsetAsync(grid, 0, L.grid_bytes, st));
    ICHK(hipMemcpyAsync(P.twx, twx.data(), twx.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    ICHK(hipMemcpyAsync(P.twy, twy.data(), twy.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    ICHK(hipMemcpyAsync(P.lapx, lapx.data(), lapx.size() * 8, hipMemcpyHostToDevice, st));
    ICHK(hipMemcpyAsync(P.lapy, lapy.data(), lapy.size() * 8, hipMemcpyHostToDevice, st));
    ICHK(hipMemcpyAsync(h->dp, &P, sizeof(Params), hipMemcpyHostToDevice, st));
    if (N > 0) {
        const size_t b = (size_t)N * 8;
        ICHK(hipMemcpyAsync(P.x[0], x, b, hipMemcpyHostToDevice, st));
        ICHK(hipMemcpyAsync(P.y[0], y, b, hipMemcpyHostToDevice, st));
        ICHK(hipMemcpyAsync(P.ux[0], ux, b, hipMemcpyHostToDevice, st));
        ICHK(hipMemcpyAsync(P.uy[0], uy, b, hipMemcpyHostToDevice, st));
        ICHK(hipMemcpyAsync(P.pz[0], uz, b, hipMemcpyHostToDevice, st));
        ICHK(hipMemcpyAsync(P.id[0], ids.data(), (size_t)N * 4, hipMemcpyHostToDevice, st));
    }
    ICHK(launch_init(P, h->dp, st));
    ICHK(hipStreamSynchronize(st));
#undef ICHK
    rc = capture(h);
    if (rc != PIC_OK) {
        g_hyb_error = h->err;
        delete h;
        return rc;
    }
    *out = h;
    return PIC_OK;
}

int pic_hyb_step(pic_hyb *h, int32_t nsteps)
{
    if (!h) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    if (nsteps < 0) return fail(&h->err, PIC_E_INVALID_ARG, "nsteps < 0");
    for (int32_t i = 0; i < nsteps; ++i) {
        if (h->gexec) HCHK(&h->err, hipGraphLaunch(h->gexec, h->stream));
        else HCHK(&h->err, launch_step(h->hp, h->dp, h->stream, nullptr, nullptr, nullptr));
    }
    return PIC_OK;
}

int pic_hyb_step_profiled(pic_hyb *h, int32_t nsteps, double *group_ms)
{
    if (!h || !group_ms) return fail(h ? &h->err : nullptr, PIC_E_INVALID_ARG, "null argument");
    if (nsteps < 0) return fail(&h->err, PIC_E_INVALID_ARG, "nsteps < 0");
    for (int g = 0; g < kGroups; ++g) group_ms[g] = 0.0;
    const int n = step_launches(h->hp);
    std::vector<hipEvent_t> ev((size_t)2 * n);
    std::vector<int> groups((size_t)n);
    for (auto &x : ev) HCHK(&h->err, hipEventCreate(&x));
    int rc = PIC_OK;
    for (int32_t s = 0; s < nsteps && rc == PIC_OK; ++s) {
        int nl = 0;
        hipError_t e = launch_step(h->hp, h->dp, h->stream, ev.data(), groups.data(), &nl);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) {
            rc = hip_fail(&h->err, e, "profiled step");
            break;
        }
        for (int k = 0; k < nl; ++k) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]) == hipSuccess) group_ms[groups[k]] += ms;
        }
    }
    for (auto &x : ev) (void)hipEventDestroy(x);
    if (rc != PIC_OK) return rc;
    return check_state(h);
}

int pic_hyb_sync(pic_hyb *h)
{
    if (!h) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    HCHK(&h->err, hipStreamSynchronize(h->stream));
    return check_state(h);
}

int pic_hyb_read_grid(pic_hyb *h, double *a, double *psi)
{
    const int rc = pic_hyb_sync(h);
    if (rc != PIC_OK) return rc;
    const size_t b = (size_t)h->hp.cells * 8;
    if (a) HCHK(&h->err, hipMemcpy(a, h->hp.a1, b, hipMemcpyDeviceToHost));
    if (psi) HCHK(&h->err, hipMemcpy(psi, h->hp.psi, b, hipMemcpyDeviceToHost));
    return PIC_OK;
}

int pic_hyb_read_particles(pic_hyb *h, double *x, double *y, double *ux, double *uy, double *pz, uint32_t *id)
{
    const int rc = pic_hyb_sync(h);
    if (rc != PIC_OK) return rc;
    State st;
    HCHK(&h->err, hipMemcpy(&st, h->hp.state, sizeof(st), hipMemcpyDeviceToHost));
    const int s = st.cur;
    const size_t b = (size_t)h->hp.np * 8;
    if (h->hp.np == 0) return PIC_OK;
    if (x) HCHK(&h->err, hipMemcpy(x, h->hp.x[s], b, hipMemcpyDeviceToHost));
    if (y) HCHK(&h->err, hipMemcpy(y, h->hp.y[s], b, hipMemcpyDeviceToHost));
    if (ux) HCHK(&h->err, hipMemcpy(ux, h->hp.ux[s], b, hipMemcpyDeviceToHost));
    if (uy) HCHK(&h->err, hipMemcpy(uy, h->hp.uy[s], b, hipMemcpyDeviceToHost));
    if (pz) HCHK(&h->err, hipMemcpy(pz, h->hp.pz[s], b, hipMemcpyDeviceToHost));
    if (id) HCHK(&h->err, hipMemcpy(id, h->hp.id[s], (size_t)h->hp.np * 4, hipMemcpyDeviceToHost));
    return PIC_OK;
}

int pic_hyb_diag_history(pic_hyb *h, pic_hyb_diag *out, int32_t max, int32_t *n)
{
    if (!h || !n || (max > 0 && !out)) return fail(h ? &h->err : nullptr, PIC_E_INVALID_ARG, "null argument");
    const int rc = pic_hyb_sync(h);
    if (rc != PIC_OK) return rc;
    State st;
    HCHK(&h->err, hipMemcpy(&st, h->hp.state, sizeof(st), hipMemcpyDeviceToHost));
    std::vector<pic_hyb_diag> ring(kRing);
    HCHK(&h->err, hipMemcpy(ring.data(), h->hp.ring, sizeof(pic_hyb_diag) * kRing, hipMemcpyDeviceToHost));
    const int cnt = std::min<int>(st.ring_count, std::max(0, max));
    for (int i = 0; i < cnt; ++i) {
        const int slot = ((st.ring_head - cnt + i) % kRing + kRing) % kRing;
        out[i] = ring[slot];
    }
    *n = cnt;
    return PIC_OK;
}

int pic_hyb_last_error(pic_hyb *h, char *buf, size_t n)
{
    if (!buf || n == 0) return PIC_E_INVALID_ARG;
    snprintf(buf, n, "%s", (h ? h->err : g_hyb_error).c_str());
    return PIC_OK;
}

int pic_hyb_destroy(pic_hyb *h)
{
    if (!h) return PIC_OK;
    (void)hipStreamSynchronize(h->stream);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    delete h;
    return PIC_OK;
}

}  // extern "C"
