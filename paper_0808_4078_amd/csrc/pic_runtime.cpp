// Host runtime of libpic: the C ABI declared in include/pic.h.
//
// It validates descriptors, carves the caller-owned device buffers into the
// particle store, field planes and scratch, writes the device-resident
// KParams block, runs the device loader, and enqueues steps (as a captured
// graph replay unless PIC_FLAG_NO_GRAPH).  It never allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pic_internal.hpp"

using namespace pic;

namespace {

thread_local std::string g_last_error;

struct Layout {
    size_t particle_bytes[kMaxSpecies] = {};
    size_t field_bytes = 0, scratch_bytes = 0, diag_bytes = 0;
    // offsets inside the particle buffer of each species
    struct Sp {
        size_t cell[3], pos[3][3], u[3][3], id[3];
        size_t start, cap, cnt_front, cnt_back;
        int64_t ncap, nominal, tile_nominal, reserve;
        uint32_t ovf_cap;
    } sp[kMaxSpecies];
    size_t F, J;                                            // field buffer
    size_t Jtile, tile_diag, field_diag, moments, state, kparams, rb[4], order, bucket;   // scratch
    size_t rho_tile, rho0, rho_n, gauss_part, cont_part;    // scratch (Gauss-law and continuity checks)
    size_t ee_tile;                                         // scratch (binary-collision counts per tile)
    size_t ee_ent = 0;                                      // scratch (binary collisions: cell-sorted participants)
    bool checks = false;                                    // PIC_FLAG_GAUSS_RESIDUAL: the above are carved
    Geometry g;
    int nj;
    size_t real;                                            // sizeof(float|double)
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; }
};

int ilog2_exact(int v)
{
    int b = 0;
    while ((1 << b) < v) ++b;
    return (1 << b) == v ? b : -1;
}

int bits_for(int v)
{
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

int fail(std::string *err, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (err) *err = buf;
    g_last_error = buf;
    return code;
}

int validate(const pic_grid_desc *g, const pic_species_desc *sp, int ns, Layout *L, std::string *err)
{
    if (!g || !sp) return fail(err, PIC_E_INVALID_ARG, "null descriptor");
    if (ns < 1 || ns > kMaxSpecies) return fail(err, PIC_E_INVALID_ARG, "nspecies %d out of 1..%d", ns, kMaxSpecies);
    if (g->ndim != 2 && g->ndim != 3) return fail(err, PIC_E_INVALID_ARG, "ndim %d", g->ndim);
    if (g->precision != PIC_PREC_FP64 && g->precision != PIC_PREC_MIXED)
        return fail(err, PIC_E_INVALID_ARG, "precision %d", g->precision);
    if (!(g->dt > 0.0) || !std::isfinite(g->dt)) return fail(err, PIC_E_INVALID_ARG, "dt must be positive");
    if (g->diag_every < 0) return fail(err, PIC_E_INVALID_ARG, "diag_every < 0");
    if (!(g->reserve >= 0.0 && g->reserve <= 8.0)) return fail(err, PIC_E_INVALID_ARG, "reserve out of [0, 8]");
    if (!(g->nu_ee >= 0.0) || !std::isfinite(g->nu_ee)) return fail(err, PIC_E_INVALID_ARG, "nu_ee must be >= 0");
    if (g->nu_ee > 0.0 && !(g->ee_vref > 0.0 && g->ee_vref < 1.0))
        return fail(err, PIC_E_INVALID_ARG, "binary collisions need 0 < ee_vref < 1");
    if (g->shape < 0 || g->shape >= kShapes)
        return fail(err, PIC_E_INVALID_ARG, "shape %d out of 0..%d", g->shape, kShapes - 1);
    if (g->shape != 0 && g->precision != PIC_PREC_MIXED)
        return fail(err, PIC_E_INVALID_ARG, "shape %d: FP64 runs take shape 0 only", g->shape);
    const double reserve = g->reserve > 0.0 ? g->reserve : 1.0;
    Geometry &G = L->g;
    memset(&G, 0, sizeof(G));
    G.ndim = g->ndim;
    G.dt = g->dt;
    G.ntiles = 1;
    G.cells = 1;
    for (int a = 0; a < 3; ++a) {
        if (a >= g->ndim) {
            G.n[a] = 1;
            G.d[a] = 1.0;
            G.tile[a] = 1;
            G.nt[a] = 1;
            continue;
        }
        if (g->n[a] <= 0) return fail(err, PIC_E_INVALID_ARG, "n[%d] = %d", a, g->n[a]);
        if (!(g->d[a] > 0.0) || !std::isfinite(g->d[a])) return fail(err, PIC_E_INVALID_ARG, "d[%d] must be positive", a);
        if (g->dt > 0.5 * g->d[a] * (1.0 + 1e-12))
            return fail(err, PIC_E_CFL, "dt %.6g exceeds d[%d]/2 = %.6g (a particle must cross less than half a cell per step)",
                        g->dt, a, 0.5 * g->d[a]);
        int t = g->tile[a];
        if (t == 0) {
            // 3D: 8^3; 2D: the largest of 16, 8 that divides both axes
            t = g->ndim == 3 ? 8 : 16;
            for (int b = 0; b < g->ndim; ++b)
                if (g->n[b] > 0 && g->n[b] % t) t = 8;
        }
        if (g->ndim == 3 && t != 8) return fail(err, PIC_E_UNSUPPORTED, "3D tiles must be 8^3 (got %d)", t);
        if (t != 8 && t != 16 && t != 32) return fail(err, PIC_E_UNSUPPORTED, "tile %d not in {8,16,32}", t);
        if (g->n[a] % t) return fail(err, PIC_E_INVALID_ARG, "n[%d] = %d is not a multiple of the tile %d", a, g->n[a], t);
        G.n[a] = g->n[a];
        G.d[a] = g->d[a];
        G.tile[a] = t;
        G.nt[a] = g->n[a] / t;
        G.tshift[a] = ilog2_exact(t);
        G.ntiles *= G.nt[a];
        G.cells *= g->n[a];
    }
    for (int a = 1; a < g->ndim; ++a)
        if (G.tile[a] != G.tile[0]) return fail(err, PIC_E_UNSUPPORTED, "tiles must be square / cubic");
    // packed cell index of the mixed mode
    int used = 0;
    for (int a = 0; a < g->ndim; ++a) {
        G.csh[a] = used;
        const int b = bits_for(G.n[a]);
        G.cmask[a] = (b >= 32) ? 0xFFFFFFFFu : ((1u << b) - 1u);
        used += b;
    }
    if (used > 32) return fail(err, PIC_E_UNSUPPORTED, "grid too large for the packed 32-bit cell index");
    const int64_t tile_cells = (int64_t)G.tile[0] * G.tile[1] * G.tile[2];
    int64_t id_total = 0;
    for (int s = 0; s < ns; ++s) {
        const pic_species_desc &S = sp[s];
        if (S.ppc <= 0) return fail(err, PIC_E_INVALID_ARG, "species %d: ppc %d", s, S.ppc);
        if (!(S.mass > 0.0)) return fail(err, PIC_E_INVALID_ARG, "species %d: mass must be positive", s);
        if (!(S.density >= 0.0)) return fail(err, PIC_E_INVALID_ARG, "species %d: density must be >= 0", s);
        if (S.nu_coll < 0.0) return fail(err, PIC_E_INVALID_ARG, "species %d: nu_coll < 0", s);
        if (!(S.u_th >= 0.0)) return fail(err, PIC_E_INVALID_ARG, "species %d: u_th < 0", s);
        if (S.coll_model != PIC_COLL_ISOTROPIC && S.coll_model != PIC_COLL_COULOMB)
            return fail(err, PIC_E_INVALID_ARG, "species %d: coll_model %d", s, S.coll_model);
        if (S.coll_model == PIC_COLL_COULOMB && S.nu_coll > 0.0 && !(S.coll_vref > 0.0 && S.coll_vref < 1.0))
            return fail(err, PIC_E_INVALID_ARG, "species %d: Coulomb scattering needs 0 < coll_vref < 1", s);
        if (S.binary != 0 && S.binary != 1) return fail(err, PIC_E_INVALID_ARG, "species %d: binary %d", s, S.binary);
        if (S.cancel_current_of >= ns || S.cancel_current_of < -1)
            return fail(err, PIC_E_INVALID_ARG, "species %d: cancel_current_of %d", s, S.cancel_current_of);
        Layout::Sp &P = L->sp[s];
        P.tile_nominal = (int64_t)S.ppc * tile_cells;
        P.nominal = P.tile_nominal * G.ntiles;
        P.reserve = std::max<int64_t>(64, (int64_t)std::ceil(reserve * (double)P.tile_nominal));
        // bins of kBinAlign-multiple capacity start on cache-line boundaries
        P.reserve = (P.tile_nominal + P.reserve + kBinAlign - 1) / kBinAlign * kBinAlign - P.tile_nominal;
        P.ncap = (P.tile_nominal + P.reserve) * G.ntiles;
        if (P.ncap * (g->precision == PIC_PREC_MIXED ? 4 : 8) >= ((int64_t)1 << 32))
            return fail(err, PIC_E_UNSUPPORTED, "species %d: a particle array would exceed 4 GiB", s);
        P.ovf_cap = (uint32_t)std::max<int64_t>(4096, P.ncap / 8);
        id_total += P.nominal;
    }
    if (id_total > 0xFFFFFFFFll) return fail(err, PIC_E_UNSUPPORTED, "more than 2^32 particles: ids do not fit");
    L->real = g->precision == PIC_PREC_MIXED ? 4 : 8;
    L->nj = G.tile[0] + 3;
    // particle buffers
    for (int s = 0; s < ns; ++s) {
        Layout::Sp &P = L->sp[s];
        Carver c;
        for (int set = 0; set < 3; ++set) {
            const size_t n = set < 2 ? (size_t)P.ncap : P.ovf_cap;
            // mixed: 16-bit in-tile cells in the bins, global 32-bit cells in the overflow list
            P.cell[set] = L->real == 4 ? c.take(n * (set < 2 ? 2 : 4)) : 0;
            for (int a = 0; a < 3; ++a) P.pos[set][a] = a < g->ndim ? c.take(n * L->real) : 0;
            for (int a = 0; a < 3; ++a) P.u[set][a] = c.take(n * L->real);
            P.id[set] = c.take(n * 4);
        }
        P.start = c.take((size_t)G.ntiles * 4);
        P.cap = c.take((size_t)G.ntiles * 4);
        P.cnt_front = c.take((size_t)G.ntiles * 8);
        P.cnt_back = c.take((size_t)G.ntiles * 8);
        L->particle_bytes[s] = c.off;
    }
    {
        Carver c;
        L->F = c.take((size_t)G.cells * 6 * L->real);
        L->J = c.take((size_t)G.cells * 3 * 8);
        L->field_bytes = c.off;
    }
    {
        Carver c;
        int64_t nj_cells = 1;
        for (int a = 0; a < g->ndim; ++a) nj_cells *= L->nj;
        L->Jtile = c.take((size_t)G.ntiles * 3 * nj_cells * L->real);
        L->tile_diag = c.take((size_t)G.ntiles * ns * kTileDiag * 8);
        L->field_diag = c.take((size_t)kFieldDiagBlocks * kFieldDiag * 8);
        L->moments = c.take((size_t)kMomentBlocks * kMomentVals * 8);
        L->state = c.take(sizeof(DevState));
        L->kparams = c.take(sizeof(KParams));
        for (int i = 0; i < 4; ++i) L->rb[i] = c.take((size_t)ns * G.ntiles * 4);
        L->order = c.take((size_t)G.ntiles * 4);
        L->bucket = c.take((size_t)G.ntiles);
        L->ee_tile = c.take((size_t)G.ntiles * 8);
        {
            // binary collisions: one 32-bit entry (slot | species << 29) per
            // store slot of each participating species
            int64_t ent = 0;
            const bool ee_on = g->nu_ee > 0.0 && !(g->flags & PIC_FLAG_NO_COLLIDE);
            for (int s = 0; ee_on && s < ns; ++s)
                if (sp[s].binary) {
                    if (L->sp[s].ncap >= ((int64_t)1 << 29))
                        return fail(err, PIC_E_CAPACITY, "species %d: binary collisions need a store below 2^29 "
                                    "slots (%lld)", s, (long long)L->sp[s].ncap);
                    ent += L->sp[s].ncap;
                }
            if (ent > 0) L->ee_ent = c.take((size_t)ent * 4);
        }
        L->checks = (g->flags & PIC_FLAG_GAUSS_RESIDUAL) != 0;
        if (L->checks) {
            int64_t n1 = 1;
            for (int a = 0; a < g->ndim; ++a) n1 *= G.tile[0] + 1;
            L->rho_tile = c.take((size_t)G.ntiles * n1 * 8);
            L->rho0 = c.take((size_t)G.cells * 8);
            L->rho_n = c.take((size_t)G.cells * 8);
            L->gauss_part = c.take((size_t)((G.cells + 255) / 256) * 2 * 8);
            L->cont_part = c.take((size_t)((G.cells + 255) / 256) * 2 * 8);
        }
        L->scratch_bytes = c.off;
    }
    L->diag_bytes = align256(sizeof(pic_diag) * kRing);
    return PIC_OK;
}

}  // namespace

struct pic_run {
    pic_grid_desc grid;
    pic_species_desc species[kMaxSpecies];
    int ns = 0;
    Layout L;
    pic_buffers buf;
    hipStream_t stream = nullptr;
    KParams hp;                 // host copy of the device-resident parameters
    KParams *dp = nullptr;      // device copy (inside scratch)
    int64_t steps_enqueued = 0;
    int64_t graph_launches = 0;  // steps enqueued as one graph replay
    int64_t direct_steps = 0;    // steps enqueued kernel by kernel
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    pic_batch *owner = nullptr;  // batch this run is a member of
    int static_device = -1;      // device whose library scratch this run holds (pic_init_static_scratch)
    std::string err;
};

struct pic_batch {
    std::vector<pic_run *> runs;
    int precision = 0, ndim = 0;
    hipStream_t stream = nullptr;
    BatchTable ht;              // host copy (device pointers inside)
    BatchTable *dt = nullptr;   // device copy (inside the caller's table buffer)
    int pblocks[kBatchGroups] = {0, 0, 0};
    int64_t graph_launches = 0, direct_steps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::string err;
};

namespace {

int hip_fail(pic_run *r, hipError_t e, const char *what)
{
    char buf[512];
    snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
    if (r) r->err = buf;
    g_last_error = buf;
    return PIC_E_HIP;
}

#define HIPCHK(r, expr)                                   \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(r, e_, #expr); \
    } while (0)

char *at(void *base, size_t off) { return (char *)base + off; }

// Uniform bin layout: capacity tile_nominal + reserve per tile.
void uniform_bins(const Layout::Sp &P, int ntiles, std::vector<int32_t> &start, std::vector<int32_t> &cap)
{
    start.resize(ntiles);
    cap.resize(ntiles);
    for (int t = 0; t < ntiles; ++t) {
        cap[t] = (int32_t)(P.tile_nominal + P.reserve);
        start[t] = (int32_t)((int64_t)t * cap[t]);
    }
}

int upload_bins(pic_run *r, int s, const std::vector<int32_t> &start, const std::vector<int32_t> &cap,
                const std::vector<uint32_t> &front0)
{
    const int nt = r->L.g.ntiles;
    const Layout::Sp &P = r->L.sp[s];
    void *b = r->buf.particles[s];
    std::vector<uint32_t> zeros((size_t)2 * nt, 0u), fr((size_t)2 * nt, 0u);
    std::copy(front0.begin(), front0.end(), fr.begin());
    HIPCHK(r, hipMemcpyAsync(at(b, P.start), start.data(), nt * 4, hipMemcpyHostToDevice, r->stream));
    HIPCHK(r, hipMemcpyAsync(at(b, P.cap), cap.data(), nt * 4, hipMemcpyHostToDevice, r->stream));
    HIPCHK(r, hipMemcpyAsync(at(b, P.cnt_front), fr.data(), (size_t)2 * nt * 4, hipMemcpyHostToDevice, r->stream));
    HIPCHK(r, hipMemcpyAsync(at(b, P.cnt_back), zeros.data(), (size_t)2 * nt * 4, hipMemcpyHostToDevice, r->stream));
    HIPCHK(r, hipStreamSynchronize(r->stream));
    return PIC_OK;
}

int read_state(pic_run *r, DevState *st)
{
    HIPCHK(r, hipStreamSynchronize(r->stream));
    HIPCHK(r, hipMemcpy(st, at(r->buf.scratch, r->L.state), sizeof(DevState), hipMemcpyDeviceToHost));
    return PIC_OK;
}

int check_fatal(pic_run *r, const DevState &st)
{
    if (st.fatal & 1) { r->err = "particle overflow list exhausted"; return PIC_E_CAPACITY; }
    if (st.fatal & 4) { r->err = "particle store reserve exhausted"; return PIC_E_CAPACITY; }
    if (st.fatal & 2) { r->err = "particle left the grid (corrupt state)"; return PIC_E_HIP; }
    if (st.fatal & 8) { r->err = "particle outside its tile's bin (corrupt state)"; return PIC_E_HIP; }
    if (st.fatal & 16) {
        r->err = "binary collisions: a cell holds more than 4096 participants";
        return PIC_E_CAPACITY;
    }
    return PIC_OK;
}

int moments(pic_run *r, int s, double delta, double out[kMomentVals])
{
    HIPCHK(r, launch_moments(r->hp, r->dp, s, delta, r->stream));
    std::vector<double> h((size_t)kMomentBlocks * kMomentVals);
    HIPCHK(r, hipMemcpyAsync(h.data(), at(r->buf.scratch, r->L.moments), h.size() * 8, hipMemcpyDeviceToHost,
                             r->stream));
    HIPCHK(r, hipStreamSynchronize(r->stream));
    for (int v = 0; v < kMomentVals; ++v) {
        double a = 0.0;
        for (int b = 0; b < kMomentBlocks; ++b) a += h[(size_t)b * kMomentVals + v];
        out[v] = a;
    }
    return PIC_OK;
}

// Loader post-processing: remove mean u_x, u_y per species; Newton shift of
// the cancelling species' u_z so that sum_s q_s w_s sum u_z/gamma = 0.
int loader_moments(pic_run *r)
{
    double m[kMomentVals];
    for (int s = 0; s < r->ns; ++s) {
        int rc = moments(r, s, 0.0, m);
        if (rc) return rc;
        if (m[5] > 0) {
            HIPCHK(r, launch_shift_u(r->hp, r->dp, s, -m[0] / m[5], -m[1] / m[5], 0.0, r->stream));
        }
    }
    for (int c = 0; c < r->ns; ++c) {
        if (r->species[c].cancel_current_of < 0) continue;
        const double qwc = r->hp.sp[c].qw;
        if (qwc == 0.0) continue;
        for (int round = 0; round < 2; ++round) {
            double other = 0.0;
            for (int s = 0; s < r->ns; ++s) {
                if (s == c) continue;
                int rc = moments(r, s, 0.0, m);
                if (rc) return rc;
                other += r->hp.sp[s].qw * m[4];
            }
            int rc = moments(r, c, 0.0, m);
            if (rc) return rc;
            const double nc = std::max(m[5], 1.0);
            double vt = -other / (qwc * nc);
            vt = std::max(-0.99, std::min(0.99, vt));
            double delta = round == 0 ? vt / std::sqrt(1.0 - vt * vt) - r->species[c].drift_u[2] : 0.0;
            for (int it = 0; it < 60; ++it) {
                rc = moments(r, c, delta, m);
                if (rc) return rc;
                const double f = other + qwc * m[2];
                const double fp = qwc * m[3];
                if (fp == 0.0) break;
                const double step = f / fp;
                delta -= step;
                if (std::fabs(step) <= 1e-16 * std::max(1.0, std::fabs(delta))) break;
            }
            HIPCHK(r, launch_shift_u(r->hp, r->dp, c, 0.0, 0.0, delta, r->stream));
        }
    }
    HIPCHK(r, hipStreamSynchronize(r->stream));
    return PIC_OK;
}

// Captures one step as a graph on a private stream.  A failure is returned
// as PIC_E_HIP (the caller can ask for kernel-by-kernel steps with
// PIC_FLAG_NO_GRAPH instead).
int capture_graph(pic_run *r)
{
    hipStream_t cs;
    HIPCHK(r, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const char *what = "hipStreamBeginCapture";
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        hipError_t le = launch_step(r->hp, r->dp, cs);
        hipGraph_t g = nullptr;
        what = "hipStreamEndCapture";
        e = hipStreamEndCapture(cs, &g);
        if (le != hipSuccess) {
            e = le;
            what = "step launch under capture";
        }
        if (e == hipSuccess) {
            what = "hipGraphInstantiate";
            e = hipGraphInstantiate(&r->gexec, g, nullptr, nullptr, 0);
            if (e == hipSuccess) r->graph = g;
            else (void)hipGraphDestroy(g);
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        r->gexec = nullptr;
        r->graph = nullptr;
        (void)hipGetLastError();
        return hip_fail(r, e, what);
    }
    return PIC_OK;
}

// Device table of a batch: BatchTable | kp[nruns] | cell blocks | work items
// of each tile group | one queue counter per group.
struct BatchLayout {
    size_t table, kp, cell_blocks, items[kBatchGroups], queues, bytes;
    int n_cell_blocks, n_items[kBatchGroups];
};

int tile_group(const pic_run *r)
{
    return r->L.g.tile[0] == 8 ? 0 : (r->L.g.tile[0] == 16 ? 1 : 2);
}

int batch_carve(int nruns, int64_t ncb, const int64_t nit[kBatchGroups], BatchLayout *B, std::string *err)
{
    if (ncb > INT32_MAX / 2) return fail(err, PIC_E_UNSUPPORTED, "batch too large");
    B->n_cell_blocks = (int)ncb;
    for (int g = 0; g < kBatchGroups; ++g) {
        if (nit[g] > INT32_MAX / 2) return fail(err, PIC_E_UNSUPPORTED, "batch too large");
        B->n_items[g] = (int)nit[g];
    }
    Carver c;
    B->table = c.take(sizeof(BatchTable));
    B->kp = c.take((size_t)nruns * sizeof(void *));
    B->cell_blocks = c.take((size_t)B->n_cell_blocks * sizeof(int2));
    for (int g = 0; g < kBatchGroups; ++g) B->items[g] = c.take((size_t)B->n_items[g] * sizeof(int2));
    B->queues = c.take(kBatchGroups * kBatchXcds * sizeof(int));
    B->bytes = c.off;
    return PIC_OK;
}

int batch_layout(int nruns, pic_run *const *runs, BatchLayout *B, std::string *err)
{
    if (nruns < 1 || !runs) return fail(err, PIC_E_INVALID_ARG, "batch needs at least one run");
    memset(B, 0, sizeof(*B));
    int64_t ncb = 0, nit[kBatchGroups] = {0, 0, 0};
    for (int i = 0; i < nruns; ++i) {
        const pic_run *r = runs[i];
        if (!r) return fail(err, PIC_E_INVALID_ARG, "run %d is NULL", i);
        if (r->grid.precision != runs[0]->grid.precision || r->grid.ndim != runs[0]->grid.ndim)
            return fail(err, PIC_E_UNSUPPORTED, "run %d: members must share precision and ndim", i);
        if (r->grid.flags & PIC_FLAG_GAUSS_RESIDUAL)
            return fail(err, PIC_E_UNSUPPORTED, "run %d: PIC_FLAG_GAUSS_RESIDUAL is for single runs", i);
        if (r->hp.binary)
            return fail(err, PIC_E_UNSUPPORTED, "run %d: binary collisions are for single runs", i);
        for (int j = 0; j < i; ++j)
            if (runs[j] == r) return fail(err, PIC_E_INVALID_ARG, "run %d listed twice", i);
        ncb += (r->L.g.cells + 255) / 256;
        nit[tile_group(r)] += r->L.g.ntiles;
    }
    return batch_carve(nruns, ncb, nit, B, err);
}

// Run-level or batch-level profiled steps: `launch(ev)` enqueues one step
// whose nk dispatches record start/stop into ev[2k], ev[2k+1].
template <typename F>
int profiled_steps(std::string *err, hipStream_t st, int32_t nsteps, int nk, const int *kgroup, double *group_ms,
                   F launch)
{
    for (int g = 0; g < kNumGroups; ++g) group_ms[g] = 0.0;
    if (nsteps == 0) return PIC_OK;
    const int ne = 2 * nk;
    std::vector<hipEvent_t> ev((size_t)nsteps * ne, nullptr);
    int rc = PIC_OK;
    auto hfail = [&](hipError_t e, const char *what) {
        return fail(err, PIC_E_HIP, "%s: %s", what, hipGetErrorString(e));
    };
    for (auto &e : ev) {
        hipError_t he = hipEventCreate(&e);
        if (he != hipSuccess) { rc = hfail(he, "hipEventCreate"); break; }
    }
    for (int32_t i = 0; rc == PIC_OK && i < nsteps; ++i) {
        hipError_t he = launch(&ev[(size_t)i * ne]);
        if (he != hipSuccess) rc = hfail(he, "step launch");
    }
    if (rc == PIC_OK) {
        hipError_t he = hipStreamSynchronize(st);
        if (he != hipSuccess) rc = hfail(he, "hipStreamSynchronize");
    }
    for (int32_t i = 0; rc == PIC_OK && i < nsteps; ++i)
        for (int k = 0; k < nk; ++k) {
            float ms = 0.f;
            hipError_t he = hipEventElapsedTime(&ms, ev[(size_t)i * ne + 2 * k], ev[(size_t)i * ne + 2 * k + 1]);
            if (he != hipSuccess) { rc = hfail(he, "hipEventElapsedTime"); break; }
            group_ms[kgroup[k]] += ms;
        }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

// One step of a batch captured as a graph; a failure is returned (hipError_t
// and the call that failed in *what).
hipError_t capture_batch_graph(pic_batch *b, const char **what)
{
    hipStream_t cs;
    *what = "hipStreamCreateWithFlags";
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    *what = "hipStreamBeginCapture";
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        hipError_t le = launch_batch_step(b->precision, b->ndim, b->ht, b->dt, b->pblocks, cs);
        hipGraph_t g = nullptr;
        *what = "hipStreamEndCapture";
        e = hipStreamEndCapture(cs, &g);
        if (le != hipSuccess) {
            e = le;
            *what = "batch step launch under capture";
        }
        if (e == hipSuccess) {
            *what = "hipGraphInstantiate";
            e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
            if (e == hipSuccess) b->graph = g;
            else (void)hipGraphDestroy(g);
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        b->gexec = nullptr;
        b->graph = nullptr;
        (void)hipGetLastError();
    }
    return e;
}

int batch_hip_fail(pic_batch *b, hipError_t e, const char *what)
{
    return fail(&b->err, PIC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define BHIPCHK(b, expr)                                          \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return batch_hip_fail(b, e_, #expr); \
    } while (0)

// Tile autotuner: where each copy of a candidate run, and the batch table
// of the copies, sit inside the workspace.
struct TuneCarve {
    pic_sizes sz;
    size_t part[kMaxSpecies], fields, scratch, diag, per_copy, table, table_bytes, bytes;
};

// Descriptors compared field by field (their padding bytes are not data).
bool same_grid(const pic_grid_desc &a, const pic_grid_desc &b, uint32_t ignore_flags)
{
    bool same = a.ndim == b.ndim && a.dt == b.dt && a.precision == b.precision && a.seed == b.seed &&
                a.run == b.run && a.diag_every == b.diag_every && a.reserve == b.reserve &&
                a.nu_ee == b.nu_ee && a.ee_vref == b.ee_vref &&
                (a.flags & ~ignore_flags) == (b.flags & ~ignore_flags);
    for (int i = 0; i < 3; ++i) same = same && a.n[i] == b.n[i] && a.d[i] == b.d[i] && a.tile[i] == b.tile[i];
    return same;
}

bool same_species(const pic_species_desc &a, const pic_species_desc &b)
{
    bool same = a.charge == b.charge && a.mass == b.mass && a.density == b.density && a.ppc == b.ppc &&
                a.u_th == b.u_th && a.cancel_current_of == b.cancel_current_of && a.nu_coll == b.nu_coll &&
                a.coll_model == b.coll_model && a.coll_vref == b.coll_vref && a.binary == b.binary;
    for (int i = 0; i < 3; ++i) same = same && a.drift_u[i] == b.drift_u[i];
    return same;
}

// Copies with zeroed padding, so that the images kept in the handle and
// written into checkpoints do not carry the caller's stack bytes.
pic_grid_desc canonical_grid(const pic_grid_desc &g)
{
    pic_grid_desc c;
    memset(&c, 0, sizeof(c));
    c.ndim = g.ndim;
    for (int i = 0; i < 3; ++i) {
        c.n[i] = g.n[i];
        c.d[i] = g.d[i];
        c.tile[i] = g.tile[i];
    }
    c.dt = g.dt;
    c.precision = g.precision;
    c.seed = g.seed;
    c.run = g.run;
    c.diag_every = g.diag_every;
    c.flags = g.flags;
    c.reserve = g.reserve;
    c.nu_ee = g.nu_ee;
    c.ee_vref = g.ee_vref;
    c.shape = g.shape;
    return c;
}

pic_species_desc canonical_species(const pic_species_desc &s)
{
    pic_species_desc c;
    memset(&c, 0, sizeof(c));
    c.charge = s.charge;
    c.mass = s.mass;
    c.density = s.density;
    c.ppc = s.ppc;
    for (int i = 0; i < 3; ++i) c.drift_u[i] = s.drift_u[i];
    c.u_th = s.u_th;
    c.cancel_current_of = s.cancel_current_of;
    c.nu_coll = s.nu_coll;
    c.coll_model = s.coll_model;
    c.coll_vref = s.coll_vref;
    c.binary = s.binary;
    return c;
}

bool tile_fits(const pic_grid_desc *g, int t)
{
    if (g->ndim == 3 && t != 8) return false;
    for (int a = 0; a < g->ndim; ++a)
        if (g->n[a] % t) return false;
    return true;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace pic {
hipError_t launch_copy_probe(const uint32_t *const *src, uint32_t *const *dst, int narrays, int64_t n,
                             int64_t chunk, hipStream_t st);    // pic_probe.hip
}

extern "C" {

int pic_copy_probe(const void *const *src, void *const *dst, int narrays, int64_t n, int64_t chunk,
                   void *hip_stream)
{
    if (!src || !dst || narrays < 1 || narrays > 8 || n < 0 || chunk < 256 || chunk % 256)
        return fail(nullptr, PIC_E_INVALID_ARG, "copy probe: bad argument");
    for (int k = 0; k < narrays; ++k)
        if (!src[k] || !dst[k]) return fail(nullptr, PIC_E_INVALID_ARG, "copy probe: NULL array %d", k);
    if (n == 0) return PIC_OK;
    const hipError_t e = pic::launch_copy_probe((const uint32_t *const *)src, (uint32_t *const *)dst, narrays, n,
                                                chunk, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, PIC_E_HIP, "copy probe: %s", hipGetErrorString(e));
    return PIC_OK;
}

const char *pic_status_string(int status)
{
    switch (status) {
    case PIC_OK: return "ok";
    case PIC_E_INVALID_ARG: return "invalid argument";
    case PIC_E_UNSUPPORTED: return "unsupported configuration";
    case PIC_E_CFL: return "time step violates the Courant condition";
    case PIC_E_BUFFER_TOO_SMALL: return "buffer too small";
    case PIC_E_HIP: return "HIP runtime error";
    case PIC_E_STATE: return "invalid state for this call";
    case PIC_E_CAPACITY: return "particle store capacity exceeded";
    default: return "unknown status";
    }
}

int pic_last_error(pic_run *run, char *buf, size_t n)
{
    if (!buf || n == 0) return PIC_E_INVALID_ARG;
    const std::string &m = run ? run->err : g_last_error;
    snprintf(buf, n, "%s", m.c_str());
    return PIC_OK;
}

int pic_query(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies, pic_sizes *out)
{
    if (!out) return fail(nullptr, PIC_E_INVALID_ARG, "null output");
    Layout L;
    const int rc = validate(grid, species, nspecies, &L, nullptr);
    if (rc) return rc;
    memset(out, 0, sizeof(*out));
    for (int s = 0; s < nspecies; ++s) out->particle_bytes[s] = L.particle_bytes[s];
    out->field_bytes = L.field_bytes;
    out->scratch_bytes = L.scratch_bytes;
    out->diag_bytes = L.diag_bytes;
    return PIC_OK;
}

int pic_init(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
             const pic_buffers *buffers, void *hip_stream, pic_run **out)
{
    return pic::init_run(grid, species, nspecies, buffers, hip_stream, out, -1);
}

}  // extern "C"

namespace {
std::mutex g_static_mu;
bool g_static_busy[kMaxDevices] = {};
}  // namespace

bool pic::claim_static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return false;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_busy[device]) return false;
    g_static_busy[device] = true;
    return true;
}

void pic::release_static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static_busy[device] = false;
}

int pic::fail_global(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int pic::init_run(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
                  const pic_buffers *buffers, void *hip_stream, pic_run **out, int static_device)
{
    if (!out || !buffers) return fail(nullptr, PIC_E_INVALID_ARG, "null argument");
    *out = nullptr;
    pic_run *r = new (std::nothrow) pic_run();
    if (!r) return fail(nullptr, PIC_E_INVALID_ARG, "host allocation failed");
    r->static_device = static_device;
    int rc = validate(grid, species, nspecies, &r->L, &r->err);
    if (rc) { delete r; return rc; }
    for (int s = 0; s < nspecies; ++s)
        if (!buffers->particles[s]) { delete r; return fail(nullptr, PIC_E_INVALID_ARG, "null particle buffer %d", s); }
    if (!buffers->fields || !buffers->scratch || !buffers->diag) {
        delete r;
        return fail(nullptr, PIC_E_INVALID_ARG, "null field, scratch or diag buffer");
    }
    r->grid = canonical_grid(*grid);
    r->ns = nspecies;
    for (int s = 0; s < nspecies; ++s) r->species[s] = canonical_species(species[s]);
    r->buf = *buffers;
    r->stream = (hipStream_t)hip_stream;
    const Layout &L = r->L;

    KParams &K = r->hp;
    memset(&K, 0, sizeof(K));
    K.g = L.g;
    K.nspecies = nspecies;
    K.precision = grid->precision;
    K.diag_every = grid->diag_every;
    K.shape = grid->shape;
    K.flags = grid->flags;
    K.seed = grid->seed;
    K.run = grid->run;
    K.nj = L.nj;
    K.nu_ee = grid->nu_ee;
    K.ee_vref = grid->ee_vref;
    int64_t id_base = 0;
    for (int s = 0; s < nspecies; ++s) {
        const pic_species_desc &S = species[s];
        const Layout::Sp &P = L.sp[s];
        SpeciesDev &D = K.sp[s];
        void *b = buffers->particles[s];
        for (int set = 0; set < 3; ++set) {
            if (set < 2) D.cell[set] = L.real == 4 ? (uint16_t *)at(b, P.cell[set]) : nullptr;
            else D.ovf_cell = L.real == 4 ? (uint32_t *)at(b, P.cell[set]) : nullptr;
            for (int a = 0; a < 3; ++a) D.pos[set][a] = a < grid->ndim ? at(b, P.pos[set][a]) : nullptr;
            for (int a = 0; a < 3; ++a) D.u[set][a] = at(b, P.u[set][a]);
            D.id[set] = (uint32_t *)at(b, P.id[set]);
        }
        D.start = (int32_t *)at(b, P.start);
        D.cap = (int32_t *)at(b, P.cap);
        D.cnt_front = (uint32_t *)at(b, P.cnt_front);
        D.cnt_back = (uint32_t *)at(b, P.cnt_back);
        D.ncap = P.ncap;
        D.nominal = P.nominal;
        D.ovf_cap = P.ovf_cap;
        D.collide = (S.nu_coll > 0.0 && !(grid->flags & PIC_FLAG_NO_COLLIDE)) ? 1 : 0;
        D.binary = (S.binary && grid->nu_ee > 0.0 && !(grid->flags & PIC_FLAG_NO_COLLIDE)) ? 1 : 0;
        if (D.binary) K.binary = 1;
        D.track_id = (D.collide || D.binary || (grid->flags & PIC_FLAG_TRACK_IDS)) ? 1 : 0;
        const double P_coll = 1.0 - std::exp(-S.nu_coll * grid->dt);
        const double thr = std::floor(P_coll * 4294967296.0);
        D.coll_thr = D.collide ? (uint32_t)std::min(4294967295.0, std::max(0.0, thr)) : 0u;
        D.coll_model = S.coll_model;
        D.coll_sig2 = S.coll_model == PIC_COLL_COULOMB
                          ? 0.5 * S.nu_coll * grid->dt * S.coll_vref * S.coll_vref * S.coll_vref
                          : 0.0;
        if (D.collide && D.coll_model == PIC_COLL_COULOMB) K.coulomb = 1;
        D.q = S.charge;
        D.m = S.mass;
        D.w = S.density / S.ppc;
        D.qmdt2 = S.charge * grid->dt / (2.0 * S.mass);
        D.qw = S.charge * D.w;
        D.ppc = S.ppc;
        D.id_base = (int32_t)id_base;
        for (int c = 0; c < 3; ++c) D.drift[c] = S.drift_u[c];
        D.uth = S.u_th;
        id_base += P.nominal;
    }
    K.F = at(buffers->fields, L.F);
    K.J = (double *)at(buffers->fields, L.J);
    K.Jtile = at(buffers->scratch, L.Jtile);
    K.tile_diag = (double *)at(buffers->scratch, L.tile_diag);
    K.field_diag = (double *)at(buffers->scratch, L.field_diag);
    K.moments = (double *)at(buffers->scratch, L.moments);
    K.state = (DevState *)at(buffers->scratch, L.state);
    K.ring = (pic_diag *)buffers->diag;
    K.rb_count = (int32_t *)at(buffers->scratch, L.rb[0]);
    K.rb_start = (int32_t *)at(buffers->scratch, L.rb[1]);
    K.rb_cap = (int32_t *)at(buffers->scratch, L.rb[2]);
    K.rb_fill = (int32_t *)at(buffers->scratch, L.rb[3]);
    r->dp = (KParams *)at(buffers->scratch, L.kparams);
    K.fd_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kFieldDiagBlocks, (L.g.cells + 2047) / 2048));
    K.order = (int32_t *)at(buffers->scratch, L.order);
    K.ee_tile = (int64_t *)at(buffers->scratch, L.ee_tile);
    K.ee_ent = L.ee_ent ? (uint32_t *)at(buffers->scratch, L.ee_ent) : nullptr;
    K.tile_bucket = (uint8_t *)at(buffers->scratch, L.bucket);
    if (L.checks) {
        K.rho_tile = (double *)at(buffers->scratch, L.rho_tile);
        K.rho0 = (double *)at(buffers->scratch, L.rho0);
        K.rho_n = (double *)at(buffers->scratch, L.rho_n);
        K.gauss_part = (double *)at(buffers->scratch, L.gauss_part);
        K.cont_part = (double *)at(buffers->scratch, L.cont_part);
    }
    {
        int64_t per_tile = 0;
        for (int s = 0; s < nspecies; ++s) per_tile += L.sp[s].tile_nominal;
        K.order_scale = 16.0 / (double)std::max<int64_t>(1, per_tile);
    }

#define INIT_CHK(expr)                                          \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) {                                 \
            int c_ = hip_fail(r, e_, #expr);                    \
            delete r;                                           \
            return c_;                                          \
        }                                                       \
    } while (0)
    INIT_CHK(hipMemcpyAsync(r->dp, &K, sizeof(K), hipMemcpyHostToDevice, r->stream));
    INIT_CHK(hipMemsetAsync(buffers->fields, 0, L.field_bytes, r->stream));
    INIT_CHK(hipMemsetAsync(K.Jtile, 0, L.tile_diag - L.Jtile, r->stream));
    INIT_CHK(hipMemsetAsync(K.tile_diag, 0, L.state - L.tile_diag, r->stream));
    INIT_CHK(hipMemsetAsync(buffers->diag, 0, L.diag_bytes, r->stream));
    DevState st0;
    memset(&st0, 0, sizeof(st0));
    INIT_CHK(hipMemcpyAsync(K.state, &st0, sizeof(st0), hipMemcpyHostToDevice, r->stream));
    std::vector<int32_t> iota((size_t)L.g.ntiles);
    for (int t = 0; t < L.g.ntiles; ++t) iota[t] = t;
    INIT_CHK(hipMemcpyAsync(K.order, iota.data(), iota.size() * 4, hipMemcpyHostToDevice, r->stream));
    INIT_CHK(hipMemsetAsync(K.tile_bucket, 0, (size_t)L.g.ntiles, r->stream));
    for (int s = 0; s < nspecies; ++s) {
        std::vector<int32_t> start, cap;
        uniform_bins(L.sp[s], L.g.ntiles, start, cap);
        const bool load = !(grid->flags & PIC_FLAG_HOST_LOAD);
        std::vector<uint32_t> front((size_t)L.g.ntiles, load ? (uint32_t)L.sp[s].tile_nominal : 0u);
        rc = upload_bins(r, s, start, cap, front);
        if (rc) { delete r; return rc; }
        if (load) INIT_CHK(launch_load_species(K, r->dp, s, r->stream));
    }
    if (!(grid->flags & PIC_FLAG_HOST_LOAD)) {
        rc = loader_moments(r);
        if (rc) { delete r; return rc; }
    }
    INIT_CHK(hipStreamSynchronize(r->stream));
    if (!(grid->flags & PIC_FLAG_NO_GRAPH)) {
        rc = capture_graph(r);
        if (rc) {
            g_last_error = r->err;
            delete r;
            return rc;
        }
    }
    *out = r;
    return PIC_OK;
}

extern "C" {

int pic_load_particles(pic_run *r, int s, const double *x, const double *u, const uint32_t *id, int64_t n)
{
    if (!r) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    if (s < 0 || s >= r->ns) return fail(&r->err, PIC_E_INVALID_ARG, "species %d", s);
    if (n < 0 || (n > 0 && (!x || !u || !id))) return fail(&r->err, PIC_E_INVALID_ARG, "bad particle arrays");
    const Layout &L = r->L;
    const Layout::Sp &P = L.sp[s];
    if (n > P.nominal) return fail(&r->err, PIC_E_BUFFER_TOO_SMALL, "n = %lld exceeds ppc*cells = %lld",
                                   (long long)n, (long long)P.nominal);
    if (r->steps_enqueued != 0) return fail(&r->err, PIC_E_STATE, "particles can only be loaded before the first step");
    const Geometry &G = L.g;
    const int nd = G.ndim;
    const int nt = G.ntiles;
    std::vector<int> cellc((size_t)n * nd), tile((size_t)n);
    std::vector<double> off((size_t)n * nd);
    std::vector<int64_t> count(nt, 0);
    for (int64_t p = 0; p < n; ++p) {
        int t = 0, mul = 1;
        for (int a = 0; a < nd; ++a) {
            const double Lx = G.n[a] * G.d[a];
            double xa = std::fmod(x[(size_t)a * n + p], Lx);
            if (xa < 0) xa += Lx;
            double X = xa / G.d[a];
            int ic = (int)std::floor(X);
            double o = X - ic;
            if (L.real == 4) {
                float of = (float)o;
                if (of >= 1.0f) { of = 0.0f; ic += 1; }
                o = of;
            } else if (o >= 1.0) { o = 0.0; ic += 1; }
            if (ic >= G.n[a]) ic -= G.n[a];
            if (ic < 0) ic += G.n[a];
            cellc[(size_t)p * nd + a] = ic;
            off[(size_t)p * nd + a] = o;
            t += (ic >> G.tshift[a]) * mul;
            mul *= G.nt[a];
        }
        tile[p] = t;
        count[t] += 1;
    }
    // reserve of tile t: m + floor(rest * count_t / n), the device re-layout's rule
    const int64_t slack = P.ncap - n;
    const int64_t m = std::min<int64_t>(64, slack / (2 * (int64_t)nt));
    const int64_t rest = slack - m * nt;
    std::vector<int32_t> start(nt), cap(nt);
    std::vector<uint32_t> front(nt);
    int64_t o = 0;
    for (int t = 0; t < nt; ++t) {
        const int64_t c = count[t];
        const int64_t v = c + m + (n > 0 ? rest * c / n : rest / nt);
        // rounded to kBinAlign slots, as the device re-layout does
        const int64_t cp = std::max((c + kBinAlign - 1) / kBinAlign * kBinAlign, v / kBinAlign * kBinAlign);
        start[t] = (int32_t)o;
        cap[t] = (int32_t)cp;
        front[t] = (uint32_t)c;
        o += cp;
    }
    if (o > P.ncap) return fail(&r->err, PIC_E_CAPACITY, "species %d: %lld particles do not fit the store", s,
                                (long long)n);
    // Inside each tile, order by (rank of the particle within its cell, cell):
    // consecutive slots then hold particles of different cells, which keeps
    // the lanes of a wave off each other's LDS current words.
    const int64_t tile_cells = (int64_t)G.tile[0] * G.tile[1] * G.tile[2];
    std::vector<int64_t> key((size_t)n);
    {
        std::vector<int32_t> rank_in_cell((size_t)G.cells, 0);
        for (int64_t p = 0; p < n; ++p) {
            int64_t cell = 0, local = 0, mul = 1, lmul = 1;
            for (int a = 0; a < nd; ++a) {
                const int ic = cellc[(size_t)p * nd + a];
                cell += ic * mul;
                mul *= G.n[a];
                local += (ic & (G.tile[a] - 1)) * lmul;
                lmul *= G.tile[a];
            }
            key[p] = (int64_t)rank_in_cell[cell]++ * tile_cells + local;
        }
    }
    std::vector<int64_t> order((size_t)n);
    for (int64_t p = 0; p < n; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        return tile[a] != tile[b] ? tile[a] < tile[b] : key[a] < key[b];
    });
    std::vector<int64_t> fill(start.begin(), start.end());
    const size_t R = L.real;
    const size_t ncap = (size_t)P.ncap;
    std::vector<uint16_t> hcell(R == 4 ? ncap : 0);
    std::vector<uint32_t> hid(ncap, 0xFFFFFFFFu);
    std::vector<char> hpos[3], hu[3];
    for (int a = 0; a < nd; ++a) hpos[a].assign(ncap * R, 0);
    for (int c = 0; c < 3; ++c) hu[c].assign(ncap * R, 0);
    for (int64_t o = 0; o < n; ++o) {
        const int64_t p = order[o];
        const int64_t slot = fill[tile[p]]++;
        if (R == 4) {
            uint32_t c = 0;     // cell within the tile
            for (int a = 0; a < nd; ++a)
                c |= ((uint32_t)cellc[(size_t)p * nd + a] & (uint32_t)(G.tile[a] - 1)) << (a * G.tshift[0]);
            hcell[slot] = (uint16_t)c;
            for (int a = 0; a < nd; ++a) ((float *)hpos[a].data())[slot] = (float)off[(size_t)p * nd + a];
            for (int c3 = 0; c3 < 3; ++c3) ((float *)hu[c3].data())[slot] = (float)u[(size_t)c3 * n + p];
        } else {
            for (int a = 0; a < nd; ++a)
                ((double *)hpos[a].data())[slot] = cellc[(size_t)p * nd + a] + off[(size_t)p * nd + a];
            for (int c3 = 0; c3 < 3; ++c3) ((double *)hu[c3].data())[slot] = u[(size_t)c3 * n + p];
        }
        hid[slot] = id[p];
    }
    void *b = r->buf.particles[s];
    if (R == 4) HIPCHK(r, hipMemcpy(at(b, P.cell[0]), hcell.data(), ncap * 2, hipMemcpyHostToDevice));
    for (int a = 0; a < nd; ++a) HIPCHK(r, hipMemcpy(at(b, P.pos[0][a]), hpos[a].data(), ncap * R, hipMemcpyHostToDevice));
    for (int c3 = 0; c3 < 3; ++c3) HIPCHK(r, hipMemcpy(at(b, P.u[0][c3]), hu[c3].data(), ncap * R, hipMemcpyHostToDevice));
    HIPCHK(r, hipMemcpy(at(b, P.id[0]), hid.data(), ncap * 4, hipMemcpyHostToDevice));
    return upload_bins(r, s, start, cap, front);
}

int pic_step(pic_run *r, int32_t nsteps)
{
    if (!r) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    if (nsteps < 0) return fail(&r->err, PIC_E_INVALID_ARG, "nsteps < 0");
    if (r->owner) return fail(&r->err, PIC_E_STATE, "run is a member of a batch; step the batch");
    for (int32_t i = 0; i < nsteps; ++i) {
        if (r->gexec) {
            HIPCHK(r, hipGraphLaunch(r->gexec, r->stream));
            r->graph_launches += 1;
        } else {
            HIPCHK(r, launch_step(r->hp, r->dp, r->stream));
            r->direct_steps += 1;
        }
        r->steps_enqueued += 1;
    }
    return PIC_OK;
}

int pic_info(pic_run *r, pic_run_info *out)
{
    if (!r || !out) return fail(r ? &r->err : nullptr, PIC_E_INVALID_ARG, "null argument");
    memset(out, 0, sizeof(*out));
    out->graph = r->gexec ? 1 : 0;
    out->static_scratch = r->static_device >= 0 ? 1 : 0;
    out->steps_enqueued = r->steps_enqueued;
    out->graph_launches = r->graph_launches;
    out->direct_steps = r->direct_steps;
    out->scratch_bytes = r->L.scratch_bytes;
    out->shape = r->hp.shape;
    out->block_threads = kShapeBlock[r->hp.shape];
    out->inflight = kShapeInflight[r->hp.shape];
    return PIC_OK;
}

int pic_step_profiled(pic_run *r, int32_t nsteps, double *group_ms)
{
    if (!r || !group_ms) return fail(r ? &r->err : nullptr, PIC_E_INVALID_ARG, "bad argument");
    if (nsteps < 0) return fail(&r->err, PIC_E_INVALID_ARG, "nsteps < 0");
    if (r->owner) return fail(&r->err, PIC_E_STATE, "run is a member of a batch; step the batch");
    int groups[32];
    const int nk = step_kernel_groups(r->hp, groups);
    if (nk <= 0 || nk > 32) return fail(&r->err, PIC_E_UNSUPPORTED, "no kernel sequence for this run");
    return profiled_steps(&r->err, r->stream, nsteps, nk, groups, group_ms, [&](hipEvent_t *ev) {
        hipError_t e = launch_step(r->hp, r->dp, r->stream, ev);
        if (e == hipSuccess) {
            r->steps_enqueued += 1;
            r->direct_steps += 1;
        }
        return e;
    });
}

int pic_sync(pic_run *r)
{
    if (!r) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    DevState st;
    int rc = read_state(r, &st);
    if (rc) return rc;
    return check_fatal(r, st);
}

int pic_diag_history(pic_run *r, pic_diag *out, int64_t max, int64_t *count)
{
    if (!r || !out || !count || max < 0) return fail(r ? &r->err : nullptr, PIC_E_INVALID_ARG, "bad argument");
    DevState st;
    int rc = read_state(r, &st);
    if (rc) return rc;
    rc = check_fatal(r, st);
    if (rc) return rc;
    const int64_t avail = std::min<int64_t>(st.ring_head, kRing);
    const int64_t n = std::min(avail, max);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t rec = st.ring_head - n + i;
        HIPCHK(r, hipMemcpy(&out[i], (char *)r->buf.diag + (rec % kRing) * sizeof(pic_diag), sizeof(pic_diag),
                            hipMemcpyDeviceToHost));
    }
    *count = n;
    return PIC_OK;
}

int pic_diagnostics(pic_run *r, pic_diag *out)
{
    if (!r || !out) return fail(r ? &r->err : nullptr, PIC_E_INVALID_ARG, "bad argument");
    int64_t n = 0;
    int rc = pic_diag_history(r, out, 1, &n);
    if (rc) return rc;
    if (n == 0) return fail(&r->err, PIC_E_STATE, "no diagnostic record yet");
    return PIC_OK;
}

int pic_read_fields(pic_run *r, double *E, double *B, double *J)
{
    if (!r) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    HIPCHK(r, hipStreamSynchronize(r->stream));
    const size_t cells = (size_t)r->L.g.cells;
    const size_t R = r->L.real;
    std::vector<char> h(cells * 6 * R);
    HIPCHK(r, hipMemcpy(h.data(), at(r->buf.fields, r->L.F), h.size(), hipMemcpyDeviceToHost));
    for (int c = 0; c < 6; ++c) {
        double *dst = c < 3 ? E : B;
        if (!dst) continue;
        dst += (size_t)(c % 3) * cells;
        for (size_t o = 0; o < cells; ++o)
            dst[o] = R == 4 ? (double)((const float *)h.data())[c * cells + o] : ((const double *)h.data())[c * cells + o];
    }
    if (J) HIPCHK(r, hipMemcpy(J, at(r->buf.fields, r->L.J), cells * 3 * 8, hipMemcpyDeviceToHost));
    return PIC_OK;
}

int pic_write_fields(pic_run *r, const double *E, const double *B)
{
    if (!r) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    HIPCHK(r, hipStreamSynchronize(r->stream));
    const size_t cells = (size_t)r->L.g.cells;
    const size_t R = r->L.real;
    for (int c = 0; c < 6; ++c) {
        const double *src = c < 3 ? E : B;
        if (!src) continue;
        src += (size_t)(c % 3) * cells;
        std::vector<char> h(cells * R);
        for (size_t o = 0; o < cells; ++o) {
            if (R == 4) ((float *)h.data())[o] = (float)src[o];
            else ((double *)h.data())[o] = src[o];
        }
        HIPCHK(r, hipMemcpy(at(r->buf.fields, r->L.F + (size_t)c * cells * R), h.data(), h.size(),
                            hipMemcpyHostToDevice));
    }
    return PIC_OK;
}

int pic_read_particles(pic_run *r, int s, double *x, double *u, uint32_t *id, int64_t cap, int64_t *count)
{
    if (!r || !count) return fail(r ? &r->err : nullptr, PIC_E_INVALID_ARG, "bad argument");
    if (s < 0 || s >= r->ns) return fail(&r->err, PIC_E_INVALID_ARG, "species %d", s);
    DevState st;
    int rc = read_state(r, &st);
    if (rc) return rc;
    rc = check_fatal(r, st);
    if (rc) return rc;
    const Layout &L = r->L;
    const Layout::Sp &P = L.sp[s];
    const Geometry &G = L.g;
    const int nt = G.ntiles, nd = G.ndim, par = st.par;
    void *b = r->buf.particles[s];
    std::vector<int32_t> start(nt), tcap(nt);
    std::vector<uint32_t> cf((size_t)2 * nt), cb((size_t)2 * nt);
    HIPCHK(r, hipMemcpy(start.data(), at(b, P.start), nt * 4, hipMemcpyDeviceToHost));
    HIPCHK(r, hipMemcpy(tcap.data(), at(b, P.cap), nt * 4, hipMemcpyDeviceToHost));
    HIPCHK(r, hipMemcpy(cf.data(), at(b, P.cnt_front), (size_t)2 * nt * 4, hipMemcpyDeviceToHost));
    HIPCHK(r, hipMemcpy(cb.data(), at(b, P.cnt_back), (size_t)2 * nt * 4, hipMemcpyDeviceToHost));
    int64_t n = 0;
    for (int t = 0; t < nt; ++t) n += (int64_t)cf[(size_t)par * nt + t] + cb[(size_t)par * nt + t];
    *count = n;
    if (n == 0) return PIC_OK;
    if (n > cap) return fail(&r->err, PIC_E_BUFFER_TOO_SMALL, "%lld particles, capacity %lld", (long long)n,
                             (long long)cap);
    if (!x || !u) return fail(&r->err, PIC_E_INVALID_ARG, "null output arrays");
    const size_t ncap = (size_t)P.ncap, R = L.real;
    std::vector<uint16_t> hcell(R == 4 ? ncap : 0);
    std::vector<uint32_t> hid(ncap);
    std::vector<char> hpos[3], hu[3];
    if (R == 4) HIPCHK(r, hipMemcpy(hcell.data(), at(b, P.cell[par]), ncap * 2, hipMemcpyDeviceToHost));
    for (int a = 0; a < nd; ++a) {
        hpos[a].resize(ncap * R);
        HIPCHK(r, hipMemcpy(hpos[a].data(), at(b, P.pos[par][a]), ncap * R, hipMemcpyDeviceToHost));
    }
    for (int c = 0; c < 3; ++c) {
        hu[c].resize(ncap * R);
        HIPCHK(r, hipMemcpy(hu[c].data(), at(b, P.u[par][c]), ncap * R, hipMemcpyDeviceToHost));
    }
    HIPCHK(r, hipMemcpy(hid.data(), at(b, P.id[par]), ncap * 4, hipMemcpyDeviceToHost));
    const bool tracked = r->hp.sp[s].track_id != 0;
    int64_t k = 0;
    for (int t = 0; t < nt; ++t) {
        const int64_t nf = cf[(size_t)par * nt + t], nb = cb[(size_t)par * nt + t];
        const int t0[3] = {(t % G.nt[0]) * G.tile[0], ((t / G.nt[0]) % G.nt[1]) * G.tile[1],
                           (t / (G.nt[0] * G.nt[1])) * G.tile[2]};
        for (int64_t j = 0; j < nf + nb; ++j, ++k) {
            const int64_t slot = j < nf ? start[t] + j : start[t] + tcap[t] - nb + (j - nf);
            for (int a = 0; a < nd; ++a) {
                double X;
                if (R == 4) {
                    const uint32_t c = hcell[slot];
                    const int ic = t0[a] + (int)((c >> (a * G.tshift[0])) & (uint32_t)(G.tile[a] - 1));
                    X = ic + (double)((const float *)hpos[a].data())[slot];
                } else {
                    X = ((const double *)hpos[a].data())[slot];
                }
                x[(size_t)a * cap + k] = X * G.d[a];
            }
            for (int c = 0; c < 3; ++c)
                u[(size_t)c * cap + k] = R == 4 ? (double)((const float *)hu[c].data())[slot]
                                              : ((const double *)hu[c].data())[slot];
            if (id) id[k] = tracked ? hid[slot] : 0xFFFFFFFFu;
        }
    }
    return PIC_OK;
}

int pic_destroy(pic_run *r)
{
    if (!r) return PIC_OK;
    if (r->owner) return fail(&r->err, PIC_E_STATE, "run is a member of a batch; destroy the batch first");
    // the caller frees the buffers once this returns: let every enqueued step finish first
    const hipError_t e = hipStreamSynchronize(r->stream);
    if (r->gexec) (void)hipGraphExecDestroy(r->gexec);
    if (r->graph) (void)hipGraphDestroy(r->graph);
    if (r->static_device >= 0) release_static_scratch(r->static_device);
    delete r;
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(nullptr, PIC_E_HIP, "pic_destroy: hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    return PIC_OK;
}

// ---------------------------------------------------------------------------
// Checkpoint / restore: a header (magic, version, descriptors, buffer sizes)
// followed by the raw contents of the four caller buffers, copied through a
// host staging buffer.

namespace {
constexpr char kCkptMagic[8] = {'P', 'I', 'C', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t kCkptVersion = 1;
struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t nspecies;
    pic_grid_desc grid;
    pic_species_desc species[kMaxSpecies];
    uint64_t bytes[kMaxSpecies + 3];   // particle buffers, fields, scratch, diag
};
constexpr size_t kStage = size_t(64) << 20;

int ckpt_buffers(const pic_run *r, void *ptr[kMaxSpecies + 3], uint64_t bytes[kMaxSpecies + 3])
{
    for (int i = 0; i < kMaxSpecies + 3; ++i) {
        ptr[i] = nullptr;
        bytes[i] = 0;
    }
    for (int s = 0; s < r->ns; ++s) {
        ptr[s] = r->buf.particles[s];
        bytes[s] = r->L.particle_bytes[s];
    }
    ptr[kMaxSpecies] = r->buf.fields;
    bytes[kMaxSpecies] = r->L.field_bytes;
    ptr[kMaxSpecies + 1] = r->buf.scratch;
    bytes[kMaxSpecies + 1] = r->L.scratch_bytes;
    ptr[kMaxSpecies + 2] = r->buf.diag;
    bytes[kMaxSpecies + 2] = r->L.diag_bytes;
    return PIC_OK;
}
}  // namespace

int pic_checkpoint(pic_run *r, const char *path)
{
    if (!r || !path) return fail(r ? &r->err : nullptr, PIC_E_INVALID_ARG, "null argument");
    DevState st;
    int rc = read_state(r, &st);
    if (rc) return rc;
    rc = check_fatal(r, st);
    if (rc) return rc;
    CkptHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kCkptMagic, sizeof(h.magic));
    h.version = kCkptVersion;
    h.nspecies = r->ns;
    h.grid = r->grid;
    for (int s = 0; s < r->ns; ++s) h.species[s] = r->species[s];
    void *ptr[kMaxSpecies + 3];
    ckpt_buffers(r, ptr, h.bytes);
    FILE *f = fopen(path, "wb");
    if (!f) return fail(&r->err, PIC_E_INVALID_ARG, "cannot open %s for writing", path);
    std::vector<char> stage(kStage);
    bool ok = fwrite(&h, sizeof(h), 1, f) == 1;
    for (int i = 0; ok && i < kMaxSpecies + 3; ++i)
        for (uint64_t o = 0; ok && o < h.bytes[i]; o += kStage) {
            const size_t n = (size_t)std::min<uint64_t>(kStage, h.bytes[i] - o);
            if (hipMemcpy(stage.data(), (char *)ptr[i] + o, n, hipMemcpyDeviceToHost) != hipSuccess) {
                fclose(f);
                return hip_fail(r, hipGetLastError(), "checkpoint copy");
            }
            ok = fwrite(stage.data(), 1, n, f) == n;
        }
    if (fclose(f) != 0) ok = false;
    if (!ok) return fail(&r->err, PIC_E_INVALID_ARG, "short write to %s", path);
    return PIC_OK;
}

int pic_restore(pic_run *r, const char *path)
{
    if (!r || !path) return fail(r ? &r->err : nullptr, PIC_E_INVALID_ARG, "null argument");
    HIPCHK(r, hipStreamSynchronize(r->stream));
    FILE *f = fopen(path, "rb");
    if (!f) return fail(&r->err, PIC_E_INVALID_ARG, "cannot open %s", path);
    CkptHeader h;
    if (fread(&h, sizeof(h), 1, f) != 1 || memcmp(h.magic, kCkptMagic, sizeof(h.magic)) != 0 ||
        h.version != kCkptVersion) {
        fclose(f);
        return fail(&r->err, PIC_E_INVALID_ARG, "%s is not a checkpoint of this library version", path);
    }
    // the checkpoint must come from a run with the same descriptors (compared
    // field by field: the structs' padding carries no meaning); flags that
    // only steer initialisation or launching may differ
    bool same = h.nspecies == r->ns && same_grid(h.grid, r->grid, PIC_FLAG_HOST_LOAD | PIC_FLAG_NO_GRAPH |
                                                                       PIC_FLAG_LATTICE_LOAD);
    for (int s = 0; same && s < r->ns; ++s) same = same_species(h.species[s], r->species[s]);
    void *ptr[kMaxSpecies + 3];
    uint64_t bytes[kMaxSpecies + 3];
    ckpt_buffers(r, ptr, bytes);
    for (int i = 0; same && i < kMaxSpecies + 3; ++i) same = bytes[i] == h.bytes[i];
    if (!same) {
        fclose(f);
        return fail(&r->err, PIC_E_STATE, "%s was written by a run with other descriptors", path);
    }
    std::vector<char> stage(kStage);
    bool ok = true;
    for (int i = 0; ok && i < kMaxSpecies + 3; ++i)
        for (uint64_t o = 0; ok && o < h.bytes[i]; o += kStage) {
            const size_t n = (size_t)std::min<uint64_t>(kStage, h.bytes[i] - o);
            ok = fread(stage.data(), 1, n, f) == n;
            if (ok && hipMemcpy((char *)ptr[i] + o, stage.data(), n, hipMemcpyHostToDevice) != hipSuccess) {
                fclose(f);
                return hip_fail(r, hipGetLastError(), "restore copy");
            }
        }
    fclose(f);
    if (!ok) return fail(&r->err, PIC_E_INVALID_ARG, "%s is truncated", path);
    // the parameter block holds this run's device addresses
    HIPCHK(r, hipMemcpy(r->dp, &r->hp, sizeof(KParams), hipMemcpyHostToDevice));
    DevState st;
    int rc = read_state(r, &st);
    if (rc) return rc;
    r->steps_enqueued = st.step;
    return check_fatal(r, st);
}

// ---------------------------------------------------------------------------
// Ensembles

int pic_batch_query(int nruns, pic_run *const *runs, size_t *table_bytes)
{
    if (!table_bytes) return fail(nullptr, PIC_E_INVALID_ARG, "null argument");
    BatchLayout B;
    int rc = batch_layout(nruns, runs, &B, nullptr);
    if (rc) return rc;
    *table_bytes = B.bytes;
    return PIC_OK;
}

int pic_batch_init(int nruns, pic_run *const *runs, void *table, size_t table_bytes, int32_t persistent_blocks,
                   uint32_t flags, pic_batch **out)
{
    if (!out || !table) return fail(nullptr, PIC_E_INVALID_ARG, "null argument");
    *out = nullptr;
    if (persistent_blocks < 0) return fail(nullptr, PIC_E_INVALID_ARG, "persistent_blocks < 0");
    BatchLayout B;
    int rc = batch_layout(nruns, runs, &B, nullptr);
    if (rc) return rc;
    if (table_bytes < B.bytes)
        return fail(nullptr, PIC_E_BUFFER_TOO_SMALL, "table buffer %zu bytes, need %zu", table_bytes, B.bytes);
    for (int i = 0; i < nruns; ++i) {
        if (runs[i]->owner) return fail(nullptr, PIC_E_STATE, "run %d already belongs to a batch", i);
        if (runs[i]->stream != runs[0]->stream)
            return fail(nullptr, PIC_E_INVALID_ARG, "run %d: members must be bound to the same stream", i);
    }
    // the members of one tile edge share one particle kernel, so one shape
    int group_shape[kBatchGroups] = {-1, -1, -1};
    for (int i = 0; i < nruns; ++i) {
        int &gs = group_shape[tile_group(runs[i])];
        if (gs >= 0 && gs != runs[i]->hp.shape)
            return fail(nullptr, PIC_E_INVALID_ARG,
                        "run %d: shape %d, but an earlier member with tile edge %d has shape %d", i,
                        runs[i]->hp.shape, runs[i]->grid.tile[0], gs);
        gs = runs[i]->hp.shape;
    }
    pic_batch *b = new (std::nothrow) pic_batch();
    if (!b) return fail(nullptr, PIC_E_INVALID_ARG, "host allocation failed");
    b->runs.assign(runs, runs + nruns);
    b->precision = runs[0]->grid.precision;
    b->ndim = runs[0]->grid.ndim;
    b->stream = runs[0]->stream;

    // host images of the table sections
    std::vector<const KParams *> kps(nruns);
    std::vector<int2> cells;
    cells.reserve(B.n_cell_blocks);
    int max_species = 0, nst = 0, max_fd = 0;
    for (int i = 0; i < nruns; ++i) {
        const pic_run *r = runs[i];
        kps[i] = r->dp;
        const int cb = (int)((r->L.g.cells + 255) / 256);
        for (int k = 0; k < cb; ++k) cells.push_back(make_int2(i, k));
        max_species = std::max(max_species, r->ns);
        nst = std::max(nst, (int)((r->ns * (int64_t)r->L.g.ntiles + 255) / 256));
        max_fd = std::max(max_fd, r->hp.fd_blocks);
    }
    // work items: runs in order of decreasing particles per tile (the longest
    // items are handed out first), all tiles of a run together
    std::vector<int64_t> load(nruns, 0);
    for (int i = 0; i < nruns; ++i)
        for (int sp = 0; sp < runs[i]->ns; ++sp) load[i] += runs[i]->L.sp[sp].tile_nominal;
    std::vector<int> order(nruns);
    for (int i = 0; i < nruns; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return load[a] > load[c]; });
    // class-major lists: class c holds the items (run, k) with k mod 8 == c
    std::vector<int2> items[kBatchGroups];
    int cls_start[kBatchGroups][kBatchXcds], cls_len[kBatchGroups][kBatchXcds];
    for (int g = 0; g < kBatchGroups; ++g)
        for (int c = 0; c < kBatchXcds; ++c) {
            cls_start[g][c] = (int)items[g].size();
            for (int i : order) {
                const pic_run *r = runs[i];
                if (tile_group(r) != g) continue;
                for (int k = c; k < r->L.g.ntiles; k += kBatchXcds) items[g].push_back(make_int2(i, k));
            }
            cls_len[g][c] = (int)items[g].size() - cls_start[g][c];
        }
    char *base = (char *)table;
    BatchTable &H = b->ht;
    memset(&H, 0, sizeof(H));
    H.nruns = nruns;
    H.n_cell_blocks = B.n_cell_blocks;
    H.nst_blocks = std::max(1, nst);
    H.max_species = max_species;
    H.max_fd_blocks = max_fd;
    H.coulomb = 0;
    for (int i = 0; i < nruns; ++i) H.coulomb |= runs[i]->hp.coulomb;
    H.kp = (const KParams *const *)(base + B.kp);
    H.cell_blocks = (const int2 *)(base + B.cell_blocks);
    for (int g = 0; g < kBatchGroups; ++g) {
        H.grp[g].shape = group_shape[g] < 0 ? 0 : group_shape[g];
        H.grp[g].n_items = (int)items[g].size();
        H.grp[g].items = (const int2 *)(base + B.items[g]);
        for (int c = 0; c < kBatchXcds; ++c) {
            H.grp[g].cls_start[c] = cls_start[g][c];
            H.grp[g].cls_len[c] = cls_len[g][c];
        }
        H.grp[g].queue = (int *)(base + B.queues) + g * kBatchXcds;
    }
    b->dt = (BatchTable *)(base + B.table);
    // persistent workgroups: as many as fit on the device at once
    int devi = 0, cus = 0;
    hipError_t he = hipGetDevice(&devi);
    if (he == hipSuccess) he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, devi);
    for (int g = 0; he == hipSuccess && g < kBatchGroups; ++g) {
        if (persistent_blocks > 0) {
            b->pblocks[g] = persistent_blocks;
            continue;
        }
        int per_cu = 0;
        he = batch_particle_occupancy(b->precision, b->ndim, g, H.coulomb != 0, H.grp[g].shape, &per_cu);
        b->pblocks[g] = std::max(1, per_cu) * std::max(1, cus);
    }
    const std::vector<int> zeros((size_t)kBatchGroups * kBatchXcds, 0);
#define BINIT_CHK(expr)                                  \
    do {                                                 \
        hipError_t e_ = (expr);                          \
        if (e_ != hipSuccess) {                          \
            int c_ = batch_hip_fail(b, e_, #expr);       \
            delete b;                                    \
            return c_;                                   \
        }                                                \
    } while (0)
    BINIT_CHK(he);
    BINIT_CHK(hipMemcpyAsync(base + B.table, &H, sizeof(H), hipMemcpyHostToDevice, b->stream));
    BINIT_CHK(hipMemcpyAsync(base + B.kp, kps.data(), kps.size() * sizeof(void *), hipMemcpyHostToDevice,
                             b->stream));
    BINIT_CHK(hipMemcpyAsync(base + B.cell_blocks, cells.data(), cells.size() * sizeof(int2), hipMemcpyHostToDevice,
                             b->stream));
    for (int g = 0; g < kBatchGroups; ++g)
        if (!items[g].empty())
            BINIT_CHK(hipMemcpyAsync(base + B.items[g], items[g].data(), items[g].size() * sizeof(int2),
                                     hipMemcpyHostToDevice, b->stream));
    BINIT_CHK(hipMemcpyAsync(base + B.queues, zeros.data(), zeros.size() * sizeof(int), hipMemcpyHostToDevice,
                             b->stream));
    BINIT_CHK(hipStreamSynchronize(b->stream));
#undef BINIT_CHK
    if (!(flags & PIC_FLAG_NO_GRAPH)) {
        const char *what = "";
        he = capture_batch_graph(b, &what);
        if (he != hipSuccess) {
            const int c = batch_hip_fail(b, he, what);
            delete b;
            return c;
        }
    }
    for (pic_run *r : b->runs) r->owner = b;
    *out = b;
    return PIC_OK;
}

int pic_batch_step(pic_batch *b, int32_t nsteps)
{
    if (!b) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    if (nsteps < 0) return fail(&b->err, PIC_E_INVALID_ARG, "nsteps < 0");
    for (int32_t i = 0; i < nsteps; ++i) {
        if (b->gexec) {
            BHIPCHK(b, hipGraphLaunch(b->gexec, b->stream));
            b->graph_launches += 1;
        } else {
            BHIPCHK(b, launch_batch_step(b->precision, b->ndim, b->ht, b->dt, b->pblocks, b->stream));
            b->direct_steps += 1;
        }
        for (pic_run *r : b->runs) r->steps_enqueued += 1;
    }
    return PIC_OK;
}

int pic_batch_launch_info(pic_batch *b, pic_run_info *out)
{
    if (!b || !out) return fail(b ? &b->err : nullptr, PIC_E_INVALID_ARG, "null argument");
    memset(out, 0, sizeof(*out));
    out->graph = b->gexec ? 1 : 0;
    out->steps_enqueued = b->graph_launches + b->direct_steps;
    out->graph_launches = b->graph_launches;
    out->direct_steps = b->direct_steps;
    return PIC_OK;
}

int pic_batch_step_profiled(pic_batch *b, int32_t nsteps, double *group_ms)
{
    if (!b || !group_ms) return fail(b ? &b->err : nullptr, PIC_E_INVALID_ARG, "bad argument");
    if (nsteps < 0) return fail(&b->err, PIC_E_INVALID_ARG, "nsteps < 0");
    return profiled_steps(&b->err, b->stream, nsteps, kBatchKernels, kBatchKernelGroup, group_ms,
                          [&](hipEvent_t *ev) {
                              hipError_t e = launch_batch_step(b->precision, b->ndim, b->ht, b->dt, b->pblocks,
                                                               b->stream, ev);
                              if (e == hipSuccess)
                                  for (pic_run *r : b->runs) r->steps_enqueued += 1;
                              return e;
                          });
}

int pic_batch_sync(pic_batch *b)
{
    if (!b) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < b->runs.size(); ++i) {
        pic_run *r = b->runs[i];
        DevState st;
        int rc = read_state(r, &st);
        if (!rc) rc = check_fatal(r, st);
        if (rc) return fail(&b->err, rc, "member %zu: %s", i, r->err.c_str());
    }
    return PIC_OK;
}

int pic_batch_diagnostics(pic_batch *b, int run, pic_diag *out)
{
    if (!b || !out) return fail(b ? &b->err : nullptr, PIC_E_INVALID_ARG, "bad argument");
    if (run < 0 || run >= (int)b->runs.size())
        return fail(&b->err, PIC_E_INVALID_ARG, "run %d out of 0..%d", run, (int)b->runs.size() - 1);
    const int rc = pic_diagnostics(b->runs[(size_t)run], out);
    if (rc != PIC_OK) b->err = b->runs[(size_t)run]->err;
    return rc;
}

int pic_batch_info(pic_batch *b, int32_t *persistent_blocks, int32_t *items, int32_t *shapes)
{
    if (!b) return fail(nullptr, PIC_E_INVALID_ARG, "null handle");
    for (int g = 0; g < kBatchGroups; ++g) {
        if (persistent_blocks) persistent_blocks[g] = b->ht.grp[g].n_items ? b->pblocks[g] : 0;
        if (items) items[g] = b->ht.grp[g].n_items;
        if (shapes) shapes[g] = b->ht.grp[g].n_items ? b->ht.grp[g].shape : -1;
    }
    return PIC_OK;
}

int pic_batch_destroy(pic_batch *b)
{
    if (!b) return PIC_OK;
    (void)hipStreamSynchronize(b->stream);
    for (pic_run *r : b->runs) r->owner = nullptr;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return PIC_OK;
}

// ---------------------------------------------------------------------------
// Tile autotuner

static int tune_carve(const pic_grid_desc *grid, const pic_species_desc *sp, int ns, int copies, int tile,
                      TuneCarve *T)
{
    pic_grid_desc g = *grid;
    for (int a = 0; a < 3; ++a) g.tile[a] = a < g.ndim ? tile : 0;
    int rc = pic_query(&g, sp, ns, &T->sz);
    if (rc) return rc;
    Carver c;
    for (int s = 0; s < ns; ++s) T->part[s] = c.take(T->sz.particle_bytes[s]);
    T->fields = c.take(T->sz.field_bytes);
    T->scratch = c.take(T->sz.scratch_bytes);
    T->diag = c.take(T->sz.diag_bytes);
    T->per_copy = c.off;
    // batch table of the copies
    int64_t cells = 1, tiles = 1;
    for (int a = 0; a < g.ndim; ++a) {
        cells *= g.n[a];
        tiles *= g.n[a] / tile;
    }
    int64_t nit[kBatchGroups] = {0, 0, 0};
    nit[tile == 8 ? 0 : (tile == 16 ? 1 : 2)] = tiles * copies;
    BatchLayout B;
    rc = batch_carve(copies, (cells + 255) / 256 * copies, nit, &B, nullptr);
    if (rc) return rc;
    T->table = T->per_copy * (size_t)copies;
    T->table_bytes = B.bytes;
    T->bytes = T->table + B.bytes;
    return PIC_OK;
}

int pic_tune_query(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies, int32_t copies,
                   size_t *workspace_bytes)
{
    if (!grid || !species || !workspace_bytes) return fail(nullptr, PIC_E_INVALID_ARG, "null argument");
    if (copies < 1 || copies > 4096) return fail(nullptr, PIC_E_INVALID_ARG, "copies %d out of 1..4096", copies);
    size_t need = 0;
    int tried = 0;
    for (int t = 8; t <= 32; t *= 2) {
        if (!tile_fits(grid, t)) continue;
        TuneCarve T;
        int rc = tune_carve(grid, species, nspecies, copies, t, &T);
        if (rc) return rc;
        need = std::max(need, T.bytes);
        ++tried;
    }
    if (!tried) return fail(nullptr, PIC_E_INVALID_ARG, "no tile edge in {8,16,32} divides the grid");
    *workspace_bytes = need;
    return PIC_OK;
}

// Milliseconds per step of `copies` fresh device-loaded runs of the described
// configuration at tile edge `tile` and particle-kernel shape `shape` (alone
// when copies == 1, as one batch otherwise), over nsteps graph-replayed steps
// after as many warm-up steps (at least 2).
static int tune_time(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies, int32_t copies,
                     void *workspace, void *hip_stream, int32_t nsteps, int tile, int shape, double *ms)
{
    hipStream_t st = (hipStream_t)hip_stream;
    TuneCarve T;
    int rc = tune_carve(grid, species, nspecies, copies, tile, &T);
    if (rc) return rc;
    std::vector<pic_run *> runs;
    pic_batch *b = nullptr;
    for (int i = 0; !rc && i < copies; ++i) {
        pic_grid_desc g = *grid;
        for (int a = 0; a < 3; ++a) g.tile[a] = a < g.ndim ? tile : 0;
        g.shape = shape;
        g.flags &= ~(uint32_t)PIC_FLAG_HOST_LOAD;
        g.run = grid->run + (uint32_t)i;
        char *base = (char *)workspace + T.per_copy * (size_t)i;
        pic_buffers buf;
        memset(&buf, 0, sizeof(buf));
        for (int s = 0; s < nspecies; ++s) buf.particles[s] = base + T.part[s];
        buf.fields = base + T.fields;
        buf.scratch = base + T.scratch;
        buf.diag = base + T.diag;
        pic_run *r = nullptr;
        rc = pic_init(&g, species, nspecies, &buf, hip_stream, &r);
        if (!rc) runs.push_back(r);
    }
    if (!rc && copies > 1)
        rc = pic_batch_init(copies, runs.data(), (char *)workspace + T.table, T.table_bytes, 0, 0, &b);
    auto steps = [&](int32_t n) { return b ? pic_batch_step(b, n) : pic_step(runs[0], n); };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float el = 0.f;
    hipError_t he = hipSuccess;
    if (!rc) he = hipEventCreate(&e0);
    if (!rc && he == hipSuccess) he = hipEventCreate(&e1);
    if (!rc && he == hipSuccess) rc = steps(std::max(2, nsteps));
    if (!rc && he == hipSuccess) he = hipEventRecord(e0, st);
    if (!rc && he == hipSuccess) rc = steps(nsteps);
    if (!rc && he == hipSuccess) he = hipEventRecord(e1, st);
    if (!rc && he == hipSuccess) he = hipEventSynchronize(e1);
    if (!rc && he == hipSuccess) he = hipEventElapsedTime(&el, e0, e1);
    if (!rc && he == hipSuccess) rc = b ? pic_batch_sync(b) : pic_sync(runs[0]);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    if (b) pic_batch_destroy(b);
    for (pic_run *r : runs) pic_destroy(r);
    if (he != hipSuccess) return fail(nullptr, PIC_E_HIP, "tuner timing: %s", hipGetErrorString(he));
    if (rc) return rc;
    *ms = (double)el / nsteps;
    return PIC_OK;
}

static int tune_prologue(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies, int32_t copies,
                         void *workspace, size_t workspace_bytes, int32_t nsteps, const void *best, const double *ms)
{
    if (!grid || !species || !workspace || !best || !ms || nsteps < 1)
        return fail(nullptr, PIC_E_INVALID_ARG, "bad argument");
    size_t need = 0;
    int rc = pic_tune_query(grid, species, nspecies, copies, &need);
    if (rc) return rc;
    if (workspace_bytes < need)
        return fail(nullptr, PIC_E_BUFFER_TOO_SMALL, "workspace %zu bytes, need %zu", workspace_bytes, need);
    return PIC_OK;
}

int pic_tune(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies, int32_t copies,
             void *workspace, size_t workspace_bytes, void *hip_stream, int32_t nsteps, int32_t *best_tile,
             double *ms)
{
    int rc = tune_prologue(grid, species, nspecies, copies, workspace, workspace_bytes, nsteps, best_tile, ms);
    if (rc) return rc;
    *best_tile = 0;
    double best = 0.0;
    for (int k = 0, t = 8; t <= 32; ++k, t *= 2) {
        ms[k] = -1.0;
        if (!tile_fits(grid, t)) continue;
        rc = tune_time(grid, species, nspecies, copies, workspace, hip_stream, nsteps, t, grid->shape, &ms[k]);
        if (rc) return rc;
        if (*best_tile == 0 || ms[k] < best) {
            best = ms[k];
            *best_tile = t;
        }
    }
    return PIC_OK;
}

int pic_tune_shape(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies, int32_t copies,
                   void *workspace, size_t workspace_bytes, void *hip_stream, int32_t nsteps, int32_t *best_shape,
                   double *ms)
{
    int rc = tune_prologue(grid, species, nspecies, copies, workspace, workspace_bytes, nsteps, best_shape, ms);
    if (rc) return rc;
    int t = grid->tile[0];
    if (t == 0) {
        t = grid->ndim == 3 ? 8 : 16;
        if (!tile_fits(grid, t)) t = 8;
    }
    if (!tile_fits(grid, t)) return fail(nullptr, PIC_E_INVALID_ARG, "tile %d does not divide the grid", t);
    const int nshapes = grid->precision == PIC_PREC_MIXED ? kShapes : 1;
    *best_shape = -1;
    double best = 0.0;
    for (int k = 0; k < kShapes; ++k) {
        ms[k] = -1.0;
        if (k >= nshapes) continue;
        rc = tune_time(grid, species, nspecies, copies, workspace, hip_stream, nsteps, t, k, &ms[k]);
        if (rc) return rc;
        if (*best_shape < 0 || ms[k] < best) {
            best = ms[k];
            *best_shape = k;
        }
    }
    return PIC_OK;
}

}  // extern "C"

