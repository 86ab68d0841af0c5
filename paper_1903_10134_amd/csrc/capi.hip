// capi.hip -- the C ABI declared in include/mdpd.h: system lifecycle, the
// timestep schedule (Alg. 1) and the read-out calls.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "mdpd.h"
#include "mdpd_internal.h"

using namespace mdpd;

namespace {

thread_local std::string g_err;

mdpd_status fail(mdpd_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(MDPD_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));         \
    } while (0)

constexpr int kTimedKernels = 6;  // sort, neighbour list, density, force, wall, adjoint pair passes

struct EventPool {
    std::vector<hipEvent_t> ev;
    size_t used = 0;
};

}  // namespace

namespace mdpd {
// Recorded trajectory for the adjoint: device checkpoints every `every`
// steps, a tape of up to every + 1 states for the recomputed segment, and
// the adjoint work arrays.
struct AdjRec {
    bool ready = false;
    int64_t nsteps = 0;
    int every = 1;
    int avg = 0;
    int tmax = 1;                 // largest type count over the replicas
    std::vector<int64_t> nfluid;  // per replica
    char *ck = nullptr;  // nck checkpoints of ck_bytes each
    uint64_t ck_bytes = 0;
    int nck = 0;
    std::vector<int> ck_lanes;  // force lane count of each checkpoint's partials
    char *tape = nullptr;  // ntape entries of tape_bytes each
    uint64_t tape_bytes = 0;
    int ntape = 0;
    Soa3 X{}, U{}, fb{}, Xo{}, Uo{};  // Xo, Uo: the step-back targets, swapped with X, U each step
    double *rhoA = nullptr, *gp = nullptr, *gpart = nullptr, *gtot = nullptr, *loss = nullptr;
    double *sdc = nullptr;  // dissipation control: s, s / S and dL/dS per slot (3 n)
    AdjConst *act = nullptr;  // 4 tables of nrep entries: seeded, unseeded, final, creation
    std::vector<AdjConst> host_act;  // host copy (kept alive while the upload may read it)
    LossConst *lct = nullptr;
    size_t gp_n = 0, gpart_n = 0;
};
}  // namespace mdpd

struct mdpd_system {
    mdpd_params p{};
    hipStream_t st = nullptr;
    int dev = 0;  // the device current at creation (where every buffer lives)
    int n = 0;
    bool fp32 = false;
    bool walls = false;
    bool slip = false;  // walls reflect with wall_slip > 0 in some replica
    bool dctl = false;  // some replica controls the fluid-solid dissipation (diss_ctrl > 0)
    uint8_t *corr_byid = nullptr;  // adjoint recording: the step's wall events by particle id
    int *perm_out = nullptr;       // adjoint recording: where the step's sorts move each slot
    int *perm_tmp = nullptr;       // walls: the two sorts of a recorded step (2 n), composed into perm_out
    int lanes[3] = {1, 4, 4};  // neighbour list (wavefronts per border cell), density (and phi), force
    // replicas (a single system is one replica)
    int nrep = 1;
    bool mt = false;  // some replica has more than one type
    std::vector<mdpd_params> params;
    std::vector<Geom> geoms;
    std::vector<PairConst> pcs;
    std::vector<int> cell_off, part_off, blk_off;  // host copies of the tables in R
    Reps R{};
    int cur = 0;
    int64_t step = 0;

    // State in the sorted order of the last list build: xs[cur], vh[cur] are
    // x(t) and the half-step velocity of the current step; the force pass
    // writes the next ones to xs[1 - cur], vh[1 - cur] (the buffers swap
    // every step).  tag[0], typ[0] are the tags and types; tag[1], typ[1],
    // tx, tv, tp the temporaries of a re-sort.
    Soa3 xs[2]{}, vh[2]{}, tx{}, tv{}, v{}, F{}, tp{};
    Soa3 xb{};  // positions at the last list build
    uint32_t *tag[2]{};
    uint8_t *typ[2]{};
    void *rho = nullptr;
    int *key = nullptr, *slot = nullptr, *counts = nullptr, *cstart = nullptr, *cnew = nullptr, *bsum = nullptr;
    int *ncnt = nullptr;    // pair list of the current positions (counts)
    uint32_t *nl = nullptr;
    int *scnt = nullptr;    // skin list of the last build (counts)
    uint32_t *sl = nullptr;
    bool perstep = false;   // every replica has skin 0: the pair list is built every step, with the
    void *nlr2 = nullptr;   // r^2 of its near entries (FP32 or FP64 as rho)
    float *bmax = nullptr;  // force-pass block maxima of the squared displacement since the build
    int *flags = nullptr;   // [nrep + 1] rebuild flags of the current step, then [nrep + 1]: done
                            // counter of the gate, [nrep + 2]: forced rebuild
    unsigned long long *nbuild = nullptr;  // replicas rebuilt since creation
    uint32_t *tmpid = nullptr;
    PartRec *rec = nullptr;  // packed neighbour records of the current step
    double *fpart = nullptr;
    int force_lanes_used = 4;  // lane count of the last force launch (its partials layout)
    int *status = nullptr;
    uint32_t *dstep = nullptr;  // noise step of the current force evaluation (advanced by the main sort)
    int *ovf = nullptr;        // [0]: overflow count, [1..n]: queued slots
    double *ovf_ve = nullptr;  // per slot: virial, pair energy of overflowed particles
    int *corr = nullptr;  // [0]: corrections this step, [1..n]: flags, then per-block counts
    uint8_t *wmask = nullptr;  // per wall sub-cell: a frozen particle within r_c of its box
    size_t wmask_bytes = 0;
    unsigned long long *ncorr_total = nullptr;
    double *tab = nullptr;
    double *obs = nullptr;       // 16 result slots per replica
    double *obs_part = nullptr;  // block partials of the observables
    double *stress = nullptr;    // 6 planes of n (allocated on first use) + 6 per replica
    double *io = nullptr;   // n x 3 staging for exports and host inputs
    double *io2 = nullptr;  // second n x 3 staging
    double *work = nullptr;

    bool timing = false;
    EventPool pool[kTimedKernels];
    std::vector<void *> allocs;
    AdjRec adj;

    // Graph mode: two timesteps captured once into a HIP graph and replayed
    // (buffers alternate every step, so a pair of steps ends where it began).
    bool use_graph = false;
    hipStream_t cap_st = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_cur = -1;
    int graph_lanes[3] = {0, 0, 0};

    ~mdpd_system()
    {
        drop_graph();
        if (cap_st) (void)hipStreamDestroy(cap_st);
        for (auto &pl : pool)
            for (auto e : pl.ev) (void)hipEventDestroy(e);
        for (void *a : allocs) (void)hipFree(a);
    }

    void drop_graph()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        graph_cur = -1;
    }

    // Capture two timesteps (device work only: every decision inside a step
    // is taken on the device) on a private stream.
    hipError_t capture_pair()
    {
        drop_graph();
        hipError_t e = hipSuccess;
        if (!cap_st) e = hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        hipStream_t user = st;
        const bool tm = timing;
        const int cur0 = cur;
        st = cap_st;
        timing = false;
        const int64_t step0 = step;
        e = hipStreamBeginCapture(cap_st, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            advance(2);
            e = hipStreamEndCapture(cap_st, &graph);
        }
        step = step0;
        st = user;
        timing = tm;
        if (e == hipSuccess && cur != cur0) e = hipErrorInvalidValue;  // cannot happen: buffers alternate
        if (e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph();
            cur = cur0;
            return e;
        }
        graph_cur = cur;
        for (int k = 0; k < 3; ++k) graph_lanes[k] = lanes[k];
        return hipSuccess;
    }

    bool graph_valid() const
    {
        return gexec && graph_cur == cur && graph_lanes[0] == lanes[0] && graph_lanes[1] == lanes[1] &&
               graph_lanes[2] == lanes[2];
    }

    // Free one allocation made by alloc() (NULL is ignored).
    void release(void *ptr)
    {
        if (!ptr) return;
        for (size_t k = 0; k < allocs.size(); ++k)
            if (allocs[k] == ptr) {
                (void)hipFree(ptr);
                allocs.erase(allocs.begin() + (long)k);
                return;
            }
    }

    template <typename T>
    mdpd_status alloc(T **out, size_t count)
    {
        void *ptr = nullptr;
        size_t bytes = count * sizeof(T);
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&ptr, bytes);
        if (e != hipSuccess) {
            *out = nullptr;
            return fail(MDPD_E_OOM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
        }
        allocs.push_back(ptr);
        *out = (T *)ptr;
        return MDPD_OK;
    }

    mdpd_status alloc3(Soa3 *a, size_t count)
    {
        double *base = nullptr;
        mdpd_status s = alloc(&base, 3 * count);
        if (s) return s;
        a->x = base;
        a->y = base + count;
        a->z = base + 2 * count;
        return MDPD_OK;
    }

    // Timing: event pair around a launch of kernel class k.
    void tic(int k)
    {
        if (!timing) return;
        EventPool &pl = pool[k];
        while (pl.ev.size() < pl.used + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            pl.ev.push_back(e);
        }
        (void)hipEventRecord(pl.ev[pl.used], st);
    }
    void toc(int k)
    {
        if (!timing) return;
        EventPool &pl = pool[k];
        if (pl.ev.size() < pl.used + 2) return;
        (void)hipEventRecord(pl.ev[pl.used + 1], st);
        pl.used += 2;
    }

    // The step's gate, then the re-sort and skin list of the replicas that
    // moved too far (every launch checks the gate's flags on the device).
    // With walls the previous positions xs[1 - cur] ride along the sort.
    // list_later (skin 0): the pair list is built after the wall corrector
    // (which may move particles back and re-sort them), not here.
    void gate_and_rebuild(bool list_later = false)
    {
        const Soa3 none{nullptr, nullptr, nullptr};
        int *dmap = perm_out && walls ? perm_tmp : perm_out;
        if (!perstep || n == 0)
            launch_gate(st, R, force_lanes_used, bmax, flags + nrep + 2, flags, flags + nrep + 1, dstep, ovf, nbuild,
                        true);
        if (!perstep) {
            rebuild(walls ? xs[1 - cur] : none, walls ? tp : none, dmap);
            return;
        }
        // skin 0: every replica rebuilds every step (no gate: the sort does
        // its bookkeeping), so the sort moves the predicted state (tx, tv)
        // straight into xs[cur], vh[cur], and x(t) from xs[1 - cur] into tp;
        // the tag and type buffers swap
        tic(0);
        launch_rebuild_sort(st, n, R, tx, tv, walls ? xs[1 - cur] : none, tag[0], typ[0], xs[cur], vh[cur],
                            walls ? tp : none, tag[1], typ[1], none, key, slot, tmpid, counts, cnew, cstart, bsum,
                            dmap, false, n > 0 ? dstep : nullptr, ovf, nbuild);
        std::swap(tag[0], tag[1]);
        std::swap(typ[0], typ[1]);
        toc(0);
        if (list_later) return;
        tic(1);
        launch_nlist(st, fp32, R, cview(xs[cur]), cstart, ncnt, nl, nlr2, true);
        toc(1);
    }

    // Where the force pass writes the next state, and where x(t) is during
    // a step (skin 0: the predicted state lives in tx, tv, and the sort puts
    // x(t) in tp).
    Soa3 next_x() const { return perstep ? tx : xs[1 - cur]; }
    Soa3 next_v() const { return perstep ? tv : vh[1 - cur]; }
    Soa3 prev_x() const { return perstep ? tp : xs[1 - cur]; }

    // The re-sort and the list of the replicas the last gate flagged: the
    // skin list, or with skin 0 the pair list itself (of every replica with
    // list_all).
    void rebuild(Soa3 xprev, Soa3 tprev, int *dmap, bool list_all = false)
    {
        tic(0);
        launch_rebuild_sort(st, n, R, xs[cur], vh[cur], xprev, tag[0], typ[0], tx, tv, tprev, tag[1], typ[1],
                            perstep ? Soa3{nullptr, nullptr, nullptr} : xb, key, slot, tmpid, counts, cnew, cstart,
                            bsum, dmap, true);
        toc(0);
        tic(1);
        if (perstep)
            launch_nlist(st, fp32, R, cview(xs[cur]), cstart, ncnt, nl, nlr2, list_all);
        else
            launch_skin_build(st, R, false, cview(xs[cur]), cstart, scnt, sl);
        toc(1);
    }

    // The build positions as the passes see them (none with skin 0: every
    // step rebuilds, nothing needs the displacement).
    Soa3c xbuild() const { return perstep ? Soa3c{nullptr, nullptr, nullptr} : cview(xb); }

    // Pair list (ncnt_out, nl_out) of the current positions from the lists
    // of the last build.
    void pair_list(int *ncnt_out, uint32_t *nl_out)
    {
        if (perstep)
            launch_nlist(st, fp32, R, cview(xs[cur]), cstart, ncnt_out, nl_out, nlr2, true);
        else {
            launch_skin_build(st, R, true, cview(xb), cstart, scnt, sl);
            launch_density(st, lanes[1], fp32, R, cview(xs[cur]), cview(vh[cur]), tag[0], typ[0], cstart, scnt, sl,
                           ncnt_out, nl_out, nullptr, nullptr);
        }
    }

    // The lists of the current state after it was restored from a
    // checkpoint: the skin list again from the build positions (the same
    // positions and cells give the same list), then the pair list at the
    // current positions (the densities are restored with the state); with
    // skin 0 the pair list from the positions and their cells.
    void restore_lists() { pair_list(ncnt, nl); }

    // Advance without synchronising (the caller checks the status word).
    void advance(int64_t nsteps)
    {
        for (int64_t k = 0; k < nsteps; ++k) {
            step += 1;
            cur = 1 - cur;
            gate_and_rebuild(walls);
            evaluate(0);
        }
    }

    void evaluate(int initial)
    {
        if (walls && !initial) {
            // phi at the predicted positions and the corrector: a flagged
            // particle goes back to x(t) = xs[1 - cur]; one that then lies
            // half the skin or more from its build position (possible right
            // after a build, for a particle faster than skin / 2 dt) makes a
            // second gate re-sort its replica and rebuild the skin list
            launch_zero_int(st, corr, 1);
            tic(4);
            launch_phi(st, lanes[1], slip, n, R, cview(xs[cur]), cview(prev_x()), xs[cur], vh[cur], tag[0],
                       cstart, wmask, corr, ncorr_total, corr_byid, xbuild(), bmax);
            toc(4);
            launch_gate(st, R, 1, bmax, flags + nrep + 2, flags, flags + nrep + 1, dstep, ovf, nbuild, false);
            const Soa3 none{nullptr, nullptr, nullptr};
            // with skin 0 the pair list of every replica is built here, once
            // per step, after the corrector and the re-sort it may need
            rebuild(none, none, perm_out ? perm_tmp + n : nullptr, perstep);
            if (perm_out) launch_compose(st, n, perm_tmp, perm_tmp + n, perm_out);
        }
        tic(2);
        if (perstep)
            launch_density_list(st, lanes[1], fp32, R, cview(xs[cur]), cview(vh[cur]), tag[0], typ[0], cstart, ncnt,
                                nlr2, rho, rec);
        else
            launch_density(st, lanes[1], fp32, R, cview(xs[cur]), cview(vh[cur]), tag[0], typ[0], cstart, scnt, sl,
                           ncnt, nl, rho, rec);
        toc(2);
        force_lanes_used = lanes[2];
        tic(3);
        launch_force(st, lanes[2], fp32, mt, dctl, R, dstep, cview(xs[cur]), cview(vh[cur]), rho, tag[0], typ[0], rec,
                     cstart, ncnt, nl, v, F, next_v(), next_x(), fpart, status, ovf, ovf + 1, ovf_ve, initial,
                     xbuild(), perstep ? nullptr : bmax);
        toc(3);
    }
};

namespace {

bool finite(double x) { return isfinite(x) != 0; }

mdpd_status validate(const mdpd_params *p, int64_t n)
{
    if (!p) return fail(MDPD_E_INVALID, "params is NULL");
    if (n < 0 || n >= (int64_t)1 << 30) return fail(MDPD_E_INVALID, "n = %lld out of range", (long long)n);
    if (p->ntypes < 1 || p->ntypes > MDPD_MAX_TYPES)
        return fail(MDPD_E_INVALID, "ntypes = %d not in 1..%d", p->ntypes, MDPD_MAX_TYPES);
    const double sc[] = {p->rc, p->rd, p->kT, p->dt, p->mass, p->phi_c, p->box[0], p->box[1], p->box[2],
                         p->body_force[0], p->body_force[1], p->body_force[2]};
    for (double v : sc)
        if (!finite(v)) return fail(MDPD_E_INVALID, "non-finite scalar parameter");
    if (!(p->rc > 0.0) || !(p->rd > 0.0) || p->rd > p->rc)
        return fail(MDPD_E_INVALID, "need 0 < rd <= rc (rc = %g, rd = %g)", p->rc, p->rd);
    if (!(p->dt > 0.0) || !(p->mass > 0.0) || p->kT < 0.0)
        return fail(MDPD_E_INVALID, "need dt > 0, mass > 0, kT >= 0");
    if (p->wall_model == MDPD_WALL_BVF && !(p->phi_c >= 0.0))
        return fail(MDPD_E_INVALID, "need phi_c >= 0 with MDPD_WALL_BVF (phi_c = %g)", p->phi_c);
    if (!(p->wall_slip >= 0.0 && p->wall_slip <= 1.0))
        return fail(MDPD_E_INVALID, "need 0 <= wall_slip <= 1 (wall_slip = %g)", p->wall_slip);
    if (p->precision != MDPD_FP64 && p->precision != MDPD_FP32_FORCES)
        return fail(MDPD_E_INVALID, "unknown precision %d", p->precision);
    if (p->wall_model != MDPD_WALL_OFF && p->wall_model != MDPD_WALL_BVF)
        return fail(MDPD_E_INVALID, "unknown wall_model %d", p->wall_model);
    const int T = p->ntypes;
    for (int a = 0; a < T; ++a)
        for (int b = 0; b < T; ++b) {
            const int ab = a * T + b, ba = b * T + a;
            if (!finite(p->A[ab]) || !finite(p->B[ab]) || !finite(p->gamma[ab]))
                return fail(MDPD_E_INVALID, "non-finite pair table entry");
            if (p->A[ab] != p->A[ba] || p->B[ab] != p->B[ba] || p->gamma[ab] != p->gamma[ba])
                return fail(MDPD_E_INVALID, "pair tables must be symmetric");
            if (p->B[ab] < 0.0 || p->gamma[ab] < 0.0) return fail(MDPD_E_INVALID, "need B, gamma >= 0");
        }
    for (int a = 0; a < 3; ++a)
        if (!(p->box[a] >= 2.0 * p->rc))
            return fail(MDPD_E_INVALID, "box edge %g is shorter than 2 r_c = %g", p->box[a], 2.0 * p->rc);
    if (!(p->skin >= 0.0) || !finite(p->skin) || p->skin > 4.0 * p->rc)
        return fail(MDPD_E_INVALID, "need 0 <= skin <= 4 r_c (skin = %g)", p->skin);
    if (!(p->diss_ctrl >= 0.0) || !finite(p->diss_ctrl))
        return fail(MDPD_E_INVALID, "need diss_ctrl >= 0 (diss_ctrl = %g)", p->diss_ctrl);
    if (p->diss_ctrl > 0.0 && (!(p->diss_rho > 0.0) || !finite(p->diss_rho)))
        return fail(MDPD_E_INVALID, "need diss_rho > 0 with diss_ctrl > 0 (diss_rho = %g)", p->diss_rho);
    return MDPD_OK;
}

// Cells per axis: the largest nc >= 1 whose edge L/nc is at least
// r_c + skin with a relative margin of 1e-12 over rounding, or exactly that
// when binning is exact (nc/L a power of two, so x * nc/L is computed without
// rounding); one cell when even that does not fit (the cell then holds every
// candidate along the axis).  The skin list is built with the test
// r^2 < (r_c + skin)^2 (1 + 1e-9) and rebuilt once a particle has moved
// skin/2 (1 - 1e-6) or more, both on the safe side of rounding.
mdpd_status make_geom(const mdpd_params *p, Geom *g)
{
    long long total = 1;
    const double rs = p->rc + p->skin;
    for (int a = 0; a < 3; ++a) {
        const double L = p->box[a];
        int nc = (int)floor(L / rs);
        while (nc >= 1) {
            const double cs = L / nc, s = nc / L;
            int e;
            const bool pow2 = frexp(s, &e) == 0.5;
            if (cs >= rs * (1.0 + 1e-12) || (pow2 && cs >= rs && L * s == (double)nc)) break;
            --nc;
        }
        if (nc < 1) nc = 1;
        // two cells on the y or z axis are each other's neighbours on both
        // sides, so a cell's search spans the whole axis either way: one cell
        // of twice the size gives the same candidates with half the cells
        // (the per-step list then sweeps twice the particles per wavefront
        // against one load of its candidates).  The x axis keeps two: the
        // list's row pieces along x need a cell on either side.
        if (nc == 2 && a > 0) nc = 1;
        g->L[a] = L;
        g->nc[a] = nc;
        g->s[a] = nc / L;
        g->cs[a] = L / nc;
        g->inv_nc[a] = 1.0 / nc;
        g->invL[a] = 1.0 / L;
        total *= nc;
    }
    if (total > (long long)4096 * 4096) return fail(MDPD_E_UNSUPPORTED, "more than 2^24 cells");
    g->ncells = (int)total;
    g->rc = p->rc;
    g->rc2 = p->rc * p->rc;
    g->rd2 = p->rd * p->rd;
    g->rs2 = rs * rs * (1.0 + 1e-9);
    g->slack = 0.5 * p->skin;
    g->gate2 = 0.25 * p->skin * p->skin * (1.0 - 1e-6);
    return MDPD_OK;
}

}  // namespace

extern "C" {

const char *mdpd_last_error(void) { return g_err.c_str(); }

void mdpd_destroy(mdpd_system *s)
{
    if (!s) return;
    if (s->st) (void)hipStreamSynchronize(s->st);
    else (void)hipDeviceSynchronize();
    delete s;
}

}  // extern "C"

namespace {

// Pair constants of one replica (device table entry; noise keys are set per
// launch from seed and step).
PairConst make_pair_const(const mdpd_params *p, const double *tab)
{
    PairConst pc{};
    for (int a = 0; a < 3; ++a) {
        pc.L[a] = p->box[a];
        pc.invL[a] = 1.0 / p->box[a];
        pc.qs[a] = 4294967296.0 / p->box[a];
        pc.qd[a] = (float)(p->box[a] / 4294967296.0);
        pc.mg[a] = p->mass * p->body_force[a];
    }
    pc.rc = p->rc;
    pc.inv_rc = 1.0 / p->rc;
    pc.rd = p->rd;
    pc.inv_rd = 1.0 / p->rd;
    pc.rd2 = p->rd * p->rd;
    pc.wrho = 15.0 / (2.0 * M_PI * p->rd * p->rd * p->rd);
    pc.hdtm = 0.5 * p->dt / p->mass;
    pc.dt = p->dt;
    pc.mass = p->mass;
    pc.phi_c = p->phi_c;
    pc.slip = p->wall_slip;
    // eta rho_f W_D, W_D = 2 pi r_c^3 / 15 (the integral of w_c^2 over the sphere)
    pc.dctl = p->diss_ctrl > 0.0 ? p->diss_ctrl * p->diss_rho * 2.0 * M_PI * p->rc * p->rc * p->rc / 15.0 : 0.0;
    pc.ntypes = p->ntypes;
    const double rdt = 1.0 / sqrt(p->dt);
    pc.A = p->A[0];
    pc.B = p->B[0];
    pc.gamma = p->gamma[0];
    pc.sig = sqrt(2.0 * p->gamma[0] * p->kT) * rdt;
    pc.Arc2 = 0.5 * p->A[0] * p->rc;
    pc.tab = tab;
    pc.seed = p->seed;
    return pc;
}

// Type-pair planes of one replica: A | B | gamma | sig | A r_c / 2.
void fill_pair_table(const mdpd_params *p, double *h)
{
    const double rdt = 1.0 / sqrt(p->dt);
    for (int k = 0; k < 320; ++k) h[k] = 0.0;
    for (int k = 0; k < p->ntypes * p->ntypes; ++k) {
        h[k] = p->A[k];
        h[64 + k] = p->B[k];
        h[128 + k] = p->gamma[k];
        h[192 + k] = sqrt(2.0 * p->gamma[k] * p->kT) * rdt;
        h[256 + k] = 0.5 * p->A[k] * p->rc;
    }
}

mdpd_status create_impl(int32_t nrep, const mdpd_params *ps, const int64_t *offsets, const double *pos,
                        const double *vel, const int32_t *type, const uint8_t *frozen, int32_t mem_kind,
                        void *stream, mdpd_system **out)
{
    if (!out) return fail(MDPD_E_INVALID, "out is NULL");
    *out = nullptr;
    if (nrep < 1 || nrep > 65536) return fail(MDPD_E_INVALID, "nrep = %d not in 1..65536", nrep);
    if (!ps || !offsets) return fail(MDPD_E_INVALID, "params or offsets is NULL");
    if (offsets[0] != 0) return fail(MDPD_E_INVALID, "offsets[0] must be 0");
    for (int r = 0; r < nrep; ++r) {
        if (offsets[r + 1] < offsets[r]) return fail(MDPD_E_INVALID, "offsets must be non-decreasing");
        mdpd_status rc = validate(&ps[r], offsets[r + 1] - offsets[r]);
        if (rc) return rc;
        if (ps[r].precision != ps[0].precision || ps[r].wall_model != ps[0].wall_model)
            return fail(MDPD_E_INVALID, "all replicas need the same precision and wall model");
    }
    const int64_t n = offsets[nrep];
    if (n >= (int64_t)1 << 30) return fail(MDPD_E_INVALID, "n = %lld out of range", (long long)n);
    if (n > 0 && (!pos || !vel || !type || !frozen)) return fail(MDPD_E_INVALID, "NULL particle array");
    if (mem_kind != MDPD_MEM_HOST && mem_kind != MDPD_MEM_DEVICE)
        return fail(MDPD_E_INVALID, "unknown mem_kind %d", mem_kind);

    mdpd_system *s = new mdpd_system();
    s->p = ps[0];
    s->st = (hipStream_t)stream;
    if (hipGetDevice(&s->dev) != hipSuccess) {
        delete s;
        return fail(MDPD_E_HIP, "hipGetDevice failed");
    }
    s->n = (int)n;
    s->nrep = nrep;
    s->fp32 = ps[0].precision == MDPD_FP32_FORCES;
    s->walls = ps[0].wall_model == MDPD_WALL_BVF;
    s->perstep = true;
    for (int r = 0; r < nrep; ++r)
        if (ps[r].skin > 0.0) s->perstep = false;
    for (int r = 0; r < nrep; ++r)
        if (s->walls && ps[r].wall_slip > 0.0) s->slip = true;
    for (int r = 0; r < nrep; ++r)
        if (ps[r].diss_ctrl > 0.0) s->dctl = true;
    s->params.assign(ps, ps + nrep);
    s->geoms.resize(nrep);
    s->cell_off.assign(nrep + 1, 0);
    s->part_off.assign(nrep + 1, 0);
    s->blk_off.assign((size_t)kLaneCounts * (nrep + 1), 0);
    int64_t cells = 0;
    for (int r = 0; r < nrep; ++r) {
        mdpd_status rc = make_geom(&ps[r], &s->geoms[r]);
        if (rc) {
            delete s;
            return rc;
        }
        cells += s->geoms[r].ncells;
        if (cells > (int64_t)1 << 26) {
            delete s;
            return fail(MDPD_E_UNSUPPORTED, "more than 2^26 cells in total");
        }
        s->cell_off[r + 1] = (int)cells;
        s->part_off[r + 1] = (int)offsets[r + 1];
        s->mt = s->mt || ps[r].ntypes > 1;
        for (int li = 0; li < kLaneCounts; ++li) {
            const int64_t P = (int64_t)1 << li;
            const int64_t nr = offsets[r + 1] - offsets[r];
            int *bo = &s->blk_off[(size_t)li * (nrep + 1)];
            bo[r + 1] = bo[r] + (int)((nr * P + kBlock - 1) / kBlock);
        }
    }

    // per-step list: the border cells (a periodic image in their 27-cell
    // stencil), replica after replica in cell order, have a launch of their
    // own; a small system takes all its cells in that one launch (the second
    // launch would cost more than it saves)
    std::vector<int> bcells, icells;
    const bool one_launch = cells <= kOneListLaunchCells;
    if (s->perstep)
        for (int r = 0; r < nrep; ++r) {
            const int *nc = s->geoms[r].nc;
            for (int cz = 0; cz < nc[2]; ++cz)
                for (int cy = 0; cy < nc[1]; ++cy)
                    for (int cx = 0; cx < nc[0]; ++cx) {
                        const int c = s->cell_off[r] + cx + nc[0] * (cy + nc[1] * cz);
                        if (one_launch || cx == 0 || cx == nc[0] - 1 || cy == 0 || cy == nc[1] - 1 || cz == 0 ||
                            cz == nc[2] - 1)
                            bcells.push_back(c);
                        else
                            icells.push_back(c);
                    }
        }
    const size_t N = (size_t)(n > 0 ? n : 1);
    const int nb_scan = (int)((cells + 4095) / 4096);
    Reps &R = s->R;
    R.nrep = nrep;
    R.ncells = (int)cells;
    R.nbcells = (int)bcells.size();
    R.list_interior = one_launch ? 0 : 1;
    R.list_split = s->lanes[0];
    // every-step sort in one workgroup per replica for a batch of many
    // replicas (measured: 256 replicas of 3,000 to 10,000 particles 1.021
    // against 1.033 ms per step; a single 6,000-particle system 47 against
    // 41 us, one workgroup being slower than five launches over the whole
    // chip), when each replica's cell offsets and ids fit its LDS (64 KiB)
    // and its particles the threads
    R.sort_small_lds = 0;
    if (s->perstep && nrep >= kSortSmallMinReplicas) {
        int64_t need = 0;
        bool fits = true;
        for (int r = 0; r < nrep; ++r) {
            const int64_t nr = offsets[r + 1] - offsets[r], mr = s->geoms[r].ncells;
            fits = fits && nr <= kSortSmallMaxN && mr <= kSortSmallMaxCells;
            need = std::max(need, 4 * (mr + 1 + nr));
        }
        if (fits && need <= kSortSmallMaxLds) R.sort_small_lds = (int)need;
    }
    for (int li = 0; li < kLaneCounts; ++li) R.nblk[li] = s->blk_off[(size_t)li * (nrep + 1) + nrep];
#define ALLOC(call)                 \
    do {                            \
        mdpd_status e_ = (call);    \
        if (e_) {                   \
            delete s;               \
            return e_;              \
        }                           \
    } while (0)
    for (int k = 0; k < 2; ++k) {
        ALLOC(s->alloc3(&s->xs[k], N));
        ALLOC(s->alloc3(&s->vh[k], N));
        ALLOC(s->alloc(&s->tag[k], N));
        ALLOC(s->alloc(&s->typ[k], N));
    }
    ALLOC(s->alloc3(&s->tx, N));
    ALLOC(s->alloc3(&s->tv, N));
    ALLOC(s->alloc3(&s->xb, N));
    ALLOC(s->alloc3(&s->v, N));
    ALLOC(s->alloc3(&s->F, N));
    if (s->walls) ALLOC(s->alloc3(&s->tp, N));
    if (s->walls) {
        // wall mask: 4 sub-cells per cell edge while it stays within 64 MiB
        R.wsub = cells <= ((int64_t)1 << 20) ? 4 : cells <= ((int64_t)1 << 23) ? 2 : 1;
        s->wmask_bytes = (size_t)cells * (size_t)(R.wsub * R.wsub * R.wsub);
        ALLOC(s->alloc(&s->wmask, s->wmask_bytes));
    }
    {
        double *r = nullptr;
        ALLOC(s->alloc(&r, N));
        s->rho = r;
    }
    ALLOC(s->alloc(&s->key, N));
    ALLOC(s->alloc(&s->slot, N));
    ALLOC(s->alloc(&s->tmpid, N));
    ALLOC(s->alloc(&s->rec, N));
    ALLOC(s->alloc(&s->ncnt, N));
    ALLOC(s->alloc(&s->nl, N * kListCap));
    if (s->perstep) {
        double *r2 = nullptr;
        ALLOC(s->alloc(&r2, s->fp32 ? N * kListCap / 2 : N * kListCap));
        s->nlr2 = r2;
    } else {
        ALLOC(s->alloc(&s->scnt, N));
        ALLOC(s->alloc(&s->sl, N * kSkinCap));
    }
    ALLOC(s->alloc(&s->bmax, (size_t)R.nblk[kLaneCounts - 1] + 1));
    ALLOC(s->alloc(&s->flags, (size_t)nrep + 3));
    ALLOC(s->alloc(&s->nbuild, 1));
    ALLOC(s->alloc(&s->counts, (size_t)cells));
    ALLOC(s->alloc(&s->cstart, (size_t)cells + 1));
    ALLOC(s->alloc(&s->cnew, (size_t)cells + 1));
    ALLOC(s->alloc(&s->bsum, (size_t)nb_scan + 1));
    ALLOC(s->alloc(&s->fpart, 2 * (size_t)(R.nblk[kLaneCounts - 1] + 1)));
    ALLOC(s->alloc(&s->status, 4));
    ALLOC(s->alloc(&s->dstep, 1));
    ALLOC(s->alloc(&s->corr, N + 1 + (size_t)R.nblk[0] + 1));
    ALLOC(s->alloc(&s->ovf, N + 1));
    ALLOC(s->alloc(&s->ovf_ve, 2 * N));
    ALLOC(s->alloc(&s->ncorr_total, 1));
    ALLOC(s->alloc(&s->tab, 320 * (size_t)nrep));
    ALLOC(s->alloc(&s->obs, 16 * (size_t)nrep));
    ALLOC(s->alloc(&s->obs_part, (size_t)obs_partials(R) + 16));
    ALLOC(s->alloc(&s->io, 3 * N));
    ALLOC(s->alloc(&s->io2, 3 * N));
    ALLOC(s->alloc(&s->work, 9 * 4096));
    Geom *dgeom = nullptr;
    PairConst *dpc = nullptr;
    int *dcell = nullptr, *dpart = nullptr, *dblk = nullptr, *dbcells = nullptr, *dcrep = nullptr;
    ALLOC(s->alloc(&dbcells, bcells.size() + 1));
    int *dicells = nullptr;
    ALLOC(s->alloc(&dicells, icells.size() + 1));
    // the replica of each cell, for the kernels with one wavefront per cell
    // (a table lookup instead of a binary search over the cell offsets)
    // and of each block of the particle launches, lane count after lane count
    std::vector<int> cell_rep, blk_rep;
    int *dbrep = nullptr;
    if (nrep > 1) {
        cell_rep.resize((size_t)cells);
        for (int r = 0; r < nrep; ++r)
            for (int c = s->cell_off[r]; c < s->cell_off[r + 1]; ++c) cell_rep[(size_t)c] = r;
        ALLOC(s->alloc(&dcrep, cell_rep.size()));
        for (int li = 0; li < kLaneCounts; ++li) {
            const int *bo = &s->blk_off[(size_t)li * (nrep + 1)];
            for (int r = 0; r < nrep; ++r)
                for (int b = bo[r]; b < bo[r + 1]; ++b) blk_rep.push_back(r);
        }
        ALLOC(s->alloc(&dbrep, blk_rep.size() + 1));
    }
    ALLOC(s->alloc(&dgeom, (size_t)nrep));
    ALLOC(s->alloc(&dpc, (size_t)nrep));
    ALLOC(s->alloc(&dcell, (size_t)nrep + 1));
    ALLOC(s->alloc(&dpart, (size_t)nrep + 1));
    ALLOC(s->alloc(&dblk, s->blk_off.size()));
#undef ALLOC
    R.geom = dgeom;
    R.pc = dpc;
    R.cell_off = dcell;
    R.cell_rep = dcrep;
    R.blk_rep = dbrep;
    R.part_off = dpart;
    R.blk_off = dblk;
    R.flag = s->flags;
    R.bcells = dbcells;
    R.icells = dicells;
    R.nicells = (int)icells.size();

    auto bail = [&](mdpd_status st) {
        delete s;
        return st;
    };
    // replica tables
    {
        std::vector<double> tabs((size_t)320 * nrep);
        s->pcs.resize(nrep);
        for (int r = 0; r < nrep; ++r) {
            fill_pair_table(&ps[r], &tabs[(size_t)320 * r]);
            s->pcs[r] = make_pair_const(&ps[r], s->tab + (size_t)320 * r);
        }
        hipError_t e = hipMemcpyAsync(s->tab, tabs.data(), tabs.size() * sizeof(double), hipMemcpyHostToDevice,
                                      s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dgeom, s->geoms.data(), nrep * sizeof(Geom), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dpc, s->pcs.data(), nrep * sizeof(PairConst), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dcell, s->cell_off.data(), (nrep + 1) * sizeof(int), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dpart, s->part_off.data(), (nrep + 1) * sizeof(int), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dblk, s->blk_off.data(), s->blk_off.size() * sizeof(int), hipMemcpyHostToDevice,
                               s->st);
        if (e == hipSuccess && !bcells.empty())
            e = hipMemcpyAsync(dbcells, bcells.data(), bcells.size() * sizeof(int), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess && !icells.empty())
            e = hipMemcpyAsync(dicells, icells.data(), icells.size() * sizeof(int), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess && !blk_rep.empty())
            e = hipMemcpyAsync(dbrep, blk_rep.data(), blk_rep.size() * sizeof(int), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess && !cell_rep.empty())
            e = hipMemcpyAsync(dcrep, cell_rep.data(), cell_rep.size() * sizeof(int), hipMemcpyHostToDevice,
                               s->st);
        if (e == hipSuccess) e = hipStreamSynchronize(s->st);
        if (e != hipSuccess) return bail(fail(MDPD_E_HIP, "upload of replica tables failed: %s", hipGetErrorString(e)));
    }

    hipError_t e = hipSuccess;
    launch_zero_int(s->st, s->status, 4);
    {
        // the gate at creation advances it to step 0
        static const uint32_t before_first = 0xFFFFFFFFu;
        e = hipMemcpyAsync(s->dstep, &before_first, sizeof before_first, hipMemcpyHostToDevice, s->st);
        if (e != hipSuccess) return bail(fail(MDPD_E_HIP, "step counter init failed: %s", hipGetErrorString(e)));
    }
    launch_zero_int(s->st, (int *)s->ncorr_total, 2);
    launch_zero_int(s->st, (int *)s->nbuild, 2);
    launch_zero_int(s->st, (int *)s->bmax, R.nblk[kLaneCounts - 1] + 1);
    launch_zero_int(s->st, s->flags, nrep + 3);
    launch_set_int(s->st, s->flags + nrep + 2, 1);  // the first gate builds every replica
    launch_zero_int(s->st, s->counts, (int)cells);
    launch_zero_int(s->st, s->corr, (int)N + 1);
    launch_zero_int(s->st, s->ovf, 1);

    // inputs: stage host arrays in device memory
    const double *dpos = pos, *dvel = vel;
    const int32_t *dtype = type;
    const uint8_t *dfz = frozen;
    int32_t *stype = nullptr;
    uint8_t *sfz = nullptr;
    if (n > 0 && mem_kind == MDPD_MEM_HOST) {
        if (s->alloc(&stype, N) || s->alloc(&sfz, N)) return bail(MDPD_E_OOM);
        e = hipMemcpyAsync(s->io, pos, 3 * N * sizeof(double), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess) e = hipMemcpyAsync(s->io2, vel, 3 * N * sizeof(double), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess) e = hipMemcpyAsync(stype, type, N * sizeof(int32_t), hipMemcpyHostToDevice, s->st);
        if (e == hipSuccess) e = hipMemcpyAsync(sfz, frozen, N, hipMemcpyHostToDevice, s->st);
        if (e != hipSuccess) return bail(fail(MDPD_E_HIP, "input upload failed: %s", hipGetErrorString(e)));
        dpos = s->io;
        dvel = s->io2;
        dtype = stype;
        dfz = sfz;
    }
    s->cur = 0;
    // the inputs become the state the first gate sorts: xs[0], vh[0], or
    // with skin 0 the predicted state tx, tv
    launch_ingest(s->st, R, dpos, dvel, dtype, dfz, s->perstep ? s->tx : s->xs[0], s->perstep ? s->tv : s->vh[0],
                  s->tag[0], s->typ[0], s->status);
    int hstatus = 0;
    e = hipMemcpyAsync(&hstatus, s->status, sizeof(int), hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return bail(fail(MDPD_E_HIP, "ingest failed: %s", hipGetErrorString(e)));
    if (stype) {
        s->release(stype);
        s->release(sfz);
    }
    if (hstatus & 2)
        return bail(fail(MDPD_E_INVALID,
                         "input has a non-finite value, a position outside [-L, 2L) or a bad type"));

    // t = 0: sort, lists, density, forces with the given velocities and noise step 0
    s->gate_and_rebuild();
    if (s->walls) {
        hipError_t ez = hipMemsetAsync(s->wmask, 0, s->wmask_bytes, s->st);
        if (ez != hipSuccess) return bail(fail(MDPD_E_HIP, "wall mask: %s", hipGetErrorString(ez)));
        launch_mark_wall_cells(s->st, R, cview(s->xs[s->cur]), s->tag[0], s->wmask);
    }
    s->evaluate(1);
    e = hipMemcpyAsync(&hstatus, s->status, sizeof(int), hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return bail(fail(MDPD_E_HIP, "initial evaluation failed: %s", hipGetErrorString(e)));
    if (hstatus) return bail(fail(MDPD_E_NONFINITE, "non-finite state after the initial evaluation"));
    *out = s;
    return MDPD_OK;
}

}  // namespace

extern "C" {

mdpd_status mdpd_create(const mdpd_params *p, int64_t n, const double *pos, const double *vel,
                        const int32_t *type, const uint8_t *frozen, int32_t mem_kind, void *stream,
                        mdpd_system **out)
{
    if (n < 0 || n >= (int64_t)1 << 30) {
        if (out) *out = nullptr;
        return fail(MDPD_E_INVALID, "n = %lld out of range", (long long)n);
    }
    const int64_t offsets[2] = {0, n};
    return create_impl(1, p, offsets, pos, vel, type, frozen, mem_kind, stream, out);
}

mdpd_status mdpd_create_batch(int32_t nrep, const mdpd_params *params, const int64_t *offsets, const double *pos,
                              const double *vel, const int32_t *type, const uint8_t *frozen, int32_t mem_kind,
                              void *stream, mdpd_system **out)
{
    return create_impl(nrep, params, offsets, pos, vel, type, frozen, mem_kind, stream, out);
}

mdpd_status mdpd_step(mdpd_system *s, int64_t nsteps)
{
    if (!s) return fail(MDPD_E_INVALID, "system is NULL");
    if (nsteps < 0) return fail(MDPD_E_INVALID, "nsteps < 0");
    if (s->use_graph && s->n > 0) {
        while (nsteps >= 2) {
            if (!s->graph_valid() && s->force_lanes_used != s->lanes[2]) {
                // the captured gate reads the block maxima of the force pass
                // in the layout of the graph's own force lanes
                s->advance(1);
                nsteps -= 1;
                continue;
            }
            if (!s->graph_valid()) HIPCHK(s->capture_pair());
            HIPCHK(hipGraphLaunch(s->gexec, s->st));
            s->step += 2;
            nsteps -= 2;
        }
    }
    s->advance(nsteps);
    int hstatus = 0;
    HIPCHK(hipMemcpyAsync(&hstatus, s->status, sizeof(int), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    HIPCHK(hipGetLastError());
    if (hstatus) return fail(MDPD_E_NONFINITE, "non-finite or out-of-box state at step %lld", (long long)s->step);
    return MDPD_OK;
}

mdpd_status mdpd_read_replica_observables(mdpd_system *s, int32_t first, int32_t count, mdpd_observables *out)
{
    if (!s || !out) return fail(MDPD_E_INVALID, "NULL argument");
    if (first < 0 || count < 0 || first + count > s->nrep)
        return fail(MDPD_E_INVALID, "replicas [%d, %d) outside [0, %d)", first, first + count, s->nrep);
    launch_observables(s->st, s->fp32, s->R, s->force_lanes_used, cview(s->v), s->rho, s->tag[0],
                       s->typ[0], s->fpart, s->ncnt, s->ovf_ve, s->obs_part, s->obs);
    std::vector<double> h((size_t)16 * (count > 0 ? count : 1));
    unsigned long long tot = 0;
    int last = 0;
    if (count > 0)
        HIPCHK(hipMemcpyAsync(h.data(), s->obs + (size_t)16 * first, (size_t)16 * count * sizeof(double),
                              hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(&tot, s->ncorr_total, sizeof tot, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(&last, s->corr, sizeof last, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    for (int k = 0; k < count; ++k) {
        const int r = first + k;
        const double *q = &h[(size_t)16 * k];
        const mdpd_params &p = s->params[r];
        const int64_t nr = s->part_off[r + 1] - s->part_off[r];
        const double m = p.mass;
        const int64_t nf = (int64_t)llround(q[6]);
        const bool driven = p.body_force[0] != 0.0 || p.body_force[1] != 0.0 || p.body_force[2] != 0.0;
        double dof = (double)nf;
        if (nf == nr && !driven) dof -= 1.0;
        const double V = p.box[0] * p.box[1] * p.box[2];
        mdpd_observables &o = out[k];
        memset(&o, 0, sizeof o);
        o.step = s->step;
        o.n = nr;
        o.n_fluid = nf;
        o.ke = 0.5 * m * q[0];
        o.kT = dof > 0 ? m * q[0] / (3.0 * dof) : 0.0;
        o.virial = q[8];
        o.pressure = (m * q[0] + q[8]) / (3.0 * V);
        o.momentum[0] = m * q[1];
        o.momentum[1] = m * q[2];
        o.momentum[2] = m * q[3];
        o.epot = q[9] + M_PI * pow(p.rd, 4) / 30.0 * q[5];
        o.mean_rho = nf > 0 ? q[4] / (double)nf : 0.0;
        o.ncorr_last = s->walls && s->step > 0 ? last : 0;
        o.ncorr_total = (int64_t)tot;
    }
    return MDPD_OK;
}

mdpd_status mdpd_read_stress(mdpd_system *s, int32_t first, int32_t count, double *out)
{
    if (!s || !out) return fail(MDPD_E_INVALID, "NULL argument");
    if (first < 0 || count < 0 || first + count > s->nrep)
        return fail(MDPD_E_INVALID, "replicas [%d, %d) outside [0, %d)", first, first + count, s->nrep);
    const size_t N = (size_t)s->n;
    if (!s->stress) {
        mdpd_status rc = s->alloc(&s->stress, 6 * (N > 0 ? N : 1) + 6 * (size_t)s->nrep);
        if (rc) return rc;
    }
    double *sums = s->stress + 6 * (N > 0 ? N : 1);
    launch_zero_int(s->st, (int *)sums, 12 * s->nrep);
    launch_stress(s->st, s->fp32, s->mt, s->n, s->R, cview(s->xs[s->cur]), cview(s->v), s->rho, s->tag[0],
                  s->typ[0], s->cstart, s->ncnt, s->nl, s->stress, false);
    if (N > 0) launch_stress_sum(s->st, s->R, s->n, s->stress, sums);
    std::vector<double> h(6 * (size_t)(count > 0 ? count : 1));
    if (count > 0)
        HIPCHK(hipMemcpyAsync(h.data(), sums + 6 * (size_t)first, 6 * (size_t)count * sizeof(double),
                              hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    for (int k = 0; k < count; ++k) {
        const mdpd_params &p = s->params[first + k];
        const double V = p.box[0] * p.box[1] * p.box[2];
        for (int a = 0; a < 6; ++a) out[6 * k + a] = h[6 * (size_t)k + a] / V;
    }
    return MDPD_OK;
}

}  // extern "C"

// Scratch of mdpd_read_stress_noalloc: a fixed array in device memory (one
// copy per GPU, held until the process ends), so that the call allocates
// nothing.  Host code reaches it only through the address hipGetSymbolAddress
// returns on each device; the array's own name is not a device address there.
constexpr size_t kNoallocScratch = (size_t)1 << 20;  // doubles: 8 MiB per GPU
static __device__ __align__(256) double scratch[kNoallocScratch];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// The scratch address on the current device, looked up once per device.
mdpd_status scratch_on_device(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(MDPD_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MDPD_E_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                        hipGetErrorString(e));
        g_scratch[dev] = (double *)p;
    }
    *out = g_scratch[dev];
    return MDPD_OK;
}

}  // namespace

extern "C" {

mdpd_status mdpd_read_stress_noalloc(mdpd_system *s, int32_t first, int32_t count, double *out, int32_t mem_kind)
{
    if (!s || !out) return fail(MDPD_E_INVALID, "NULL argument");
    if (first < 0 || count < 0 || first + count > s->nrep)
        return fail(MDPD_E_INVALID, "replicas [%d, %d) outside [0, %d)", first, first + count, s->nrep);
    if (mem_kind != MDPD_MEM_HOST && mem_kind != MDPD_MEM_DEVICE)
        return fail(MDPD_E_INVALID, "unknown mem_kind %d", mem_kind);
    if (count == 0) return MDPD_OK;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != s->dev)
        return fail(MDPD_E_STATE, "device %d is current; the system lives on device %d", dev, s->dev);
    const size_t nb = (size_t)s->R.nblk[lanes_index(kStressLanes)];
    const size_t need = 6 * nb + 6 * (size_t)count;
    if (need > kNoallocScratch)
        return fail(MDPD_E_UNSUPPORTED,
                    "%zu scratch doubles needed (%zu blocks), the fixed scratch holds %zu (about %zu particles)",
                    need, nb, kNoallocScratch, kNoallocScratch / 6 * (kBlock / kStressLanes));
    double *ptr = nullptr;
    mdpd_status rc = scratch_on_device(dev, &ptr);
    if (rc) return rc;
    double *parts = ptr, *res = ptr + 6 * nb;
    // every block writes its partial sums and the reduction writes every
    // result, so nothing left by an earlier call is read
    launch_stress(s->st, s->fp32, s->mt, s->n, s->R, cview(s->xs[s->cur]), cview(s->v), s->rho, s->tag[0],
                  s->typ[0], s->cstart, s->ncnt, s->nl, parts, true);
    launch_stress_part_sum(s->st, s->R, first, count, parts, mem_kind == MDPD_MEM_DEVICE ? out : res);
    HIPCHK(hipGetLastError());
    if (mem_kind == MDPD_MEM_HOST) {
        HIPCHK(hipMemcpyAsync(out, res, 6 * (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
    }
    return MDPD_OK;
}

mdpd_status mdpd_read_list_builds(mdpd_system *s, int64_t *builds)
{
    if (!s || !builds) return fail(MDPD_E_INVALID, "NULL argument");
    unsigned long long b = 0;
    HIPCHK(hipMemcpyAsync(&b, s->nbuild, sizeof b, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    *builds = (int64_t)b;
    return MDPD_OK;
}

mdpd_status mdpd_read_observables(mdpd_system *s, mdpd_observables *out)
{
    if (!s || !out) return fail(MDPD_E_INVALID, "NULL argument");
    if (s->nrep != 1) return fail(MDPD_E_STATE, "a batch of replicas: use mdpd_read_replica_observables");
    return mdpd_read_replica_observables(s, 0, 1, out);
}

mdpd_status mdpd_read_profile(mdpd_system *s, int32_t axis, int32_t nbins, int32_t quantity, double *out)
{
    if (!s || !out) return fail(MDPD_E_INVALID, "NULL argument");
    if (s->nrep != 1) return fail(MDPD_E_UNSUPPORTED, "profiles are for single systems");
    if (axis < 0 || axis > 2 || nbins < 1 || nbins > 4096 || quantity < 0 || quantity > 5)
        return fail(MDPD_E_INVALID, "bad profile request (axis %d, nbins %d, quantity %d)", axis, nbins,
                    quantity);
    const double binvol = s->p.box[0] * s->p.box[1] * s->p.box[2] / nbins;
    double *res = s->work + 9 * nbins;
    if ((size_t)(10 * nbins) > (size_t)9 * 4096) res = s->io;  // large nbins: use staging
    launch_profile(s->st, s->fp32, s->n, axis, nbins, quantity, s->p.box[axis], binvol, s->p.mass,
                   cview(s->xs[s->cur]), cview(s->v), s->rho, s->tag[0], s->work, res);
    HIPCHK(hipMemcpyAsync(out, res, nbins * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return MDPD_OK;
}

mdpd_status mdpd_get_state(mdpd_system *s, double *pos, double *vel, double *rho, int32_t mem_kind)
{
    if (!s) return fail(MDPD_E_INVALID, "system is NULL");
    if (mem_kind != MDPD_MEM_HOST && mem_kind != MDPD_MEM_DEVICE)
        return fail(MDPD_E_INVALID, "unknown mem_kind %d", mem_kind);
    const size_t N = (size_t)s->n;
    if (N == 0) return MDPD_OK;
    if (mem_kind == MDPD_MEM_DEVICE) {
        launch_export(s->st, s->fp32, s->R, cview(s->xs[s->cur]), cview(s->v), s->rho, s->tag[0], pos,
                      vel, rho);
        HIPCHK(hipStreamSynchronize(s->st));
        return MDPD_OK;
    }
    launch_export(s->st, s->fp32, s->R, cview(s->xs[s->cur]), cview(s->v), s->rho, s->tag[0],
                  pos ? s->io : nullptr, vel ? s->io2 : nullptr, nullptr);
    if (pos) HIPCHK(hipMemcpyAsync(pos, s->io, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s->st));
    if (vel) HIPCHK(hipMemcpyAsync(vel, s->io2, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    if (rho) {
        launch_export(s->st, s->fp32, s->R, cview(s->xs[s->cur]), cview(s->v), s->rho, s->tag[0],
                      nullptr, nullptr, s->io);
        HIPCHK(hipMemcpyAsync(rho, s->io, N * sizeof(double), hipMemcpyDeviceToHost, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
    }
    return MDPD_OK;
}

}  // extern "C"

// Checkpoint layout: header, parameters, then the arrays in the order of
// ckpt_fields(); every field starts on a 256-byte boundary.
namespace {

constexpr uint64_t kCkptMagic = 0x3250544b4350444dull;  // "MDPDCKP2": version 2 (skin-list state)
constexpr uint64_t kCkptAlign = 256;

struct CkptHeader {
    uint64_t magic;
    int64_t n;
    int64_t step;
    int64_t force_lanes;
    int64_t ncells;
    int64_t nrep;
    int64_t reserved[2];
};

struct CkptField {
    void *dev;
    uint64_t bytes;
};

std::vector<CkptField> ckpt_fields(mdpd_system *s)
{
    const uint64_t N = (uint64_t)s->n;
    const int c = s->cur;
    const uint64_t rb = s->fp32 ? 4 : 8;
    const uint64_t nb = (uint64_t)s->R.nblk[kLaneCounts - 1];
    return {
        {s->xs[c].x, 24 * N},          {s->v.x, 24 * N},         {s->F.x, 24 * N},
        {s->next_x().x, 24 * N},       {s->next_v().x, 24 * N},  {s->rho, rb * N},
        {s->tag[0], 4 * N},            {s->typ[0], N},           {s->ovf_ve, 16 * N},
        {s->cstart, 4 * ((uint64_t)s->R.ncells + 1)},
        {s->fpart, 16 * nb},
        {s->ncorr_total, 8},           {s->corr, 4},
        {s->dstep, 4},
        {s->xb.x, s->perstep ? 0 : 24 * N}, {s->bmax, 4 * nb},   {s->nbuild, 8},
    };
}

uint64_t align_up(uint64_t x) { return (x + kCkptAlign - 1) / kCkptAlign * kCkptAlign; }

// Bytes of the state arrays of a checkpoint (without header and parameters).
uint64_t state_bytes(mdpd_system *s)
{
    uint64_t off = 0;
    for (const CkptField &f : ckpt_fields(s)) off += align_up(f.bytes);
    return off;
}

// Header and the parameters of every replica.
uint64_t head_bytes(const mdpd_system *s) { return align_up(sizeof(CkptHeader) + s->nrep * sizeof(mdpd_params)); }

uint64_t ckpt_bytes(mdpd_system *s) { return head_bytes(s) + state_bytes(s); }

// The parameters stored in a checkpoint equal the system's, byte for byte.
bool params_match(mdpd_system *s, const char *in, hipMemcpyKind hk)
{
    std::vector<mdpd_params> q(s->nrep);
    if (hipMemcpyAsync(q.data(), in + sizeof(CkptHeader), s->nrep * sizeof(mdpd_params), hk, s->st) != hipSuccess)
        return false;
    if (hipStreamSynchronize(s->st) != hipSuccess) return false;
    return memcmp(q.data(), s->params.data(), s->nrep * sizeof(mdpd_params)) == 0;
}

// Enqueue copies of the state arrays to / from dst (kind: the direction).
hipError_t state_copy(mdpd_system *s, char *buf, bool save, hipMemcpyKind kind)
{
    uint64_t off = 0;
    for (const CkptField &f : ckpt_fields(s)) {
        if (f.bytes) {
            hipError_t e = save ? hipMemcpyAsync(buf + off, f.dev, f.bytes, kind, s->st)
                                : hipMemcpyAsync(f.dev, buf + off, f.bytes, kind, s->st);
            if (e != hipSuccess) return e;
        }
        off += align_up(f.bytes);
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

mdpd_status mdpd_checkpoint_size(const mdpd_system *s, uint64_t *bytes)
{
    if (!s || !bytes) return fail(MDPD_E_INVALID, "NULL argument");
    *bytes = ckpt_bytes(const_cast<mdpd_system *>(s));
    return MDPD_OK;
}

mdpd_status mdpd_save_checkpoint(mdpd_system *s, void *buf, uint64_t bytes, int32_t mem_kind)
{
    if (!s || !buf) return fail(MDPD_E_INVALID, "NULL argument");
    if (mem_kind != MDPD_MEM_HOST && mem_kind != MDPD_MEM_DEVICE)
        return fail(MDPD_E_INVALID, "unknown mem_kind %d", mem_kind);
    const uint64_t need = ckpt_bytes(s);
    if (bytes < need) return fail(MDPD_E_INVALID, "checkpoint buffer of %llu bytes, need %llu",
                                  (unsigned long long)bytes, (unsigned long long)need);
    const hipMemcpyKind dk = mem_kind == MDPD_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    const hipMemcpyKind hk = mem_kind == MDPD_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyHostToDevice;
    CkptHeader h{};
    h.magic = kCkptMagic;
    h.n = s->n;
    h.step = s->step;
    h.force_lanes = s->force_lanes_used;
    h.ncells = s->R.ncells;
    h.nrep = s->nrep;
    char *out = (char *)buf;
    HIPCHK(hipMemcpyAsync(out, &h, sizeof h, hk, s->st));
    HIPCHK(hipMemcpyAsync(out + sizeof h, s->params.data(), s->nrep * sizeof(mdpd_params), hk, s->st));
    HIPCHK(state_copy(s, out + head_bytes(s), true, dk));
    HIPCHK(hipStreamSynchronize(s->st));
    return MDPD_OK;
}

mdpd_status mdpd_load_checkpoint(mdpd_system *s, const void *buf, uint64_t bytes, int32_t mem_kind)
{
    if (!s || !buf) return fail(MDPD_E_INVALID, "NULL argument");
    if (mem_kind != MDPD_MEM_HOST && mem_kind != MDPD_MEM_DEVICE)
        return fail(MDPD_E_INVALID, "unknown mem_kind %d", mem_kind);
    const uint64_t need = ckpt_bytes(s);
    if (bytes < head_bytes(s)) return fail(MDPD_E_INVALID, "checkpoint buffer too small");
    const char *in = (const char *)buf;
    const hipMemcpyKind hk = mem_kind == MDPD_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost;
    const hipMemcpyKind dk = mem_kind == MDPD_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    CkptHeader h{};
    HIPCHK(hipMemcpyAsync(&h, in, sizeof h, hk, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    if (h.magic != kCkptMagic) return fail(MDPD_E_INVALID, "buffer does not hold an mdpd checkpoint");
    if (h.n != s->n || h.ncells != s->R.ncells || h.nrep != s->nrep || !params_match(s, in, hk))
        return fail(MDPD_E_INVALID, "checkpoint was saved from a system with other parameters or n");
    if (bytes < need) return fail(MDPD_E_INVALID, "checkpoint buffer of %llu bytes, need %llu",
                                  (unsigned long long)bytes, (unsigned long long)need);
    if (h.force_lanes != 1 && h.force_lanes != 2 && h.force_lanes != 4 && h.force_lanes != 8 &&
        h.force_lanes != 16)
        return fail(MDPD_E_INVALID, "corrupt checkpoint");
    s->force_lanes_used = (int)h.force_lanes;
    s->step = h.step;
    HIPCHK(state_copy(s, const_cast<char *>(in) + head_bytes(s), false, dk));
    launch_zero_int(s->st, s->status, 1);  // the loaded state's own status starts clean
    if (s->walls) {  // the wall mask follows the frozen particles of the loaded state
        HIPCHK(hipMemsetAsync(s->wmask, 0, s->wmask_bytes, s->st));
        launch_mark_wall_cells(s->st, s->R, cview(s->xs[s->cur]), s->tag[0], s->wmask);
    }
    s->restore_lists();
    HIPCHK(hipStreamSynchronize(s->st));
    HIPCHK(hipGetLastError());
    return MDPD_OK;
}

mdpd_status mdpd_debug_forces(mdpd_system *s, double *force)
{
    if (!s || !force) return fail(MDPD_E_INVALID, "NULL argument");
    const size_t N = (size_t)s->n;
    if (N == 0) return MDPD_OK;
    launch_export(s->st, false, s->R, cview(s->F), Soa3c{nullptr, nullptr, nullptr}, nullptr, s->tag[0],
                  s->io, nullptr, nullptr);
    HIPCHK(hipMemcpyAsync(force, s->io, 3 * N * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return MDPD_OK;
}

mdpd_status mdpd_debug_neighbors(mdpd_system *s, double cutoff, int64_t *count, uint64_t *hash)
{
    if (!s || !count || !hash) return fail(MDPD_E_INVALID, "NULL argument");
    for (const mdpd_params &q : s->params)
        if (!(cutoff > 0.0) || cutoff > q.rc) return fail(MDPD_E_INVALID, "cutoff must be in (0, rc]");
    const size_t N = (size_t)s->n;
    if (N == 0) return MDPD_OK;
    int64_t *dc = (int64_t *)s->io;
    uint64_t *dh = (uint64_t *)s->io2;
    launch_debug_neighbors(s->st, s->R, cutoff * cutoff, cview(s->xs[s->cur]), s->tag[0], s->cstart,
                           s->ncnt, s->nl, dc, dh);
    HIPCHK(hipMemcpyAsync(count, dc, N * sizeof(int64_t), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(hash, dh, N * sizeof(uint64_t), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    return MDPD_OK;
}

mdpd_status mdpd_set_kernel_timing(mdpd_system *s, int32_t enable)
{
    if (!s) return fail(MDPD_E_INVALID, "system is NULL");
    s->timing = enable != 0;
    return MDPD_OK;
}

mdpd_status mdpd_read_kernel_timing(mdpd_system *s, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!s || !total_ms || !launches) return fail(MDPD_E_INVALID, "NULL argument");
    if (kernel < 0 || kernel >= kTimedKernels) return fail(MDPD_E_INVALID, "kernel class %d", kernel);
    HIPCHK(hipStreamSynchronize(s->st));
    EventPool &pl = s->pool[kernel];
    double tot = 0.0;
    for (size_t k = 0; k + 1 < pl.used; k += 2) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, pl.ev[k], pl.ev[k + 1]));
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)(pl.used / 2);
    pl.used = 0;
    return MDPD_OK;
}

mdpd_status mdpd_set_graph(mdpd_system *s, int32_t enable)
{
    if (!s) return fail(MDPD_E_INVALID, "system is NULL");
    s->use_graph = enable != 0;
    if (!s->use_graph) {
        HIPCHK(s->st ? hipStreamSynchronize(s->st) : hipDeviceSynchronize());
        s->drop_graph();
    }
    return MDPD_OK;
}

mdpd_status mdpd_set_lanes(mdpd_system *s, int32_t pass, int32_t lanes)
{
    if (!s) return fail(MDPD_E_INVALID, "system is NULL");
    if (pass < 0 || pass > 2) return fail(MDPD_E_INVALID, "pass %d not in 0..2", pass);
    if (lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16)
        return fail(MDPD_E_INVALID, "lanes %d not in {1, 2, 4, 8, 16}", lanes);
    s->lanes[pass] = lanes;
    s->R.list_split = s->lanes[0];
    return MDPD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner: lanes per particle of the density and force passes, timed with
// HIP events on the system's own stream, cached per shape for the process.
// ---------------------------------------------------------------------------
namespace {

using TuneKey = std::tuple<int, int, int, int, int, int>;  // n, cells, nrep, fp32, types > 1, walls

std::mutex g_tune_mu;
std::map<TuneKey, std::vector<int>> g_tune_cache;

TuneKey tune_key(const mdpd_system *s)
{
    return TuneKey{s->n, s->R.ncells, s->nrep, s->fp32 ? 1 : 0, s->mt ? 1 : 0, s->walls ? 1 : 0};
}

}  // namespace

extern "C" {

mdpd_status mdpd_autotune(mdpd_system *s, int32_t steps, int32_t *lanes_out)
{
    if (!s) return fail(MDPD_E_INVALID, "system is NULL");
    if (steps < 1) return fail(MDPD_E_INVALID, "steps must be >= 1");
    const TuneKey key = tune_key(s);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            for (int k = 0; k < 3; ++k) s->lanes[k] = it->second[k];
            s->R.list_split = s->lanes[0];
            if (lanes_out)
                for (int k = 0; k < 3; ++k) lanes_out[k] = s->lanes[k];
            return MDPD_OK;
        }
    }
    // keep the state: the trial steps must leave no trace
    char *save = nullptr;
    mdpd_status rc = s->alloc(&save, state_bytes(s));
    if (rc) return rc;
    const int cur0 = s->cur, lanes_used0 = s->force_lanes_used;
    const int64_t step0 = s->step;
    const bool timing0 = s->timing;
    HIPCHK(state_copy(s, save, true, hipMemcpyDeviceToDevice));
    s->timing = true;
    const int cand[5] = {1, 2, 4, 8, 16};
    // the list split (skin 0), density (and phi), force
    const int passes[3] = {0, 1, 2}, classes[3] = {1, 2, 3};
    mdpd_status err = MDPD_OK;
    for (int q = s->perstep ? 0 : 1; q < 3 && !err; ++q) {
        double best = 1e300;
        int best_l = s->lanes[passes[q]];
        for (int l : cand) {
            s->lanes[passes[q]] = l;
            s->R.list_split = s->lanes[0];
            s->advance(1);  // warm-up of this instantiation
            double ms = 0.0;
            int64_t cnt = 0;
            if ((err = mdpd_read_kernel_timing(s, classes[q], &ms, &cnt))) break;
            s->advance(steps);
            if ((err = mdpd_read_kernel_timing(s, classes[q], &ms, &cnt))) break;
            if (ms < best) {
                best = ms;
                best_l = l;
            }
        }
        s->lanes[passes[q]] = best_l;
        s->R.list_split = s->lanes[0];
    }
    for (int k = 0; k < kTimedKernels; ++k) {
        double ms;
        int64_t cnt;
        (void)mdpd_read_kernel_timing(s, k, &ms, &cnt);  // clear
    }
    s->timing = timing0;
    s->cur = cur0;
    s->step = step0;
    s->force_lanes_used = lanes_used0;
    HIPCHK(state_copy(s, save, false, hipMemcpyDeviceToDevice));
    launch_zero_int(s->st, s->status, 1);
    s->restore_lists();
    HIPCHK(hipStreamSynchronize(s->st));
    s->release(save);
    if (err) return err;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = std::vector<int>{s->lanes[0], s->lanes[1], s->lanes[2]};
    }
    if (lanes_out)
        for (int k = 0; k < 3; ++k) lanes_out[k] = s->lanes[k];
    return MDPD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adjoint: recorded trajectory, recomputation per segment, backward steps.
// ---------------------------------------------------------------------------
namespace {

// One tape entry: the state of step n in its sorted order, as the backward
// step needs it (x_n, the half-step velocity u_{n-1} its forces used, v_n,
// rho_n, tags, types, cell offsets).
// One recomputed state of a segment: positions, velocities, densities, ids,
// types, cell offsets, and the neighbour list the forward step built for it
// (the backward step reads the same list instead of building it again).
struct TapeEntry {
    Soa3 x, u, v;
    void *rho;
    uint32_t *tag;
    uint8_t *typ;
    int *cstart;
    int *ncnt;
    uint32_t *nl;
    int *perm;      // slot in this state of the particle at slot i of the state before
    uint8_t *corr;  // walls: 1 for the particles (by global id) the corrector sent back in this step
};

uint64_t tape_entry_bytes(mdpd_system *s)
{
    const uint64_t N = (uint64_t)(s->n > 0 ? s->n : 1);
    const uint64_t rb = s->fp32 ? 4 : 8;
    return 3 * align_up(24 * N) + align_up(rb * N) + align_up(4 * N) + align_up(N) +
           align_up(4 * ((uint64_t)s->R.ncells + 1)) + align_up(4 * N) + align_up(4 * N * kListCap) +
           align_up(4 * N) + (s->walls ? align_up(N) : 0);
}

TapeEntry tape_entry(mdpd_system *s, int k)
{
    const uint64_t N = (uint64_t)(s->n > 0 ? s->n : 1);
    const uint64_t rb = s->fp32 ? 4 : 8;
    char *b = s->adj.tape + (uint64_t)k * s->adj.tape_bytes;
    TapeEntry e;
    Soa3 *planes[3] = {&e.x, &e.u, &e.v};
    for (Soa3 *pl : planes) {
        double *d = (double *)b;
        *pl = Soa3{d, d + N, d + 2 * N};
        b += align_up(24 * N);
    }
    e.rho = b;
    b += align_up(rb * N);
    e.tag = (uint32_t *)b;
    b += align_up(4 * N);
    e.typ = (uint8_t *)b;
    b += align_up(N);
    e.cstart = (int *)b;
    b += align_up(4 * ((uint64_t)s->R.ncells + 1));
    e.ncnt = (int *)b;
    b += align_up(4 * N);
    e.nl = (uint32_t *)b;
    b += align_up(4 * N * kListCap);
    e.perm = (int *)b;
    b += align_up(4 * N);
    e.corr = s->walls ? (uint8_t *)b : nullptr;
    return e;
}

// Restores the system's list buffers (and stops recording wall events) when
// it goes out of scope.
struct ListRedirect {
    mdpd_system *s;
    int *ncnt;
    uint32_t *nl;
    ~ListRedirect()
    {
        s->ncnt = ncnt;
        s->nl = nl;
        s->corr_byid = nullptr;
        s->perm_out = nullptr;
    }
};

// The lists of the restored state, its pair list written to tape entry k.
void tape_list(mdpd_system *s, int k)
{
    const TapeEntry e = tape_entry(s, k);
    s->pair_list(e.ncnt, e.nl);
}

// Copy the current state into tape entry k; u is the half-step velocity the
// last force evaluation used (for the state at creation: v(0)).
hipError_t tape_record(mdpd_system *s, int k, bool creation)
{
    const TapeEntry e = tape_entry(s, k);
    const size_t N = (size_t)s->n;
    const int c = s->cur;
    const hipMemcpyKind d2d = hipMemcpyDeviceToDevice;
    hipError_t r = hipSuccess;
    auto cp = [&](void *dst, const void *src, size_t bytes) {
        if (r == hipSuccess && bytes) r = hipMemcpyAsync(dst, src, bytes, d2d, s->st);
    };
    cp(e.x.x, s->xs[c].x, 24 * N);
    cp(e.u.x, creation ? s->v.x : s->vh[c].x, 24 * N);
    cp(e.v.x, s->v.x, 24 * N);
    cp(e.rho, s->rho, (s->fp32 ? 4 : 8) * N);
    cp(e.tag, s->tag[0], 4 * N);
    cp(e.typ, s->typ[0], N);
    cp(e.cstart, s->cstart, 4 * ((size_t)s->R.ncells + 1));
    return r;
}

hipError_t ckpt_store(mdpd_system *s, int k)
{
    s->adj.ck_lanes[k] = s->force_lanes_used;
    return state_copy(s, s->adj.ck + (uint64_t)k * s->adj.ck_bytes, true, hipMemcpyDeviceToDevice);
}

hipError_t ckpt_restore(mdpd_system *s, int k, int64_t step)
{
    s->force_lanes_used = s->adj.ck_lanes[k];
    s->step = step;
    return state_copy(s, s->adj.ck + (uint64_t)k * s->adj.ck_bytes, false, hipMemcpyDeviceToDevice);
}

int64_t ckpt_step(const AdjRec &a, int k) { return k * (int64_t)a.every < a.nsteps ? k * (int64_t)a.every : a.nsteps; }

// Loss weight of state n: the mean over steps 1..N, or the final state.
double seed_weight(const AdjRec &a, int64_t n)
{
    if (a.avg) return n >= 1 ? 1.0 / (double)a.nsteps : 0.0;
    return n == a.nsteps ? 1.0 : 0.0;
}

// Per-replica constants of a backward step with seed weight sw (creation:
// the force adjoint takes h U and there is no drift).
void fill_adj_table(mdpd_system *s, const double *w, double sw, bool creation, AdjConst *out)
{
    for (int r = 0; r < s->nrep; ++r) {
        const mdpd_params &p = s->params[r];
        const double V3 = 3.0 * p.box[0] * p.box[1] * p.box[2];
        const int64_t nf = s->adj.nfluid[r];
        const double inf = nf > 0 ? 1.0 / (double)nf : 0.0;
        const double h = 0.5 * p.dt / p.mass;
        AdjConst &ac = out[r];
        ac.cU = creation ? h : 2.0 * h;
        ac.cv = creation ? 0.0 : h;
        ac.wrho_nf = sw * w[3 * r] * inf;
        ac.wP_3V = sw * w[3 * r + 1] / V3;
        ac.wvx_nf = sw * w[3 * r + 2] * inf;
        ac.mass = p.mass;
        ac.dt = creation ? 0.0 : p.dt;
        ac.pad = 0.0;
    }
}

// Backward step for the state in tape entry k at step n with the
// per-replica constants act.
void adjoint_step(mdpd_system *s, int k, int64_t n, const AdjConst *act)
{
    AdjRec &a = s->adj;
    const TapeEntry e = tape_entry(s, k);
    launch_adj_seed(s->st, s->R, act, cview(e.v), e.tag, a.U, a.fb, a.rhoA);
    s->tic(5);
    if (s->dctl)
        launch_adj_dscale(s->st, s->lanes[1], s->R, cview(e.x), e.tag, e.cstart, e.ncnt, e.nl, a.sdc, a.sdc + s->n);
    launch_adj_force(s->st, s->lanes[2], s->fp32, s->mt, s->dctl, s->n, a.tmax, s->R, (uint32_t)n, act, cview(e.x),
                     cview(e.u), e.rho, e.tag, e.typ, e.cstart, e.ncnt, e.nl, cview(a.fb), a.X, a.U, a.rhoA,
                     a.gp, a.sdc, s->dctl ? a.sdc + s->n : nullptr, s->dctl ? a.sdc + 2 * (size_t)s->n : nullptr);
    launch_adj_density(s->st, s->lanes[1], s->R, cview(e.x), e.cstart, e.ncnt, e.nl, a.rhoA, a.X,
                       s->dctl ? a.sdc + 2 * (size_t)s->n : nullptr);
    s->toc(5);
    launch_adj_params(s->st, s->R, s->n, a.tmax, e.typ, a.gp, a.gpart, a.gtot);
}

}  // namespace

extern "C" {

mdpd_status mdpd_forward_record(mdpd_system *s, int64_t nsteps, int32_t every, int32_t average, double *loss)
{
    if (!s || !loss) return fail(MDPD_E_INVALID, "NULL argument");
    if (nsteps < 0 || every < 1) return fail(MDPD_E_INVALID, "need nsteps >= 0 and every >= 1");
    if (average && nsteps < 1) return fail(MDPD_E_INVALID, "a time average needs nsteps >= 1");
    if (s->slip)
        return fail(MDPD_E_UNSUPPORTED, "the adjoint differentiates the bounce-back wall corrector only (wall_slip = 0)");
    if (s->step != 0) return fail(MDPD_E_STATE, "recording starts from the state given to mdpd_create");
    AdjRec &a = s->adj;
    a.ready = false;
    std::vector<mdpd_observables> o((size_t)s->nrep);
    mdpd_status rc = mdpd_read_replica_observables(s, 0, s->nrep, o.data());
    if (rc) return rc;
    a.nfluid.resize((size_t)s->nrep);
    a.tmax = 1;
    std::vector<LossConst> lc((size_t)s->nrep);
    for (int r = 0; r < s->nrep; ++r) {
        const mdpd_params &p = s->params[r];
        a.nfluid[r] = o[r].n_fluid;
        a.tmax = p.ntypes > a.tmax ? p.ntypes : a.tmax;
        lc[r].inv_nf = o[r].n_fluid > 0 ? 1.0 / (double)o[r].n_fluid : 0.0;
        lc[r].inv3V = 1.0 / (3.0 * p.box[0] * p.box[1] * p.box[2]);
        lc[r].mass = p.mass;
        lc[r].pad = 0.0;
    }
    a.nsteps = nsteps;
    a.every = every;
    a.avg = average ? 1 : 0;
    const int K = (int)((nsteps + every - 1) / every);
    const size_t N = (size_t)(s->n > 0 ? s->n : 1);
    // (re)allocate what the recording needs
    const uint64_t ckb = state_bytes(s), tpb = tape_entry_bytes(s);
    const int ntape = (int)((nsteps < every ? nsteps : every) + 1);
    if (!a.ck || a.nck < K + 1 || a.ck_bytes != ckb) {
        s->release(a.ck);
        a.ck = nullptr;
        rc = s->alloc(&a.ck, (size_t)(K + 1) * ckb);
        if (rc) return rc;
        a.nck = K + 1;
        a.ck_bytes = ckb;
    }
    a.ck_lanes.assign((size_t)K + 1, 4);
    if (!a.tape || a.ntape < ntape || a.tape_bytes != tpb) {
        s->release(a.tape);
        a.tape = nullptr;
        rc = s->alloc(&a.tape, (size_t)ntape * tpb);
        if (rc) return rc;
        a.ntape = ntape;
        a.tape_bytes = tpb;
    }
    const size_t nrep = (size_t)s->nrep;
    if (!a.rhoA) {
        Soa3 *v3[5] = {&a.X, &a.U, &a.fb, &a.Xo, &a.Uo};
        for (Soa3 *q : v3)
            if ((rc = s->alloc3(q, N))) return rc;
        if ((rc = s->alloc(&a.rhoA, N))) return rc;
        if (s->walls && (rc = s->alloc(&s->perm_tmp, 2 * N))) return rc;
        if (s->dctl && (rc = s->alloc(&a.sdc, 3 * N))) return rc;
        if ((rc = s->alloc(&a.gtot, 3 * 64 * nrep))) return rc;
        if ((rc = s->alloc(&a.loss, 3 * nrep + 1))) return rc;
        if ((rc = s->alloc(&a.act, 4 * nrep))) return rc;
        if ((rc = s->alloc(&a.lct, nrep))) return rc;
    }
    if (a.gp_n < 3 * (size_t)a.tmax * N) {
        s->release(a.gp);
        a.gp = nullptr;
        a.gp_n = 3 * (size_t)a.tmax * N;
        if ((rc = s->alloc(&a.gp, a.gp_n))) return rc;
    }
    if (a.gpart_n < (size_t)adj_param_partials(s->R, a.tmax)) {
        s->release(a.gpart);
        a.gpart = nullptr;
        a.gpart_n = (size_t)adj_param_partials(s->R, a.tmax);
        if ((rc = s->alloc(&a.gpart, a.gpart_n))) return rc;
    }
    // run and checkpoint; the loss terms accumulate on the device
    HIPCHK(hipMemcpyAsync(a.lct, lc.data(), nrep * sizeof(LossConst), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipMemsetAsync(a.loss, 0, (3 * nrep + 1) * sizeof(double), s->st));
    auto accum = [&](int64_t n) {
        const double sw = seed_weight(a, n);
        if (sw == 0.0) return;
        launch_observables(s->st, s->fp32, s->R, s->force_lanes_used, cview(s->v), s->rho, s->tag[0],
                           s->typ[0], s->fpart, s->ncnt, s->ovf_ve, s->obs_part, s->obs);
        launch_loss_accum(s->st, s->nrep, s->obs, a.lct, a.loss, sw);
    };
    HIPCHK(ckpt_store(s, 0));
    accum(0);
    for (int k = 1; k <= K; ++k) {
        const int64_t s0 = ckpt_step(a, k - 1), s1 = ckpt_step(a, k);
        for (int64_t n = s0 + 1; n <= s1; ++n) {
            s->advance(1);
            accum(n);
        }
        HIPCHK(ckpt_store(s, k));
    }
    int hstatus = 0;
    HIPCHK(hipMemcpyAsync(loss, a.loss, 3 * nrep * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(&hstatus, s->status, sizeof(int), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    HIPCHK(hipGetLastError());
    if (hstatus) return fail(MDPD_E_NONFINITE, "non-finite or out-of-box state during the recording");
    a.ready = true;
    return MDPD_OK;
}

mdpd_status mdpd_backward(mdpd_system *s, const double *w, double *dA, double *dB, double *dgamma, double *dx0,
                          double *dv0, int32_t mem_kind)
{
    if (!s || !w) return fail(MDPD_E_INVALID, "NULL argument");
    if (mem_kind != MDPD_MEM_HOST && mem_kind != MDPD_MEM_DEVICE)
        return fail(MDPD_E_INVALID, "unknown mem_kind %d", mem_kind);
    AdjRec &a = s->adj;
    if (!a.ready) return fail(MDPD_E_STATE, "no recorded trajectory (call mdpd_forward_record first)");
    const size_t N = (size_t)s->n;
    const size_t nrep = (size_t)s->nrep;
    const int K = (int)((a.nsteps + a.every - 1) / a.every);
    // per-replica constants: steps with the mean-loss weight, steps without a
    // loss term, the final step, and the evaluation at creation
    {
        std::vector<AdjConst> &tab = a.host_act;
        tab.assign(4 * nrep, AdjConst{});
        const double wmid = a.avg ? 1.0 / (double)(a.nsteps > 0 ? a.nsteps : 1) : 0.0;
        fill_adj_table(s, w, wmid, false, &tab[0]);
        fill_adj_table(s, w, 0.0, false, &tab[nrep]);
        fill_adj_table(s, w, a.avg ? wmid : 1.0, false, &tab[2 * nrep]);
        fill_adj_table(s, w, seed_weight(a, 0), true, &tab[3 * nrep]);
        HIPCHK(hipMemcpyAsync(a.act, tab.data(), tab.size() * sizeof(AdjConst), hipMemcpyHostToDevice, s->st));
    }
    auto table = [&](int64_t n) -> const AdjConst * {
        if (n == a.nsteps) return a.act + 2 * nrep;
        return seed_weight(a, n) != 0.0 ? a.act : a.act + nrep;
    };
    HIPCHK(hipMemsetAsync(a.gtot, 0, 3 * 64 * nrep * sizeof(double), s->st));
    if (N > 0) {
        launch_zero_int(s->st, (int *)a.X.x, (int)(6 * N));
        launch_zero_int(s->st, (int *)a.U.x, (int)(6 * N));
    }
    // segments from the last to the first: recompute, then step back
    for (int k = K; k >= 1; --k) {
        const int64_t s0 = ckpt_step(a, k - 1), s1 = ckpt_step(a, k);
        HIPCHK(ckpt_restore(s, k - 1, s0));
        HIPCHK(tape_record(s, 0, s0 == 0));
        tape_list(s, 0);
        {
            // each recomputed step builds its list straight into its tape
            // entry; the system's own list buffers are back at scope exit
            const ListRedirect keep{s, s->ncnt, s->nl};
            for (int m = 1; m <= (int)(s1 - s0); ++m) {
                const TapeEntry e = tape_entry(s, m);
                s->ncnt = e.ncnt;
                s->nl = e.nl;
                if (e.corr) {  // the step's wall events, by particle id
                    launch_zero_int(s->st, (int *)e.corr, (int)((N + 3) / 4));
                    s->corr_byid = e.corr;
                }
                s->perm_out = e.perm;  // where the step's sort moves each slot
                s->advance(1);
                HIPCHK(tape_record(s, m, false));
            }
        }
        for (int m = (int)(s1 - s0); m >= 1; --m) {
            const AdjConst *act = table(s0 + m);
            adjoint_step(s, m, s0 + m, act);
            const TapeEntry cur = tape_entry(s, m), prev = tape_entry(s, m - 1);
            launch_adj_step_back(s->st, s->R, act, prev.tag, cur.perm, cview(a.X), cview(a.U), a.Xo, a.Uo,
                                 cur.corr);
            std::swap(a.X, a.Xo);
            std::swap(a.U, a.Uo);
        }
    }
    if (K == 0) {
        HIPCHK(ckpt_restore(s, 0, 0));
        HIPCHK(tape_record(s, 0, true));
        tape_list(s, 0);
    }
    // the evaluation at creation, then export in input order
    adjoint_step(s, 0, 0, a.act + 3 * nrep);
    std::vector<double> g(3 * 64 * nrep);
    HIPCHK(hipMemcpyAsync(g.data(), a.gtot, g.size() * sizeof(double), hipMemcpyDeviceToHost, s->st));
    const hipMemcpyKind dk = mem_kind == MDPD_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (N > 0) {
        // sorted SoA planes to n x 3 rows in id order (U of frozen particles is 0)
        launch_export(s->st, false, s->R, cview(a.X), cview(a.U), nullptr, tape_entry(s, 0).tag, s->io, s->io2,
                      nullptr);
        if (dx0) HIPCHK(hipMemcpyAsync(dx0, s->io, 3 * N * sizeof(double), dk, s->st));
        if (dv0) HIPCHK(hipMemcpyAsync(dv0, s->io2, 3 * N * sizeof(double), dk, s->st));
    }
    HIPCHK(hipStreamSynchronize(s->st));
    // per replica, its ntypes^2 table entries, replica after replica
    double *outs[3] = {dA, dB, dgamma};
    for (int q = 0; q < 3; ++q) {
        if (!outs[q]) continue;
        size_t off = 0;
        for (size_t r = 0; r < nrep; ++r) {
            const int T = s->params[r].ntypes;
            for (int ab = 0; ab < T * T; ++ab) outs[q][off + ab] = g[r * 192 + q * 64 + ab];
            off += (size_t)T * T;
        }
    }
    // back to the state at the end of the recording
    HIPCHK(ckpt_restore(s, K, a.nsteps));
    s->restore_lists();
    HIPCHK(hipStreamSynchronize(s->st));
    HIPCHK(hipGetLastError());
    return MDPD_OK;
}

}  // extern "C"
