// mdpd_internal.h -- shared declarations of the gfx950 mDPD library.
//
// Data layout in device memory (all arrays indexed by the current sorted
// slot k, particles ordered by cell, x fastest, then y, then z, and by
// particle id inside a cell, as of the last list build):
//   positions, velocities, forces : three FP64 planes (SoA), x | y | z
//   tag                           : uint32, particle id in bits 0..30,
//                                   bit 31 set for frozen wall particles
//   type                          : uint8
//   rho                           : FP64 (FP64 form) or FP32 (FP32 form)
//   skin list                     : kSkinCap entries per particle, particle-major:
//                                   u32 slot of every neighbour closer than
//                                   r_c + skin at the last build, with a
//                                   flag for pairs that may need the minimum
//                                   image, and a count per particle
//   pair list                     : kListCap entries per particle: the skin
//                                   entries closer than r_c at the current
//                                   positions (flag for r < r_d), and a count
//   cell_start                    : ncells + 1 offsets into the sorted order
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mdpd {

constexpr int kListCap = 64;    // pair-list slots per particle
constexpr int kSkinCap = 128;   // skin-list slots per particle
constexpr int kOneListLaunchCells = 8192;  // per-step list: up to this many cells it is one launch
static_assert((kListCap & (kListCap - 1)) == 0, "far-buffer positions wrap with a mask");
constexpr int kBlock = 256;    // threads per block of the particle kernels
// every-step sort in one workgroup per replica (sort.hip, k_sort_small):
// limits per replica of particles (12 per thread of 1024), cells, and LDS
constexpr int kSortSmallMaxN = 12 * 1024;
constexpr int kSortSmallMaxCells = 4096;
constexpr int kSortSmallMaxLds = 65536 - 256;
constexpr int kSortSmallMinReplicas = 64;  // below that the multi-pass sort is faster
constexpr uint32_t kFrozenBit = 0x80000000u;
// wall slip: the particle was sent back by the corrector in the last step
// (ids are below 2^30, so bit 30 is free)
constexpr uint32_t kRejectBit = 0x40000000u;
constexpr uint32_t kIdMask = 0x3fffffffu;

struct Soa3 {
    double *x, *y, *z;
};
struct Soa3c {
    const double *x, *y, *z;
};
inline Soa3c cview(const Soa3 &a) { return Soa3c{a.x, a.y, a.z}; }

// Everything the force pass reads of a neighbour, packed in one record per
// slot (written by the density pass), so that one neighbour costs one
// sector instead of eight scattered loads: 64 bytes in the FP64 form (this
// one), 32 in the FP32 form (PartRec32 below).
struct alignas(16) PartRec {
    double x, y, z;     // position
    double vx, vy, vz;  // half-step velocity (0 for frozen particles)
    double rho;         // many-body density (the FP32 form's value, exactly)
    uint32_t tag;       // id | frozen bit
    uint32_t typ;       // type
};
static_assert(sizeof(PartRec) == 64, "PartRec must be one 64-byte sector");

// The neighbour record of the FP32 form: half the bytes per gathered
// neighbour (the type, with several types, comes from the type array).  The position is fixed point in units of L / 2^32 per
// axis (q = round(x 2^32 / L) mod 2^32): the difference of two, read as a
// signed 32-bit integer, is the minimum-image difference, exact, with a
// resolution of L / 2^32 (1.3e-8 at L = 56).
struct alignas(32) PartRec32 {
    uint32_t qx, qy, qz;  // fixed-point position
    float vx, vy, vz;     // half-step velocity (0 for frozen particles)
    float rho;            // many-body density
    uint32_t tag;         // id | flag bits
};
static_assert(sizeof(PartRec32) == 32, "PartRec32 must be one 32-byte sector");

// Cell lattice: nc[a] cells of edge L[a]/nc[a] >= r_c + skin per axis.
// The cells and the skin list are built together; until the next build a
// particle moves less than half the skin (slack), so a cell scan stays
// complete when its clipping allows for that slack.
struct Geom {
    double L[3];
    double s[3];   // cells per unit length, nc / L
    double cs[3];  // cell edge, L / nc
    double inv_nc[3];  // 1 / nc: splits a cell index into its coordinates
    double invL[3];    // 1 / L
    int nc[3];
    int ncells;
    double rc, rc2, rd2;
    double rs2;    // squared cutoff of the skin-list build, (r_c + skin)^2 (1 + 1e-9)
    double gate2;  // a squared displacement since the build at or above this forces a rebuild
    double slack;  // half the skin: the most a particle moves between builds
};

// Scalars of one pair pass (one launch).
struct PairConst {
    double L[3], invL[3];
    double rc, inv_rc, rd, inv_rd, rd2;
    double wrho;        // 15 / (2 pi r_d^3)
    double hdtm, dt;    // dt / (2 m), dt
    double mass;
    double mg[3];       // body force m g on fluid
    double A, B, gamma, sig, Arc2;  // single-type values; sig = sqrt(2 gamma kT / dt)
    double phi_c;
    double slip;        // wall reflection: tangential factor 2 slip - 1 (0: bounce-back)
    double qs[3];       // 2^32 / L: fixed-point scale of the 32-byte records
    float qd[3];        // L / 2^32
    double dctl;        // dissipation control: eta rho_f W_D (0: off); fluid-frozen pairs of
                        // fluid i take gamma s_i, sigma sqrt(s_i), s_i = dctl / sum_{j, r<r_c} w_c^2
    const double *tab;  // ntypes > 1: A | B | gamma | sig | Arc2 planes of 64
    int ntypes;
    uint32_t seed;      // key word 0 of the pair noise
    uint32_t ks0, ks1;  // Threefry key words added to the counter
    uint32_t inj0[5], inj1[5];  // Threefry key injections after rounds 4, 8, ..., 20
};

// Replicas: independent periodic systems stored back to back.  Replica r
// owns the global cells [cell_off[r], cell_off[r+1]) and, since the sort key
// is replica-major and particles never change replica, the sorted slots
// [part_off[r], part_off[r+1]).  The particle kernels run replica-aligned
// blocks: with P lanes per particle, replica r owns the blocks
// [blk[r], blk[r+1]) of blk = blk_off + lanes_index(P) * (nrep + 1), so every
// block reads one replica's constants (scalar loads).  A single system is
// one replica.
constexpr int kLaneCounts = 5;  // P = 1, 2, 4, 8, 16
struct Reps {
    const Geom *geom;       // [nrep]
    const PairConst *pc;    // [nrep]; noise keys are set per launch from (seed, step)
    const int *cell_off;    // [nrep + 1]
    const int *cell_rep;    // [ncells] replica of each global cell (NULL with one replica)
    const int *blk_rep;     // per lane count, replica of each block (NULL with one replica)
    const int *part_off;    // [nrep + 1]
    const int *blk_off;     // [kLaneCounts][nrep + 1]
    const int *flag;        // [nrep + 1]: 1 = replica r rebuilds its lists this step; [nrep]: any does
    const int *bcells;      // [nbcells] per-step list: global indices of the border cells (a periodic image in the stencil)
    const int *icells;      // [nicells] per-step list: global indices of the other (interior) cells
    int nicells;
    int nrep;
    int ncells;             // total cells
    int nbcells;
    int list_interior;      // per-step list: 1 = interior cells have a launch of their own; 0 = bcells holds every cell
    int list_split;         // per-step list: wavefronts per cell of the border launch (its particles dealt round robin)
    int sort_small_lds;     // > 0: every replica fits one workgroup's sort (LDS bytes it needs); 0: multi-pass sort
    int wsub;               // wall mask: sub-cells per cell edge (walls on)
    int nblk[kLaneCounts];  // total blocks per lane count
};

__host__ __device__ constexpr int lanes_index(int P) { return P == 1 ? 0 : P == 2 ? 1 : P == 4 ? 2 : P == 8 ? 3 : 4; }

// Read-only table entry through the constant address space: the tables
// never change while a kernel runs, so uniform reads become scalar loads and
// the values live in scalar registers.
template <typename T>
__device__ __forceinline__ T cload(const T *p, int k)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(4))) T *)p)[k];
#else
    return p[k];  // host pass: never called
#endif
}

// Largest r with off[r] <= x (off ascending, off[0] = 0 <= x).  With a
// wave-uniform x the search is uniform.
__device__ __forceinline__ int find_rep(const int *__restrict__ off, int nrep, int x)
{
    int lo = 0, hi = nrep;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cload(off, mid) <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The replica of block blk of a launch with lane count index li (off: that
// lane count's block offsets): a table lookup with several replicas (one
// scalar load instead of a search of dependent loads), 0 with one.
__device__ __forceinline__ int block_replica(const Reps &R, int li, const int *off, int blk)
{
    if (!R.blk_rep) return __builtin_amdgcn_readfirstlane(find_rep(off, R.nrep, blk));
    int base = 0;
    for (int l = 0; l < li; ++l) base += R.nblk[l];
    return cload(R.blk_rep, base + blk);
}

// Threefry key schedule for key (seed, step): ks2 = 0x1BD11BDA ^ k0 ^ k1 and
// the injection after rounds 4s adds (ks[s % 3], ks[(s + 1) % 3] + s).
__host__ __device__ inline void set_noise_keys(PairConst &pc, uint32_t step)
{
    const uint32_t k0 = pc.seed, k1 = step;
    const uint32_t ks[3] = {k0, k1, 0x1BD11BDAu ^ k0 ^ k1};
    pc.ks0 = ks[0];
    pc.ks1 = ks[1];
    for (uint32_t s = 1; s <= 5; ++s) {
        pc.inj0[s - 1] = ks[s % 3];
        pc.inj1[s - 1] = ks[(s + 1) % 3] + s;
    }
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
// Cell index along one axis, clamped to [0, nc - 1]; a non-finite coordinate
// (a run that blew up, reported through the status word) maps to cell 0, so
// no launch can index outside the cell arrays.
__device__ __forceinline__ int cell_coord(double x, double s, int nc)
{
    double t = x * s;
    if (!(t >= 0.0)) t = 0.0;
    const int c = t < (double)nc ? (int)t : nc - 1;
    return c;
}

// Squared distance with no fused multiply-add, evaluated ((dx dx + dy dy) + dz dz):
// the neighbour test must round exactly like a plain sequence of products and sums.
__device__ __forceinline__ double exact_r2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    double a = dx * dx;
    double b = dy * dy;
    double c = dz * dz;
    double s = a + b;
    s = s + c;
    return s;
}

// Minimum image of a difference |d| < L: d - L * rint(d / L).  For pairs
// closer than L/2 the multiple is -1, 0 or +1, L*k is exact, so the result is
// the correctly rounded d - L, d or d + L.
__device__ __forceinline__ double min_image(double d, double L, double invL)
{
    return fma(-L, rint(d * invL), d);
}

// 1/sqrt(a) for a > 0 to full double precision: hardware estimate and two
// Newton steps.
__device__ __forceinline__ double rsqrt_f64(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    double h = 0.5 * a;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

__device__ __forceinline__ uint32_t rotl32(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

// First output word of Threefry-2x32 with 20 rounds (Salmon et al., SC'11),
// counter (c0, c1); the key enters through ks0, ks1 and the five injections
// precomputed on the host from (seed, step).
__device__ __forceinline__ uint32_t threefry2x32_20_w0(uint32_t c0, uint32_t c1, const PairConst &k)
{
    uint32_t x0 = c0 + k.ks0, x1 = c1 + k.ks1;
#define MDPD_TF_ROUND(R) \
    x0 += x1;            \
    x1 = rotl32(x1, R);  \
    x1 ^= x0;
    MDPD_TF_ROUND(13) MDPD_TF_ROUND(15) MDPD_TF_ROUND(26) MDPD_TF_ROUND(6)
    x0 += k.inj0[0]; x1 += k.inj1[0];
    MDPD_TF_ROUND(17) MDPD_TF_ROUND(29) MDPD_TF_ROUND(16) MDPD_TF_ROUND(24)
    x0 += k.inj0[1]; x1 += k.inj1[1];
    MDPD_TF_ROUND(13) MDPD_TF_ROUND(15) MDPD_TF_ROUND(26) MDPD_TF_ROUND(6)
    x0 += k.inj0[2]; x1 += k.inj1[2];
    MDPD_TF_ROUND(17) MDPD_TF_ROUND(29) MDPD_TF_ROUND(16) MDPD_TF_ROUND(24)
    x0 += k.inj0[3]; x1 += k.inj1[3];
    MDPD_TF_ROUND(13) MDPD_TF_ROUND(15) MDPD_TF_ROUND(26) MDPD_TF_ROUND(6)
    x0 += k.inj0[4];
#undef MDPD_TF_ROUND
    return x0;
}

// Pair noise: top 24 bits k of the first Threefry word with counter
// (min id, max id) give t = (2k + 1 - 2^24) 2^-24, exact in both FP32 and
// FP64; theta = sqrt(3) t is uniform with zero mean and unit variance.
__device__ __forceinline__ int theta_int(uint32_t ida, uint32_t idb, const PairConst &k)
{
    uint32_t lo = ida < idb ? ida : idb;
    uint32_t hi = ida < idb ? idb : ida;
    uint32_t w = threefry2x32_20_w0(lo, hi, k);
    return (int)((w >> 8) << 1) + 1 - 16777216;
}

// Scalars of one backward step of the adjoint for one replica (adjoint.hip;
// one table entry per replica).  Loss weights are zero at states that carry
// no loss term.
#define MDPD_ADJ_MAX_TYPES 8
struct AdjConst {
    double cU;       // coefficient of U = dL/du_n in the force adjoint: 2h, or h at creation
    double cv;       // coefficient of the velocity seed in the force adjoint: h, or 0 at creation
    double wrho_nf;  // weight of the mean fluid density / N_f
    double wP_3V;    // weight of the virial pressure / (3 V)
    double wvx_nf;   // weight of the mean fluid x-velocity / N_f
    double mass;
    double dt;       // drift of the step (0 at creation)
    double pad;
};

// Per-replica constants of the loss terms (mean fluid density, virial
// pressure, mean fluid x-velocity) accumulated during a recording.
struct LossConst {
    double inv_nf, inv3V, mass, pad;
};

// Host-side launchers (defined in the .hip files).  n is the total number
// of particles over all replicas.
void launch_ingest(hipStream_t st, const Reps &R, const double *pos, const double *vel,
                   const int32_t *type, const uint8_t *frozen, Soa3 xp, Soa3 vp, uint32_t *tag,
                   uint8_t *typ, int *status);
// The list gate of one step: for each replica, the largest squared
// displacement since its last list build (block maxima written by the force
// pass, which ran with `lanes` lanes per particle) against its threshold
// gate2, or a forced rebuild, gives flags[r] (1 = rebuild this step);
// flags[nrep] = any.  The same launch advances the noise step and clears the
// force pass's overflow count.  force: read and cleared; done: a counter
// that must be zero and is left zero; nbuild accumulates the replicas
// rebuilt.  first = false: a second gate of the same step (after the wall
// corrector, on its block maxima, laid out for one lane per particle): no
// bookkeeping, and a rebuild there is counted too.
void launch_gate(hipStream_t st, const Reps &R, int lanes, const float *bmax, int *force, int *flags, int *done,
                 uint32_t *step_ctr, int *ovf_count, unsigned long long *nbuild, bool first);
// out[i] = b[a[i]] (two permutations of slots, one after the other).
void launch_compose(hipStream_t st, int n, const int *a, const int *b, int *out);
// Sort of the replicas whose flag is set into (cell, id) order: positions x,
// half-step velocities v, tags, types and, with walls, the previous
// positions xprev (nullable) are permuted in place through the temporaries
// t*; the replica's cell offsets in cstart are replaced and its sorted
// positions copied to xbuild.  dmap (nullable): dmap[i] = the slot the
// particle at slot i moves to (the identity for replicas not rebuilt).
// copy_back = false: every replica is sorted whatever the flags say (the
// caller rebuilds every step), the sorted arrays stay in the t* arrays,
// which the caller then takes as the state (and x, v, xprev, tag, typ as the
// next temporaries); step_ctr, ovf_count, nbuild (nullable): the once-per-step
// bookkeeping of the gate, done by the sort instead (n > 0).
void launch_rebuild_sort(hipStream_t st, int n, const Reps &R, Soa3 x, Soa3 v, Soa3 xprev, uint32_t *tag,
                         uint8_t *typ, Soa3 tx, Soa3 tv, Soa3 tp, uint32_t *ttag, uint8_t *ttyp, Soa3 xbuild,
                         int *key, int *slot, uint32_t *tmpid, int *counts, int *cnew, int *cstart, int *bsum,
                         int *dmap, bool copy_back, uint32_t *step_ctr = nullptr, int *ovf_count = nullptr,
                         unsigned long long *nbuild = nullptr);
// Per-step neighbour list (skin 0) of the replicas whose flag is set (every
// replica with all): the pairs closer than r_c at the positions xs, the near
// ones (r < r_d) flagged, with their r^2 in nlr2 (FP32 or FP64 as rho; FP32
// rows split into 16-entry heads and a tail area, n slots x 64 entries in all).
void launch_nlist(hipStream_t st, bool fp32, const Reps &R, Soa3c xs, const int *cstart, int *ncnt,
                  uint32_t *nl, void *nlr2, bool all);
// Density from the per-step list's stored r^2, and the packed records.
void launch_density_list(hipStream_t st, int lanes, bool fp32, const Reps &R, Soa3c xs, Soa3c vh,
                         const uint32_t *tag, const uint8_t *typ, const int *cstart, const int *ncnt,
                         const void *nlr2, void *rho, PartRec *rec);
// Skin list of the replicas whose flag is set (every replica with all):
// for each particle the slots of all others closer than sqrt(rs2) at the
// positions xs, scnt = their number (a row of more than kSkinCap is not
// stored; the passes then scan the cells directly).
void launch_skin_build(hipStream_t st, const Reps &R, bool all, Soa3c xs, const int *cstart, int *scnt,
                       uint32_t *sl);
// Pair list at the current positions from the skin list (exact FP64 test
// against r_c, flag for r < r_d), the many-body density, and the packed
// neighbour records of every slot (rho and rec NULL: the pair list only).
void launch_density(hipStream_t st, int lanes, bool fp32, const Reps &R, Soa3c xs, Soa3c vh,
                    const uint32_t *tag, const uint8_t *typ, const int *cstart, const int *scnt,
                    const uint32_t *sl, int *ncnt, uint32_t *nl, void *rho, PartRec *rec);
// Walls: the sub-cell mask of where a frozen particle is in reach (once), and
// phi + corrector for one step (cell scan at the predicted positions).
void launch_mark_wall_cells(hipStream_t st, const Reps &R, Soa3c xs, const uint32_t *tag, uint8_t *wmask);
// ncorr: [0] corrections of this step (written), [1..n] per-slot flags,
// then one count per kBlock slots (scratch); ncorr_total accumulates.
// slip: some replica reflects with wall_slip > 0 (the wall normal is needed;
// the corrector keeps kRejectBit of each fluid tag up to date).
// byid (nullable, n bytes by global particle id): set to 1 for every particle
// corrected in this step (the adjoint's record of the wall events).
// A corrected particle goes back to xprev; cmax receives, per block of
// kBlock slots (replica-aligned, the layout of one lane per particle), the
// largest squared distance of a corrected particle from its build position
// xbuild (0 without corrections), for the step's second gate.
void launch_phi(hipStream_t st, int lanes, bool slip, int n, const Reps &R, Soa3c xs, Soa3c xprev, Soa3 xfix,
                Soa3 vfix, uint32_t *tag, const int *cstart, const uint8_t *wmask, int *ncorr,
                unsigned long long *ncorr_total, uint8_t *byid, Soa3c xbuild, float *cmax);
// stepp: device word holding the noise step (advanced by the gate).  The
// epilogue writes the next positions and half-step velocities to xpred,
// vpred and the block maxima of their squared displacement from xbuild to
// bmax (float, rounded up; the gate of the next step reads them).
// dc: some replica controls the fluid-solid dissipation (PairConst::dctl > 0).
void launch_force(hipStream_t st, int lanes, bool fp32, bool mt, bool dc, const Reps &R, const uint32_t *stepp,
                  Soa3c xs, Soa3c vh, const void *rho, const uint32_t *tag, const uint8_t *typ,
                  const PartRec *rec, const int *cstart, const int *ncnt, const uint32_t *nl, Soa3 vout,
                  Soa3 fout,
                  Soa3 vpred, Soa3 xpred, double *part, int *status, int *ovf_count, int *ovf,
                  double *ovf_ve, int initial, Soa3c xbuild, float *bmax);
// Number of virial/energy block partials the force pass writes with this
// lane count (one per block; replica r owns its blocks' range).
int force_partials(const Reps &R, int lanes);
// Adjoint launchers: ac is a device table of one AdjConst per replica; gp
// holds 3 x ntypes parameter shares per slot; gtot accumulates per replica
// 3 planes of MDPD_ADJ_MAX_TYPES^2 (A, B, gamma) over the backward steps.
void launch_adj_seed(hipStream_t st, const Reps &R, const AdjConst *ac, Soa3c v, const uint32_t *tag, Soa3 U,
                     Soa3 fb, double *rhoA);
// Dissipation control (dc): sdc[i] = s_i, qdc[i] = s_i / S_i per slot of the
// state (1 and 0 where the control does not act); the force adjoint then
// writes adc[i] = dL/dS_i, which the density adjoint (adc non-NULL) turns
// into the position adjoint of the w_c^2 sums.
void launch_adj_dscale(hipStream_t st, int lanes, const Reps &R, Soa3c xs, const uint32_t *tag, const int *cstart,
                       const int *ncnt, const uint32_t *nl, double *sdc, double *qdc);
void launch_adj_force(hipStream_t st, int lanes, bool fp32, bool mt, bool dc, int n, int tmax, const Reps &R,
                      uint32_t step, const AdjConst *ac, Soa3c xs, Soa3c u, const void *rho,
                      const uint32_t *tag, const uint8_t *typ, const int *cstart, const int *ncnt,
                      const uint32_t *nl, Soa3c fb, Soa3 X, Soa3 U, double *rhoA, double *gp,
                      const double *sdc, const double *qdc, double *adc);
void launch_adj_density(hipStream_t st, int lanes, const Reps &R, Soa3c xs, const int *cstart,
                        const int *ncnt, const uint32_t *nl, const double *rhoA, Soa3 X, const double *adc);
// Drift adjoint and reorder in one pass: perm[i] = slot in step n of the
// particle at slot i of step n - 1 (tag_prev: its tags); X, U in the order
// of step n to Xo, Uo in the order of step n - 1; corr (nullable): the
// step's wall-event bytes by global particle id.
void launch_adj_step_back(hipStream_t st, const Reps &R, const AdjConst *ac, const uint32_t *tag_prev,
                          const int *perm, Soa3c X, Soa3c U, Soa3 Xo, Soa3 Uo, const uint8_t *corr);
int adj_param_partials(const Reps &R, int tmax);
void launch_adj_params(hipStream_t st, const Reps &R, int n, int tmax, const uint8_t *typ, const double *gp,
                       double *part, double *gtot);
void launch_loss_accum(hipStream_t st, int nrep, const double *obs, const LossConst *lc, double *acc,
                       double scale);
// Observables per replica: part needs obs_partials(R) doubles, out 16 per
// replica (sums as listed at k_obs_final).
int obs_partials(const Reps &R);
void launch_observables(hipStream_t st, bool fp32, const Reps &R, int force_lanes, Soa3c v,
                        const void *rho, const uint32_t *tag, const uint8_t *typ,
                        const double *fpart, const int *ncnt, const double *ovf_ve, double *part,
                        double *out);
void launch_profile(hipStream_t st, bool fp32, int n, int axis, int nbins, int quantity, double La,
                    double binvol, double mass, Soa3c x, Soa3c v, const void *rho,
                    const uint32_t *tag, double *work, double *out);
void launch_export(hipStream_t st, bool fp32, const Reps &R, Soa3c x, Soa3c v, const void *rho,
                   const uint32_t *tag, double *pos, double *vel, double *rho_out);
void launch_debug_neighbors(hipStream_t st, const Reps &R, double cutoff2, Soa3c xs,
                            const uint32_t *tag, const int *cstart, const int *ncnt,
                            const uint32_t *nl, int64_t *count, uint64_t *hash);
void launch_zero_int(hipStream_t st, int *p, int n);
void launch_set_int(hipStream_t st, int *p, int v);
// Pressure tensor: per-slot planes (6 x n, xx yy zz xy xz yz), then per-replica
// sums into out[6 r + a] (still to be divided by the replica's volume).
// per_block: instead of planes, six sums per block of kStressLanes lanes per
// particle (R.nblk[lanes_index(kStressLanes)] blocks, block b at out[6 b]),
// reduced per replica by launch_stress_part_sum into
// out[6 k + a] = sum / volume for replicas first + k, k < count.
constexpr int kStressLanes = 4;
void launch_stress(hipStream_t st, bool fp32, bool mt, int n, const Reps &R, Soa3c xs, Soa3c v,
                   const void *rho, const uint32_t *tag, const uint8_t *typ, const int *cstart,
                   const int *ncnt, const uint32_t *nl, double *out, bool per_block);
void launch_stress_sum(hipStream_t st, const Reps &R, int n, const double *planes, double *out);
void launch_stress_part_sum(hipStream_t st, const Reps &R, int first, int count, const double *parts,
                            double *out);

}  // namespace mdpd
