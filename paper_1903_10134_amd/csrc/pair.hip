// pair.hip -- the pair passes of one mDPD timestep on gfx950.
//
//   k_nlist_cell, k_nlist_border
//                 skin 0, every step: one wavefront per cell builds the pair
//                 list of its particles from the candidates of the cells
//                 around it (exact FP64 test), each entry flagged for
//                 r < r_d, and stores the near entries' r^2
//   k_density_list
//                 skin 0: the many-body density
//                 rho_i = sum_{j != i, r < r_d} w_rho(r_ij) (Sec. 2.1) from
//                 the stored r^2; packs the neighbour records the force pass
//                 gathers (32 bytes in the FP32 form, 64 in the FP64 form)
//   k_skin_build  skin > 0: one wavefront per cell: the neighbours within
//                 r_c + skin of every particle of the cell at the build
//                 positions (exact FP64 test), written to a fixed-capacity
//                 skin list; runs only in the steps the gate asks for a
//                 rebuild
//   k_density     skin > 0, every step: the skin entries closer than r_c at
//                 the current positions (the same exact test) become the
//                 step's pair list, each with a flag for r < r_d, and the
//                 density is summed over them; also packs the records
//   k_phi         boundary volume fraction of fluid particles at the predicted
//                 positions (direct cell scan, only where a sub-cell mask puts
//                 a frozen particle in reach) and the predictor-corrector flag
//                 (Sec. 2.2, 3.2)
//   k_force       Eq. 1 conservative force, dissipative and random forces
//                 (Sec. 2.1), body force, and the velocity-Verlet update fused
//                 in the epilogue: v(t+dt), the next half-step velocity and the
//                 next predicted position (Alg. 1), and how far the particles
//                 have moved since the list build (for the next gate)
//
// In the list passes P lanes of a 64-wide wavefront cooperate on one particle
// (P = 1, 2, 4, 8 or 16): they split its list entries and combine their partial
// sums with a butterfly of lane shuffles inside the group, so every sum has
// one fixed order.  A particle with more than kSkinCap skin neighbours, or
// more than kListCap pair neighbours, is served by a direct scan of the
// cells with the same exact test (the cells of the last build, their
// clipping widened by the half skin the particles may have moved since).
#include "pair_common.h"

namespace mdpd {

namespace {

// Stores into one list row go through a buffer resource whose range is the
// row: a lane with nothing to store gives an offset past the range, and the
// hardware drops the store, so the emission needs no branch.
constexpr int kDropOffset = (int)0x80000000;
constexpr int kRawBufferConfig = 0x00020000;  // 32-bit data format, no swizzle

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(void *row, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(row, (short)0, bytes, kRawBufferConfig);
}

// ---------------------------------------------------------------------------
// Per-step neighbour list (skin 0): one wavefront per cell.
//
// Interior cells (no periodic image in the stencil): the 27 stencil cells are
// 9 rows of 3 x-adjacent cells, each row contiguous in the sorted order.  The
// rows of one dz form a batch of up to 128 candidates held in two register
// slots (lane q holds candidate q and q + 64), so all candidates of the cell
// are loaded once.  The wave then loops uniformly over the particles i of the
// cell, broadcasts i's position, and tests the batches with the exact FP64
// test, 64 pairs per instruction.  A ballot and mbcnt append the hits to i's
// list in candidate order; i's count is a wave-uniform scalar.
//
// Border cells (a periodic image in the stencil) take the same register path
// when every axis has at least four cells: away from the x faces their rows
// are still contiguous (wrapped in y and z), on an x face a row is two pieces,
// and the minimum image is taken on the axes where the cell touches the
// boundary.  Otherwise (fewer cells, or a batch above 128 candidates) the
// general path walks the batches 64 candidates at a time with the shifts of
// each row piece, and i's running count lives in lane (i mod 64); with two
// cells on an axis the other cell is visited with both shifts, and a pair
// closer than r_c <= L/2 matches one of them only.
//
// Each entry is the neighbour's slot, with kNearBit set when r < r_d and
// kWrapBit set when the pair is seen through a periodic image (its difference
// then needs the minimum-image shift).  A row holds its entries with no gap
// (a row of the usual ~25 entries is one 128-byte line): in candidate order
// from the register path, near entries first from the general path.  The
// exact r^2 of the near entries go back to back into a parallel row (R2 =
// FP32 or FP64, the arithmetic of the density pass; layout at R2Row), which
// is all the density pass reads.  In the general path near hits are stored
// as they are found and far hits wait in LDS until the particle's near count
// is known.

__device__ __forceinline__ void store_r2(__amdgpu_buffer_rsrc_t r, int k, bool keep, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, keep ? k * 4 : kDropOffset, 0, 0);
}

__device__ __forceinline__ void store_r2(__amdgpu_buffer_rsrc_t r, int k, bool keep, double v)
{
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const u32x2 w = {(unsigned)b, (unsigned)(b >> 32)};
    __builtin_amdgcn_raw_buffer_store_b64(w, r, keep ? k * 8 : kDropOffset, 0, 0);
}

// The near-r^2 row of particle i (n: the slots of all replicas).  FP64: the
// kListCap entries at i kListCap.  FP32: the first kR2Head entries of every
// row side by side, 64 bytes a particle, so two neighbouring particles share
// a 128-byte line and the density pass fetches half a line for a row of the
// usual ten or so entries (a full line with rows kListCap apart); entries
// kR2Head and up of particle i in a tail area after the n heads.
constexpr int kR2Head = 16;

template <typename R2>
struct R2Row {
    static constexpr bool kSplit = sizeof(R2) == 4;
    __amdgpu_buffer_rsrc_t head, tail;
    __device__ __forceinline__ R2Row(R2 *base, size_t n, int i)
    {
        if constexpr (kSplit) {
            head = row_rsrc(base + (size_t)i * kR2Head, kR2Head * 4);
            tail = row_rsrc(base + n * kR2Head + (size_t)i * (kListCap - kR2Head), (kListCap - kR2Head) * 4);
        } else {
            head = tail = row_rsrc(base + (size_t)i * kListCap, kListCap * 8);
        }
    }
    // this lane's entry k, when keep
    __device__ __forceinline__ void put(int k, bool keep, R2 v) const
    {
        if constexpr (kSplit) {
            store_r2(head, k, keep && k < kR2Head, v);
            store_r2(tail, k - kR2Head, keep && k >= kR2Head, v);
        } else {
            store_r2(head, k, keep, v);
        }
    }
    // a whole row: lane k holds entry k, count entries (wave-uniform)
    __device__ __forceinline__ void put_row(int count, R2 v) const
    {
        const int lane = threadIdx.x & 63;
        if constexpr (kSplit) {
            store_r2(head, lane, lane < count && lane < kR2Head, v);
            if (count > kR2Head) store_r2(tail, lane - kR2Head, lane >= kR2Head && lane < count, v);
        } else {
            store_r2(head, lane, lane < count, v);
        }
    }
};

// Where the density pass reads entry k of particle i's near-r^2 row: head + k
// below kR2Head, tail + k from there (the same pointer twice in FP64).
template <typename R2>
__device__ __forceinline__ void r2_row_ptrs(const R2 *base, size_t n, int i, const R2 *&head, const R2 *&tail)
{
    if constexpr (sizeof(R2) == 4) {
        head = base + (size_t)i * kR2Head;
        tail = base + n * kR2Head + (size_t)i * (kListCap - kR2Head) - kR2Head;
    } else {
        head = tail = base + (size_t)i * kListCap;
    }
}

// Hits of one 64-candidate test for particle i: mn marks the lanes whose
// candidate is within r_d, mf those within r_c but not r_d; cn / cf are i's
// near / far counts before this test.  A near hit goes to row position
// cn + (near hits in lower lanes) with its r^2 beside it; a far hit goes to
// position cf + (far hits in lower lanes) of the far buffer fb (lanes
// without one write to their own slot of dump).  A row whose counts
// add up to more than kListCap is never read (direct scan): its positions past
// the row are dropped by the store range check, and the far buffer index is
// kept inside the buffer.
template <typename R2>
__device__ __forceinline__ void emit_hits(__amdgpu_buffer_rsrc_t ro, const R2Row<R2> &rr, uint32_t *fb,
                                          uint32_t *dump, unsigned long long mn, unsigned long long mf, int cn,
                                          int cf, uint32_t e, double r2)
{
    const int lane = threadIdx.x & 63;
    const bool near = __builtin_amdgcn_inverse_ballot_w64(mn);
    const bool far = __builtin_amdgcn_inverse_ballot_w64(mf);
    const int pn = lanes_below(mn, cn);
    const int pf = lanes_below(mf, cf) & (kListCap - 1);
    __builtin_amdgcn_raw_buffer_store_b32(e | kNearBit, ro, near ? pn * 4 : kDropOffset, 0, 0);
    rr.put(pn, near, (R2)r2);
    *(far ? fb + pf : dump + lane) = e;
}

// The far hits of particle i, held in fb[0 .. cf), appended to its row after
// its cn near hits.
__device__ __forceinline__ void flush_far(__amdgpu_buffer_rsrc_t ro, const uint32_t *fb, int cn, int cf)
{
    const int lane = threadIdx.x & 63;
    const uint32_t e = fb[lane];
    __builtin_amdgcn_raw_buffer_store_b32(e, ro, lane < cf ? (cn + lane) * 4 : kDropOffset, 0, 0);
}

// Row assembly in LDS (the single-particle sweep).  The hits of one
// 64-candidate test (hm: within r_c) go to row positions ct + (hits in lower
// lanes) of nb, in candidate order, flagged kNearBit when within r_d (mn);
// the near hits' r^2 go to rb at cn + (near hits in lower lanes), so the
// density pass reads them back to back.  ct / cn are the row's entries / near
// entries before this test.  flush_row (BatchRows::flush in the interior
// kernel) then writes the row and the near r^2 with one store each.  A row past kListCap entries is never read; its
// excess goes to the lane's dump slot.
template <typename R2>
__device__ __forceinline__ void stage_hits(uint32_t *nb, R2 *rb, uint32_t *dump, unsigned long long hm,
                                           unsigned long long mn, int ct, int cn, uint32_t e, double r2)
{
    const int lane = threadIdx.x & 63;
    const bool hit = __builtin_amdgcn_inverse_ballot_w64(hm);
    const bool near = __builtin_amdgcn_inverse_ballot_w64(mn);
    const int p = lanes_below(hm, ct);
    const int pn = lanes_below(mn, cn);
    *(hit && p < kListCap ? nb + p : dump + lane) = near ? e | kNearBit : e;
    if (near && pn < kListCap) rb[pn] = (R2)r2;
}

template <typename R2>
__device__ __forceinline__ void flush_row(__amdgpu_buffer_rsrc_t ro, const R2Row<R2> &rr, const uint32_t *nb,
                                          const R2 *rb, int ct, int cn)
{
    const int lane = threadIdx.x & 63;
    __builtin_amdgcn_raw_buffer_store_b32(nb[lane], ro, lane < ct ? lane * 4 : kDropOffset, 0, 0);
    rr.put_row(cn, rb[lane]);
}

// The rows of the particles i0 .. i0 + nb - 1 (nb <= 64, one batch of a
// cell's sweep) behind one buffer resource per array, whose range is the
// batch: particle u's row starts at the scalar offset u times the row's
// bytes, and a lane's entry k at the vector offset k times the entry's, so
// the sweep builds no descriptor and no address per particle.  A kept entry
// lies inside the batch and a dropped one (kDropOffset) beyond it however
// the range check counts the scalar offset.
template <typename R2>
struct BatchRows {
    static constexpr bool kSplit = sizeof(R2) == 4;
    __amdgpu_buffer_rsrc_t nlr, head, tail;
    __device__ __forceinline__ BatchRows(uint32_t *nl, R2 *nlr2, size_t n, int i0, int nb)
    {
        nlr = row_rsrc(nl + (size_t)i0 * kListCap, nb * kListCap * 4);
        if constexpr (kSplit) {
            head = row_rsrc(nlr2 + (size_t)i0 * kR2Head, nb * kR2Head * 4);
            tail = row_rsrc(nlr2 + n * kR2Head + (size_t)i0 * (kListCap - kR2Head), nb * (kListCap - kR2Head) * 4);
        } else {
            head = tail = row_rsrc(nlr2 + (size_t)i0 * kListCap, nb * kListCap * 8);
        }
    }
    // particle u's row staged in LDS: entries nb[0 .. ct), near r^2 rb[0 .. cn)
    __device__ __forceinline__ void flush(int u, const uint32_t *nb, const R2 *rb, int ct, int cn) const
    {
        const int lane = threadIdx.x & 63;
        __builtin_amdgcn_raw_buffer_store_b32(nb[lane], nlr, lane < ct ? lane * 4 : kDropOffset, u * kListCap * 4,
                                              0);
        const R2 v = rb[lane];
        if constexpr (kSplit) {
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), head,
                                                  lane < cn && lane < kR2Head ? lane * 4 : kDropOffset,
                                                  u * kR2Head * 4, 0);
            if (cn > kR2Head)
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), tail,
                                                      lane < cn && lane >= kR2Head ? (lane - kR2Head) * 4
                                                                                   : kDropOffset,
                                                      u * (kListCap - kR2Head) * 4, 0);
        } else {
            typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
            const unsigned long long b = (unsigned long long)__double_as_longlong((double)v);
            const u32x2 w = {(unsigned)b, (unsigned)(b >> 32)};
            __builtin_amdgcn_raw_buffer_store_b64(w, head, lane < cn ? lane * 8 : kDropOffset, u * kListCap * 8, 0);
        }
    }
};

// LDS of one wavefront: the far buffers of up to kGenBatch particles (one in
// the interior path) and one slot per lane for lanes without a far hit.
constexpr int kGenBatch = 8;
constexpr int kFarLds = (kGenBatch + 1) * kListCap;

// The list of global cell cg, built by one wavefront.  far_lds: the
// wavefront's kFarLds words of LDS.  The interior instantiation
// (BORDER = false) returns at once for a border cell; the border one is given
// the border cells (every cell of a small system, interior ones included).
// part, nsplit: this wavefront takes the particles part, part + nsplit, ...
// of the cell (nsplit wavefronts share a cell; each loads the candidates).
template <typename R2, bool BORDER>
__device__ __forceinline__ void nlist_cell(const Reps &R, int cg, Soa3c xs, const int *__restrict__ cstart_all,
                                           int *__restrict__ ncnt, uint32_t *__restrict__ nl,
                                           R2 *__restrict__ nlr2, uint32_t *far_lds, int all, int part = 0,
                                           int nsplit = 1)
{
    const int lane = threadIdx.x & 63;
    uint32_t *const dump = far_lds + kGenBatch * kListCap;
    // the replica of this cell: its lattice, and its cell offsets (global slots)
    const int rep = R.cell_rep ? cload(R.cell_rep, cg) : 0;
    if (!all && cload(R.flag, rep) == 0) return;  // the replica keeps its list this time
    const size_t nslots = (size_t)cload(R.part_off, R.nrep);
    const Geom g = cload(R.geom, rep);
    const int c = cg - cload(R.cell_off, rep);
    const int *__restrict__ cstart = cstart_all + cload(R.cell_off, rep);
    const int i0 = cstart[c], ni = cstart[c + 1] - i0;
    if (ni == 0) return;
    const int nx = g.nc[0], ny = g.nc[1], nz = g.nc[2];
    // cell coordinates: the quotients are exact in FP64 (at most 2^24 cells),
    // which avoids integer division
    const int cyz = __builtin_amdgcn_readfirstlane((int)(((double)c + 0.5) * g.inv_nc[0]));
    const int cz = __builtin_amdgcn_readfirstlane((int)(((double)cyz + 0.5) * g.inv_nc[1]));
    const int cx = c - cyz * nx, cy = cyz - cz * ny;
    const double rc2 = g.rc2, rd2 = g.rd2;

    const bool interior = cx > 0 && cx < nx - 1 && cy > 0 && cy < ny - 1 && cz > 0 && cz < nz - 1;
    if (!BORDER && !interior) return;
    // Border cells take the register path too when every axis has at least
    // four cells: a stencil candidate then differs by less than L/2 in a
    // coordinate unless it is seen through that boundary, and by more than L/2
    // if it is, so the minimum image by rounding picks exactly the pairs
    // through a boundary and gives the same difference as the general path's
    // explicit shift (a pair whose difference rounds to L/2 itself is more
    // than r_c apart either way).  A thin y or z axis (one cell; two are
    // merged into one when the lattice is made, but also handled here)
    // takes it too: each distinct cell of the axis is visited once (offsets
    // 0 and +1 with two cells, 0 with one), every difference is taken through
    // the minimum image on that axis (every cell touches its boundary), and
    // the rows off the own cell on it -- with one cell, all rows -- carry the
    // wrap flag, since such a pair may be closest through the boundary.
    // (interior cells need three cells per axis, so only the border
    // instantiation can see a thin axis)
    const bool thin_y = BORDER && ny <= 2, thin_z = BORDER && nz <= 2;
    bool fast = interior || (nx >= 4 && (ny >= 4 || thin_y) && (nz >= 4 || thin_z));
    // away from the x faces the stencil is 9 rows of 3 x-adjacent cells, each
    // contiguous in the sorted order
    const bool xin = cx > 0 && cx < nx - 1;
    int qz[3] = {0, 0, 0};
    int rb[9], rl[9];                 // rows: the 9 rows of 3 cells
    uint32_t rwrap = 0;               // rows: bit r = row r is seen through a y or z boundary
    int pb[18], pl[18];               // x faces: per dz, per dy, piece A then piece B
    uint32_t pwrap = 0;               // x faces: bit k = piece k is seen through a boundary
    int left = 0;                     // x faces: candidates of the own row before the own cell
    if (fast && xin) {
        // row r = (dy + 1) + 3 (dz + 1) spans the cells cx - 1 .. cx + 1 of
        // the (wrapped) row cy + dy, cz + dz
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const int dy = r % 3 - 1, dz = r / 3 - 1;
            const int yy = cy + dy, zz = cz + dz;
            const bool skip = (thin_y && (ny == 1 ? dy != 0 : dy < 0)) || (thin_z && (nz == 1 ? dz != 0 : dz < 0));
            const bool w = yy < 0 || yy >= ny || zz < 0 || zz >= nz || (thin_y && (dy != 0 || ny == 1)) ||
                           (thin_z && (dz != 0 || nz == 1));
            const int base = cx + nx * (wrap_index(yy, ny) + ny * wrap_index(zz, nz));
            rb[r] = cstart[base - 1];
            rl[r] = skip ? 0 : cstart[base + 2] - rb[r];
            rwrap |= (w ? 1u : 0u) << r;
        }
#pragma unroll
        for (int z = 0; z < 3; ++z) qz[z] = rl[3 * z] + rl[3 * z + 1] + rl[3 * z + 2];
    } else if (fast) {
        // the rows of a cell on an x face: a row that wraps in x is two pieces
#pragma unroll
        for (int z = 0; z < 3; ++z) {
            const int dz = z - 1;
            const int zz = wrap_index(cz + dz, nz);
            const bool wz = cz + dz < 0 || cz + dz >= nz || (thin_z && (dz != 0 || nz == 1));
            const bool skz = thin_z && (nz == 1 ? dz != 0 : dz < 0);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int dy = r - 1;
                const int yy = wrap_index(cy + dy, ny);
                const bool wy = cy + dy < 0 || cy + dy >= ny || (thin_y && (dy != 0 || ny == 1));
                const bool skip = skz || (thin_y && (ny == 1 ? dy != 0 : dy < 0));
                const int base = nx * (yy + ny * zz);
                int a0, a1, b0, b1;
                bool wa = wz || wy, wb = wz || wy;
                if (cx == 0) {           // cells nx-1 (through the boundary), then 0, 1
                    a0 = base + nx - 1;
                    a1 = base + nx;
                    b0 = base;
                    b1 = base + 2;
                    wa = true;
                } else if (cx == nx - 1) {  // cells nx-2, nx-1, then 0 (through the boundary)
                    a0 = base + nx - 2;
                    a1 = base + nx;
                    b0 = base;
                    b1 = base + 1;
                    wb = true;
                } else {                 // cells cx-1 .. cx+1
                    a0 = base + cx - 1;
                    a1 = base + cx + 2;
                    b0 = b1 = base;
                }
                const int k = 6 * z + 2 * r;
                pb[k] = cstart[a0];
                pl[k] = skip ? 0 : cstart[a1] - pb[k];
                pb[k + 1] = cstart[b0];
                pl[k + 1] = skip ? 0 : cstart[b1] - pb[k + 1];
                pwrap |= (wa ? 1u : 0u) << k;
                pwrap |= (wb ? 1u : 0u) << (k + 1);
                qz[z] += pl[k] + pl[k + 1];
            }
        }
        // the own row (dz = dy = 0) starts with the cell left of the own cell
        const int cl = nx * cyz + (cx == 0 ? nx - 1 : cx - 1);
        left = cstart[cl + 1] - cstart[cl];
    }
#pragma unroll
    for (int z = 0; z < 3; ++z)
        if (qz[z] > 128) fast = false;
    if (fast) {
        double cxj[6], cyj[6], czj[6];
        int cs[6];
        unsigned long long vm[6];  // the lanes of each slot that hold a candidate
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const int z = s >> 1;
            const int q = (s & 1) * 64 + lane;
            int slot = -1;
            uint32_t wrap = 0;
            if (q < qz[z]) {
                if (xin) {
                    const int l0 = rl[3 * z], l1 = rl[3 * z + 1];
                    const int row = q < l0 ? 3 * z : (q < l0 + l1 ? 3 * z + 1 : 3 * z + 2);
                    slot = q < l0 ? rb[3 * z] + q
                                  : (q < l0 + l1 ? rb[3 * z + 1] + (q - l0) : rb[3 * z + 2] + (q - l0 - l1));
                    if constexpr (BORDER) wrap = (rwrap >> row) & 1u ? kWrapBit : 0u;
                } else {
                    int off = q;
#pragma unroll
                    for (int k = 6 * z; k < 6 * z + 6; ++k) {
                        if (off >= 0 && off < pl[k]) {
                            slot = pb[k] + off;
                            wrap = (pwrap >> k) & 1u ? kWrapBit : 0u;
                        }
                        off -= pl[k];
                    }
                }
            }
            vm[s] = __builtin_amdgcn_ballot_w64(slot >= 0);
            const int js = slot >= 0 ? slot : i0;
            cs[s] = slot >= 0 ? (int)((uint32_t)slot | wrap) : -1;
            cxj[s] = ld(xs.x, js);
            cyj[s] = ld(xs.y, js);
            czj[s] = ld(xs.z, js);
        }
        // the single-particle sweep assembles each row in the wavefront's
        // LDS (where the general path keeps its batch buffers)
        uint32_t *const row_lds = far_lds;
        R2 *const near_r2 = reinterpret_cast<R2 *>(far_lds + 2 * kListCap);
        // particle i is candidate selfq0 + i of the dz = 0 batch: after the
        // dy = -1 row and the own row's cells left of the own cell
        const int selfq0 = xin ? rl[3] - rb[4] : pl[6] + pl[7] + left - i0;
        // the sweep over the particles of the cell, with the minimum image
        // taken only on the axis where a face cell touches the boundary (on
        // the others every stencil candidate is less than L/2 away, where the
        // minimum image is the identity); edge and corner cells take it on
        // all three axes
        auto sweep = [&](auto WX, auto WY, auto WZ) {
            for (int ib = 0; ib < ni; ib += 64) {
                const int nic = ni - ib < 64 ? ni - ib : 64;
                const int me = i0 + ib + (lane < nic ? lane : 0);
                const double pxi = ld(xs.x, me), pyi = ld(xs.y, me), pzi = ld(xs.z, me);
                // stages particle u's row in LDS: ct entries, cn of them near
                auto test = [&](int u, int &ct, int &cn) {
                    const double xi = bcast_d(pxi, u), yi = bcast_d(pyi, u), zi = bcast_d(pzi, u);
                    const int sq = selfq0 + i0 + ib + u;
                    ct = 0;
                    cn = 0;
#pragma unroll
                    for (int s = 0; s < 6; ++s) {
                        if ((s & 1) && qz[s >> 1] <= 64) continue;
                        double dx = xi - cxj[s], dy = yi - cyj[s], dz = zi - czj[s];
                        if constexpr (decltype(WX)::value) dx = min_image(dx, g.L[0], g.invL[0]);
                        if constexpr (decltype(WY)::value) dy = min_image(dy, g.L[1], g.invL[1]);
                        if constexpr (decltype(WZ)::value) dz = min_image(dz, g.L[2], g.invL[2]);
                        const double r2 = exact_r2(dx, dy, dz);
                        unsigned long long hm = __builtin_amdgcn_ballot_w64(r2 < rc2) & vm[s];
                        if ((s >> 1) == 1 && (sq >> 6) == (s & 1)) hm &= ~(1ull << (sq & 63));
                        const unsigned long long mn = hm & __builtin_amdgcn_ballot_w64(r2 < rd2);
                        stage_hits<R2>(row_lds, near_r2, dump, hm, mn, ct, cn, (uint32_t)cs[s], r2);
                        ct += __popcll(hm);
                        cn += __popcll(mn);
                    }
                };
                if constexpr (!BORDER) {
                    // interior cells: the batch's rows behind one descriptor
                    // per array, and its counts stored once (lane u holds
                    // particle u's); the border kernel, which holds more
                    // scalar state across this loop, would spill those
                    // descriptors, so there each particle builds its own
                    const BatchRows<R2> rows(nl, nlr2, nslots, i0 + ib, nic);
                    int counts = 0;
                    for (int u = part; u < nic; u += nsplit) {
                        int ct, cn;
                        test(u, ct, cn);
                        rows.flush(u, row_lds, near_r2, ct, cn);
                        if (lane == u) counts = cn | ((ct - cn) << 16);
                    }
                    if (lane < nic && lane >= part && (lane - part) % nsplit == 0) ncnt[i0 + ib + lane] = counts;
                } else {
                    for (int u = part; u < nic; u += nsplit) {
                        const int i = i0 + ib + u;
                        int ct, cn;
                        test(u, ct, cn);
                        flush_row<R2>(row_rsrc(nl + (size_t)i * kListCap, kListCap * 4), R2Row<R2>(nlr2, nslots, i),
                                      row_lds, near_r2, ct, cn);
                        if (lane == 0) ncnt[i] = cn | ((ct - cn) << 16);
                    }
                }
            }
        };
        using T = std::true_type;
        using F = std::false_type;
        if constexpr (!BORDER) {
            sweep(F{}, F{}, F{});
        } else {
            const bool bx = !interior && (cx == 0 || cx == nx - 1);
            const bool by = !interior && (cy == 0 || cy == ny - 1);
            const bool bz = !interior && (cz == 0 || cz == nz - 1);
            switch ((bx ? 1 : 0) | (by ? 2 : 0) | (bz ? 4 : 0)) {
            case 0: sweep(F{}, F{}, F{}); break;
            case 1: sweep(T{}, F{}, F{}); break;
            case 2: sweep(F{}, T{}, F{}); break;
            case 4: sweep(F{}, F{}, T{}); break;
            default: sweep(T{}, T{}, T{}); break;  // edges and corners
            }
        }
        return;
    }

    if (part != 0) return;  // the general path runs the whole cell in one wavefront
    // general path
    const bool wl = cx == 0, wr = cx == nx - 1;  // the row wraps on the left / right
    // particles in batches of kGenBatch, each with its far buffer
    for (int ib = 0; ib < ni; ib += kGenBatch) {
        const int nic = ni - ib < kGenBatch ? ni - ib : kGenBatch;
        const int me = i0 + ib + (lane < nic ? lane : 0);
        const double pxi = ld(xs.x, me), pyi = ld(xs.y, me), pzi = ld(xs.z, me);
        int cnt = 0;  // lane u: near count | far count << 16 of particle i0 + ib + u
        for (int dz = -1; dz <= 1; ++dz) {
            const int zz = wrap_index(cz + dz, nz);
            const double sz = cz + dz < 0 ? g.L[2] : (cz + dz >= nz ? -g.L[2] : 0.0);
            // six pieces (wave-uniform): per row dy, piece A then piece B
            int pb[6], pl[6];
            double psx[6], psy[6];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int dy = r - 1;
                const int yy = wrap_index(cy + dy, ny);
                const double sy = cy + dy < 0 ? g.L[1] : (cy + dy >= ny ? -g.L[1] : 0.0);
                const int base = nx * (yy + ny * zz);
                int a0, a1, b0, b1;
                double asx = 0.0, bsx = 0.0;
                if (wl) {         // cells nx-1 (shifted +L), then 0, 1
                    a0 = base + nx - 1;
                    a1 = base + nx;
                    asx = g.L[0];
                    b0 = base;
                    b1 = base + 2;
                } else if (wr) {  // cells nx-2, nx-1, then 0 (shifted -L)
                    a0 = base + nx - 2;
                    a1 = base + nx;
                    b0 = base;
                    b1 = base + 1;
                    bsx = -g.L[0];
                } else {          // cells cx-1 .. cx+1
                    a0 = base + cx - 1;
                    a1 = base + cx + 2;
                    b0 = b1 = base;
                }
                pb[2 * r] = cstart[a0];
                pl[2 * r] = cstart[a1] - pb[2 * r];
                pb[2 * r + 1] = cstart[b0];
                pl[2 * r + 1] = cstart[b1] - pb[2 * r + 1];
                psx[2 * r] = asx;
                psx[2 * r + 1] = bsx;
                psy[2 * r] = sy;
                psy[2 * r + 1] = sy;
            }
            int Q = 0;
#pragma unroll
            for (int k = 0; k < 6; ++k) Q += pl[k];
            for (int q0 = 0; q0 < Q; q0 += 64) {
                int off = q0 + lane, slot = -1;
                double sx = 0.0, sy = 0.0;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    if (off >= 0 && off < pl[k]) {
                        slot = pb[k] + off;
                        sx = psx[k];
                        sy = psy[k];
                    }
                    off -= pl[k];
                }
                const int js = slot >= 0 ? slot : i0;
                const double xj = ld(xs.x, js), yj = ld(xs.y, js), zj = ld(xs.z, js);
                for (int u = 0; u < nic; ++u) {
                    const double xi = bcast_d(pxi, u), yi = bcast_d(pyi, u), zi = bcast_d(pzi, u);
                    const int i = i0 + ib + u;
                    const double r2 = exact_r2((xi - xj) + sx, (yi - yj) + sy, (zi - zj) + sz);
                    const unsigned long long hm = __builtin_amdgcn_ballot_w64(slot >= 0 && slot != i && r2 < rc2);
                    if (hm) {
                        const unsigned long long nm = __builtin_amdgcn_ballot_w64(r2 < rd2);
                        const unsigned long long mn = hm & nm, mf = hm & ~nm;
                        const int base = bcast_i(cnt, u);
                        emit_hits<R2>(row_rsrc(nl + (size_t)i * kListCap, kListCap * 4), R2Row<R2>(nlr2, nslots, i),
                                      far_lds + u * kListCap, dump, mn, mf, base & 0xffff, base >> 16,
                                      (uint32_t)slot | (sx != 0.0 || sy != 0.0 || sz != 0.0 ? kWrapBit : 0u), r2);
                        if (lane == u) cnt += __popcll(mn) + (__popcll(mf) << 16);
                    }
                }
            }
        }
        for (int u = 0; u < nic; ++u) {
            const int i = i0 + ib + u, c2 = bcast_i(cnt, u);
            flush_far(row_rsrc(nl + (size_t)i * kListCap, kListCap * 4), far_lds + u * kListCap, c2 & 0xffff,
                      c2 >> 16);
        }
        if (lane < nic) ncnt[i0 + ib + lane] = cnt;
    }
}

// Interior cells (and, for the border kernel, border cells) at eight waves
// per SIMD: the interior path fits in 64 VGPRs.
template <typename R2>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_nlist_cell(
    Reps R, Soa3c xs, const int *__restrict__ cstart_all, int *__restrict__ ncnt, uint32_t *__restrict__ nl,
    R2 *__restrict__ nlr2, int all)
{
    if (!all && cload(R.flag, R.nrep) == 0) return;
    __shared__ __align__(16) uint32_t lds[kWavesPerBlock * kFarLds];
    const int w = __builtin_amdgcn_readfirstlane(xcd_block() * kWavesPerBlock + (int)(threadIdx.x >> 6));
    if (w >= R.nicells) return;
    const int cg = cload(R.icells, w);
    nlist_cell<R2, false>(R, cg, xs, cstart_all, ncnt, nl, nlr2, lds + (threadIdx.x >> 6) * kFarLds, all);
}

template <typename R2>
__global__ __launch_bounds__(kBlock) void k_nlist_border(Reps R, Soa3c xs, const int *__restrict__ cstart_all,
                                                         int *__restrict__ ncnt, uint32_t *__restrict__ nl,
                                                         R2 *__restrict__ nlr2, int all)
{
    if (!all && cload(R.flag, R.nrep) == 0) return;
    __shared__ __align__(16) uint32_t lds[kWavesPerBlock * kFarLds];
    const int w = __builtin_amdgcn_readfirstlane(xcd_block() * kWavesPerBlock + (int)(threadIdx.x >> 6));
    const int S = R.list_split;
    if (w >= R.nbcells * S) return;
    nlist_cell<R2, true>(R, cload(R.bcells, w / S), xs, cstart_all, ncnt, nl, nlr2,
                         lds + (threadIdx.x >> 6) * kFarLds, all, w % S, S);
}

// ---------------------------------------------------------------------------
// Skin list: one wavefront per cell.
//
// The distinct cells around the cell (offsets -1, 0, +1 per axis with three
// cells or more on it, 0 and +1 with two, 0 with one) are taken one z layer
// at a time; a layer is up to three rows of x-adjacent cells, each one or two
// contiguous pieces of the sorted order.  The wave loads 64 candidates of the
// layer at a time (lane q holds candidate q) and tests them against every
// particle of the cell, broadcast through the scalar unit, with the exact
// FP64 test: a ballot and mbcnt append the hits to the particle's row in
// candidate order; its running count lives in lane (particle mod 64).
// Cells within two cells of a box face take the minimum image of every
// difference (the torus distance) and flag their entries: such a pair may
// cross a face before the next build, the others cannot (both particles
// stay more than a cell edge minus half the skin inside the box).
template <bool ALL>
__device__ __forceinline__ void skin_cell(const Reps &R, int cg, Soa3c xs, const int *__restrict__ cstart_all,
                                          int *__restrict__ scnt, uint32_t *__restrict__ sl)
{
    const int lane = threadIdx.x & 63;
    const int rep = R.cell_rep ? cload(R.cell_rep, cg) : 0;
    if (!ALL && cload(R.flag, rep) == 0) return;
    const Geom g = cload(R.geom, rep);
    const int c = cg - cload(R.cell_off, rep);
    const int *__restrict__ cstart = cstart_all + cload(R.cell_off, rep);
    const int i0 = cstart[c], ni = cstart[c + 1] - i0;
    if (ni == 0) return;
    const int nx = g.nc[0], ny = g.nc[1], nz = g.nc[2];
    // cell coordinates: the quotients are exact in FP64 (at most 2^24 cells),
    // which avoids integer division
    const int cyz = __builtin_amdgcn_readfirstlane((int)(((double)c + 0.5) * g.inv_nc[0]));
    const int cz = __builtin_amdgcn_readfirstlane((int)(((double)cyz + 0.5) * g.inv_nc[1]));
    const int cx = c - cyz * nx, cy = cyz - cz * ny;
    const bool face = cx < 2 || cx >= nx - 2 || cy < 2 || cy >= ny - 2 || cz < 2 || cz >= nz - 2;
    const uint32_t wrap = face ? kWrapBit : 0u;
    const double rs2 = g.rs2;
    const int oz0 = nz >= 3 ? -1 : 0, oz1 = nz >= 2 ? 1 : 0;
    const int oy0 = ny >= 3 ? -1 : 0, oy1 = ny >= 2 ? 1 : 0;
    // the x cells of a row: [a0, a1) and, when the row wraps, [b0, b1)
    int a0 = 0, a1 = nx, b0 = 0, b1 = 0;
    if (nx >= 3) {
        if (cx == 0) {
            a0 = nx - 1;
            b1 = 2;
        } else if (cx == nx - 1) {
            a0 = nx - 2;
            b1 = 1;
        } else {
            a0 = cx - 1;
            a1 = cx + 2;
        }
    }
    for (int ib = 0; ib < ni; ib += 64) {
        const int nic = ni - ib < 64 ? ni - ib : 64;
        const int me = i0 + ib + (lane < nic ? lane : 0);
        const double pxi = ld(xs.x, me), pyi = ld(xs.y, me), pzi = ld(xs.z, me);
        int cnt = 0;  // lane u: entries of particle i0 + ib + u so far
        for (int oz = oz0; oz <= oz1; ++oz) {
            const int zz = wrap_index(cz + oz, nz);
            int pb[6], pl[6];
            int Q = 0;
            for (int oy = oy0; oy <= oy1; ++oy) {
                const int yy = wrap_index(cy + oy, ny);
                const int base = nx * (yy + ny * zz);
                const int r = oy - oy0;
                pb[2 * r] = cstart[base + a0];
                pl[2 * r] = cstart[base + a1] - pb[2 * r];
                pb[2 * r + 1] = cstart[base + b0];
                pl[2 * r + 1] = cstart[base + b1] - pb[2 * r + 1];
                Q += pl[2 * r] + pl[2 * r + 1];
            }
            const int npieces = 2 * (oy1 - oy0 + 1);
            for (int q0 = 0; q0 < Q; q0 += 64) {
                int off = q0 + lane, slot = -1;
                for (int k = 0; k < npieces; ++k) {
                    if (off >= 0 && off < pl[k]) slot = pb[k] + off;
                    off -= pl[k];
                }
                const int js = slot >= 0 ? slot : i0;
                const double xj = ld(xs.x, js), yj = ld(xs.y, js), zj = ld(xs.z, js);
                for (int u = 0; u < nic; ++u) {
                    const double xi = bcast_d(pxi, u), yi = bcast_d(pyi, u), zi = bcast_d(pzi, u);
                    const int i = i0 + ib + u;
                    double dx = xi - xj, dy = yi - yj, dz = zi - zj;
                    if (face) {
                        dx = min_image(dx, g.L[0], g.invL[0]);
                        dy = min_image(dy, g.L[1], g.invL[1]);
                        dz = min_image(dz, g.L[2], g.invL[2]);
                    }
                    const double r2 = exact_r2(dx, dy, dz);
                    const bool hit = slot >= 0 && slot != i && r2 < rs2;
                    const unsigned long long hm = __builtin_amdgcn_ballot_w64(hit);
                    if (hm) {
                        const int pos = lanes_below(hm, bcast_i(cnt, u));
                        const __amdgpu_buffer_rsrc_t ro = row_rsrc(sl + (size_t)i * kSkinCap, kSkinCap * 4);
                        __builtin_amdgcn_raw_buffer_store_b32((uint32_t)slot | wrap, ro, hit ? pos * 4 : kDropOffset,
                                                              0, 0);
                        if (lane == u) cnt += (int)__popcll(hm);
                    }
                }
            }
        }
        if (lane < nic) scnt[i0 + ib + lane] = cnt;
    }
}

template <bool ALL>
__global__ __launch_bounds__(kBlock) void k_skin_build(Reps R, Soa3c xs, const int *__restrict__ cstart_all,
                                                       int *__restrict__ scnt, uint32_t *__restrict__ sl)
{
    if (!ALL && cload(R.flag, R.nrep) == 0) return;
    const int cg = __builtin_amdgcn_readfirstlane(xcd_block() * kWavesPerBlock + (int)(threadIdx.x >> 6));
    if (cg >= R.ncells) return;
    skin_cell<ALL>(R, cg, xs, cstart_all, scnt, sl);
}

// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R w_rho(const PairConst &pc, R r2);

template <>
__device__ __forceinline__ double w_rho<double>(const PairConst &pc, double r2)
{
    const double r = __builtin_sqrt(r2);
    const double u = 1.0 - r * pc.inv_rd;
    return pc.wrho * u * u;
}

template <>
__device__ __forceinline__ float w_rho<float>(const PairConst &pc, float r2)
{
    const float r = __builtin_sqrtf(r2);
    const float u = 1.0f - r * (float)pc.inv_rd;
    return (float)pc.wrho * u * u;
}

// ---------------------------------------------------------------------------
// The neighbour record of slot i and its density rho_i, written by the P lanes
// of i (sub = lane in the group).  The FP32 form writes the 32-byte
// fixed-point record, the FP64 form the 64-byte one.  With P = 4 the four
// lanes write a quarter of the record each, so one store instruction covers
// 16 whole records.
template <int P, typename R>
__device__ __forceinline__ void put_record(const PairConst &pc, int i, int sub, Soa3c xs, Soa3c vh,
                                           const uint32_t *__restrict__ tag, const uint8_t *__restrict__ typ,
                                           R acc, R *__restrict__ rho, PartRec *__restrict__ rec)
{
    if (sub == 0) rho[i] = acc;
    const uint32_t tg = tag[i];
    const bool fz = (tg & kFrozenBit) != 0;
    if constexpr (sizeof(R) == 4) {
        // qx qy | qz vx | vy vz | rho tag
        PartRec32 *const r32 = reinterpret_cast<PartRec32 *>(rec);
        auto vel = [&](double u) { return __float_as_uint(fz ? 0.0f : (float)u); };
        if constexpr (P == 4) {
            const double *pa = sub == 0 ? xs.x : (sub == 1 ? xs.z : vh.y);
            const double *pb = sub == 0 ? xs.y : (sub == 1 ? vh.x : vh.z);
            uint2 w;
            if (sub < 3) {
                const double a = pa[i], b = pb[i];
                w.x = sub < 2 ? qfix(a, sub == 0 ? pc.qs[0] : pc.qs[2]) : vel(a);
                w.y = sub == 0 ? qfix(b, pc.qs[1]) : vel(b);
            } else {
                w = make_uint2(__float_as_uint((float)acc), tg);
            }
            reinterpret_cast<uint2 *>(r32 + i)[sub] = w;
        } else if (sub == 0) {
            PartRec32 o;
            o.qx = qfix(xs.x[i], pc.qs[0]);
            o.qy = qfix(xs.y[i], pc.qs[1]);
            o.qz = qfix(xs.z[i], pc.qs[2]);
            o.vx = __uint_as_float(vel(vh.x[i]));
            o.vy = __uint_as_float(vel(vh.y[i]));
            o.vz = __uint_as_float(vel(vh.z[i]));
            o.rho = (float)acc;
            o.tag = tg;
            r32[i] = o;
        }
    } else if constexpr (P == 4) {
        // x y | z vx | vy vz | rho tag typ
        const double *pa = sub == 0 ? xs.x : (sub == 1 ? xs.z : vh.y);
        const double *pb = sub == 0 ? xs.y : (sub == 1 ? vh.x : vh.z);
        double a = pa[i], b = pb[i];
        if (fz && sub >= 1) {
            b = 0.0;
            if (sub >= 2) a = 0.0;
        }
        if (sub == 3) {
            a = (double)acc;
            b = __longlong_as_double((long long)((unsigned long long)tg | ((unsigned long long)typ[i] << 32)));
        }
        reinterpret_cast<double2 *>(rec + i)[sub] = make_double2(a, b);
    } else if (sub == 0) {
        PartRec o;
        o.x = xs.x[i];
        o.y = xs.y[i];
        o.z = xs.z[i];
        o.vx = fz ? 0.0 : vh.x[i];
        o.vy = fz ? 0.0 : vh.y[i];
        o.vz = fz ? 0.0 : vh.z[i];
        o.rho = (double)acc;
        o.tag = tg;
        o.typ = typ[i];
        rec[i] = o;
    }
}

// Density from the per-step list: the stored r^2 of the near entries (r < r_d
// first in the row), or a direct scan for a row that overflowed; also packs
// the neighbour records.
template <int P, typename R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_density_list(Reps Rp, Soa3c xs, Soa3c vh, const uint32_t *__restrict__ tag,
                                                    const uint8_t *__restrict__ typ,
                                                    const int *__restrict__ cstart_all,
                                                    const int *__restrict__ ncnt,
                                                    const R *__restrict__ nlr2, R *__restrict__ rho,
                                                    PartRec *__restrict__ rec)
{
    const BlockRep br = block_rep<P>(Rp, xcd_block());
    const int i = br.i0 + (int)threadIdx.x / P;
    const int sub = threadIdx.x & (P - 1);
    if (i >= br.i1) return;
    const PairConst pc = cload(Rp.pc, br.r);
    const Geom g = cload(Rp.geom, br.r);
    const int *__restrict__ cstart = cstart_all + cload(Rp.cell_off, br.r);
    const int packed = ncnt[i];
    R acc = 0;
    if (list_total(packed) <= kListCap) {
        const int nnear = list_near(packed);
        const R *hd, *tl;
        r2_row_ptrs<R>(nlr2, (size_t)cload(Rp.part_off, Rp.nrep), i, hd, tl);
        for (int k = sub; k < nnear; k += P) acc += w_rho<R>(pc, *(k < kR2Head ? hd + k : tl + k));
    } else {
        const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
        for_each_row(g, xi, yi, zi, cstart, [&](int b, int e) {
            for (int j = b + sub; j < e; j += P) {
                if (j == i) continue;
                double dx = xi - xs.x[j], dy = yi - xs.y[j], dz = zi - xs.z[j];
                min_image3(g, dx, dy, dz);
                const double r2 = exact_r2(dx, dy, dz);
                if (r2 < g.rd2) acc += w_rho<R>(pc, (R)r2);
            }
        });
    }
    acc = group_sum<P>(acc);
    put_record<P, R>(pc, i, sub, xs, vh, tag, typ, acc, rho, rec);
}

// Pair list and density.  The P lanes of particle i take its skin entries in
// turns; each entry closer than r_c at the current positions is appended to
// i's pair row (flag kNearBit when r < r_d) at the group's running count plus
// the group's hits in lower lanes, so the row keeps the skin order.  The near
// count and the far count are packed in ncnt (near | far << 16); a row over
// kListCap entries is not read (the passes scan the cells directly).
template <int P, typename R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_density_skin(
    Reps Rp, Soa3c xs, Soa3c vh, const uint32_t *__restrict__ tag, const uint8_t *__restrict__ typ,
    const int *__restrict__ cstart_all, const int *__restrict__ scnt, const uint32_t *__restrict__ sl,
    int *__restrict__ ncnt, uint32_t *__restrict__ nl, R *__restrict__ rho, PartRec *__restrict__ rec)
{
    const BlockRep br = block_rep<P>(Rp, xcd_block());
    const int i = br.i0 + (int)threadIdx.x / P;
    const int sub = threadIdx.x & (P - 1);
    if (i >= br.i1) return;
    const PairConst pc = cload(Rp.pc, br.r);
    const Geom g = cload(Rp.geom, br.r);
    const int *__restrict__ cstart = cstart_all + cload(Rp.cell_off, br.r);
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    const int ns = scnt[i];
    R acc = 0;
    if (ns <= kSkinCap) {
        const int lane = threadIdx.x & 63;
        const unsigned long long gmask = (P == 64 ? ~0ull : ((1ull << P) - 1ull)) << (lane & ~(P - 1));
        const uint32_t *__restrict__ srow = sl + (size_t)i * kSkinCap;
        const __amdgpu_buffer_rsrc_t ro = row_rsrc(nl + (size_t)i * kListCap, kListCap * 4);
        int cn = 0, cf = 0;
        for (int k0 = 0; k0 < ns; k0 += P) {
            const int k = k0 + sub;
            const bool valid = k < ns;
            const uint32_t e = valid ? srow[k] : 0u;
            const int j = (int)(e & kSlotMask);
            double dx = xi - ld(xs.x, j), dy = yi - ld(xs.y, j), dz = zi - ld(xs.z, j);
            if (e & kWrapBit) {
                dx = min_image(dx, pc.L[0], pc.invL[0]);
                dy = min_image(dy, pc.L[1], pc.invL[1]);
                dz = min_image(dz, pc.L[2], pc.invL[2]);
            }
            const double r2 = exact_r2(dx, dy, dz);
            const bool hit = valid && r2 < g.rc2;
            const bool near = hit && r2 < g.rd2;
            if (near) acc += w_rho<R>(pc, (R)r2);
            const unsigned long long mh = __builtin_amdgcn_ballot_w64(hit) & gmask;
            const unsigned long long mn = __builtin_amdgcn_ballot_w64(near) & gmask;
            const int pos = lanes_below(mh, cn + cf);
            __builtin_amdgcn_raw_buffer_store_b32((e & (kSlotMask | kWrapBit)) | (near ? kNearBit : 0u), ro,
                                                  hit ? pos * 4 : kDropOffset, 0, 0);
            const int h = (int)__popcll(mh), hn = (int)__popcll(mn);
            cn += hn;
            cf += h - hn;
        }
        if (sub == 0) ncnt[i] = cn | (cf << 16);
    } else {
        for_each_row(g, xi, yi, zi, cstart, [&](int b, int e) {
            for (int j = b + sub; j < e; j += P) {
                if (j == i) continue;
                double dx = xi - xs.x[j], dy = yi - xs.y[j], dz = zi - xs.z[j];
                min_image3(g, dx, dy, dz);
                const double r2 = exact_r2(dx, dy, dz);
                if (r2 < g.rd2) acc += w_rho<R>(pc, (R)r2);
            }
        });
        if (sub == 0) ncnt[i] = (kListCap + 1) << 16;  // not a list: the passes scan the cells
    }
    acc = group_sum<P>(acc);
    if (!rho) return;  // the pair list only
    put_record<P, R>(pc, i, sub, xs, vh, tag, typ, acc, rho, rec);
}

// ---------------------------------------------------------------------------
// Wall mask: the cell lattice refined R.wsub times per axis; a sub-cell is
// marked when its box comes closer than r_c (plus a relative margin of 1e-6
// that covers the rounding of the sub-cell coordinate) to a frozen particle
// or one of its periodic images.  A fluid particle in an unmarked sub-cell has
// no frozen neighbour within r_c, so phi = 0 and it is never flagged.  Frozen
// particles never move, so the mask is built once (a plain store of 1 from
// every writer).
__device__ __forceinline__ int wrap_any(int a, int n)
{
    const int m = a % n;
    return m < 0 ? m + n : m;
}

__device__ __forceinline__ double box_gap(double p, int a, double h)
{
    return fmax(0.0, fmax(a * h - p, p - (a + 1) * h));
}

__global__ __launch_bounds__(kBlock) void k_mark_wall_cells(Reps R, Soa3c xs, const uint32_t *__restrict__ tag,
                                                            uint8_t *__restrict__ wmask)
{
    const BlockRep br = block_rep<1>(R, blockIdx.x);
    const int i = br.i0 + (int)threadIdx.x;
    if (i >= br.i1 || !(tag[i] & kFrozenBit)) return;
    const Geom g = cload(R.geom, br.r);
    const int k = R.wsub;
    uint8_t *const m = wmask + (size_t)cload(R.cell_off, br.r) * (size_t)(k * k * k);
    const double reach = g.rc * (1.0 + 1e-6), reach2 = reach * reach;
    const double p[3] = {xs.x[i], xs.y[i], xs.z[i]};
    int lo[3], hi[3], N[3];
    double h[3];
    for (int a = 0; a < 3; ++a) {
        N[a] = g.nc[a] * k;
        h[a] = g.cs[a] / k;
        lo[a] = (int)floor((p[a] - reach) / h[a]);
        hi[a] = (int)floor((p[a] + reach) / h[a]);
    }
    for (int az = lo[2]; az <= hi[2]; ++az) {
        const double ez = box_gap(p[2], az, h[2]);
        const int wz = wrap_any(az, N[2]);
        for (int ay = lo[1]; ay <= hi[1]; ++ay) {
            const double ey = box_gap(p[1], ay, h[1]);
            const double q = ey * ey + ez * ez;
            if (!(q < reach2)) continue;
            const size_t row = (size_t)N[0] * (wrap_any(ay, N[1]) + (size_t)N[1] * wz);
            for (int ax = lo[0]; ax <= hi[0]; ++ax) {
                const double ex = box_gap(p[0], ax, h[0]);
                if (ex * ex + q < reach2) m[row + wrap_any(ax, N[0])] = 1;
            }
        }
    }
}

// phi_i = sum_{frozen j} w_c^2 / sum_j w_c^2 over neighbours within r_c at the
// predicted positions, by a direct scan of the cells (the exact test of the
// neighbour list); flag[i] = 0 when phi_i <= phi_c, else 1 (bounce-back: the
// corrector negates the half-step velocity) or, with NRM and wall_slip > 0,
// 2: the half-step velocity is reflected here about the wall normal
// n = unit(sum_{frozen j} w_c^2 (x_i - x_j) / r), normal part negated,
// tangential part times 2 slip - 1 (a zero normal sum gives flag 1).  Frozen
// particles and fluid particles in unmarked sub-cells have flag 0 and are not
// scanned.  Each wavefront takes 64 slots, packs the ones to scan in LDS, and
// runs them in rounds of 64 / P particles with P lanes each, so skipped
// particles leave no idle lanes.
// Without the wall normal the kernel fits the budget of six waves per SIMD
// (80 VGPRs, no spills, against 92 and five waves unbounded: ring cells at
// 1M particles 174 -> 167 us per step for phi and the corrector).
template <int P, bool NRM>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(NRM ? 1 : 6))) void k_phi(Reps R, Soa3c xs, const uint32_t *__restrict__ tag,
                                                const int *__restrict__ cstart_all,
                                                const uint8_t *__restrict__ wmask, int *__restrict__ flag, Soa3 vh)
{
    __shared__ int pick[kBlock];
    const BlockRep br = block_rep<1>(R, xcd_block());
    const int lane = (int)threadIdx.x & 63;
    int *const wp = pick + ((int)threadIdx.x & ~63);
    const int i = br.i0 + (int)threadIdx.x;
    const Geom g = cload(R.geom, br.r);
    const int coff = cload(R.cell_off, br.r);
    bool scan = false;
    if (i < br.i1) {
        if (!(tag[i] & kFrozenBit)) {
            const int k = R.wsub;
            const int sx = cell_coord(xs.x[i], g.s[0] * k, g.nc[0] * k);
            const int sy = cell_coord(xs.y[i], g.s[1] * k, g.nc[1] * k);
            const int sz = cell_coord(xs.z[i], g.s[2] * k, g.nc[2] * k);
            scan = wmask[(size_t)coff * (size_t)(k * k * k) + sx +
                         (size_t)g.nc[0] * k * (sy + (size_t)g.nc[1] * k * sz)] != 0;
        }
        if (!scan) flag[i] = 0;
    }
    const uint64_t m = __builtin_amdgcn_ballot_w64(scan);
    if (m == 0) return;
    if (scan) wp[lanes_below(m)] = i;
    __builtin_amdgcn_wave_barrier();
    const int cnt = (int)__popcll(m);
    const PairConst pc = cload(R.pc, br.r);
    const int *__restrict__ cstart = cstart_all + coff;
    const int sub = lane & (P - 1);
    for (int q = lane / P; q < cnt; q += 64 / P) {  // uniform over the P lanes of a particle
        const int ii = wp[q];
        const double xi = xs.x[ii], yi = xs.y[ii], zi = xs.z[ii];
        double num = 0.0, den = 0.0, nx = 0.0, ny = 0.0, nz = 0.0;
        for_each_row(g, xi, yi, zi, cstart, [&](int b, int e) {
            for (int j = b + sub; j < e; j += P) {
                if (j == ii) continue;
                double dx = xi - xs.x[j], dy = yi - xs.y[j], dz = zi - xs.z[j];
                min_image3(g, dx, dy, dz);
                const double r2 = exact_r2(dx, dy, dz);
                if (!(r2 < g.rc2)) continue;
                const double r = __builtin_sqrt(r2);
                const double w = 1.0 - r * pc.inv_rc;
                den += w * w;
                if (tag[j] & kFrozenBit) {
                    num += w * w;
                    if constexpr (NRM) {
                        if (r2 > 0.0) {
                            const double c = w * w / r;
                            nx += c * dx;
                            ny += c * dy;
                            nz += c * dz;
                        }
                    }
                }
            }
        });
        num = group_sum<P>(num);
        den = group_sum<P>(den);
        const bool hit = den > 0.0 && num / den > pc.phi_c;
        int f = hit ? 1 : 0;
        if constexpr (NRM) {
            nx = group_sum<P>(nx);
            ny = group_sum<P>(ny);
            nz = group_sum<P>(nz);
            const double n2 = nx * nx + ny * ny + nz * nz;
            // a particle also sent back in the last step is bounced back
            // (flag 1) so that it leaves the wall the way it came
            if (hit && pc.slip > 0.0 && n2 > 0.0 && sub == 0 && !(tag[ii] & kRejectBit)) {
                const double inv = 1.0 / __builtin_sqrt(n2);
                const double ux = nx * inv, uy = ny * inv, uz = nz * inv;
                const double vx = vh.x[ii], vy = vh.y[ii], vz = vh.z[ii];
                const double vn = vx * ux + vy * uy + vz * uz;
                const double tx = vx - vn * ux, ty = vy - vn * uy, tz = vz - vn * uz;
                const double ft = 2.0 * pc.slip - 1.0;
                vh.x[ii] = ft * tx - vn * ux;
                vh.y[ii] = ft * ty - vn * uy;
                vh.z[ii] = ft * tz - vn * uz;
                f = 2;
            }
        }
        if (sub == 0) flag[ii] = f;
    }
}

// Applies the corrector to flagged particles: x <- x(t), and for flag 1
// v_half <- -v_half (flag 2: k_phi has reflected v_half already).  Blocks are
// replica-aligned (kBlock slots of one replica); each writes its number of
// corrections to part[blockIdx.x] and the largest squared distance of a
// corrected particle from its build position to cmax[blockIdx.x]: the list
// covers a particle sent back as long as that stays below half the skin,
// which the step's second gate checks.  With byid (the adjoint's recording)
// a corrected particle also sets byid[part_off[r] + id].
__global__ __launch_bounds__(kBlock) void k_correct(Reps R, const int *__restrict__ flag, Soa3c xprev, Soa3 xs,
                                                    Soa3 vh, int *__restrict__ part,
                                                    uint32_t *__restrict__ tag, uint8_t *__restrict__ byid,
                                                    Soa3c xbuild, float *__restrict__ cmax)
{
    __shared__ int cnt[kWavesPerBlock];
    __shared__ float far[kWavesPerBlock];
    const BlockRep br = block_rep<1>(R, blockIdx.x);
    const int i = br.i0 + (int)threadIdx.x;
    int hit = 0;
    float d2 = 0.0f;
    const int f = i < br.i1 ? flag[i] : 0;
    if (i < br.i1 && cload(R.pc, br.r).slip > 0.0) {
        // wall slip: remember which fluid particles were sent back this step
        const uint32_t tg = tag[i];
        if (!(tg & kFrozenBit) && ((tg & kRejectBit) != 0) != (f != 0))
            tag[i] = f ? (tg | kRejectBit) : (tg & ~kRejectBit);
    }
    if (f) {
        const double px = xprev.x[i], py = xprev.y[i], pz = xprev.z[i];
        xs.x[i] = px;
        xs.y[i] = py;
        xs.z[i] = pz;
        if (f == 1) {
            vh.x[i] = -vh.x[i];
            vh.y[i] = -vh.y[i];
            vh.z[i] = -vh.z[i];
        }
        if (xbuild.x) {
            const Geom g = cload(R.geom, br.r);
            const double dx = min_image(px - xbuild.x[i], g.L[0], g.invL[0]);
            const double dy = min_image(py - xbuild.y[i], g.L[1], g.invL[1]);
            const double dz = min_image(pz - xbuild.z[i], g.L[2], g.invL[2]);
            d2 = (float)((dx * dx + dy * dy + dz * dz) * (1.0 + 1e-6));
        } else {
            d2 = 1.0f;  // skin 0: any particle moved back re-sorts its replica
        }
        if (byid) byid[(size_t)cload(R.part_off, br.r) + (tag[i] & kIdMask)] = 1;
        hit = 1;
    }
    const int w = (int)__popcll(__ballot(hit));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d2 = fmaxf(d2, __shfl_xor(d2, o, 64));
    if ((threadIdx.x & 63) == 0) {
        cnt[threadIdx.x >> 6] = w;
        far[threadIdx.x >> 6] = d2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        float m = 0.0f;
        for (int k = 0; k < kWavesPerBlock; ++k) {
            t += cnt[k];
            m = fmaxf(m, far[k]);
        }
        part[blockIdx.x] = t;
        cmax[blockIdx.x] = m;
    }
}

// The step's number of corrections (the re-sort gate) and the running total,
// from the block counts of k_correct (one block, no atomics).
__global__ __launch_bounds__(kBlock) void k_correct_sum(int nb, const int *__restrict__ part,
                                                        int *__restrict__ ncorr,
                                                        unsigned long long *__restrict__ ncorr_total)
{
    __shared__ int cnt[kWavesPerBlock];
    int t = 0;
    for (int k = (int)threadIdx.x; k < nb; k += kBlock) t += part[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        int sum = 0;
        for (int k = 0; k < kWavesPerBlock; ++k) sum += cnt[k];
        *ncorr = sum;
        *ncorr_total += (unsigned long long)sum;
    }
}

// ---------------------------------------------------------------------------
// Force pass with the velocity-Verlet epilogue.
__device__ __forceinline__ double wrap_coord(double x, double L)
{
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    return x;
}

// Dissipation control (DC): the dissipative and random parts of particle
// i's fluid-frozen pairs summed apart from the rest, and the sum of w_c^2
// over all its neighbours that gives s_i = dctl / w2; the parts are scaled
// by s_i and sqrt(s_i) once the neighbour loop is done.
template <typename R, bool DC>
struct WallDiss {};
template <typename R>
struct WallDiss<R, true> {
    R w2 = 0, dx = 0, dy = 0, dz = 0, rx = 0, ry = 0, rz = 0;
};

// Force of one neighbour j on i (Eq. 1 + dissipative + random), added to f;
// the conservative virial and the A-term pair energy, with weight c, to vir
// and ep.  d = x_i - x_j (minimum image), dv = v_half,i - v_half,j.  A
// coincident pair (r = 0) contributes nothing.  DC: w_c^2 goes to wd.w2, and
// for a fluid-frozen pair under the control (wall) the dissipative and random
// parts go to wd instead of f.
template <typename R, bool DC = false>
__device__ __forceinline__ void pair_force(const PairConst &pc, double A, double B, double gam, double sig,
                                           double Arc2, double dx, double dy, double dz, double dvx,
                                           double dvy, double dvz, bool near, R rhoij, int th, double c,
                                           R &fx, R &fy, R &fz, double &vir, double &ep,
                                           WallDiss<R, DC> *wd = nullptr, bool wall = false)
{
    if constexpr (DC) {
        // the same terms as below, kept apart
        const R r2 = (R)(dx * dx + dy * dy + dz * dz);
        const bool pos = r2 > (R)0;
        R rinv;
        if constexpr (sizeof(R) == 8) rinv = pos ? rsqrt_f64(r2) : 0.0;
        else rinv = pos ? __builtin_amdgcn_rsqf(r2) : 0.0f;
        const R r = r2 * rinv;
        const R wc = (R)1 - r * (R)pc.inv_rc;
        R fc = (R)A * wc;
        if (near) fc += (R)B * rhoij * ((R)1 - r * (R)pc.inv_rd);
        const R ex = (R)dx * rinv, ey = (R)dy * rinv, ez = (R)dz * rinv;
        const R ev = ex * (R)dvx + ey * (R)dvy + ez * (R)dvz;
        const R fd = -(R)gam * wc * wc * ev;
        R fr;
        if constexpr (sizeof(R) == 8) fr = sig * wc * ((double)th * kSqrt3Scaled);
        else fr = (float)sig * wc * ((float)th * kSqrt3ScaledF);
        wd->w2 += wc * wc;
        if (wall) {
            wd->dx += fd * ex;
            wd->dy += fd * ey;
            wd->dz += fd * ez;
            wd->rx += fr * ex;
            wd->ry += fr * ey;
            wd->rz += fr * ez;
            fx += fc * ex;
            fy += fc * ey;
            fz += fc * ez;
        } else {
            const R fs = fc + fd + fr;
            fx += fs * ex;
            fy += fs * ey;
            fz += fs * ez;
        }
        vir += c * (double)(fc * r);
        ep += pos ? c * Arc2 * (double)(wc * wc) : 0.0;
    } else if constexpr (sizeof(R) == 8) {
        const double r2 = dx * dx + dy * dy + dz * dz;
        const bool pos = r2 > 0.0;
        const double rinv = pos ? rsqrt_f64(r2) : 0.0;
        const double r = r2 * rinv;
        const double wc = 1.0 - r * pc.inv_rc;
        double fc = A * wc;
        if (near) fc += B * rhoij * (1.0 - r * pc.inv_rd);
        const double ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
        const double ev = ex * dvx + ey * dvy + ez * dvz;
        const double fs = fc - gam * wc * wc * ev + sig * wc * ((double)th * kSqrt3Scaled);
        fx += fs * ex;
        fy += fs * ey;
        fz += fs * ez;
        vir += c * fc * r;
        ep += pos ? c * Arc2 * wc * wc : 0.0;
    } else {
        const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
        const float r2 = fdx * fdx + fdy * fdy + fdz * fdz;
        const bool pos = r2 > 0.0f;
        const float rinv = pos ? __builtin_amdgcn_rsqf(r2) : 0.0f;
        const float r = r2 * rinv;
        const float wc = 1.0f - r * (float)pc.inv_rc;
        float fc = (float)A * wc;
        if (near) fc += (float)B * rhoij * (1.0f - r * (float)pc.inv_rd);
        const float ex = fdx * rinv, ey = fdy * rinv, ez = fdz * rinv;
        const float ev = ex * (float)dvx + ey * (float)dvy + ez * (float)dvz;
        const float fs = fc - (float)gam * wc * wc * ev + (float)sig * wc * ((float)th * kSqrt3ScaledF);
        fx += fs * ex;
        fy += fs * ey;
        fz += fs * ez;
        vir += c * (double)(fc * r);
        ep += pos ? c * Arc2 * (double)(wc * wc) : 0.0;
    }
}

// Outputs of the force pass.
struct ForceOut {
    Soa3 v, f, vpred, xpred;  // v(t+dt), F(t+dt), next half-step velocity, next predicted x
    double *part;             // per-block virial and pair-energy partials
    int *status;              // bit 0: non-finite or out-of-box state
    int *ovf_count, *ovf;     // particles whose list overflowed, for k_force_overflow
    int initial;              // 1 at creation: v(t) is the given velocity
    Soa3c xbuild;             // positions at the last list build
    float *bmax;              // per block: largest squared displacement of xpred from xbuild (nullable)
};

// Squared distance (minimum image) of a new position from its build
// position, rounded up to FP32 for the gate's block maxima.
__device__ __forceinline__ float moved2(const PairConst &pc, const Soa3c &xb, int i, double qx, double qy, double qz)
{
    if (!xb.x) return 0.0f;  // skin 0: every step rebuilds anyway
    const double dx = min_image(qx - xb.x[i], pc.L[0], pc.invL[0]);
    const double dy = min_image(qy - xb.y[i], pc.L[1], pc.invL[1]);
    const double dz = min_image(qz - xb.z[i], pc.L[2], pc.invL[2]);
    const double d2 = dx * dx + dy * dy + dz * dz;
    return (float)(d2 * (1.0 + 1e-6));
}

// Force on particle i (slot), its velocity-Verlet epilogue, and its share of
// the virial and pair energy.  SCAN = false: the neighbours come from the
// list; SCAN = true: from a direct scan of the cells (lists that overflowed).
// Both are separate instantiations so the list kernel keeps the small
// register footprint of the list loop.
// LDS bytes per quad for the regrouping of four 64-byte records (padded
// against bank conflicts)
constexpr int kQuadXch = 4 * 64 + 16;

template <int P, bool MT, bool DC, bool SCAN, typename R>
__device__ __forceinline__ void force_particle(const PairConst &pc, const Geom &g, int i, int sub, Soa3c xs,
                                               Soa3c vh, const R *__restrict__ rho,
                                               const uint32_t *__restrict__ tag,
                                               const uint8_t *__restrict__ typ,
                                               const int *__restrict__ cstart, int packed,
                                               const uint32_t *__restrict__ lst,
                                               const PartRec *__restrict__ rec, const ForceOut &out,
                                               const double *__restrict__ tab, double &vir, double &ep,
                                               float &moved)
{
    const uint32_t tgi = tag[i];
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    if (tgi & kFrozenBit) {
        if (sub == 0) {
            out.v.x[i] = out.v.y[i] = out.v.z[i] = 0.0;
            out.f.x[i] = out.f.y[i] = out.f.z[i] = 0.0;
            out.vpred.x[i] = out.vpred.y[i] = out.vpred.z[i] = 0.0;
            out.xpred.x[i] = xi;
            out.xpred.y[i] = yi;
            out.xpred.z[i] = zi;
        }
        return;
    }
    const uint32_t idi = tgi & kIdMask;
    const double vxi = vh.x[i], vyi = vh.y[i], vzi = vh.z[i];
    const R rhoi = rho[i];
    const int T = pc.ntypes;
    const int ti = MT ? (int)typ[i] : 0;
    R fx = 0, fy = 0, fz = 0;
    WallDiss<R, DC> wd;
    const bool dc_on = DC && pc.dctl > 0.0;
    // pair arithmetic for one neighbour whose data is already loaded
    // (dv = v_half,i - v_half,j)
    auto pair = [&](double dx, double dy, double dz, double dvx, double dvy, double dvz, R rj, uint32_t tgj,
                    int tj, bool near) {
        double A = pc.A, B = pc.B, gam = pc.gamma, sig = pc.sig, Arc2 = pc.Arc2;
        if (MT) {
            const int tt = ti * T + tj;
            A = tab[tt];
            B = tab[64 + tt];
            gam = tab[128 + tt];
            sig = tab[192 + tt];
            Arc2 = tab[256 + tt];
        }
        const int th = theta_int(idi, tgj & kIdMask, pc);
        const double c = (tgj & kFrozenBit) ? 1.0 : 0.5;
        if (dc_on) {
            pair_force<R, DC>(pc, A, B, gam, sig, Arc2, dx, dy, dz, dvx, dvy, dvz, near, rhoi + rj, th, c, fx, fy,
                              fz, vir, ep, &wd, (tgj & kFrozenBit) != 0);
        } else {
            pair_force<R>(pc, A, B, gam, sig, Arc2, dx, dy, dz, dvx, dvy, dvz, near, rhoi + rj, th, c, fx, fy, fz,
                          vir, ep);
        }
    };
    // the FP32 form reads the 32-byte fixed-point records (the type of a
    // neighbour, with several types, from the type array)
    constexpr bool Q = sizeof(R) == 4;
    if constexpr (Q && !SCAN) {
        const PartRec32 *__restrict__ r32 = reinterpret_cast<const PartRec32 *>(rec);
        const uint32_t qxi = qfix(xi, pc.qs[0]), qyi = qfix(yi, pc.qs[1]), qzi = qfix(zi, pc.qs[2]);
        const float vxf = (float)vxi, vyf = (float)vyi, vzf = (float)vzi;
        // Each lane loads its own neighbour's record: two 16-byte loads of one
        // 32-byte sector (regrouping a quad's four records through LDS, as
        // the 64-byte records do, measured slower here: force pass 166
        // against 159 us at 1M particles).  The next record is loaded one
        // iteration ahead (155 against 159 us) and the entry after it two
        // ahead, so the record loads never wait on the row (146 against 147
        // us).  Entries past the row stand in as slot 0.
        const int cnt = list_total(packed);
        uint32_t e = sub < cnt ? lst[sub] : 0u;
        uint32_t en = sub + P < cnt ? lst[sub + P] : 0u;
        uint4 p0 = ((const uint4 *)(r32 + (int)(e & kSlotMask)))[0];  // qx qy qz vx
        uint4 p1 = ((const uint4 *)(r32 + (int)(e & kSlotMask)))[1];  // vy vz rho tag
        for (int k = sub; k < cnt; k += P) {
            const uint32_t enn = k + 2 * P < cnt ? lst[k + 2 * P] : 0u;
            const uint4 *rn = (const uint4 *)(r32 + (int)(en & kSlotMask));
            const uint4 n0 = rn[0], n1 = rn[1];
            pair(qdiff(qxi, p0.x, pc.qd[0]), qdiff(qyi, p0.y, pc.qd[1]), qdiff(qzi, p0.z, pc.qd[2]),
                 vxf - __uint_as_float(p0.w), vyf - __uint_as_float(p1.x), vzf - __uint_as_float(p1.y),
                 __uint_as_float(p1.z), p1.w, MT ? (int)typ[e & kSlotMask] : 0, (e & kNearBit) != 0);
            e = en;
            en = enn;
            p0 = n0;
            p1 = n1;
        }
    } else if constexpr (SCAN) {
        for_each_neighbor<P>(pc, g, i, sub, xi, yi, zi, xs, cstart, packed, nullptr,
                             [&](int j, double dx, double dy, double dz, bool near) {
                                 pair(dx, dy, dz, vxi - ld(vh.x, j), vyi - ld(vh.y, j), vzi - ld(vh.z, j),
                                      ld(rho, j), ld(tag, j),
                                      MT ? (int)ld(typ, j) : 0, near);
                             });
    } else if constexpr (P >= 4) {
        // Each quad of lanes loads its four neighbours' records together: lane
        // q of the quad fetches bytes [16 q, 16 q + 16) of all four, so a load
        // instruction touches one 64-byte sector per quad instead of one per
        // lane, and the pieces are regrouped through the quad's LDS slice.  A
        // quad lies inside one particle's lane group, so its lanes run the
        // same number of iterations.
        __shared__ __align__(16) unsigned char xch[(kBlock / 4) * kQuadXch];
        unsigned char *const qb = xch + (threadIdx.x >> 2) * kQuadXch;
        const int q = threadIdx.x & 3;
        const int cnt = list_total(packed);
        // the next entry is loaded one iteration ahead (two types, ring cells
        // at 1M particles: 227 against 201 us); slot 0 stands in for a
        // missing entry
        uint32_t en = sub < cnt ? lst[sub] : 0u;
        for (int k0 = 0; k0 < cnt; k0 += P) {
            const int k = k0 + sub;
            const uint32_t e = en;
            en = k + P < cnt ? lst[k + P] : 0u;
            const int j = (int)(e & kSlotMask);
            const int jq[4] = {__builtin_amdgcn_mov_dpp(j, 0x00, 0xF, 0xF, false),
                               __builtin_amdgcn_mov_dpp(j, 0x55, 0xF, 0xF, false),
                               __builtin_amdgcn_mov_dpp(j, 0xAA, 0xF, 0xF, false),
                               __builtin_amdgcn_mov_dpp(j, 0xFF, 0xF, 0xF, false)};
            uint4 piece[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) piece[t] = *((const uint4 *)(rec + jq[t]) + q);
#pragma unroll
            for (int t = 0; t < 4; ++t) *(uint4 *)(qb + t * 64 + q * 16) = piece[t];
            const uint4 *mine = (const uint4 *)(qb + q * 64);
            const uint4 p0 = mine[0], p1 = mine[1], p2 = mine[2], p3 = mine[3];
            if (k < cnt) {
                const double2 a = __builtin_bit_cast(double2, p0);  // x, y
                const double2 b = __builtin_bit_cast(double2, p1);  // z, v_x
                const double2 c = __builtin_bit_cast(double2, p2);  // v_y, v_z
                const R rj = (R)__longlong_as_double((long long)(((unsigned long long)p3.y << 32) | p3.x));
                const uint32_t tgj = p3.z;
                const int tj = MT ? (int)p3.w : 0;
                double dx = xi - a.x, dy = yi - a.y, dz = zi - b.x;
                if (e & kWrapBit) {  // pairs through a periodic image (border cells only)
                    dx = min_image(dx, pc.L[0], pc.invL[0]);
                    dy = min_image(dy, pc.L[1], pc.invL[1]);
                    dz = min_image(dz, pc.L[2], pc.invL[2]);
                }
                pair(dx, dy, dz, vxi - b.y, vyi - c.x, vzi - c.y, rj, tgj, tj, (e & kNearBit) != 0);
            }
        }
    } else {
        const int cnt = list_total(packed);
        // the next entry is loaded one iteration ahead, so a neighbour costs one
        // memory round trip (its record) instead of two
        uint32_t e = sub < cnt ? lst[sub] : 0u;
        for (int k = sub; k < cnt; k += P) {
            const uint32_t en = k + P < cnt ? lst[k + P] : 0u;
            const int j = (int)(e & kSlotMask);
            // the neighbour's packed record: four 16-byte loads of one sector
            const double2 *q = (const double2 *)(rec + j);
            const double2 a = q[0], b = q[1], c = q[2];
            const uint4 d = *(const uint4 *)(q + 3);
            const R rj = (R)__longlong_as_double((long long)(((unsigned long long)d.y << 32) | d.x));
            const uint32_t tgj = d.z;
            const int tj = MT ? (int)d.w : 0;
            double dx = xi - a.x, dy = yi - a.y, dz = zi - b.x;
            if (e & kWrapBit) {  // pairs through a periodic image (border cells only)
                dx = min_image(dx, pc.L[0], pc.invL[0]);
                dy = min_image(dy, pc.L[1], pc.invL[1]);
                dz = min_image(dz, pc.L[2], pc.invL[2]);
            }
            pair(dx, dy, dz, vxi - b.y, vyi - c.x, vzi - c.y, rj, tgj, tj, (e & kNearBit) != 0);
            e = en;
        }
    }
    fx = group_sum<P>(fx);
    fy = group_sum<P>(fy);
    fz = group_sum<P>(fz);
    double Fx = (double)fx + pc.mg[0];
    double Fy = (double)fy + pc.mg[1];
    double Fz = (double)fz + pc.mg[2];
    if constexpr (DC) {
        if (dc_on) {
            const R w2 = group_sum<P>(wd.w2);
            const R dxs = group_sum<P>(wd.dx), dys = group_sum<P>(wd.dy), dzs = group_sum<P>(wd.dz);
            const R rxs = group_sum<P>(wd.rx), rys = group_sum<P>(wd.ry), rzs = group_sum<P>(wd.rz);
            const double si = w2 > (R)0 ? pc.dctl / (double)w2 : 1.0;
            const double ri = __builtin_sqrt(si);
            Fx += si * (double)dxs + ri * (double)rxs;
            Fy += si * (double)dys + ri * (double)rys;
            Fz += si * (double)dzs + ri * (double)rzs;
        }
    }
    if (sub != 0) return;
    const double vx = out.initial ? vxi : vxi + pc.hdtm * Fx;
    const double vy = out.initial ? vyi : vyi + pc.hdtm * Fy;
    const double vz = out.initial ? vzi : vzi + pc.hdtm * Fz;
    const double px = vx + pc.hdtm * Fx;
    const double py = vy + pc.hdtm * Fy;
    const double pz = vz + pc.hdtm * Fz;
    const double qx = wrap_coord(xi + pc.dt * px, pc.L[0]);
    const double qy = wrap_coord(yi + pc.dt * py, pc.L[1]);
    const double qz = wrap_coord(zi + pc.dt * pz, pc.L[2]);
    out.v.x[i] = vx;
    out.v.y[i] = vy;
    out.v.z[i] = vz;
    out.f.x[i] = Fx;
    out.f.y[i] = Fy;
    out.f.z[i] = Fz;
    out.vpred.x[i] = px;
    out.vpred.y[i] = py;
    out.vpred.z[i] = pz;
    out.xpred.x[i] = qx;
    out.xpred.y[i] = qy;
    out.xpred.z[i] = qz;
    const bool ok = __builtin_isfinite(qx) && __builtin_isfinite(qy) && __builtin_isfinite(qz) &&
                    __builtin_isfinite(px) && __builtin_isfinite(py) && __builtin_isfinite(pz) && qx >= 0.0 &&
                    qx < pc.L[0] && qy >= 0.0 && qy < pc.L[1] && qz >= 0.0 && qz < pc.L[2];
    if (!ok) atomicOr(out.status, 1);
    moved = ok ? moved2(pc, out.xbuild, i, qx, qy, qz) : __builtin_inff();
}

// Fixed-order block sum of the per-lane virial and pair-energy partials, and
// the block maximum of the squared displacements (for the gate).
__device__ __forceinline__ void block_partials(double vir, double ep, float moved, double *part, float *bmax,
                                               int slot)
{
    __shared__ double red_v[kBlock];
    __shared__ double red_e[kBlock];
    __shared__ float red_m[kWavesPerBlock];
    red_v[threadIdx.x] = vir;
    red_e[threadIdx.x] = ep;
    if (bmax) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) moved = fmaxf(moved, __shfl_xor(moved, o, 64));
        if ((threadIdx.x & 63) == 0) red_m[threadIdx.x >> 6] = moved;
    }
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red_v[threadIdx.x] += red_v[threadIdx.x + s];
            red_e[threadIdx.x] += red_e[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * slot] = red_v[0];
        part[2 * slot + 1] = red_e[0];
        if (bmax) {
            float m = red_m[0];
            for (int w = 1; w < kWavesPerBlock; ++w) m = fmaxf(m, red_m[w]);
            bmax[slot] = m;
        }
    }
}

template <int P, bool MT, bool DC, typename R>
__global__ __launch_bounds__(kBlock) void k_force(Reps Rp, const uint32_t *__restrict__ stepp, Soa3c xs, Soa3c vh,
                                                  const R *__restrict__ rho,
                                                  const uint32_t *__restrict__ tag,
                                                  const uint8_t *__restrict__ typ,
                                                  const PartRec *__restrict__ rec,
                                                  const int *__restrict__ ncnt,
                                                  const uint32_t *__restrict__ nl, ForceOut out)
{
    const int blk = xcd_block();
    const BlockRep br = block_rep<P>(Rp, blk);
    const int i = br.i0 + (int)threadIdx.x / P;
    const int sub = threadIdx.x & (P - 1);
    PairConst pc = cload(Rp.pc, br.r);
    set_noise_keys(pc, cload(stepp, 0));
    const Geom g = cload(Rp.geom, br.r);
    // the type-pair planes of the block's replica, staged in LDS
    __shared__ double ptab[MT ? 320 : 1];
    if constexpr (MT) {
        for (int k = (int)threadIdx.x; k < 320; k += kBlock) ptab[k] = pc.tab[k];
        __syncthreads();
    }
    double vir = 0.0, ep = 0.0;
    float moved = 0.0f;
    if (i < br.i1) {
        const int packed = ncnt[i];
        if (list_total(packed) <= kListCap) {
            force_particle<P, MT, DC, false, R>(pc, g, i, sub, xs, vh, rho, tag, typ, nullptr, packed,
                                            nl + (size_t)i * kListCap, rec, out, ptab, vir, ep, moved);
        } else if (sub == 0) {
            out.ovf[atomicAdd(out.ovf_count, 1)] = i;  // served by k_force_overflow (its move too)
        }
    }
    block_partials(vir, ep, moved, out.part, out.bmax, blk);
}

// Particles whose neighbour list overflowed: a fixed grid walks the queue
// that k_force filled, scanning the cells directly.  The queue order depends
// on atomic timing, so each particle's virial and pair-energy share goes to
// its own slot of ovf_ve (summed per particle in a fixed order) and the
// observables reduction adds it back in slot order.
constexpr int kOverflowBlocks = 32;

// The squared move of a queued particle goes into the block maximum of the
// force launch's block that holds its slot (with fl_idx the lane index of
// that launch), by an integer maximum on the float's bits, which orders
// non-negative floats and does not depend on the order of the updates.
template <bool MT, bool DC, typename R>
__global__ __launch_bounds__(kBlock) void k_force_overflow(Reps Rp, const uint32_t *__restrict__ stepp, Soa3c xs,
                                                           Soa3c vh,
                                                           const R *__restrict__ rho,
                                                           const uint32_t *__restrict__ tag,
                                                           const uint8_t *__restrict__ typ,
                                                           const int *__restrict__ cstart_all,
                                                           const int *__restrict__ ncnt, ForceOut out,
                                                           double *__restrict__ ovf_ve, int fl_idx)
{
    constexpr int P = 4;
    const int count = *out.ovf_count;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int groups = gridDim.x * (kBlock / P);
    const int sub = t & (P - 1);
    for (int q = t / P; q < count; q += groups) {
        const int i = out.ovf[q];
        const int r = find_rep(Rp.part_off, Rp.nrep, i);  // per lane: queued particles mix replicas
        PairConst pc = Rp.pc[r];
        set_noise_keys(pc, *stepp);
        const Geom g = Rp.geom[r];
        double vir = 0.0, ep = 0.0;
        float moved = 0.0f;
        force_particle<P, MT, DC, true, R>(pc, g, i, sub, xs, vh, rho, tag, typ, cstart_all + cload(Rp.cell_off, r),
                                       ncnt[i], nullptr, nullptr, out, pc.tab, vir, ep, moved);
        vir = group_sum<P>(vir);
        ep = group_sum<P>(ep);
        if (sub == 0) {
            ovf_ve[2 * (size_t)i] = vir;
            ovf_ve[2 * (size_t)i + 1] = ep;
            const int per = kBlock >> fl_idx;  // particles per block of the force launch
            const int blk = Rp.blk_off[fl_idx * (Rp.nrep + 1) + r] + (i - Rp.part_off[r]) / per;
            if (out.bmax) atomicMax((unsigned int *)&out.bmax[blk], __float_as_uint(moved));
        }
    }
}

// ---------------------------------------------------------------------------
// Pressure tensor per slot (read-out, not part of a step): for fluid i,
// m v_a v_b + sum_j c_ij d_a d_b / r F^C(r), F^C = A w_c + B (rho_i + rho_j)
// w_d, c_ij = 1/2 for fluid j and 1 for frozen j; frozen slots give 0.
// PART = false: out holds six FP64 planes (xx, yy, zz, xy, xz, yz) of n
// entries.  PART = true: out holds six sums per block (block b at 6 b, in
// the fixed order of a tree over the block's particles); every block of the
// launch writes its six values, so nothing needs clearing first.
template <int P, bool MT, typename R, bool PART>
__global__ __launch_bounds__(kBlock) void k_stress(Reps Rp, Soa3c xs, Soa3c v, const R *__restrict__ rho,
                                                   const uint32_t *__restrict__ tag,
                                                   const uint8_t *__restrict__ typ,
                                                   const int *__restrict__ cstart_all,
                                                   const int *__restrict__ ncnt,
                                                   const uint32_t *__restrict__ nl, int n,
                                                   double *__restrict__ out)
{
    const int blk = xcd_block();
    const BlockRep br = block_rep<P>(Rp, blk);
    const int i = br.i0 + (int)threadIdx.x / P;
    const int sub = threadIdx.x & (P - 1);
    const bool live = i < br.i1;
    if (!PART && !live) return;
    const PairConst pc = cload(Rp.pc, br.r);
    const Geom g = cload(Rp.geom, br.r);
    const int *__restrict__ cstart = cstart_all + cload(Rp.cell_off, br.r);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (live && !(tag[i] & kFrozenBit)) {
        const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
        const double rhoi = (double)rho[i];
        const int T = pc.ntypes;
        const int ti = MT ? (int)typ[i] : 0;
        for_each_neighbor<P>(pc, g, i, sub, xi, yi, zi, xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                             [&](int j, double dx, double dy, double dz, bool near) {
            const double r2 = exact_r2(dx, dy, dz);
            if (!(r2 > 0.0)) return;
            const double r = __builtin_sqrt(r2);
            double A = pc.A, B = pc.B;
            if (MT) {
                const int tt = ti * T + (int)typ[j];
                A = pc.tab[tt];
                B = pc.tab[64 + tt];
            }
            double fc = A * (1.0 - r * pc.inv_rc);
            if (near) fc += B * (rhoi + (double)rho[j]) * (1.0 - r * pc.inv_rd);
            const double k = ((tag[j] & kFrozenBit) ? 1.0 : 0.5) * fc / r;
            acc[0] += k * dx * dx;
            acc[1] += k * dy * dy;
            acc[2] += k * dz * dz;
            acc[3] += k * dx * dy;
            acc[4] += k * dx * dz;
            acc[5] += k * dy * dz;
        });
        if (sub == 0) {
            const double m = pc.mass;
            const double vx = v.x[i], vy = v.y[i], vz = v.z[i];
            acc[0] += m * vx * vx;
            acc[1] += m * vy * vy;
            acc[2] += m * vz * vz;
            acc[3] += m * vx * vy;
            acc[4] += m * vx * vz;
            acc[5] += m * vy * vz;
        }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) acc[a] = group_sum<P>(acc[a]);
    if constexpr (!PART) {
        if (sub == 0)
#pragma unroll
            for (int a = 0; a < 6; ++a) out[(size_t)a * n + i] = acc[a];
    } else {
        // one value per particle (lane sub = 0 of its group), then a tree
        __shared__ double sh[6][kBlock];
#pragma unroll
        for (int a = 0; a < 6; ++a) sh[a][threadIdx.x] = sub == 0 ? acc[a] : 0.0;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
#pragma unroll
                for (int a = 0; a < 6; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0)
#pragma unroll
            for (int a = 0; a < 6; ++a) out[6 * (size_t)blk + a] = sh[a][0];
    }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_debug_neighbors(Reps R, double cut2,
                                                            Soa3c xs, const uint32_t *__restrict__ tag,
                                                            const int *__restrict__ cstart_all,
                                                            const int *__restrict__ ncnt,
                                                            const uint32_t *__restrict__ nl,
                                                            int64_t *__restrict__ count,
                                                            uint64_t *__restrict__ hash)
{
    const BlockRep br = block_rep<1>(R, blockIdx.x);
    const int i = br.i0 + (int)threadIdx.x;
    if (i >= br.i1) return;
    const PairConst pc = cload(R.pc, br.r);
    const Geom g = cload(R.geom, br.r);
    const int *__restrict__ cstart = cstart_all + cload(R.cell_off, br.r);
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    int64_t c = 0;
    uint64_t h = 0;
    for_each_neighbor<1>(pc, g, i, 0, xi, yi, zi, xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                         [&](int j, double dx, double dy, double dz, bool) {
                             if (exact_r2(dx, dy, dz) < cut2) {
                                 ++c;
                                 h += mix64((uint64_t)(tag[j] & kIdMask));
                             }
                         });
    const size_t out = (size_t)cload(R.part_off, br.r) + (tag[i] & kIdMask);  // input order
    count[out] = c;
    hash[out] = h;
}

}  // namespace

int force_partials(const Reps &R, int lanes) { return R.nblk[lanes_index(lanes)]; }

void launch_nlist(hipStream_t st, bool fp32, const Reps &R, Soa3c xs, const int *cstart, int *ncnt,
                  uint32_t *nl, void *nlr2, bool all)
{
    if (R.ncells <= 0) return;
    const int blocks = (R.nicells + kWavesPerBlock - 1) / kWavesPerBlock;
    const int bblocks = (R.nbcells * R.list_split + kWavesPerBlock - 1) / kWavesPerBlock;
    if (fp32) {
        if (R.list_interior && blocks > 0)
            k_nlist_cell<float><<<blocks, kBlock, 0, st>>>(R, xs, cstart, ncnt, nl, (float *)nlr2, all ? 1 : 0);
        if (bblocks > 0)
            k_nlist_border<float><<<bblocks, kBlock, 0, st>>>(R, xs, cstart, ncnt, nl, (float *)nlr2, all ? 1 : 0);
    } else {
        if (R.list_interior && blocks > 0)
            k_nlist_cell<double><<<blocks, kBlock, 0, st>>>(R, xs, cstart, ncnt, nl, (double *)nlr2, all ? 1 : 0);
        if (bblocks > 0)
            k_nlist_border<double><<<bblocks, kBlock, 0, st>>>(R, xs, cstart, ncnt, nl, (double *)nlr2, all ? 1 : 0);
    }
}

void launch_density_list(hipStream_t st, int lanes, bool fp32, const Reps &R, Soa3c xs, Soa3c vh, const uint32_t *tag,
                    const uint8_t *typ, const int *cstart, const int *ncnt, const void *nlr2, void *rho,
                    PartRec *rec)
{
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        const int nb = R.nblk[lanes_index(L)];
        if (nb <= 0) return;
        if (fp32)
            k_density_list<L, float><<<nb, kBlock, 0, st>>>(R, xs, vh, tag, typ, cstart, ncnt, (const float *)nlr2,
                                                       (float *)rho, rec);
        else
            k_density_list<L, double><<<nb, kBlock, 0, st>>>(R, xs, vh, tag, typ, cstart, ncnt, (const double *)nlr2,
                                                        (double *)rho, rec);
    });
}

void launch_skin_build(hipStream_t st, const Reps &R, bool all, Soa3c xs, const int *cstart, int *scnt,
                       uint32_t *sl)
{
    if (R.ncells <= 0) return;
    const int blocks = (R.ncells + kWavesPerBlock - 1) / kWavesPerBlock;
    if (all)
        k_skin_build<true><<<blocks, kBlock, 0, st>>>(R, xs, cstart, scnt, sl);
    else
        k_skin_build<false><<<blocks, kBlock, 0, st>>>(R, xs, cstart, scnt, sl);
}

void launch_density(hipStream_t st, int lanes, bool fp32, const Reps &R, Soa3c xs, Soa3c vh, const uint32_t *tag,
                    const uint8_t *typ, const int *cstart, const int *scnt, const uint32_t *sl, int *ncnt,
                    uint32_t *nl, void *rho, PartRec *rec)
{
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        const int nb = R.nblk[lanes_index(L)];
        if (nb <= 0) return;
        if (fp32)
            k_density_skin<L, float><<<nb, kBlock, 0, st>>>(R, xs, vh, tag, typ, cstart, scnt, sl, ncnt, nl,
                                                            (float *)rho, rec);
        else
            k_density_skin<L, double><<<nb, kBlock, 0, st>>>(R, xs, vh, tag, typ, cstart, scnt, sl, ncnt, nl,
                                                             (double *)rho, rec);
    });
}

void launch_mark_wall_cells(hipStream_t st, const Reps &R, Soa3c xs, const uint32_t *tag, uint8_t *wmask)
{
    if (R.nblk[0] > 0) k_mark_wall_cells<<<R.nblk[0], kBlock, 0, st>>>(R, xs, tag, wmask);
}

void launch_phi(hipStream_t st, int lanes, bool slip, int n, const Reps &R, Soa3c xs, Soa3c xprev, Soa3 xfix,
                Soa3 vfix, uint32_t *tag, const int *cstart, const uint8_t *wmask, int *flag_and_count,
                unsigned long long *ncorr_total, uint8_t *byid, Soa3c xbuild, float *cmax)
{
    if (n <= 0) return;
    int *ncorr = flag_and_count;       // [0]: corrections this step
    int *flag = flag_and_count + 1;    // [1..n]: per-slot flags
    int *part = flag + n;              // [n+1 ..]: corrections per block of k_correct
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        if (R.nblk[0] <= 0) return;
        if (slip)
            k_phi<L, true><<<R.nblk[0], kBlock, 0, st>>>(R, xs, tag, cstart, wmask, flag, vfix);
        else
            k_phi<L, false><<<R.nblk[0], kBlock, 0, st>>>(R, xs, tag, cstart, wmask, flag, vfix);
    });
    const int nb = R.nblk[0];
    k_correct<<<nb, kBlock, 0, st>>>(R, flag, xprev, xfix, vfix, part, tag, byid, xbuild, cmax);
    k_correct_sum<<<1, kBlock, 0, st>>>(nb, part, ncorr, ncorr_total);
}

void launch_force(hipStream_t st, int lanes, bool fp32, bool mt, bool dc, const Reps &R, const uint32_t *stepp,
                  Soa3c xs, Soa3c vh, const void *rho, const uint32_t *tag, const uint8_t *typ, const PartRec *rec,
                  const int *cstart,
                  const int *ncnt, const uint32_t *nl, Soa3 vout, Soa3 fout, Soa3 vpred, Soa3 xpred,
                  double *part, int *status, int *ovf_count, int *ovf, double *ovf_ve, int initial, Soa3c xbuild,
                  float *bmax)
{
    const ForceOut out{vout, fout, vpred, xpred, part, status, ovf_count, ovf, initial, xbuild, bmax};
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        const int nb = R.nblk[lanes_index(L)];
        if (nb <= 0) return;
        auto go = [&](auto mtc, auto dcc, auto rc) {
            constexpr bool M = decltype(mtc)::value;
            constexpr bool D = decltype(dcc)::value;
            using RT = typename decltype(rc)::type;
            k_force<L, M, D, RT><<<nb, kBlock, 0, st>>>(R, stepp, xs, vh, (const RT *)rho, tag, typ, rec, ncnt,
                                                        nl, out);
            k_force_overflow<M, D, RT><<<kOverflowBlocks, kBlock, 0, st>>>(R, stepp, xs, vh, (const RT *)rho,
                                                                           tag, typ, cstart, ncnt, out, ovf_ve,
                                                                           lanes_index(L));
        };
        using T = std::true_type;
        using F = std::false_type;
        // the control takes the type-table path (its tables hold every
        // replica's values, one type included)
        if (fp32) {
            if (dc) go(T{}, T{}, Tid<float>{});
            else if (mt) go(T{}, F{}, Tid<float>{});
            else go(F{}, F{}, Tid<float>{});
        } else {
            if (dc) go(T{}, T{}, Tid<double>{});
            else if (mt) go(T{}, F{}, Tid<double>{});
            else go(F{}, F{}, Tid<double>{});
        }
    });
}

void launch_stress(hipStream_t st, bool fp32, bool mt, int n, const Reps &R, Soa3c xs, Soa3c v, const void *rho,
                   const uint32_t *tag, const uint8_t *typ, const int *cstart, const int *ncnt, const uint32_t *nl,
                   double *out, bool per_block)
{
    const int nb = R.nblk[lanes_index(kStressLanes)];
    if (nb <= 0) return;
    auto go = [&](auto mtc, auto rc) {
        constexpr bool M = decltype(mtc)::value;
        using RT = typename decltype(rc)::type;
        if (per_block)
            k_stress<kStressLanes, M, RT, true><<<nb, kBlock, 0, st>>>(R, xs, v, (const RT *)rho, tag, typ, cstart,
                                                                       ncnt, nl, n, out);
        else
            k_stress<kStressLanes, M, RT, false><<<nb, kBlock, 0, st>>>(R, xs, v, (const RT *)rho, tag, typ,
                                                                        cstart, ncnt, nl, n, out);
    };
    if (fp32) {
        if (mt) go(std::true_type{}, Tid<float>{});
        else go(std::false_type{}, Tid<float>{});
    } else {
        if (mt) go(std::true_type{}, Tid<double>{});
        else go(std::false_type{}, Tid<double>{});
    }
}

void launch_debug_neighbors(hipStream_t st, const Reps &R, double cut2, Soa3c xs, const uint32_t *tag,
                            const int *cstart, const int *ncnt, const uint32_t *nl, int64_t *count,
                            uint64_t *hash)
{
    const int nb = R.nblk[0];
    if (nb <= 0) return;
    k_debug_neighbors<<<nb, kBlock, 0, st>>>(R, cut2, xs, tag, cstart, ncnt, nl, count, hash);
}

}  // namespace mdpd
