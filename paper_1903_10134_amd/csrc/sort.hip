// sort.hip -- the list gate, cell binning and the deterministic stable
// reorder into SoA.
//
// Every step the gate decides, per replica, whether its particles have moved
// far enough since the last list build (half the skin) to need new cells and
// a new skin list.  The replicas that do are re-binned into cells of edge
// >= r_c + skin and all their per-particle arrays rewritten in (cell,
// particle id) order:
//   k_gate         per-replica rebuild flags from the force pass's block
//                  maxima of the displacement; advances the noise step
//   k_bin          cell key per particle and its arrival slot in the cell
//                  (integer atomics: the counts are exact, the slots are not
//                  ordered)
//   k_scan_*       exclusive scan of the cell counts -> new cell offsets in
//                  two passes: tiles, then tile offsets (the counts are
//                  cleared as they are read); a rebuilt replica's offsets
//                  replace its cell_start
//   k_scatter_id   writes each particle's id at its arrival slot
//   k_rank_gather  rank of the particle inside its cell = number of particles
//                  of that cell with a smaller id; moves every array of a
//                  rebuilt replica to cell_start + rank in temporaries
//   k_copy_back    the temporaries back in place, and the build positions.
//   k_sort_small   the every-step sort of replicas small enough for one
//                  workgroup each: binning, scan, id lists and ranks in LDS
//                  (one launch instead of five, the same order).
// The result depends only on positions and ids, not on the previous order or
// the atomics' arrival order, so runs and restarts are bitwise reproducible,
// and a replica's schedule of builds depends on its own particles only.
#include "mdpd_internal.h"

namespace mdpd {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kWaves = kBlock / 64;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

inline int blocks_for(int64_t threads) { return (int)((threads + kBlock - 1) / kBlock); }

// Cell key and arrival slot.  Particles arrive almost in cell order (they
// were sorted at the last build), so lanes whose key equals the previous
// lane's form runs; the first lane of a run reserves the whole run with one
// atomic and the others take consecutive slots after it.
// Blocks are replica-aligned (kBlock particles of one replica), and the key
// is the global cell: the replica's first cell plus its local cell.  When any
// replica rebuilds, every particle is binned (the scan needs all counts).
__global__ __launch_bounds__(kBlock) void k_bin(Reps R, Soa3c x, int *__restrict__ key,
                                                int *__restrict__ slot, int *__restrict__ counts, int all,
                                                uint32_t *__restrict__ step_ctr, int *__restrict__ ovf_count,
                                                unsigned long long *__restrict__ nbuild)
{
    if (!all && cload(R.flag, R.nrep) == 0) return;
    if (step_ctr && blockIdx.x == 0 && threadIdx.x == 0) {
        // the step's bookkeeping when no gate runs (every replica rebuilds)
        *step_ctr += 1;
        *ovf_count = 0;
        *nbuild += (unsigned long long)R.nrep;
    }
    const int *boff = R.blk_off;  // lane count 1
    const int r = block_replica(R, 0, boff, blockIdx.x);
    const int i = cload(R.part_off, r) + (blockIdx.x - cload(boff, r)) * kBlock + threadIdx.x;
    const int n = cload(R.part_off, r + 1);  // end of this replica's slots
    const Geom g = cload(R.geom, r);
    const int lane = threadIdx.x & 63;
    int c = -1;
    if (i < n) {
        const int cx = cell_coord(x.x[i], g.s[0], g.nc[0]);
        const int cy = cell_coord(x.y[i], g.s[1], g.nc[1]);
        const int cz = cell_coord(x.z[i], g.s[2], g.nc[2]);
        c = cload(R.cell_off, r) + cx + g.nc[0] * (cy + g.nc[1] * cz);
        key[i] = c;
    }
    const int prev = __shfl_up(c, 1, 64);
    const bool head = i < n && (lane == 0 || prev != c);
    const unsigned long long heads = __ballot(head);
    // first lane of my run, and the first lane of the next run (or 64)
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int first = 63 - __clzll(heads & upto);
    const unsigned long long after = heads & ~upto;
    const int next = after ? __ffsll((long long)after) - 1 : 64;
    int base = 0;
    if (head) {
        int len = next - lane;
        const int last_valid = n - 1 - (i - lane);  // lanes beyond n are not in any run
        if (lane + len - 1 > last_valid) len = last_valid - lane + 1;
        base = atomicAdd(&counts[c], len);
    }
    base = __shfl(base, first, 64);
    if (i < n) slot[i] = base + (lane - first);
}

// Inclusive scan across one block of kScanThreads threads; returns the
// inclusive prefix of v and the block total in *total.
__device__ __forceinline__ int block_inclusive_scan(int v, int *sh, int *total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) sh[wave] = v;
    __syncthreads();
    if (wave == 0) {
        constexpr int nw = kScanThreads / 64;
        int w = lane < nw ? sh[lane] : 0;
#pragma unroll
        for (int o = 1; o < nw; o <<= 1) {
            const int u = __shfl_up(w, o, 64);
            if (lane >= o) w += u;
        }
        if (lane < nw) sh[lane] = w;
    }
    __syncthreads();
    if (wave > 0) v += sh[wave - 1];
    *total = sh[kScanThreads / 64 - 1];
    return v;
}

// Local exclusive scan of tile b of counts into out; clears counts.  With a
// single tile (cstart set) the scan is complete here: the offsets also go to
// cstart (of rebuilt replicas) and the total to out[m] and cstart[m], as
// k_scan_add would write them.
__global__ __launch_bounds__(kScanThreads) void k_scan_local(Reps R, int m, int *__restrict__ counts,
                                                             int *__restrict__ out,
                                                             int *__restrict__ bsum, int all,
                                                             int *__restrict__ cstart)
{
    if (!all && cload(R.flag, R.nrep) == 0) return;
    __shared__ int sh[kScanThreads / 64];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int v[kScanPer];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int idx = base + k;
        v[k] = idx < m ? counts[idx] : 0;
        if (idx < m) counts[idx] = 0;
        s += v[k];
    }
    int total;
    const int incl = block_inclusive_scan(s, sh, &total);
    int run = incl - s;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int idx = base + k;
        if (idx < m) {
            out[idx] = run;
            if (cstart && (all || cload(R.flag, R.cell_rep ? R.cell_rep[idx] : 0))) cstart[idx] = run;
        }
        run += v[k];
    }
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = total;
        if (cstart) out[m] = cstart[m] = total;
    }
}

// Adds to tile b of out the sum of the totals of tiles 0 .. b-1 (the first
// wavefront sums them; integer sums do not depend on the order); the last
// tile also writes the grand total to out[m].  The offsets of the cells of
// rebuilt replicas also go to cstart.
__global__ __launch_bounds__(kScanThreads) void k_scan_add(Reps R, int m, int nb, const int *__restrict__ bsum,
                                                           int *__restrict__ out, int *__restrict__ cstart, int all)
{
    if (!all && cload(R.flag, R.nrep) == 0) return;
    __shared__ int sh;
    if (threadIdx.x < 64) {
        int v = 0;
        for (int k = (int)threadIdx.x; k < (int)blockIdx.x; k += 64) v += bsum[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (threadIdx.x == 0) {
            sh = v;
            if ((int)blockIdx.x == nb - 1) out[m] = cstart[m] = v + bsum[nb - 1];
        }
    }
    __syncthreads();
    const int add = sh;
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int c = base + k;
        if (c < m) {
            const int v = out[c] + add;
            out[c] = v;
            if (all || cload(R.flag, R.cell_rep ? R.cell_rep[c] : 0)) cstart[c] = v;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter_id(Reps R, int n, const int *__restrict__ key,
                                                       const int *__restrict__ slot,
                                                       const int *__restrict__ cnew,
                                                       const uint32_t *__restrict__ tag,
                                                       uint32_t *__restrict__ tmpid, int all)
{
    if (!all && cload(R.flag, R.nrep) == 0) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    tmpid[cnew[key[i]] + slot[i]] = tag[i] & kIdMask;
}

// Particles of rebuilt replicas: new slot = cell start + rank, every array
// written there in the temporaries.  dmap (nullable) records the move (the
// identity for replicas not rebuilt).
__global__ __launch_bounds__(kBlock) void k_rank_gather(Reps R, const int *__restrict__ key,
                                                        const int *__restrict__ cnew,
                                                        const uint32_t *__restrict__ tmpid, Soa3c xin,
                                                        Soa3c vin, Soa3c pin,
                                                        const uint32_t *__restrict__ tag_in,
                                                        const uint8_t *__restrict__ typ_in, Soa3 xout,
                                                        Soa3 vout, Soa3 pout,
                                                        uint32_t *__restrict__ tag_out,
                                                        uint8_t *__restrict__ typ_out, int *__restrict__ dmap,
                                                        int all)
{
    const int *boff = R.blk_off;  // lane count 1
    const int r = block_replica(R, 0, boff, blockIdx.x);
    const int i = cload(R.part_off, r) + (blockIdx.x - cload(boff, r)) * kBlock + threadIdx.x;
    if (i >= cload(R.part_off, r + 1)) return;
    if (!all && cload(R.flag, r) == 0) {
        if (dmap) dmap[i] = i;
        return;
    }
    const uint32_t tg = tag_in[i];
    const int c = key[i];
    const int b = cnew[c], e = cnew[c + 1];
    const uint32_t id = tg & kIdMask;
    int rank = 0;
    for (int k = b; k < e; ++k) rank += tmpid[k] < id ? 1 : 0;
    const int dst = b + rank;
    if (dmap) dmap[i] = dst;
    xout.x[dst] = xin.x[i];
    xout.y[dst] = xin.y[i];
    xout.z[dst] = xin.z[i];
    vout.x[dst] = vin.x[i];
    vout.y[dst] = vin.y[i];
    vout.z[dst] = vin.z[i];
    if (pin.x) {
        pout.x[dst] = pin.x[i];
        pout.y[dst] = pin.y[i];
        pout.z[dst] = pin.z[i];
    }
    tag_out[dst] = tg;
    typ_out[dst] = typ_in[i];
}

// Every-step sort of small replicas: one workgroup of kScanThreads threads
// per replica bins its particles into cells (LDS counts), scans them, lists
// the ids of every cell in arrival order and ranks each particle inside its
// cell, all in LDS with workgroup barriers, and moves the arrays to
// part_off[r] + cell offset + rank -- the (cell, id) order of the multi-pass
// sort, which it replaces in one launch.  Dynamic LDS: the replica's cell
// offsets (cells + 1) then its ids (n_r); a thread keeps the keys and arrival
// slots of its (at most kSmallPer) particles in registers.
constexpr int kSmallPer = kSortSmallMaxN / kScanThreads;
static_assert(kSmallPer * kScanThreads == kSortSmallMaxN, "particles per thread of the one-workgroup sort");
static_assert(kScanPer * kScanThreads >= kSortSmallMaxCells, "the scan takes up to kScanPer cells per thread");

__global__ __launch_bounds__(kScanThreads) void k_sort_small(Reps R, Soa3c xin, Soa3c vin, Soa3c pin,
                                                            const uint32_t *__restrict__ tag_in,
                                                            const uint8_t *__restrict__ typ_in, Soa3 xout,
                                                            Soa3 vout, Soa3 pout, uint32_t *__restrict__ tag_out,
                                                            uint8_t *__restrict__ typ_out, int *__restrict__ cstart,
                                                            int *__restrict__ cnew, int *__restrict__ dmap,
                                                            uint32_t *__restrict__ step_ctr,
                                                            int *__restrict__ ovf_count,
                                                            unsigned long long *__restrict__ nbuild)
{
    extern __shared__ int lds[];
    __shared__ int sh[kScanThreads / 64];
    const int r = blockIdx.x;
    const int p0 = cload(R.part_off, r), p1 = cload(R.part_off, r + 1);
    const int c0 = cload(R.cell_off, r), m = cload(R.cell_off, r + 1) - c0;
    const Geom g = cload(R.geom, r);
    int *const off = lds;          // [m + 1]: counts, then offsets
    int *const ids = lds + m + 1;  // [p1 - p0]
    const int t = (int)threadIdx.x;
    if (step_ctr && r == 0 && t == 0) {
        // the step's bookkeeping when no gate runs (every replica rebuilds)
        *step_ctr += 1;
        *ovf_count = 0;
        *nbuild += (unsigned long long)R.nrep;
    }
    for (int c = t; c <= m; c += kScanThreads) off[c] = 0;
    __syncthreads();
    int key[kSmallPer], slot[kSmallPer];
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
        const int i = p0 + t + k * kScanThreads;
        key[k] = 0;
        slot[k] = 0;
        if (i < p1) {
            const int cx = cell_coord(xin.x[i], g.s[0], g.nc[0]);
            const int cy = cell_coord(xin.y[i], g.s[1], g.nc[1]);
            const int cz = cell_coord(xin.z[i], g.s[2], g.nc[2]);
            key[k] = cx + g.nc[0] * (cy + g.nc[1] * cz);
            slot[k] = atomicAdd(&off[key[k]], 1);
        }
    }
    __syncthreads();
    // exclusive scan of the counts: kScanPer consecutive cells per thread
    int v[kScanPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int c = t * kScanPer + k;
        v[k] = c < m ? off[c] : 0;
        sum += v[k];
    }
    int total;
    int run = block_inclusive_scan(sum, sh, &total) - sum;  // its barriers also end the reads above
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int c = t * kScanPer + k;
        if (c < m) {
            off[c] = run;
            cstart[c0 + c] = cnew[c0 + c] = p0 + run;
        }
        run += v[k];
    }
    if (t == 0) {
        off[m] = total;
        if (r == R.nrep - 1) cstart[c0 + m] = cnew[c0 + m] = p0 + total;  // the grand total
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
        const int i = p0 + t + k * kScanThreads;
        if (i < p1) ids[off[key[k]] + slot[k]] = (int)(tag_in[i] & kIdMask);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSmallPer; ++k) {
        const int i = p0 + t + k * kScanThreads;
        if (i >= p1) continue;
        const uint32_t tg = tag_in[i];
        const int id = (int)(tg & kIdMask);
        const int b = off[key[k]], e = off[key[k] + 1];
        int rank = 0;
        for (int q = b; q < e; ++q) rank += ids[q] < id ? 1 : 0;
        const int dst = p0 + b + rank;
        if (dmap) dmap[i] = dst;
        xout.x[dst] = xin.x[i];
        xout.y[dst] = xin.y[i];
        xout.z[dst] = xin.z[i];
        vout.x[dst] = vin.x[i];
        vout.y[dst] = vin.y[i];
        vout.z[dst] = vin.z[i];
        if (pin.x) {
            pout.x[dst] = pin.x[i];
            pout.y[dst] = pin.y[i];
            pout.z[dst] = pin.z[i];
        }
        tag_out[dst] = tg;
        typ_out[dst] = typ_in[i];
    }
}

// The sorted temporaries of rebuilt replicas back in place; the positions
// also become the build positions (xb, unless NULL).
__global__ __launch_bounds__(kBlock) void k_copy_back(Reps R, Soa3c tx, Soa3c tv, Soa3c tp,
                                                      const uint32_t *__restrict__ ttag,
                                                      const uint8_t *__restrict__ ttyp, Soa3 x, Soa3 v,
                                                      Soa3 p, uint32_t *__restrict__ tag,
                                                      uint8_t *__restrict__ typ, Soa3 xb)
{
    const int *boff = R.blk_off;  // lane count 1
    const int r = block_replica(R, 0, boff, blockIdx.x);
    if (cload(R.flag, r) == 0) return;
    const int i = cload(R.part_off, r) + (blockIdx.x - cload(boff, r)) * kBlock + threadIdx.x;
    if (i >= cload(R.part_off, r + 1)) return;
    const double px = tx.x[i], py = tx.y[i], pz = tx.z[i];
    x.x[i] = px;
    x.y[i] = py;
    x.z[i] = pz;
    if (xb.x) {
        xb.x[i] = px;
        xb.y[i] = py;
        xb.z[i] = pz;
    }
    v.x[i] = tv.x[i];
    v.y[i] = tv.y[i];
    v.z[i] = tv.z[i];
    if (tp.x) {
        p.x[i] = tp.x[i];
        p.y[i] = tp.y[i];
        p.z[i] = tp.z[i];
    }
    tag[i] = ttag[i];
    typ[i] = ttyp[i];
}

// The gate: one block per replica takes the maximum of its force blocks'
// maxima; the last block to finish (a counter, reset by that block) forms
// the OR of the flags and does the once-per-step bookkeeping.
__global__ __launch_bounds__(kBlock) void k_gate(Reps R, int lane_idx, const float *__restrict__ bmax,
                                                 int *__restrict__ force, int *__restrict__ flags,
                                                 int *__restrict__ done, uint32_t *__restrict__ step_ctr,
                                                 int *__restrict__ ovf_count, unsigned long long *__restrict__ nbuild,
                                                 int first)
{
    __shared__ float red[kWaves];
    __shared__ int last;
    const int r = blockIdx.x;
    const int *off = R.blk_off + lane_idx * (R.nrep + 1);
    float m = 0.0f;
    for (int k = cload(off, r) + (int)threadIdx.x; k < cload(off, r + 1); k += kBlock) m = fmaxf(m, bmax[k]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) m = fmaxf(m, red[w]);
        const Geom g = cload(R.geom, r);
        // the second gate of a step rebuilds only for a particle that was
        // moved back at all (with skin 0 the threshold is 0)
        const bool far = (double)m >= g.gate2 && (first || m > 0.0f);
        const int f = (__hip_atomic_load(force, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || far) ? 1 : 0;
        __hip_atomic_store(&flags[r], f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        last = atomicAdd(done, 1) == R.nrep - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    int any = 0;
    for (int q = (int)threadIdx.x; q < R.nrep; q += kBlock)
        any += __hip_atomic_load(&flags[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) any += __shfl_xor(any, o, 64);
    __shared__ int tot[kWaves];
    if ((threadIdx.x & 63) == 0) tot[threadIdx.x >> 6] = any;
    __syncthreads();
    if (threadIdx.x == 0) {
        int sum = 0;
        for (int w = 0; w < kWaves; ++w) sum += tot[w];
        flags[R.nrep] = sum > 0 ? 1 : 0;
        *nbuild += (unsigned long long)sum;
        *force = 0;
        *done = 0;
        if (first) {
            *step_ctr += 1;  // noise step of this step's force pass
            *ovf_count = 0;  // the force pass of this step refills it
        }
    }
}

// Input arrays (AoS n x 3, caller order: replica after replica) to SoA
// predicted state; validates against the replica's box and type count.  The
// id of a particle is its index inside its replica.
__global__ __launch_bounds__(kBlock) void k_ingest(Reps R, const double *__restrict__ pos,
                                                   const double *__restrict__ vel,
                                                   const int32_t *__restrict__ type,
                                                   const uint8_t *__restrict__ frozen, Soa3 xp, Soa3 vp,
                                                   uint32_t *__restrict__ tag,
                                                   uint8_t *__restrict__ typ, int *__restrict__ status)
{
    const int *boff = R.blk_off;  // lane count 1
    const int r = block_replica(R, 0, boff, blockIdx.x);
    const int i = cload(R.part_off, r) + (blockIdx.x - cload(boff, r)) * kBlock + threadIdx.x;
    if (i >= cload(R.part_off, r + 1)) return;
    const Geom g = cload(R.geom, r);
    const int ntypes = cload(R.pc, r).ntypes;
    const bool fz = frozen[i] != 0;
    double q[3], w[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
        double x = pos[3 * (size_t)i + a];
        const double L = g.L[a];
        ok = ok && __builtin_isfinite(x) && x >= -L && x < 2.0 * L;
        if (x < 0.0) x += L;
        if (x >= L) x -= L;
        q[a] = x;
        const double v = vel[3 * (size_t)i + a];
        ok = ok && __builtin_isfinite(v);
        w[a] = fz ? 0.0 : v;
    }
    const int t = type[i];
    ok = ok && t >= 0 && t < ntypes;
    if (!ok) atomicOr(status, 2);
    xp.x[i] = q[0];
    xp.y[i] = q[1];
    xp.z[i] = q[2];
    vp.x[i] = w[0];
    vp.y[i] = w[1];
    vp.z[i] = w[2];
    tag[i] = (uint32_t)(i - cload(R.part_off, r)) | (fz ? kFrozenBit : 0u);
    typ[i] = (uint8_t)(t >= 0 && t < ntypes ? t : 0);
}

__global__ void k_zero_int(int *p, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

}  // namespace

void launch_zero_int(hipStream_t st, int *p, int n)
{
    if (n > 0) k_zero_int<<<blocks_for(n), kBlock, 0, st>>>(p, n);
}

void launch_set_int(hipStream_t st, int *p, int v) { k_set_int<<<1, 1, 0, st>>>(p, v); }

void launch_ingest(hipStream_t st, const Reps &R, const double *pos, const double *vel, const int32_t *type,
                   const uint8_t *frozen, Soa3 xp, Soa3 vp, uint32_t *tag, uint8_t *typ, int *status)
{
    if (R.nblk[0] <= 0) return;
    k_ingest<<<R.nblk[0], kBlock, 0, st>>>(R, pos, vel, type, frozen, xp, vp, tag, typ, status);
}

void launch_gate(hipStream_t st, const Reps &R, int lanes, const float *bmax, int *force, int *flags, int *done,
                 uint32_t *step_ctr, int *ovf_count, unsigned long long *nbuild, bool first)
{
    k_gate<<<R.nrep, kBlock, 0, st>>>(R, lanes_index(lanes), bmax, force, flags, done, step_ctr, ovf_count, nbuild,
                                      first ? 1 : 0);
}

__global__ __launch_bounds__(kBlock) void k_compose(int n, const int *__restrict__ a, const int *__restrict__ b,
                                                    int *__restrict__ out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = b[a[i]];
}

void launch_compose(hipStream_t st, int n, const int *a, const int *b, int *out)
{
    if (n > 0) k_compose<<<blocks_for(n), kBlock, 0, st>>>(n, a, b, out);
}

void launch_rebuild_sort(hipStream_t st, int n, const Reps &R, Soa3 x, Soa3 v, Soa3 xprev, uint32_t *tag,
                         uint8_t *typ, Soa3 tx, Soa3 tv, Soa3 tp, uint32_t *ttag, uint8_t *ttyp, Soa3 xbuild,
                         int *key, int *slot, uint32_t *tmpid, int *counts, int *cnew, int *cstart, int *bsum,
                         int *dmap, bool copy_back, uint32_t *step_ctr, int *ovf_count,
                         unsigned long long *nbuild)
{
    const int m = R.ncells;
    const int nb = (m + kScanTile - 1) / kScanTile;
    const int all = copy_back ? 0 : 1;
    if (!copy_back && R.sort_small_lds > 0) {
        k_sort_small<<<R.nrep, kScanThreads, R.sort_small_lds, st>>>(
            R, cview(x), cview(v), xprev.x ? cview(xprev) : Soa3c{nullptr, nullptr, nullptr}, tag, typ, tx, tv, tp,
            ttag, ttyp, cstart, cnew, dmap, n > 0 ? step_ctr : nullptr, ovf_count, nbuild);
        return;
    }
    if (n > 0) k_bin<<<R.nblk[0], kBlock, 0, st>>>(R, cview(x), key, slot, counts, all, step_ctr, ovf_count, nbuild);
    // one tile: the local scan is the whole scan
    k_scan_local<<<nb, kScanThreads, 0, st>>>(R, m, counts, cnew, bsum, all, nb == 1 ? cstart : nullptr);
    if (nb > 1) k_scan_add<<<nb, kScanThreads, 0, st>>>(R, m, nb, bsum, cnew, cstart, all);
    if (n > 0) {
        const Soa3c none{nullptr, nullptr, nullptr};
        k_scatter_id<<<blocks_for(n), kBlock, 0, st>>>(R, n, key, slot, cnew, tag, tmpid, all);
        k_rank_gather<<<R.nblk[0], kBlock, 0, st>>>(R, key, cnew, tmpid, cview(x), cview(v),
                                                    xprev.x ? cview(xprev) : none, tag, typ, tx, tv, tp, ttag,
                                                    ttyp, dmap, all);
        if (copy_back)
            k_copy_back<<<R.nblk[0], kBlock, 0, st>>>(R, cview(tx), cview(tv), xprev.x ? cview(tp) : none, ttag,
                                                      ttyp, x, v, xprev, tag, typ, xbuild);
    }
}

}  // namespace mdpd
