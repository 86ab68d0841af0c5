// sort.hip -- cell binning and the deterministic stable reorder into SoA.
//
// Every step the predicted positions are binned into cells of edge >= r_c and
// all per-particle arrays are rewritten in (cell, particle id) order:
//   k_bin          cell key per particle and its arrival slot in the cell
//                  (integer atomics: the counts are exact, the slots are not
//                  ordered)
//   k_scan_*       exclusive scan of the cell counts -> cell_start[ncells + 1]
//                  in two passes: tiles, then tile offsets (the counts are
//                  cleared as they are read)
//   k_scatter_id   writes each particle's id at its arrival slot
//   k_rank_gather  rank of the particle inside its cell = number of particles
//                  of that cell with a smaller id; moves every array to
//                  cell_start + rank.
// The result depends only on positions and ids, not on the previous order or
// the atomics' arrival order, so runs and restarts are bitwise reproducible.
#include "mdpd_internal.h"

namespace mdpd {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

inline int blocks_for(int64_t threads) { return (int)((threads + kBlock - 1) / kBlock); }

// Cell key and arrival slot.  Particles arrive almost in cell order (they
// were sorted one step ago), so lanes whose key equals the previous lane's
// form runs; the first lane of a run reserves the whole run with one atomic
// and the others take consecutive slots after it.
// Blocks are replica-aligned (kBlock particles of one replica), and the key
// is the global cell: the replica's first cell plus its local cell.
__global__ __launch_bounds__(kBlock) void k_bin(Reps R, Soa3c x, int *__restrict__ key,
                                                int *__restrict__ slot, int *__restrict__ counts,
                                                const int *__restrict__ gate, int *__restrict__ ovf_count,
                                                uint32_t *__restrict__ step_ctr)
{
    if (gate && *gate == 0) return;
    const int *boff = R.blk_off;  // lane count 1
    const int r = __builtin_amdgcn_readfirstlane(find_rep(boff, R.nrep, blockIdx.x));
    const int i = cload(R.part_off, r) + (blockIdx.x - cload(boff, r)) * kBlock + threadIdx.x;
    const int n = cload(R.part_off, r + 1);  // end of this replica's slots
    if (ovf_count && i == 0) {
        *ovf_count = 0;  // the force pass of this step refills it
        *step_ctr += 1;  // noise step of this step's force pass
    }
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

// Local exclusive scan of tile b of counts into out; clears counts.
__global__ __launch_bounds__(kScanThreads) void k_scan_local(int m, int *__restrict__ counts,
                                                             int *__restrict__ out,
                                                             int *__restrict__ bsum,
                                                             const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
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
        if (idx < m) out[idx] = run;
        run += v[k];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Adds to tile b of out the sum of the totals of tiles 0 .. b-1 (the first
// wavefront sums them; integer sums do not depend on the order); the last
// tile also writes the grand total to out[m].
__global__ __launch_bounds__(kScanThreads) void k_scan_add(int m, int nb, const int *__restrict__ bsum,
                                                           int *__restrict__ out,
                                                           const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    __shared__ int sh;
    if (threadIdx.x < 64) {
        int v = 0;
        for (int k = (int)threadIdx.x; k < (int)blockIdx.x; k += 64) v += bsum[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (threadIdx.x == 0) {
            sh = v;
            if ((int)blockIdx.x == nb - 1) out[m] = v + bsum[nb - 1];
        }
    }
    __syncthreads();
    const int add = sh;
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanPer;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < m) out[base + k] += add;
}

__global__ __launch_bounds__(kBlock) void k_scatter_id(int n, const int *__restrict__ key,
                                                       const int *__restrict__ slot,
                                                       const int *__restrict__ cstart,
                                                       const uint32_t *__restrict__ tag,
                                                       uint32_t *__restrict__ tmpid,
                                                       const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    tmpid[cstart[key[i]] + slot[i]] = tag[i] & kIdMask;
}

// With gate == 0 (nothing moved since the last sort) the arrays are copied in
// place order so the caller's buffer swap stays valid.
__global__ __launch_bounds__(kBlock) void k_rank_gather(int n, const int *__restrict__ key,
                                                        const int *__restrict__ cstart,
                                                        const uint32_t *__restrict__ tmpid, Soa3c xin,
                                                        Soa3c vin, Soa3c pin,
                                                        const uint32_t *__restrict__ tag_in,
                                                        const uint8_t *__restrict__ typ_in, Soa3 xout,
                                                        Soa3 vout, Soa3 pout,
                                                        uint32_t *__restrict__ tag_out,
                                                        uint8_t *__restrict__ typ_out,
                                                        const int *__restrict__ gate, int *__restrict__ dmap)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t tg = tag_in[i];
    int dst = i;
    if (!(gate && *gate == 0)) {
        const int c = key[i];
        const int b = cstart[c], e = cstart[c + 1];
        const uint32_t id = tg & kIdMask;
        int rank = 0;
        for (int k = b; k < e; ++k) rank += tmpid[k] < id ? 1 : 0;
        dst = b + rank;
    }
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
    const int r = __builtin_amdgcn_readfirstlane(find_rep(boff, R.nrep, blockIdx.x));
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

}  // namespace

void launch_zero_int(hipStream_t st, int *p, int n)
{
    if (n > 0) k_zero_int<<<blocks_for(n), kBlock, 0, st>>>(p, n);
}

void launch_ingest(hipStream_t st, const Reps &R, const double *pos, const double *vel, const int32_t *type,
                   const uint8_t *frozen, Soa3 xp, Soa3 vp, uint32_t *tag, uint8_t *typ, int *status)
{
    if (R.nblk[0] <= 0) return;
    k_ingest<<<R.nblk[0], kBlock, 0, st>>>(R, pos, vel, type, frozen, xp, vp, tag, typ, status);
}

void launch_sort(hipStream_t st, int n, const Reps &R, Soa3c xin, Soa3c vin, Soa3c xprev_in,
                 const uint32_t *tag_in, const uint8_t *typ_in, Soa3 xout, Soa3 vout, Soa3 xprev_out,
                 uint32_t *tag_out, uint8_t *typ_out, int *key, int *slot, uint32_t *tmpid, int *counts,
                 int *cstart, int *bsum, const int *gate, int *ovf_count, uint32_t *step_ctr, int *dmap)
{
    const int m = R.ncells;
    const int nb = (m + kScanTile - 1) / kScanTile;
    if (n > 0) k_bin<<<R.nblk[0], kBlock, 0, st>>>(R, xin, key, slot, counts, gate, ovf_count, step_ctr);
    k_scan_local<<<nb, kScanThreads, 0, st>>>(m, counts, cstart, bsum, gate);
    k_scan_add<<<nb, kScanThreads, 0, st>>>(m, nb, bsum, cstart, gate);
    if (n > 0) {
        k_scatter_id<<<blocks_for(n), kBlock, 0, st>>>(n, key, slot, cstart, tag_in, tmpid, gate);
        k_rank_gather<<<blocks_for(n), kBlock, 0, st>>>(n, key, cstart, tmpid, xin, vin, xprev_in,
                                                        tag_in, typ_in, xout, vout, xprev_out, tag_out,
                                                        typ_out, gate, dmap);
    }
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

}  // namespace mdpd
