// reduce.hip -- read-out of the state: observables, bin profiles and export
// to caller (id) order.  All sums are FP64 with a fixed reduction order
// (per-thread strided partials, then a block tree), so results are
// deterministic.
#include "mdpd_internal.h"

namespace mdpd {

namespace {

constexpr int kRed = 256;
constexpr int kObs = 10;  // partial slots per block

inline int blocks_for(int64_t threads) { return (int)((threads + kBlock - 1) / kBlock); }

template <int W>
__device__ __forceinline__ void block_tree(double (*sh)[kRed], double *v)
{
#pragma unroll
    for (int k = 0; k < W; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = kRed / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < W; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = sh[k][0];
}

// Block partials over one replica-aligned block of kRed particles:
// [0] sum m-less |v|^2, [1..3] sum v, [4] sum rho, [5] sum B_ii rho^2,
// [6] fluid count, [8] virial and [9] pair-energy shares of particles whose
// neighbour list overflowed.
template <typename R>
__global__ __launch_bounds__(kRed) void k_obs_partial(Reps Rp, Soa3c v, const R *rho, const uint32_t *tag,
                                                      const uint8_t *typ, const int *ncnt, const double *ovf_ve,
                                                      double *part)
{
    __shared__ double sh[kObs][kRed];
    double acc[kObs] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int *boff = Rp.blk_off;  // lane count 1
    const int r = block_replica(Rp, 0, boff, blockIdx.x);
    const int i = cload(Rp.part_off, r) + (blockIdx.x - cload(boff, r)) * kRed + threadIdx.x;
    const PairConst pc = cload(Rp.pc, r);
    if (i < cload(Rp.part_off, r + 1)) {
        const int c = ncnt[i];
        if ((c & 0xffff) + (c >> 16) > kListCap) {  // list overflowed: force pass wrote its share here
            acc[8] += ovf_ve[2 * (size_t)i];
            acc[9] += ovf_ve[2 * (size_t)i + 1];
        }
        const double rr = (double)rho[i];
        const int t = pc.ntypes > 1 ? (int)typ[i] : 0;
        const double B = pc.ntypes > 1 ? pc.tab[64 + t * pc.ntypes + t] : pc.B;
        acc[5] += B * rr * rr;
        if (!(tag[i] & kFrozenBit)) {
            const double vx = v.x[i], vy = v.y[i], vz = v.z[i];
            acc[0] += vx * vx + vy * vy + vz * vz;
            acc[1] += vx;
            acc[2] += vy;
            acc[3] += vz;
            acc[4] += rr;
            acc[6] += 1.0;
        }
    }
    block_tree<kObs>(sh, acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < kObs; ++k) part[(size_t)blockIdx.x * kObs + k] = acc[k];
}

// One block per replica, fixed-order sums: out[16 r + 0..7] observables
// partials, [8] virial, [9] pair energy (force-pass block partials of the
// replica's blocks plus the overflowed particles' shares).
__global__ __launch_bounds__(kRed) void k_obs_final(Reps Rp, int force_li, const double *part,
                                                    const double *fpart, double *out)
{
    __shared__ double sh[10][kRed];
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int r = blockIdx.x;
    const int *b1 = Rp.blk_off;
    const int *bf = Rp.blk_off + force_li * (Rp.nrep + 1);
    for (int b = b1[r] + threadIdx.x; b < b1[r + 1]; b += kRed)
        for (int k = 0; k < kObs; ++k) acc[k] += part[(size_t)b * kObs + k];
    if (fpart)
        for (int b = bf[r] + threadIdx.x; b < bf[r + 1]; b += kRed) {
            acc[8] += fpart[2 * (size_t)b];
            acc[9] += fpart[2 * (size_t)b + 1];
        }
    block_tree<10>(sh, acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < 10; ++k) out[16 * r + k] = acc[k];
}

// Bin sums for one bin per block: count, sum v (3), sum rho, and (second
// pass) sum |v - mean|^2.
template <typename R>
__global__ __launch_bounds__(kRed) void k_profile_bin(int n, int axis, int nbins, double La,
                                                      Soa3c x, Soa3c v, const R *rho,
                                                      const uint32_t *tag, const double *mean,
                                                      double *work)
{
    __shared__ double sh[6][kRed];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int b = blockIdx.x;
    const double *xa = axis == 0 ? x.x : (axis == 1 ? x.y : x.z);
    for (int i = threadIdx.x; i < n; i += kRed) {
        if (tag[i] & kFrozenBit) continue;
        int bi = (int)(xa[i] / La * nbins);
        bi = bi < 0 ? 0 : (bi >= nbins ? nbins - 1 : bi);
        if (bi != b) continue;
        const double vx = v.x[i], vy = v.y[i], vz = v.z[i];
        acc[0] += 1.0;
        acc[1] += vx;
        acc[2] += vy;
        acc[3] += vz;
        acc[4] += (double)rho[i];
        if (mean) {
            const double ux = vx - mean[3 * b], uy = vy - mean[3 * b + 1], uz = vz - mean[3 * b + 2];
            acc[5] += ux * ux + uy * uy + uz * uz;
        }
    }
    block_tree<6>(sh, acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) work[6 * b + k] = acc[k];
}

__global__ void k_profile_mean(int nbins, const double *work, double *mean)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    const double c = work[6 * b];
    for (int a = 0; a < 3; ++a) mean[3 * b + a] = c > 0.0 ? work[6 * b + 1 + a] / c : 0.0;
}

__global__ void k_profile_final(int nbins, int quantity, double binvol, double mass,
                                const double *work, double *out)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    const double c = work[6 * b];
    double r = 0.0;
    if (quantity == 0)
        r = c / binvol;
    else if (quantity >= 1 && quantity <= 3)
        r = c > 0.0 ? work[6 * b + quantity] / c : 0.0;
    else if (quantity == 4)
        r = c > 0.0 ? mass * work[6 * b + 5] / (3.0 * c) : 0.0;
    else
        r = c > 0.0 ? work[6 * b + 4] / c : 0.0;
    out[b] = r;
}

// Scatter to input order: replica r's particle with id k goes to row
// part_off[r] + k.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_export(Reps Rp, Soa3c x, Soa3c v, const R *rho,
                                                   const uint32_t *tag, double *pos, double *vel,
                                                   double *rho_out)
{
    const int *boff = Rp.blk_off;  // lane count 1
    const int r = block_replica(Rp, 0, boff, blockIdx.x);
    const int i = cload(Rp.part_off, r) + (blockIdx.x - cload(boff, r)) * kBlock + threadIdx.x;
    if (i >= cload(Rp.part_off, r + 1)) return;
    const size_t id = (size_t)cload(Rp.part_off, r) + (tag[i] & kIdMask);
    if (pos) {
        pos[3 * id] = x.x[i];
        pos[3 * id + 1] = x.y[i];
        pos[3 * id + 2] = x.z[i];
    }
    if (vel) {
        vel[3 * id] = v.x[i];
        vel[3 * id + 1] = v.y[i];
        vel[3 * id + 2] = v.z[i];
    }
    if (rho_out) rho_out[id] = (double)rho[i];
}

// Per-replica sums of the six pressure-tensor planes written by k_stress:
// one block per replica, fixed order (strided partials, then a tree).
__global__ __launch_bounds__(kRed) void k_stress_sum(Reps Rp, int n, const double *planes, double *out)
{
    __shared__ double sh[6][kRed];
    const int r = blockIdx.x;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int b = cload(Rp.part_off, r), e = cload(Rp.part_off, r + 1);
    for (int i = b + threadIdx.x; i < e; i += kRed)
        for (int a = 0; a < 6; ++a) acc[a] += planes[(size_t)a * n + i];
    block_tree<6>(sh, acc);
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) out[6 * r + a] = acc[a];
}

// Pressure tensor from the per-block sums of k_stress: one block per
// replica r = first + blockIdx.x sums its blocks' partials in a fixed order
// and divides by the replica's volume.
__global__ __launch_bounds__(kRed) void k_stress_part_sum(Reps Rp, int first, const double *parts, double *out)
{
    __shared__ double sh[6][kRed];
    const int r = first + (int)blockIdx.x;
    const int *off = Rp.blk_off + lanes_index(kStressLanes) * (Rp.nrep + 1);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int b = cload(off, r), e = cload(off, r + 1);
    for (int k = b + (int)threadIdx.x; k < e; k += kRed)
        for (int a = 0; a < 6; ++a) acc[a] += parts[6 * (size_t)k + a];
    block_tree<6>(sh, acc);
    if (threadIdx.x == 0) {
        const Geom g = cload(Rp.geom, r);
        const double V = g.L[0] * g.L[1] * g.L[2];
        for (int a = 0; a < 6; ++a) out[6 * (size_t)blockIdx.x + a] = acc[a] / V;
    }
}

// acc[3r + 0..2] += scale * (mean fluid rho, virial pressure, mean fluid
// v_x) of replica r from the final sums of k_obs_final.
__global__ void k_loss_accum(int nrep, const double *obs, const LossConst *lc, double *acc, double scale)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    const double *o = obs + 16 * (size_t)r;
    const LossConst c = lc[r];
    acc[3 * r] += scale * o[4] * c.inv_nf;
    acc[3 * r + 1] += scale * (c.mass * o[0] + o[8]) * c.inv3V;
    acc[3 * r + 2] += scale * o[1] * c.inv_nf;
}

}  // namespace

void launch_stress_sum(hipStream_t st, const Reps &R, int n, const double *planes, double *out)
{
    k_stress_sum<<<R.nrep, kRed, 0, st>>>(R, n, planes, out);
}

void launch_stress_part_sum(hipStream_t st, const Reps &R, int first, int count, const double *parts,
                            double *out)
{
    if (count <= 0) return;
    k_stress_part_sum<<<count, kRed, 0, st>>>(R, first, parts, out);
}

void launch_loss_accum(hipStream_t st, int nrep, const double *obs, const LossConst *lc, double *acc,
                       double scale)
{
    k_loss_accum<<<(nrep + 255) / 256, 256, 0, st>>>(nrep, obs, lc, acc, scale);
}

int obs_partials(const Reps &R) { return R.nblk[0] * kObs; }

void launch_observables(hipStream_t st, bool fp32, const Reps &R, int force_lanes, Soa3c v, const void *rho,
                        const uint32_t *tag, const uint8_t *typ, const double *fpart, const int *ncnt,
                        const double *ovf_ve, double *part, double *out)
{
    if (R.nblk[0] > 0) {
        if (fp32)
            k_obs_partial<float><<<R.nblk[0], kRed, 0, st>>>(R, v, (const float *)rho, tag, typ, ncnt, ovf_ve, part);
        else
            k_obs_partial<double><<<R.nblk[0], kRed, 0, st>>>(R, v, (const double *)rho, tag, typ, ncnt, ovf_ve,
                                                              part);
    }
    k_obs_final<<<R.nrep, kRed, 0, st>>>(R, lanes_index(force_lanes), part, fpart, out);
}

void launch_profile(hipStream_t st, bool fp32, int n, int axis, int nbins, int quantity, double La,
                    double binvol, double mass, Soa3c x, Soa3c v, const void *rho, const uint32_t *tag,
                    double *work, double *out)
{
    double *mean = work + 6 * nbins;
    double *wk = work;
    auto pass = [&](const double *mn) {
        if (fp32)
            k_profile_bin<float><<<nbins, kRed, 0, st>>>(n, axis, nbins, La, x, v, (const float *)rho,
                                                         tag, mn, wk);
        else
            k_profile_bin<double><<<nbins, kRed, 0, st>>>(n, axis, nbins, La, x, v,
                                                          (const double *)rho, tag, mn, wk);
    };
    pass(nullptr);
    if (quantity == 4) {
        k_profile_mean<<<(nbins + 255) / 256, 256, 0, st>>>(nbins, wk, mean);
        pass(mean);
    }
    k_profile_final<<<(nbins + 255) / 256, 256, 0, st>>>(nbins, quantity, binvol, mass, wk, out);
}

void launch_export(hipStream_t st, bool fp32, const Reps &R, Soa3c x, Soa3c v, const void *rho,
                   const uint32_t *tag, double *pos, double *vel, double *rho_out)
{
    if (R.nblk[0] <= 0) return;
    if (fp32)
        k_export<float><<<R.nblk[0], kBlock, 0, st>>>(R, x, v, (const float *)rho, tag, pos, vel, rho_out);
    else
        k_export<double><<<R.nblk[0], kBlock, 0, st>>>(R, x, v, (const double *)rho, tag, pos, vel, rho_out);
}

}  // namespace mdpd
