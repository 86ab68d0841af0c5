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

template <typename R>
__global__ __launch_bounds__(kRed) void k_obs_partial(int n, PairConst pc, Soa3c v, const R *rho,
                                                      const uint32_t *tag, const uint8_t *typ,
                                                      const int *ncnt, const double *ovf_ve, double *part)
{
    __shared__ double sh[kObs][kRed];
    double acc[kObs] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = blockIdx.x * kRed + threadIdx.x; i < n; i += gridDim.x * kRed) {
        const int c = ncnt[i];
        if ((c & 0xffff) + (c >> 16) > kListCap) {  // list overflowed: force pass wrote its share here
            acc[8] += ovf_ve[2 * (size_t)i];
            acc[9] += ovf_ve[2 * (size_t)i + 1];
        }
        const double r = (double)rho[i];
        const int t = pc.ntypes > 1 ? (int)typ[i] : 0;
        const double B = pc.ntypes > 1 ? pc.tab[64 + t * pc.ntypes + t] : pc.B;
        acc[5] += B * r * r;
        if (tag[i] & kFrozenBit) continue;
        const double vx = v.x[i], vy = v.y[i], vz = v.z[i];
        acc[0] += vx * vx + vy * vy + vz * vz;
        acc[1] += vx;
        acc[2] += vy;
        acc[3] += vz;
        acc[4] += r;
        acc[6] += 1.0;
    }
    block_tree<kObs>(sh, acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < kObs; ++k) part[blockIdx.x * kObs + k] = acc[k];
}

// Final fixed-order sums: out[0..7] observables partials, out[8] virial,
// out[9] pair energy (force-pass block partials plus the overflowed
// particles' shares).
__global__ __launch_bounds__(kRed) void k_obs_final(int nb, const double *part, int nf,
                                                    const double *fpart, double *out)
{
    __shared__ double sh[10][kRed];
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kRed)
        for (int k = 0; k < kObs; ++k) acc[k] += part[b * kObs + k];
    for (int b = threadIdx.x; b < nf; b += kRed) {
        acc[8] += fpart[2 * b];
        acc[9] += fpart[2 * b + 1];
    }
    block_tree<10>(sh, acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < 10; ++k) out[k] = acc[k];
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

template <typename R>
__global__ __launch_bounds__(kBlock) void k_export(int n, Soa3c x, Soa3c v, const R *rho,
                                                   const uint32_t *tag, double *pos, double *vel,
                                                   double *rho_out)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t id = tag[i] & kIdMask;
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

// acc[0..2] += scale * (mean fluid rho, virial pressure, mean fluid v_x)
// from the final sums of k_obs_final.
__global__ void k_loss_accum(const double *obs, double *acc, double inv_nf, double inv3V, double mass,
                             double scale)
{
    if (threadIdx.x != 0) return;
    acc[0] += scale * obs[4] * inv_nf;
    acc[1] += scale * (mass * obs[0] + obs[8]) * inv3V;
    acc[2] += scale * obs[1] * inv_nf;
}

}  // namespace

void launch_loss_accum(hipStream_t st, const double *obs16, double *acc, double inv_nf, double inv3V,
                       double mass, double scale)
{
    k_loss_accum<<<1, 64, 0, st>>>(obs16, acc, inv_nf, inv3V, mass, scale);
}

void launch_observables(hipStream_t st, bool fp32, int n, const PairConst &pc, Soa3c v, const void *rho,
                        const uint32_t *tag, const uint8_t *typ, const double *fpart, int nfpart,
                        const int *ncnt, const double *ovf_ve, double *out16)
{
    // out16: 16 result slots followed by up to 1024 x kObs block partials.
    const int nb = n > 0 ? (blocks_for(n) < 1024 ? blocks_for(n) : 1024) : 0;
    double *part = out16 + 16;
    if (nb > 0) {
        if (fp32)
            k_obs_partial<float><<<nb, kRed, 0, st>>>(n, pc, v, (const float *)rho, tag, typ, ncnt, ovf_ve,
                                                      part);
        else
            k_obs_partial<double><<<nb, kRed, 0, st>>>(n, pc, v, (const double *)rho, tag, typ, ncnt, ovf_ve,
                                                       part);
    }
    k_obs_final<<<1, kRed, 0, st>>>(nb, part, nfpart, fpart, out16);
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

void launch_export(hipStream_t st, bool fp32, int n, Soa3c x, Soa3c v, const void *rho, const uint32_t *tag,
                   double *pos, double *vel, double *rho_out)
{
    if (n <= 0) return;
    if (fp32)
        k_export<float><<<blocks_for(n), kBlock, 0, st>>>(n, x, v, (const float *)rho, tag, pos, vel,
                                                          rho_out);
    else
        k_export<double><<<blocks_for(n), kBlock, 0, st>>>(n, x, v, (const double *)rho, tag, pos, vel,
                                                           rho_out);
}

}  // namespace mdpd
