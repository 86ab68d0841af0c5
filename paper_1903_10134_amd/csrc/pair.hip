// pair.hip -- the pair passes of one mDPD timestep on gfx950.
//
//   k_nlist    cell scan: for every particle the neighbours within r_c (exact
//              FP64 test on FP64 positions), written to a fixed-capacity list
//   k_density  many-body density rho_i = sum_{j != i, r < r_d} w_rho(r_ij)
//              (Sec. 2.1) over the list
//   k_phi      boundary volume fraction of fluid particles at the predicted
//              positions and the predictor-corrector flag (Sec. 2.2, Sec. 3.2)
//   k_force    Eq. 1 conservative force, dissipative and random forces
//              (Sec. 2.1), body force, and the velocity-Verlet update fused in
//              the epilogue: v(t+dt), the next half-step velocity and the next
//              predicted position (Alg. 1)
//
// Work decomposition: P lanes of a 64-wide wavefront cooperate on one
// particle i (P = 1, 2, 4, 8 or 16).  In the cell scan the P lanes stride
// through each contiguous run of candidate slots (three x-adjacent cells are
// contiguous in the sorted order), and a wavefront ballot compacts the hits
// into the list in scan order.  In the list passes the P lanes split the
// list entries and combine their partial sums with a butterfly of lane
// shuffles inside the group, so every sum has one fixed order.
#include "mdpd_internal.h"

namespace mdpd {

namespace {

constexpr double kSqrt3Scaled = 1.7320508075688772 / 16777216.0;  // sqrt(3) 2^-24
constexpr float kSqrt3ScaledF = 1.7320508075688772f / 16777216.0f;

// Calls fn(begin, end, sx, sy, sz) for the contiguous slot ranges holding the
// 27 cells around the cell of (xi, yi, zi); (sx, sy, sz) is the periodic shift
// to add to x_i - x_j for candidates of that range.
template <typename Fn>
__device__ __forceinline__ void for_each_row(const Geom &g, double xi, double yi, double zi,
                                             const int *__restrict__ cstart, Fn &&fn)
{
    const int nx = g.nc[0], ny = g.nc[1], nz = g.nc[2];
    const int cx = cell_coord(xi, g.s[0], nx);
    const int cy = cell_coord(yi, g.s[1], ny);
    const int cz = cell_coord(zi, g.s[2], nz);
    for (int dz = -1; dz <= 1; ++dz) {
        int zz = cz + dz;
        double sz = 0.0;
        if (zz < 0) {
            zz += nz;
            sz = g.L[2];
        } else if (zz >= nz) {
            zz -= nz;
            sz = -g.L[2];
        }
        for (int dy = -1; dy <= 1; ++dy) {
            int yy = cy + dy;
            double sy = 0.0;
            if (yy < 0) {
                yy += ny;
                sy = g.L[1];
            } else if (yy >= ny) {
                yy -= ny;
                sy = -g.L[1];
            }
            const int base = nx * (yy + ny * zz);
            if (cx > 0 && cx < nx - 1) {
                fn(cstart[base + cx - 1], cstart[base + cx + 2], 0.0, sy, sz);
            } else if (cx == 0) {
                fn(cstart[base + nx - 1], cstart[base + nx], g.L[0], sy, sz);
                fn(cstart[base], cstart[base + 2], 0.0, sy, sz);
            } else {
                fn(cstart[base + nx - 2], cstart[base + nx], 0.0, sy, sz);
                fn(cstart[base], cstart[base + 1], -g.L[0], sy, sz);
            }
        }
    }
}

// Sum over the P lanes of a group (butterfly, fixed order).
template <int P, typename T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int m = 1; m < P; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Visits every neighbour j (r_ij < r_c, j != i) of slot i: from the list when
// it did not overflow, else by a direct cell scan with the same exact test.
// fn(j, dx, dy, dz) receives the minimum-image difference x_i - x_j.
template <int P, typename Fn>
__device__ __forceinline__ void for_each_neighbor(const PairConst &pc, const Geom &g, int i, int sub,
                                                  double xi, double yi, double zi, Soa3c xs,
                                                  const int *__restrict__ cstart, int cnt,
                                                  const int *__restrict__ lst, Fn &&fn)
{
    if (cnt <= kListCap) {
        for (int k = sub; k < cnt; k += P) {
            const int j = lst[k];
            const double dx = min_image(xi - xs.x[j], pc.L[0], pc.invL[0]);
            const double dy = min_image(yi - xs.y[j], pc.L[1], pc.invL[1]);
            const double dz = min_image(zi - xs.z[j], pc.L[2], pc.invL[2]);
            fn(j, dx, dy, dz);
        }
    } else {
        for_each_row(g, xi, yi, zi, cstart, [&](int b, int e, double sx, double sy, double sz) {
            for (int j = b + sub; j < e; j += P) {
                if (j == i) continue;
                const double dx = (xi - xs.x[j]) + sx;
                const double dy = (yi - xs.y[j]) + sy;
                const double dz = (zi - xs.z[j]) + sz;
                if (exact_r2(dx, dy, dz) < g.rc2) fn(j, dx, dy, dz);
            }
        });
    }
}

// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_nlist(Geom g, int n, Soa3c xs,
                                                  const int *__restrict__ cstart,
                                                  int *__restrict__ ncnt, int *__restrict__ nl,
                                                  const int *__restrict__ gate)
{
    if (gate && *gate == 0) return;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int i = t / P;
    const int sub = t & (P - 1);
    if (i >= n) return;
    const int gbase = (threadIdx.x & 63) & ~(P - 1);
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    int *out = nl + (size_t)i * kListCap;
    int cnt = 0;
    for_each_row(g, xi, yi, zi, cstart, [&](int b, int e, double sx, double sy, double sz) {
        for (int j0 = b; j0 < e; j0 += P) {
            const int j = j0 + sub;
            bool hit = false;
            if (j < e && j != i) {
                const double dx = (xi - xs.x[j]) + sx;
                const double dy = (yi - xs.y[j]) + sy;
                const double dz = (zi - xs.z[j]) + sz;
                hit = exact_r2(dx, dy, dz) < g.rc2;
            }
            const unsigned long long m = __ballot(hit);
            const unsigned long long gm =
                P == 64 ? m : ((m >> gbase) & ((1ull << (P & 63)) - 1ull));
            const int pre = __popcll(gm & ((1ull << sub) - 1ull));
            if (hit && cnt + pre < kListCap) out[cnt + pre] = j;
            cnt += __popcll(gm);
        }
    });
    if (sub == 0) ncnt[i] = cnt;
}

// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R w_rho(const PairConst &pc, double r2);

template <>
__device__ __forceinline__ double w_rho<double>(const PairConst &pc, double r2)
{
    const double r = __builtin_sqrt(r2);
    const double u = 1.0 - r * pc.inv_rd;
    return pc.wrho * u * u;
}

template <>
__device__ __forceinline__ float w_rho<float>(const PairConst &pc, double r2)
{
    const float r = __builtin_sqrtf((float)r2);
    const float u = 1.0f - r * (float)pc.inv_rd;
    return (float)pc.wrho * u * u;
}

template <int P, typename R>
__global__ __launch_bounds__(kBlock) void k_density(PairConst pc, Geom g, int n, Soa3c xs,
                                                    const int *__restrict__ cstart,
                                                    const int *__restrict__ ncnt,
                                                    const int *__restrict__ nl, R *__restrict__ rho)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int i = t / P;
    const int sub = t & (P - 1);
    if (i >= n) return;
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    R acc = 0;
    for_each_neighbor<P>(pc, g, i, sub, xi, yi, zi, xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                         [&](int, double dx, double dy, double dz) {
                             const double r2 = exact_r2(dx, dy, dz);
                             if (r2 < pc.rd2) acc += w_rho<R>(pc, r2);
                         });
    acc = group_sum<P>(acc);
    if (sub == 0) rho[i] = acc;
}

// ---------------------------------------------------------------------------
// phi_i = sum_{frozen j} w_c^2 / sum_j w_c^2 over neighbours within r_c at the
// predicted positions; flag[i] = 1 when phi_i > phi_c (fluid only).
template <int P>
__global__ __launch_bounds__(kBlock) void k_phi(PairConst pc, Geom g, int n, Soa3c xs,
                                                const uint32_t *__restrict__ tag,
                                                const int *__restrict__ cstart,
                                                const int *__restrict__ ncnt,
                                                const int *__restrict__ nl, int *__restrict__ flag)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int i = t / P;
    const int sub = t & (P - 1);
    if (i >= n) return;
    if (tag[i] & kFrozenBit) {
        if (sub == 0) flag[i] = 0;
        return;
    }
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    double num = 0.0, den = 0.0;
    for_each_neighbor<P>(pc, g, i, sub, xi, yi, zi, xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                         [&](int j, double dx, double dy, double dz) {
                             const double r = __builtin_sqrt(exact_r2(dx, dy, dz));
                             const double w = 1.0 - r * pc.inv_rc;
                             den += w * w;
                             if (tag[j] & kFrozenBit) num += w * w;
                         });
    num = group_sum<P>(num);
    den = group_sum<P>(den);
    if (sub == 0) flag[i] = (den > 0.0 && num / den > pc.phi_c) ? 1 : 0;
}

// Applies the corrector to flagged particles: x <- x(t), v_half <- -v_half.
__global__ __launch_bounds__(kBlock) void k_correct(int n, const int *__restrict__ flag, Soa3c xprev,
                                                    Soa3 xs, Soa3 vh, int *__restrict__ ncorr,
                                                    unsigned long long *__restrict__ ncorr_total)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    int hit = 0;
    if (i < n && flag[i]) {
        xs.x[i] = xprev.x[i];
        xs.y[i] = xprev.y[i];
        xs.z[i] = xprev.z[i];
        vh.x[i] = -vh.x[i];
        vh.y[i] = -vh.y[i];
        vh.z[i] = -vh.z[i];
        hit = 1;
    }
    const unsigned long long m = __ballot(hit);
    if ((threadIdx.x & 63) == 0 && m) {
        atomicAdd(ncorr, (int)__popcll(m));
        atomicAdd(ncorr_total, (unsigned long long)__popcll(m));
    }
}

// ---------------------------------------------------------------------------
// Force pass with the velocity-Verlet epilogue.
template <typename R>
struct Acc3 {
    R x, y, z;
};

__device__ __forceinline__ double wrap_coord(double x, double L)
{
    if (x < 0.0) x += L;
    if (x >= L) x -= L;
    return x;
}

template <int P, bool MT, typename R>
__global__ __launch_bounds__(kBlock) void k_force(PairConst pc, Geom g, int n, Soa3c xs, Soa3c vh,
                                                  const R *__restrict__ rho,
                                                  const uint32_t *__restrict__ tag,
                                                  const uint8_t *__restrict__ typ,
                                                  const int *__restrict__ cstart,
                                                  const int *__restrict__ ncnt,
                                                  const int *__restrict__ nl, Soa3 vout, Soa3 fout,
                                                  Soa3 vpred, Soa3 xpred, double *__restrict__ part,
                                                  int *__restrict__ status, int initial)
{
    __shared__ double red_v[kBlock];
    __shared__ double red_e[kBlock];
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int i = t / P;
    const int sub = t & (P - 1);
    double vir = 0.0, ep = 0.0;
    if (i < n) {
        const uint32_t tgi = tag[i];
        const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
        if (!(tgi & kFrozenBit)) {
            const uint32_t idi = tgi & kIdMask;
            const double vxi = vh.x[i], vyi = vh.y[i], vzi = vh.z[i];
            const R rhoi = rho[i];
            const int T = pc.ntypes;
            const int ti = MT ? (int)typ[i] : 0;
            R fx = 0, fy = 0, fz = 0;
            for_each_neighbor<P>(
                pc, g, i, sub, xi, yi, zi, xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                [&](int j, double dx, double dy, double dz) {
                    const double r2 = exact_r2(dx, dy, dz);
                    if (r2 == 0.0) return;  // coincident pair: no direction, no force
                    const uint32_t tgj = tag[j];
                    double A = pc.A, B = pc.B, gam = pc.gamma, sig = pc.sig, Arc2 = pc.Arc2;
                    if (MT) {
                        const int tt = ti * T + (int)typ[j];
                        A = pc.tab[tt];
                        B = pc.tab[64 + tt];
                        gam = pc.tab[128 + tt];
                        sig = pc.tab[192 + tt];
                        Arc2 = pc.tab[256 + tt];
                    }
                    const int th = theta_int(idi, tgj & kIdMask, pc);
                    const double dvx = vxi - vh.x[j], dvy = vyi - vh.y[j], dvz = vzi - vh.z[j];
                    const bool near = r2 < pc.rd2;
                    double fc_d;  // conservative magnitude, kept in FP64 for the virial
                    double wc_d;
                    if constexpr (sizeof(R) == 8) {
                        const double rinv = rsqrt_f64(r2);
                        const double r = r2 * rinv;
                        const double wc = 1.0 - r * pc.inv_rc;
                        double fc = A * wc;
                        if (near) fc += B * (rhoi + rho[j]) * (1.0 - r * pc.inv_rd);
                        const double ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
                        const double ev = ex * dvx + ey * dvy + ez * dvz;
                        const double fs = fc - gam * wc * wc * ev + sig * wc * ((double)th * kSqrt3Scaled);
                        fx += fs * ex;
                        fy += fs * ey;
                        fz += fs * ez;
                        fc_d = fc * r;
                        wc_d = wc;
                    } else {
                        const float r2f = (float)r2;
                        const float rinv = __builtin_amdgcn_rsqf(r2f);
                        const float r = r2f * rinv;
                        const float wc = 1.0f - r * (float)pc.inv_rc;
                        float fc = (float)A * wc;
                        if (near) fc += (float)B * (rhoi + rho[j]) * (1.0f - r * (float)pc.inv_rd);
                        const float ex = (float)dx * rinv, ey = (float)dy * rinv, ez = (float)dz * rinv;
                        const float ev = ex * (float)dvx + ey * (float)dvy + ez * (float)dvz;
                        const float fs = fc - (float)gam * wc * wc * ev +
                                         (float)sig * wc * ((float)th * kSqrt3ScaledF);
                        fx += fs * ex;
                        fy += fs * ey;
                        fz += fs * ez;
                        fc_d = (double)(fc * r);
                        wc_d = (double)wc;
                    }
                    const double c = (tgj & kFrozenBit) ? 1.0 : 0.5;
                    vir += c * fc_d;
                    ep += c * Arc2 * wc_d * wc_d;
                });
            fx = group_sum<P>(fx);
            fy = group_sum<P>(fy);
            fz = group_sum<P>(fz);
            if (sub == 0) {
                const double Fx = (double)fx + pc.mg[0];
                const double Fy = (double)fy + pc.mg[1];
                const double Fz = (double)fz + pc.mg[2];
                const double vx = initial ? vxi : vxi + pc.hdtm * Fx;
                const double vy = initial ? vyi : vyi + pc.hdtm * Fy;
                const double vz = initial ? vzi : vzi + pc.hdtm * Fz;
                const double px = vx + pc.hdtm * Fx;
                const double py = vy + pc.hdtm * Fy;
                const double pz = vz + pc.hdtm * Fz;
                const double qx = wrap_coord(xi + pc.dt * px, pc.L[0]);
                const double qy = wrap_coord(yi + pc.dt * py, pc.L[1]);
                const double qz = wrap_coord(zi + pc.dt * pz, pc.L[2]);
                vout.x[i] = vx;
                vout.y[i] = vy;
                vout.z[i] = vz;
                fout.x[i] = Fx;
                fout.y[i] = Fy;
                fout.z[i] = Fz;
                vpred.x[i] = px;
                vpred.y[i] = py;
                vpred.z[i] = pz;
                xpred.x[i] = qx;
                xpred.y[i] = qy;
                xpred.z[i] = qz;
                const bool ok = __builtin_isfinite(qx) && __builtin_isfinite(qy) &&
                                __builtin_isfinite(qz) && __builtin_isfinite(px) &&
                                __builtin_isfinite(py) && __builtin_isfinite(pz) &&
                                qx >= 0.0 && qx < pc.L[0] && qy >= 0.0 && qy < pc.L[1] &&
                                qz >= 0.0 && qz < pc.L[2];
                if (!ok) atomicOr(status, 1);
            }
        } else if (sub == 0) {
            vout.x[i] = vout.y[i] = vout.z[i] = 0.0;
            fout.x[i] = fout.y[i] = fout.z[i] = 0.0;
            vpred.x[i] = vpred.y[i] = vpred.z[i] = 0.0;
            xpred.x[i] = xi;
            xpred.y[i] = yi;
            xpred.z[i] = zi;
        }
    }
    // block partials of the virial and the pair energy (fixed-order tree)
    red_v[threadIdx.x] = vir;
    red_e[threadIdx.x] = ep;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red_v[threadIdx.x] += red_v[threadIdx.x + s];
            red_e[threadIdx.x] += red_e[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = red_v[0];
        part[2 * blockIdx.x + 1] = red_e[0];
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

__global__ __launch_bounds__(kBlock) void k_debug_neighbors(PairConst pc, Geom g, int n, double cut2,
                                                            Soa3c xs, const uint32_t *__restrict__ tag,
                                                            const int *__restrict__ cstart,
                                                            const int *__restrict__ ncnt,
                                                            const int *__restrict__ nl,
                                                            int64_t *__restrict__ count,
                                                            uint64_t *__restrict__ hash)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    int64_t c = 0;
    uint64_t h = 0;
    for_each_neighbor<1>(pc, g, i, 0, xi, yi, zi, xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                         [&](int j, double dx, double dy, double dz) {
                             if (exact_r2(dx, dy, dz) < cut2) {
                                 ++c;
                                 h += mix64((uint64_t)(tag[j] & kIdMask));
                             }
                         });
    const uint32_t id = tag[i] & kIdMask;
    count[id] = c;
    hash[id] = h;
}

template <typename K>
void launch_lanes(int lanes, K &&k)
{
    switch (lanes) {
    case 1: k(std::integral_constant<int, 1>{}); break;
    case 2: k(std::integral_constant<int, 2>{}); break;
    case 4: k(std::integral_constant<int, 4>{}); break;
    case 8: k(std::integral_constant<int, 8>{}); break;
    default: k(std::integral_constant<int, 16>{}); break;
    }
}

inline int blocks_for(int64_t threads) { return (int)((threads + kBlock - 1) / kBlock); }

}  // namespace

int force_blocks(int lanes, int n) { return blocks_for((int64_t)n * lanes); }

void launch_nlist(hipStream_t st, int lanes, int n, Geom g, Soa3c xs, const int *cstart, int *ncnt,
                  int *nl, const int *gate)
{
    if (n <= 0) return;
    launch_lanes(lanes, [&](auto P) {
        k_nlist<decltype(P)::value><<<blocks_for((int64_t)n * P), kBlock, 0, st>>>(g, n, xs, cstart,
                                                                                   ncnt, nl, gate);
    });
}

void launch_density(hipStream_t st, int lanes, bool fp32, int n, const PairConst &pc, Geom g,
                    Soa3c xs, const int *cstart, const int *ncnt, const int *nl, void *rho)
{
    if (n <= 0) return;
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        if (fp32)
            k_density<L, float><<<blocks_for((int64_t)n * L), kBlock, 0, st>>>(
                pc, g, n, xs, cstart, ncnt, nl, (float *)rho);
        else
            k_density<L, double><<<blocks_for((int64_t)n * L), kBlock, 0, st>>>(
                pc, g, n, xs, cstart, ncnt, nl, (double *)rho);
    });
}

void launch_phi(hipStream_t st, int lanes, int n, const PairConst &pc, Geom g, Soa3c xs, Soa3c xprev,
                Soa3 xfix, Soa3 vfix, const uint32_t *tag, const int *cstart, const int *ncnt,
                const int *nl, int *flag_and_count, unsigned long long *ncorr_total)
{
    if (n <= 0) return;
    int *ncorr = flag_and_count;       // [0]: corrections this step
    int *flag = flag_and_count + 1;    // [1..n]: per-slot flags
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        k_phi<L><<<blocks_for((int64_t)n * L), kBlock, 0, st>>>(pc, g, n, xs, tag, cstart, ncnt, nl,
                                                                flag);
    });
    k_correct<<<blocks_for(n), kBlock, 0, st>>>(n, flag, xprev, xfix, vfix, ncorr, ncorr_total);
}

void launch_force(hipStream_t st, int lanes, bool fp32, int n, const PairConst &pc, Geom g, Soa3c xs,
                  Soa3c vh, const void *rho, const uint32_t *tag, const uint8_t *typ,
                  const int *cstart, const int *ncnt, const int *nl, Soa3 vout, Soa3 fout,
                  Soa3 vpred, Soa3 xpred, double *part, int *status, int initial)
{
    if (n <= 0) return;
    const bool mt = pc.ntypes > 1;
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        const int nb = blocks_for((int64_t)n * L);
        if (fp32) {
            if (mt)
                k_force<L, true, float><<<nb, kBlock, 0, st>>>(pc, g, n, xs, vh, (const float *)rho, tag,
                                                               typ, cstart, ncnt, nl, vout, fout, vpred,
                                                               xpred, part, status, initial);
            else
                k_force<L, false, float><<<nb, kBlock, 0, st>>>(pc, g, n, xs, vh, (const float *)rho, tag,
                                                                typ, cstart, ncnt, nl, vout, fout, vpred,
                                                                xpred, part, status, initial);
        } else {
            if (mt)
                k_force<L, true, double><<<nb, kBlock, 0, st>>>(pc, g, n, xs, vh, (const double *)rho,
                                                                tag, typ, cstart, ncnt, nl, vout, fout,
                                                                vpred, xpred, part, status, initial);
            else
                k_force<L, false, double><<<nb, kBlock, 0, st>>>(pc, g, n, xs, vh, (const double *)rho,
                                                                 tag, typ, cstart, ncnt, nl, vout, fout,
                                                                 vpred, xpred, part, status, initial);
        }
    });
}

void launch_debug_neighbors(hipStream_t st, int n, Geom g, const PairConst &pc, double cutoff2,
                            Soa3c xs, const uint32_t *tag, const int *cstart, const int *ncnt,
                            const int *nl, int64_t *count, uint64_t *hash)
{
    if (n <= 0) return;
    k_debug_neighbors<<<blocks_for(n), kBlock, 0, st>>>(pc, g, n, cutoff2, xs, tag, cstart, ncnt, nl,
                                                        count, hash);
}

}  // namespace mdpd
