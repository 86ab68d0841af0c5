// adjoint.hip -- reverse-mode derivative of one mDPD timestep (the adjoint
// of the pair passes and of velocity-Verlet), for gradients of trajectory
// losses with respect to the pair tables A, B, gamma and the initial state.
//
// Forward recurrence of one step n (walls off), with u_n the half-step
// velocity v(t_n + dt/2) and h = dt / (2 m):
//     x_n = x_{n-1} + dt u_{n-1}              (drift, Alg. 1)
//     rho_n = rho(x_n)                         (Sec. 2.1)
//     F_n = F(x_n, u_{n-1}, rho_n; theta_n)    (Eq. 1 and Sec. 2.1)
//     v_n = u_{n-1} + h F_n,   u_n = u_{n-1} + 2 h F_n
// The noise theta_ij depends on (seed, step, ids) only, so it is a constant of
// the derivative.  Given the adjoints X = dL/dx_n and U = dL/du_n, one
// backward step computes, per sorted slot of step n:
//   k_adj_seed     loss seeds of the state n (mean fluid density, virial
//                  pressure, mean fluid x-velocity), the force adjoint
//                  fbar = 2h U + h vbar, and U += vbar
//   k_adj_force    the pair VJP of the force pass with the full neighbour
//                  list: for f_ij = fs(r, e.u_ij, rho_i + rho_j) e (f_ji =
//                  -f_ij) and g_ij = fbar_i - fbar_j every particle gathers
//                  its own share, X_i += J_x(ij)^T g_ij, U_i += J_u(ij)^T g_ij,
//                  rhobar_i += B w_d (e . g_ij), and half of each pair's
//                  parameter derivative (the pair is visited from both ends),
//                  so no atomics are needed; plus the virial seed's terms
//   k_adj_density  X_i += sum_j (rhobar_i + rhobar_j) w_rho'(r) e_ij
//   k_adj_scatter  U += dt X (drift) and reorder X, U by particle id
//   k_adj_gather   X, U into the sorted order of step n - 1
// Parameter shares are written per particle (3 x ntypes values, by the type
// of the neighbour) and reduced per step in a fixed order (k_adj_params).
// All adjoint arithmetic is FP64.
#include "pair_common.h"

namespace mdpd {

namespace {

// Pair constants of the type pair (ti, tj).
struct PairTab {
    double A, B, gam, sig;
};

template <bool MT>
__device__ __forceinline__ PairTab pair_tab(const PairConst &pc, int ti, int tj)
{
    if (!MT) return PairTab{pc.A, pc.B, pc.gamma, pc.sig};
    const int tt = ti * pc.ntypes + tj;
    return PairTab{pc.tab[tt], pc.tab[64 + tt], pc.tab[128 + tt], pc.tab[192 + tt]};
}

__global__ __launch_bounds__(kBlock) void k_adj_seed(int n, AdjConst ac, Soa3c v, const uint32_t *__restrict__ tag,
                                                    Soa3 U, Soa3 fb, double *__restrict__ rhoA)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (tag[i] & kFrozenBit) {
        U.x[i] = U.y[i] = U.z[i] = 0.0;
        fb.x[i] = fb.y[i] = fb.z[i] = 0.0;
        rhoA[i] = 0.0;
        return;
    }
    const double kv = 2.0 * ac.mass * ac.wP_3V;
    const double bx = kv * v.x[i] + ac.wvx_nf, by = kv * v.y[i], bz = kv * v.z[i];
    const double ux = U.x[i], uy = U.y[i], uz = U.z[i];
    fb.x[i] = ac.cU * ux + ac.cv * bx;
    fb.y[i] = ac.cU * uy + ac.cv * by;
    fb.z[i] = ac.cU * uz + ac.cv * bz;
    U.x[i] = ux + bx;
    U.y[i] = uy + by;
    U.z[i] = uz + bz;
    rhoA[i] = ac.wrho_nf;
}

template <int P, bool MT, typename R>
__global__ __launch_bounds__(kBlock) void k_adj_force(Reps Rp, uint32_t step, AdjConst ac, int n, Soa3c xs,
                                                     Soa3c u, const R *__restrict__ rho,
                                                     const uint32_t *__restrict__ tag,
                                                     const uint8_t *__restrict__ typ,
                                                     const int *__restrict__ cstart_all,
                                                     const int *__restrict__ ncnt,
                                                     const uint32_t *__restrict__ nl, Soa3c fb, Soa3 X, Soa3 U,
                                                     double *__restrict__ rhoA, double *__restrict__ gp)
{
    constexpr int TM = MT ? MDPD_ADJ_MAX_TYPES : 1;
    const BlockRep br = block_rep<P>(Rp, xcd_block());
    const int i = br.i0 + (int)threadIdx.x / P;
    const int sub = threadIdx.x & (P - 1);
    if (i >= br.i1) return;  // uniform over the P lanes of particle i
    PairConst pc = cload(Rp.pc, br.r);
    set_noise_keys(pc, step);
    const Geom g = cload(Rp.geom, br.r);
    const int *__restrict__ cstart = cstart_all + cload(Rp.cell_off, br.r);
    const uint32_t tgi = tag[i];
    const bool fzi = (tgi & kFrozenBit) != 0;
    const uint32_t idi = tgi & kIdMask;
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    const double uxi = fzi ? 0.0 : u.x[i], uyi = fzi ? 0.0 : u.y[i], uzi = fzi ? 0.0 : u.z[i];
    const double fxi = fb.x[i], fyi = fb.y[i], fzi_ = fb.z[i];
    const double rhoi = (double)rho[i];
    const int T = MT ? pc.ntypes : 1;
    const int ti = MT ? (int)typ[i] : 0;
    const double wP = ac.wP_3V;
    double ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0, ar = 0;
    double pA[TM], pB[TM], pG[TM];
#pragma unroll
    for (int k = 0; k < TM; ++k) pA[k] = pB[k] = pG[k] = 0.0;
    for_each_neighbor<P>(pc, g, i, sub, xi, yi, zi, xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                         [&](int j, double dx, double dy, double dz, bool near) {
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 > 0.0)) return;
        const uint32_t tgj = ld(tag, j);
        const bool fzj = (tgj & kFrozenBit) != 0;
        const int tj = MT ? (int)ld(typ, j) : 0;
        const PairTab pt = pair_tab<MT>(pc, ti, tj);
        const double rinv = rsqrt_f64(r2);
        const double r = r2 * rinv;
        const double ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
        const double uxj = fzj ? 0.0 : ld(u.x, j), uyj = fzj ? 0.0 : ld(u.y, j), uzj = fzj ? 0.0 : ld(u.z, j);
        const double gx = fxi - ld(fb.x, j), gy = fyi - ld(fb.y, j), gz = fzi_ - ld(fb.z, j);
        const double rs = rhoi + (double)ld(rho, j);
        const double vx = uxi - uxj, vy = uyi - uyj, vz = uzi - uzj;
        const double wc = 1.0 - r * pc.inv_rc;
        const double wd = near ? 1.0 - r * pc.inv_rd : 0.0;
        const double Bn = near ? pt.B : 0.0;
        const double ev = ex * vx + ey * vy + ez * vz;
        const double th = (double)theta_int(idi, tgj & kIdMask, pc) * kSqrt3Scaled;
        const double fc = pt.A * wc + Bn * rs * wd;
        const double fs = fc - pt.gam * wc * wc * ev + pt.sig * wc * th;
        const double gE = gx * ex + gy * ey + gz * ez;
        // derivatives of fs in r (at fixed e.u_ij) and in e.u_ij
        const double dfc_dr = -pt.A * pc.inv_rc - Bn * rs * pc.inv_rd;
        const double dfs_dr = dfc_dr + 2.0 * pt.gam * wc * ev * pc.inv_rc - pt.sig * th * pc.inv_rc;
        const double dfs_dev = -pt.gam * wc * wc;
        // X_i += gE dfs_dr e + fs (g - gE e) / r + gE dfs_dev (u_ij - ev e) / r
        double ce = gE * dfs_dr - fs * gE * rinv - gE * dfs_dev * ev * rinv;
        const double cg = fs * rinv, cu = gE * dfs_dev * rinv;
        // virial seed: each end takes the whole derivative of r fc for its
        // own coordinate; pairs of two frozen particles are not in the virial
        const double q = (fzi && fzj) ? 0.0 : wP;
        ce += q * (fc + r * dfc_dr);
        ax += ce * ex + cg * gx + cu * vx;
        ay += ce * ey + cg * gy + cu * vy;
        az += ce * ez + cg * gz + cu * vz;
        const double cb = dfs_dev * gE;
        bx += cb * ex;
        by += cb * ey;
        bz += cb * ez;
        ar += Bn * wd * (gE + q * r);
        // half of the pair's parameter derivatives (the other end adds the rest)
        const double dsig = pt.gam > 0.0 ? pt.sig / (2.0 * pt.gam) : 0.0;
        const double sA = 0.5 * wc * (gE + q * r);
        const double sB = 0.5 * rs * wd * (gE + q * r) * (near ? 1.0 : 0.0);
        const double sG = 0.5 * gE * (-wc * wc * ev + dsig * wc * th);
#pragma unroll
        for (int k = 0; k < TM; ++k) {
            const bool hit = !MT || k == tj;
            pA[k] += hit ? sA : 0.0;
            pB[k] += hit ? sB : 0.0;
            pG[k] += hit ? sG : 0.0;
        }
    });
    ax = group_sum<P>(ax);
    ay = group_sum<P>(ay);
    az = group_sum<P>(az);
    bx = group_sum<P>(bx);
    by = group_sum<P>(by);
    bz = group_sum<P>(bz);
    ar = group_sum<P>(ar);
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        pA[k] = group_sum<P>(pA[k]);
        pB[k] = group_sum<P>(pB[k]);
        pG[k] = group_sum<P>(pG[k]);
    }
    if (sub != 0) return;
    X.x[i] += ax;
    X.y[i] += ay;
    X.z[i] += az;
    if (!fzi) {
        U.x[i] += bx;
        U.y[i] += by;
        U.z[i] += bz;
    }
    rhoA[i] += ar;
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        if (k < T) {
            gp[(size_t)(0 * T + k) * n + i] = pA[k];
            gp[(size_t)(1 * T + k) * n + i] = pB[k];
            gp[(size_t)(2 * T + k) * n + i] = pG[k];
        }
    }
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_density(Reps Rp, Soa3c xs, const int *__restrict__ cstart_all,
                                                       const int *__restrict__ ncnt,
                                                       const uint32_t *__restrict__ nl,
                                                       const double *__restrict__ rhoA, Soa3 X)
{
    const BlockRep br = block_rep<P>(Rp, xcd_block());
    const int i = br.i0 + (int)threadIdx.x / P;
    const int sub = threadIdx.x & (P - 1);
    if (i >= br.i1) return;
    const PairConst pc = cload(Rp.pc, br.r);
    const Geom g = cload(Rp.geom, br.r);
    const int *__restrict__ cstart = cstart_all + cload(Rp.cell_off, br.r);
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    const double rai = rhoA[i];
    const double k2 = -2.0 * pc.wrho * pc.inv_rd;  // w_rho'(r) = k2 (1 - r / r_d)
    double ax = 0, ay = 0, az = 0;
    for_each_neighbor<P>(pc, g, i, sub, xi, yi, zi, xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                         [&](int j, double dx, double dy, double dz, bool near) {
        if (!near) return;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 > 0.0)) return;
        const double rinv = rsqrt_f64(r2);
        const double r = r2 * rinv;
        const double c = (rai + ld(rhoA, j)) * k2 * (1.0 - r * pc.inv_rd) * rinv;
        ax += c * dx;
        ay += c * dy;
        az += c * dz;
    });
    ax = group_sum<P>(ax);
    ay = group_sum<P>(ay);
    az = group_sum<P>(az);
    if (sub != 0) return;
    X.x[i] += ax;
    X.y[i] += ay;
    X.z[i] += az;
}

// Drift adjoint (U += dt X for fluid) and reorder by particle id.
__global__ __launch_bounds__(kBlock) void k_adj_scatter(int n, double dt, const uint32_t *__restrict__ tag,
                                                       Soa3c X, Soa3c U, Soa3 Xid, Soa3 Uid)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t tg = tag[i];
    const size_t id = tg & kIdMask;
    const double x = X.x[i], y = X.y[i], z = X.z[i];
    Xid.x[id] = x;
    Xid.y[id] = y;
    Xid.z[id] = z;
    if (tg & kFrozenBit) {
        Uid.x[id] = Uid.y[id] = Uid.z[id] = 0.0;
    } else {
        Uid.x[id] = U.x[i] + dt * x;
        Uid.y[id] = U.y[i] + dt * y;
        Uid.z[id] = U.z[i] + dt * z;
    }
}

__global__ __launch_bounds__(kBlock) void k_adj_gather(int n, const uint32_t *__restrict__ tag, Soa3c Xid,
                                                      Soa3c Uid, Soa3 X, Soa3 U)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t id = tag[i] & kIdMask;
    X.x[i] = Xid.x[id];
    X.y[i] = Xid.y[id];
    X.z[i] = Xid.z[id];
    U.x[i] = Uid.x[id];
    U.y[i] = Uid.y[id];
    U.z[i] = Uid.z[id];
}

// Parameter shares: for one (quantity q, type a) pass, block partials of
// sum over particles i of type a of gp[q][b][i], for every b < T.
constexpr int kAdjRedBlocks = 512;

__global__ __launch_bounds__(kBlock) void k_adj_params(int n, int T, int q, int a, const uint8_t *__restrict__ typ,
                                                      const double *__restrict__ gp, double *__restrict__ part)
{
    __shared__ double sh[MDPD_ADJ_MAX_TYPES][kBlock];
    double acc[MDPD_ADJ_MAX_TYPES];
#pragma unroll
    for (int b = 0; b < MDPD_ADJ_MAX_TYPES; ++b) acc[b] = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        if (T > 1 && (int)typ[i] != a) continue;
#pragma unroll
        for (int b = 0; b < MDPD_ADJ_MAX_TYPES; ++b)
            if (b < T) acc[b] += gp[(size_t)(q * T + b) * n + i];
    }
#pragma unroll
    for (int b = 0; b < MDPD_ADJ_MAX_TYPES; ++b) sh[b][threadIdx.x] = acc[b];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int b = 0; b < T; ++b) sh[b][threadIdx.x] += sh[b][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int b = 0; b < T; ++b) part[(size_t)b * gridDim.x + blockIdx.x] = sh[b][0];
}

// total[q][a][b] += sum over blocks (fixed order) of the partials.
__global__ __launch_bounds__(kBlock) void k_adj_params_final(int nb, int T, int q, int a,
                                                            const double *__restrict__ part,
                                                            double *__restrict__ total)
{
    __shared__ double sh[kBlock];
    for (int b = 0; b < T; ++b) {
        double s = 0.0;
        for (int k = threadIdx.x; k < nb; k += kBlock) s += part[(size_t)b * nb + k];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) total[q * 64 + a * T + b] += sh[0];
        __syncthreads();
    }
}

}  // namespace

void launch_adj_seed(hipStream_t st, int n, const AdjConst &ac, Soa3c v, const uint32_t *tag, Soa3 U, Soa3 fb,
                     double *rhoA)
{
    if (n > 0) k_adj_seed<<<blocks_for(n), kBlock, 0, st>>>(n, ac, v, tag, U, fb, rhoA);
}

void launch_adj_force(hipStream_t st, int lanes, bool fp32, bool mt, int n, const Reps &R, uint32_t step,
                      const AdjConst &ac, Soa3c xs, Soa3c u, const void *rho, const uint32_t *tag,
                      const uint8_t *typ, const int *cstart, const int *ncnt, const uint32_t *nl, Soa3c fb,
                      Soa3 X, Soa3 U, double *rhoA, double *gp)
{
    if (n <= 0) return;
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        const int nb = R.nblk[lanes_index(L)];
        if (fp32) {
            if (mt)
                k_adj_force<L, true, float><<<nb, kBlock, 0, st>>>(R, step, ac, n, xs, u, (const float *)rho, tag,
                                                                   typ, cstart, ncnt, nl, fb, X, U, rhoA, gp);
            else
                k_adj_force<L, false, float><<<nb, kBlock, 0, st>>>(R, step, ac, n, xs, u, (const float *)rho,
                                                                    tag, typ, cstart, ncnt, nl, fb, X, U, rhoA,
                                                                    gp);
        } else {
            if (mt)
                k_adj_force<L, true, double><<<nb, kBlock, 0, st>>>(R, step, ac, n, xs, u, (const double *)rho,
                                                                    tag, typ, cstart, ncnt, nl, fb, X, U, rhoA,
                                                                    gp);
            else
                k_adj_force<L, false, double><<<nb, kBlock, 0, st>>>(R, step, ac, n, xs, u, (const double *)rho,
                                                                     tag, typ, cstart, ncnt, nl, fb, X, U, rhoA,
                                                                     gp);
        }
    });
}

void launch_adj_density(hipStream_t st, int lanes, const Reps &R, Soa3c xs, const int *cstart, const int *ncnt,
                        const uint32_t *nl, const double *rhoA, Soa3 X)
{
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        const int nb = R.nblk[lanes_index(L)];
        if (nb > 0) k_adj_density<L><<<nb, kBlock, 0, st>>>(R, xs, cstart, ncnt, nl, rhoA, X);
    });
}

void launch_adj_scatter(hipStream_t st, int n, double dt, const uint32_t *tag, Soa3c X, Soa3c U, Soa3 Xid,
                        Soa3 Uid)
{
    if (n > 0) k_adj_scatter<<<blocks_for(n), kBlock, 0, st>>>(n, dt, tag, X, U, Xid, Uid);
}

void launch_adj_gather(hipStream_t st, int n, const uint32_t *tag, Soa3c Xid, Soa3c Uid, Soa3 X, Soa3 U)
{
    if (n > 0) k_adj_gather<<<blocks_for(n), kBlock, 0, st>>>(n, tag, Xid, Uid, X, U);
}

int adj_param_partials(int ntypes) { return kAdjRedBlocks * ntypes; }

void launch_adj_params(hipStream_t st, int n, int ntypes, const uint8_t *typ, const double *gp, double *part,
                       double *total)
{
    if (n <= 0) return;
    const int nb = blocks_for(n) < kAdjRedBlocks ? blocks_for(n) : kAdjRedBlocks;
    for (int q = 0; q < 3; ++q)
        for (int a = 0; a < ntypes; ++a) {
            k_adj_params<<<nb, kBlock, 0, st>>>(n, ntypes, q, a, typ, gp, part);
            k_adj_params_final<<<1, kBlock, 0, st>>>(nb, ntypes, q, a, part, total);
        }
}

}  // namespace mdpd
