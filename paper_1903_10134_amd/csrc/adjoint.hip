// adjoint.hip -- reverse-mode derivative of one mDPD timestep (the adjoint
// of the pair passes and of velocity-Verlet), for gradients of trajectory
// losses with respect to the pair tables A, B, gamma and the initial state.
//
// Forward recurrence of one step n, with u_n the half-step velocity
// v(t_n + dt/2) and h = dt / (2 m) (a particle the bounce-back wall corrector
// sends back instead keeps x_n = x_{n-1} and moves on with -u_{n-1}):
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
// With the fluid-solid dissipation control (DC) a fluid particle's
// fluid-solid pairs carry gamma s_i and sigma sqrt(s_i), s_i = dctl / S_i,
// S_i = sum over its neighbours of w_c^2: k_adj_dscale computes s_i and
// s_i / S_i per state, k_adj_force scales those pairs and returns
// a_i = dL/dS_i = -(s_i / S_i) dL/ds_i, and k_adj_density adds
// X_i += sum_j (a_i + a_j) 2 w_c w_c' e_ij over every neighbour.
//   k_adj_step_back  U += dt X (drift) and X, U into the sorted order of
//                  step n - 1 through the recorded sort permutation
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

// Replica and slot of thread threadIdx.x in a replica-aligned block of
// kBlock particles (lane count 1); i >= i1 means no particle.
__device__ __forceinline__ BlockRep elem_rep(const Reps &R) { return block_rep<1>(R, blockIdx.x); }

__global__ __launch_bounds__(kBlock) void k_adj_seed(Reps Rp, const AdjConst *__restrict__ act, Soa3c v,
                                                    const uint32_t *__restrict__ tag, Soa3 U, Soa3 fb,
                                                    double *__restrict__ rhoA)
{
    const BlockRep br = elem_rep(Rp);
    const int i = br.i0 + (int)threadIdx.x;
    if (i >= br.i1) return;
    if (tag[i] & kFrozenBit) {
        U.x[i] = U.y[i] = U.z[i] = 0.0;
        fb.x[i] = fb.y[i] = fb.z[i] = 0.0;
        rhoA[i] = 0.0;
        return;
    }
    const AdjConst ac = cload(act, br.r);
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

// DC: s_i = dctl / S_i and s_i / S_i of every fluid particle (1 and 0
// without the control, for frozen particles and for S_i = 0).
template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_dscale(Reps Rp, Soa3c xs, const uint32_t *__restrict__ tag,
                                                      const int *__restrict__ cstart_all,
                                                      const int *__restrict__ ncnt,
                                                      const uint32_t *__restrict__ nl, double *__restrict__ sdc,
                                                      double *__restrict__ qdc)
{
    const BlockRep br = block_rep<P>(Rp, xcd_block());
    const int i = br.i0 + (int)threadIdx.x / P;
    const int sub = threadIdx.x & (P - 1);
    if (i >= br.i1) return;
    const PairConst pc = cload(Rp.pc, br.r);
    if (!(pc.dctl > 0.0) || (tag[i] & kFrozenBit)) {
        if (sub == 0) {
            sdc[i] = 1.0;
            qdc[i] = 0.0;
        }
        return;
    }
    const Geom g = cload(Rp.geom, br.r);
    const int *__restrict__ cstart = cstart_all + cload(Rp.cell_off, br.r);
    double S = 0.0;
    for_each_neighbor<P>(pc, g, i, sub, xs.x[i], xs.y[i], xs.z[i], xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                         [&](int, double dx, double dy, double dz, bool) {
        const double r = __builtin_sqrt(dx * dx + dy * dy + dz * dz);
        const double w = 1.0 - r * pc.inv_rc;
        S += w * w;
    });
    S = group_sum<P>(S);
    if (sub == 0) {
        const double si = S > 0.0 ? pc.dctl / S : 1.0;
        sdc[i] = si;
        qdc[i] = S > 0.0 ? si / S : 0.0;
    }
}

// One type: the register budget of three waves per SIMD (at most 168 VGPRs,
// against 175 unbounded, so two waves) costs 12 bytes of spills in the FP32
// form and none in FP64, and the batched backward pass runs 7% faster; with
// the type tables that budget would spill hundreds of bytes, so those keep
// theirs.
template <int P, bool MT, bool DC, typename R>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MT ? 1 : 3))) void k_adj_force(Reps Rp, uint32_t step, const AdjConst *__restrict__ act,
                                                     int n, int tmax, Soa3c xs,
                                                     Soa3c u, const R *__restrict__ rho,
                                                     const uint32_t *__restrict__ tag,
                                                     const uint8_t *__restrict__ typ,
                                                     const int *__restrict__ cstart_all,
                                                     const int *__restrict__ ncnt,
                                                     const uint32_t *__restrict__ nl, Soa3c fb, Soa3 X, Soa3 U,
                                                     double *__restrict__ rhoA, double *__restrict__ gp,
                                                     const double *__restrict__ sdc,
                                                     const double *__restrict__ qdc, double *__restrict__ adc)
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
    const AdjConst ac = cload(act, br.r);
    const uint32_t tgi = tag[i];
    const bool fzi = (tgi & kFrozenBit) != 0;
    const uint32_t idi = tgi & kIdMask;
    const double xi = xs.x[i], yi = xs.y[i], zi = xs.z[i];
    const double uxi = fzi ? 0.0 : u.x[i], uyi = fzi ? 0.0 : u.y[i], uzi = fzi ? 0.0 : u.z[i];
    const double fxi = fb.x[i], fyi = fb.y[i], fzi_ = fb.z[i];
    const double rhoi = (double)rho[i];
    const int T = MT ? pc.ntypes : 1;  // this replica's types (shares stored with stride tmax)
    const int ti = MT ? (int)typ[i] : 0;
    const double wP = ac.wP_3V;
    double ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0, ar = 0;
    double cs = 0.0;  // DC: dL/ds_i over i's fluid-solid pairs
    const bool dc_on = DC && pc.dctl > 0.0;
    const double si = dc_on && !fzi ? sdc[i] : 1.0;
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
        // DC: a fluid-solid pair takes gamma s and sigma sqrt(s), s of its fluid end
        double sp = 1.0;
        if (dc_on && fzi != fzj) sp = fzj ? si : ld(sdc, j);
        const double rsp = dc_on ? __builtin_sqrt(sp) : 1.0;
        const double gam = pt.gam * sp, sig = pt.sig * rsp;
        const double fc = pt.A * wc + Bn * rs * wd;
        const double fs = fc - gam * wc * wc * ev + sig * wc * th;
        const double gE = gx * ex + gy * ey + gz * ez;
        // derivatives of fs in r (at fixed e.u_ij) and in e.u_ij
        const double dfc_dr = -pt.A * pc.inv_rc - Bn * rs * pc.inv_rd;
        const double dfs_dr = dfc_dr + 2.0 * gam * wc * ev * pc.inv_rc - sig * th * pc.inv_rc;
        const double dfs_dev = -gam * wc * wc;
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
        const double sG = 0.5 * gE * (-sp * wc * wc * ev + rsp * dsig * wc * th);
        if (dc_on && !fzi && fzj)  // d/ds of s (-gamma w^2 ev) + sqrt(s) sigma w th, along g
            cs += gE * (-pt.gam * wc * wc * ev + 0.5 / rsp * pt.sig * wc * th);
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
    if (dc_on) cs = group_sum<P>(cs);
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
    if constexpr (DC) adc[i] = dc_on && !fzi ? -qdc[i] * cs : 0.0;  // dL/dS_i
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        if (k < T) {
            gp[(size_t)(0 * tmax + k) * n + i] = pA[k];
            gp[(size_t)(1 * tmax + k) * n + i] = pB[k];
            gp[(size_t)(2 * tmax + k) * n + i] = pG[k];
        }
    }
}

template <int P, bool DC>
__global__ __launch_bounds__(kBlock) void k_adj_density(Reps Rp, Soa3c xs, const int *__restrict__ cstart_all,
                                                       const int *__restrict__ ncnt,
                                                       const uint32_t *__restrict__ nl,
                                                       const double *__restrict__ rhoA, Soa3 X,
                                                       const double *__restrict__ adc)
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
    const double aai = DC ? adc[i] : 0.0;
    double ax = 0, ay = 0, az = 0;
    for_each_neighbor<P>(pc, g, i, sub, xi, yi, zi, xs, cstart, ncnt[i], nl + (size_t)i * kListCap,
                         [&](int j, double dx, double dy, double dz, bool near) {
        if (!DC && !near) return;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (!(r2 > 0.0)) return;
        const double rinv = rsqrt_f64(r2);
        const double r = r2 * rinv;
        double c = near ? (rai + ld(rhoA, j)) * k2 * (1.0 - r * pc.inv_rd) * rinv : 0.0;
        if constexpr (DC) {
            // dS/dx through w_c^2: 2 w_c w_c' e, w_c' = -1/r_c
            c += (aai + ld(adc, j)) * 2.0 * (1.0 - r * pc.inv_rc) * (-pc.inv_rc) * rinv;
        }
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

// Drift adjoint (U += dt X for fluid) and the reorder from the sorted order
// of step n to that of step n - 1 through the recorded sort permutation (the
// particles barely move between steps, so perm is close to the identity and
// the reads stay almost coalesced).  A particle the wall corrector sent back
// in step n (corr[part_off[r] + id] != 0) kept x and had its half-step
// velocity negated: its U is negated and gets no dt X.
__global__ __launch_bounds__(kBlock) void k_adj_step_back(Reps Rp, const AdjConst *__restrict__ act,
                                                         const uint32_t *__restrict__ tag_prev,
                                                         const int *__restrict__ perm, Soa3c X, Soa3c U,
                                                         Soa3 Xo, Soa3 Uo, const uint8_t *__restrict__ corr)
{
    const BlockRep br = elem_rep(Rp);
    const int i = br.i0 + (int)threadIdx.x;
    if (i >= br.i1) return;
    const double dt = cload(act, br.r).dt;
    const uint32_t tg = tag_prev[i];
    const int k = perm[i];
    const double x = X.x[k], y = X.y[k], z = X.z[k];
    Xo.x[i] = x;
    Xo.y[i] = y;
    Xo.z[i] = z;
    if (tg & kFrozenBit) {
        Uo.x[i] = Uo.y[i] = Uo.z[i] = 0.0;
    } else if (corr && corr[(size_t)cload(Rp.part_off, br.r) + (tg & kIdMask)]) {
        Uo.x[i] = -U.x[k];
        Uo.y[i] = -U.y[k];
        Uo.z[i] = -U.z[k];
    } else {
        Uo.x[i] = U.x[k] + dt * x;
        Uo.y[i] = U.y[k] + dt * y;
        Uo.z[i] = U.z[k] + dt * z;
    }
}

// Parameter shares, first level: for each replica-aligned block of kBlock
// particles and each (quantity q, type a of i, type b of j) the fixed-order
// block sum of gp over the block's particles of type a.  part holds
// 3 * tmax * tmax sums per block.
__global__ __launch_bounds__(kBlock) void k_adj_params(Reps Rp, int n, int tmax,
                                                      const uint8_t *__restrict__ typ,
                                                      const double *__restrict__ gp, double *__restrict__ part)
{
    __shared__ double sh[kBlock];
    const BlockRep br = elem_rep(Rp);
    const int i = br.i0 + (int)threadIdx.x;
    const bool in = i < br.i1;
    const int T = cload(Rp.pc, br.r).ntypes;
    const int ti = in ? (int)typ[i] : -1;
    double *out = part + (size_t)blockIdx.x * 3 * tmax * tmax;
    for (int q = 0; q < 3; ++q)
        for (int a = 0; a < T; ++a)
            for (int b = 0; b < T; ++b) {
                sh[threadIdx.x] = (in && ti == a) ? gp[(size_t)(q * tmax + b) * n + i] : 0.0;
                __syncthreads();
                for (int w = kBlock / 2; w > 0; w >>= 1) {
                    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
                    __syncthreads();
                }
                if (threadIdx.x == 0) out[(q * tmax + a) * tmax + b] = sh[0];
                __syncthreads();
            }
}

// Second level, one block per replica: gtot[r][q][a T + b] += sum over the
// replica's blocks in order.
__global__ __launch_bounds__(kBlock) void k_adj_params_final(Reps Rp, int tmax, const double *__restrict__ part,
                                                            double *__restrict__ gtot)
{
    const int r = blockIdx.x;
    const int T = cload(Rp.pc, r).ntypes;
    const int *boff = Rp.blk_off;  // lane count 1
    const int b0 = cload(boff, r), b1 = cload(boff, r + 1);
    const int e = threadIdx.x;
    if (e >= 3 * T * T) return;
    const int q = e / (T * T), a = (e / T) % T, b = e % T;
    double s = 0.0;
    for (int k = b0; k < b1; ++k) s += part[(size_t)k * 3 * tmax * tmax + (q * tmax + a) * tmax + b];
    gtot[(size_t)r * 3 * 64 + q * 64 + a * T + b] += s;
}

}  // namespace

void launch_adj_seed(hipStream_t st, const Reps &R, const AdjConst *ac, Soa3c v, const uint32_t *tag, Soa3 U,
                     Soa3 fb, double *rhoA)
{
    if (R.nblk[0] > 0) k_adj_seed<<<R.nblk[0], kBlock, 0, st>>>(R, ac, v, tag, U, fb, rhoA);
}

void launch_adj_dscale(hipStream_t st, int lanes, const Reps &R, Soa3c xs, const uint32_t *tag, const int *cstart,
                       const int *ncnt, const uint32_t *nl, double *sdc, double *qdc)
{
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        const int nb = R.nblk[lanes_index(L)];
        if (nb > 0) k_adj_dscale<L><<<nb, kBlock, 0, st>>>(R, xs, tag, cstart, ncnt, nl, sdc, qdc);
    });
}

void launch_adj_force(hipStream_t st, int lanes, bool fp32, bool mt, bool dc, int n, int tmax, const Reps &R,
                      uint32_t step, const AdjConst *ac, Soa3c xs, Soa3c u, const void *rho, const uint32_t *tag,
                      const uint8_t *typ, const int *cstart, const int *ncnt, const uint32_t *nl, Soa3c fb,
                      Soa3 X, Soa3 U, double *rhoA, double *gp, const double *sdc, const double *qdc, double *adc)
{
    if (n <= 0) return;
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        const int nb = R.nblk[lanes_index(L)];
        auto go = [&](auto mtc, auto dcc, auto rc) {
            constexpr bool M = decltype(mtc)::value;
            constexpr bool D = decltype(dcc)::value;
            using RT = typename decltype(rc)::type;
            k_adj_force<L, M, D, RT><<<nb, kBlock, 0, st>>>(R, step, ac, n, tmax, xs, u, (const RT *)rho, tag, typ,
                                                            cstart, ncnt, nl, fb, X, U, rhoA, gp, sdc, qdc, adc);
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

void launch_adj_density(hipStream_t st, int lanes, const Reps &R, Soa3c xs, const int *cstart, const int *ncnt,
                        const uint32_t *nl, const double *rhoA, Soa3 X, const double *adc)
{
    launch_lanes(lanes, [&](auto P) {
        constexpr int L = decltype(P)::value;
        const int nb = R.nblk[lanes_index(L)];
        if (nb <= 0) return;
        if (adc) k_adj_density<L, true><<<nb, kBlock, 0, st>>>(R, xs, cstart, ncnt, nl, rhoA, X, adc);
        else k_adj_density<L, false><<<nb, kBlock, 0, st>>>(R, xs, cstart, ncnt, nl, rhoA, X, nullptr);
    });
}

void launch_adj_step_back(hipStream_t st, const Reps &R, const AdjConst *ac, const uint32_t *tag_prev,
                          const int *perm, Soa3c X, Soa3c U, Soa3 Xo, Soa3 Uo, const uint8_t *corr)
{
    if (R.nblk[0] > 0) k_adj_step_back<<<R.nblk[0], kBlock, 0, st>>>(R, ac, tag_prev, perm, X, U, Xo, Uo, corr);
}

int adj_param_partials(const Reps &R, int tmax) { return (R.nblk[0] + 1) * 3 * tmax * tmax; }

void launch_adj_params(hipStream_t st, const Reps &R, int n, int tmax, const uint8_t *typ, const double *gp,
                       double *part, double *gtot)
{
    if (n <= 0 || R.nblk[0] <= 0) return;
    k_adj_params<<<R.nblk[0], kBlock, 0, st>>>(R, n, tmax, typ, gp, part);
    k_adj_params_final<<<R.nrep, kBlock, 0, st>>>(R, tmax, part, gtot);
}

}  // namespace mdpd
