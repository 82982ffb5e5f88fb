// Reverse-mode (adjoint) kernels of one predictor-corrector step.
//
// Forward step (fluid particles):  v = u + dt/2 a;  x' = x + dt v;
// a' = A(x', v; nu);  u' = v + dt/2 a'.  With lhat = lam_a' + dt/2 lam_u'
// (the adjoint reaching a'), the reverse needs (dA/dx')^T lhat,
// (dA/dv)^T lhat and (dA/dnu)^T lhat.  A_i sums pair terms
//   T_ij = m_j [ -(P_i + P_j) F(r) r_ij + 4 nu G(r)/(rho_i + rho_j) v_ij ],
//   F = (dW/dr)/r,  G = F r^2/(r^2 + eta h^2),
// and P_k = p(rho_k)/rho_k^2 with rho_k = sum_l m_l W(r_kl).
//
// Both ends of a pair are written by gathering over the neighbour set of the
// destination: the predicate is exactly symmetric (r_ji = -r_ij bitwise), so
// the transpose of "i gathers from j" is "j gathers from i" and no scatter or
// atomic is needed.  With w = m_j lhat_i - m_i lhat_j the pair (i, j)
// contributes to particle i:
//   lam_x  += -(P_i+P_j) (F w + F1 (r.w) r) + 4 nu/(rho_i+rho_j) G1 (v_ij.w) r
//   lam_v  += 4 nu G/(rho_i+rho_j) w
//   lam_P  += -F (r.w)
//   lam_rho+= -4 nu G/(rho_i+rho_j)^2 (v_ij.w)
//   lam_nu += 4 m_j G/(rho_i+rho_j) (lhat_i.v_ij)
// with F1 = (d2W/dr2 - F)/r^2 and G1 = (dG/dr)/r.  A second gather maps
// lam_rho (including lam_P dP/drho) to positions:
//   lam_x_i += sum_j (lam_rho_i m_j + lam_rho_j m_i) F r_ij.
#pragma once

#include "sph_kernels.hpp"

namespace sph {

// F = (dW/dr)/r and F1 = (d2W/dr2 - F)/r^2 as functions of q = r/h.
//   cubic, q < 1:  F = s2 (-3 + 2.25 q),          F1 = s4 2.25 / q
//   cubic, q < 2:  F = -0.75 s2 (2-q)^2 / q,       F1 = s4 (1.5 (2-q) + 0.75 (2-q)^2/q) / q^2
//   Wendland:      F = -5 s2 (1-q/2)^3,            F1 = 7.5 s4 (1-q/2)^2 / q
//   quintic, q < 1: F = s2 (-120 + q^2 (120 - 50 q)), F1 = s4 (240 - 150 q)
//   quintic, q < 3: F = s2 w'/q,                   F1 = s4 (w'' - w'/q) / q^2
//     w' = -5 (3-q)^4 + 30 (2-q)_+^4,  w'' = 20 (3-q)^3 - 120 (2-q)_+^3
// with s2 = sigma/h^2, s4 = sigma/h^4.
template <int KERNEL, typename T>
__device__ __forceinline__ void kernel_f_f1(T q, T inv_q, T s2, T s4, T* F, T* F1) {
    if (KERNEL == 2) {
        if (q < T(1)) {
            *F = s2 * (T(-120) + q * q * (T(120) - T(50) * q));
            *F1 = s4 * (T(240) - T(150) * q);
        } else {
            const T t3 = T(3) - q, t2 = pos_part(T(2) - q);
            const T dw = quintic_dw(q);
            const T d2w = T(20) * t3 * t3 * t3 - T(120) * t2 * t2 * t2;
            *F = s2 * dw * inv_q;
            *F1 = s4 * (d2w - dw * inv_q) * inv_q * inv_q;
        }
    } else if (KERNEL == 0) {
        if (q < T(1)) {
            *F = s2 * (T(-3) + T(2.25) * q);
            *F1 = s4 * T(2.25) * inv_q;
        } else {
            const T t = T(2) - q;
            *F = T(-0.75) * s2 * t * t * inv_q;
            *F1 = s4 * (T(1.5) * t + T(0.75) * t * t * inv_q) * inv_q * inv_q;
        }
    } else {
        const T t = T(1) - T(0.5) * q;
        *F = T(-5) * s2 * t * t * t;
        *F1 = T(7.5) * s4 * t * t * inv_q;
    }
}

// lhat = lam_a + dt/2 lam_u for fluid particles (0 for walls), packed as a
// pair record.  Source index of slot s is gather[s] (identity if null).
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void k_adj_seed(int n, const double* __restrict__ lam_u,
                                                     const double* __restrict__ lam_a, int64_t ld,
                                                     double hdt, const uint8_t* __restrict__ type,
                                                     const uint32_t* __restrict__ gather,
                                                     typename Vec4<T>::type* __restrict__ lhat) {
#pragma clang fp contract(off)
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int64_t src = gather ? (int64_t)gather[s] : (int64_t)s;
    T l[3] = {T(0), T(0), T(0)};
    if (type[s] == 0) {
        for (int k = 0; k < DIM; ++k) {
            double v = lam_a[k * ld + src];
            if (lam_u) v += hdt * lam_u[k * ld + src];
            l[k] = (T)v;
        }
    }
    typename Vec4<T>::type r;
    r.x = l[0]; r.y = l[1]; r.z = l[2]; r.w = T(0);
    lhat[s] = r;
}

// First gather: direct position and velocity adjoints, lam_rho, nu partials.
template <int DIM, int SR, int KERNEL, typename T>
__global__ __launch_bounds__(kBlock) void k_adj_pair1(
    int n, Grid G, PairConst<T> C, const uint32_t* __restrict__ skey,
    const typename Rec<T>::type* __restrict__ pos, const typename Vec4<T>::type* __restrict__ vel,
    const typename Vec2<T>::type* __restrict__ rp, const typename Vec4<T>::type* __restrict__ lhat,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend,
    const uint32_t* __restrict__ list, const uint32_t* __restrict__ ncnt, uint32_t cap,
    double* __restrict__ lx, double* __restrict__ lv, T* __restrict__ lrho,
    double* __restrict__ nupart) {
    const int i = xcd_block() * kBlock + threadIdx.x;
    if (i >= n) return;
    const typename Rec<T>::type ri = pos[i];
    const typename Vec4<T>::type vi = vel[i];
    const typename Vec2<T>::type rpi = load_rp<DIM, T>(vi, rp, (uint32_t)i);
    const typename Vec4<T>::type li = lhat[i];
    const T h = p_rcp(C.inv_h);
    const T mi = rec_mass(ri);
    T gx = 0, gy = 0, gz = 0, hx = 0, hy = 0, hz = 0, lP = 0, lR = 0, nu_acc = 0;
    struct Pay {
        typename Vec4<T>::type v;
        typename Vec2<T>::type rp;
        typename Vec4<T>::type l;
    };
    for_each_neighbor_p<DIM, SR, T>(
        i, G, C, ri, pos, skey, cstart, cend, (uint32_t)n, list, ncnt, cap,
        [&](uint32_t j) {
            typename Vec4<T>::type v = vel[j];
            keep_whole<DIM>(v);
            return Pay{v, load_rp<DIM, T>(v, rp, j), lhat[j]};
        },
        [&](uint32_t j, const typename Rec<T>::type& rj, const Pay& pj, const Geom<T>& g) {
            const T r2 = g.r2;
            const T dx = g.d[0], dy = g.d[1], dz = g.d[2];
            if (j == (uint32_t)i || r2 == T(0)) return;
            const typename Vec4<T>::type vj = pj.v;
            const typename Vec2<T>::type rpj = pj.rp;
            const typename Vec4<T>::type lj = pj.l;
            const T r = p_sqrt(r2);
            const T inv_r = p_rcp(r);
            const T q = r * C.inv_h;
            const T inv_q = h * inv_r;
            T F, F1;
            kernel_f_f1<KERNEL, T>(q, inv_q, C.sigma_h2, C.sigma_h4, &F, &F1);
            const T inv_den = p_rcp(r2 + C.eta_h2);
            const T Gv = F * r2 * inv_den;
            const T G1 = F1 * r2 * inv_den + T(2) * F * C.eta_h2 * inv_den * inv_den;
            const T inv_rs = p_rcp(rpi.x + rpj.x);
            const T c4 = C.four_nu * inv_rs;
            const T mj = rec_mass(rj);
            const T wx = mj * li.x - mi * lj.x;
            const T wy = mj * li.y - mi * lj.y;
            const T wz = DIM == 3 ? mj * li.z - mi * lj.z : T(0);
            const T vx = vi.x - vj.x, vy = vi.y - vj.y, vz = DIM == 3 ? vi.z - vj.z : T(0);
            const T rw = dx * wx + dy * wy + (DIM == 3 ? dz * wz : T(0));
            const T vw = vx * wx + vy * wy + (DIM == 3 ? vz * wz : T(0));
            const T Ps = rpi.y + rpj.y;
            const T cr = -Ps * F1 * rw + c4 * G1 * vw;
            const T cw = -Ps * F;
            gx += cw * wx + cr * dx;
            gy += cw * wy + cr * dy;
            const T cv = c4 * Gv;
            hx += cv * wx;
            hy += cv * wy;
            if (DIM == 3) {
                gz += cw * wz + cr * dz;
                hz += cv * wz;
            }
            lP -= F * rw;
            lR -= cv * inv_rs * vw;
            const T lv_ = li.x * vx + li.y * vy + (DIM == 3 ? li.z * vz : T(0));
            nu_acc += T(4) * mj * Gv * inv_rs * lv_;
        });
    // dP/drho = p'(rho)/rho^2 - 2 P / rho,  p'(rho) = 7 B (rho/rho0)^6 / rho0
    const T rho = rpi.x;
    const T rr = rho * C.inv_rho0;
    const T rr2 = rr * rr;
    const T dP = C.b7 * rr2 * rr2 * rr2 / (rho * rho) - T(2) * rpi.y / rho;
    lrho[i] = lR + lP * dP;
    lx[i] = (double)gx;
    lx[(int64_t)n + i] = (double)gy;
    lv[i] = (double)hx;
    lv[(int64_t)n + i] = (double)hy;
    if (DIM == 3) {
        lx[2 * (int64_t)n + i] = (double)gz;
        lv[2 * (int64_t)n + i] = (double)hz;
    }
    nupart[i] = (double)nu_acc;
}

// Second gather: lam_x_i += sum_j (lam_rho_i m_j + lam_rho_j m_i) F r_ij.
template <int DIM, int SR, int KERNEL, typename T>
__global__ __launch_bounds__(kBlock) void k_adj_pair2(
    int n, Grid G, PairConst<T> C, const uint32_t* __restrict__ skey,
    const typename Rec<T>::type* __restrict__ pos, const T* __restrict__ lrho,
    const uint32_t* __restrict__ cstart, const uint32_t* __restrict__ cend,
    const uint32_t* __restrict__ list, const uint32_t* __restrict__ ncnt, uint32_t cap,
    double* __restrict__ lx) {
    const int i = xcd_block() * kBlock + threadIdx.x;
    if (i >= n) return;
    const typename Rec<T>::type ri = pos[i];
    const T lri = lrho[i];
    const T mi = rec_mass(ri);
    T ax = 0, ay = 0, az = 0;
    for_each_neighbor_p<DIM, SR, T>(
        i, G, C, ri, pos, skey, cstart, cend, (uint32_t)n, list, ncnt, cap,
        [&](uint32_t j) { return lrho[j]; },
        [&](uint32_t j, const typename Rec<T>::type& rj, const T& lrj, const Geom<T>& g) {
            if (j == (uint32_t)i || g.r2 == T(0)) return;
            const T q = p_sqrt(g.r2) * C.inv_h;
            const T F = kernel_f<KERNEL, T>(q, C.sigma_h2);
            const T c = (lri * rec_mass(rj) + lrj * mi) * F;
            ax += c * g.d[0];
            ay += c * g.d[1];
            if (DIM == 3) az += c * g.d[2];
        });
    lx[i] += (double)ax;
    lx[(int64_t)n + i] += (double)ay;
    if (DIM == 3) lx[2 * (int64_t)n + i] += (double)az;
}

// Reverse of the kicks and the drift, written in the order before the sort:
//   lam_x' = lam_x_in + (dA/dx')^T lhat;  lam_v = lam_u_in + (dA/dv)^T lhat + dt lam_x'
//   out: lam_x = lam_x', lam_u = lam_v, lam_a = dt/2 lam_v   (walls: 0).
// Layout of lam buffers: [x (dim arrays)][u (dim arrays)][a (dim arrays)].
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_adj_kick(int n, const double* __restrict__ lam_in,
                                                     const double* __restrict__ lxd,
                                                     const double* __restrict__ lvd,
                                                     const uint8_t* __restrict__ type,
                                                     const uint32_t* __restrict__ perm, double dt,
                                                     double hdt, double* __restrict__ lam_out) {
#pragma clang fp contract(off)
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int64_t d = perm[s];
    const int64_t N = n;
    const bool fluid = type[s] == 0;
    for (int k = 0; k < DIM; ++k) {
        double lxp = 0.0, lvv = 0.0;
        if (fluid) {
            lxp = lam_in[k * N + s] + lxd[k * N + s];
            lvv = lam_in[(DIM + k) * N + s] + lvd[k * N + s];
            lvv = lvv + dt * lxp;
        }
        lam_out[k * N + d] = lxp;
        lam_out[(DIM + k) * N + d] = lvv;
        lam_out[(2 * DIM + k) * N + d] = hdt * lvv;
    }
}

// Adjoint of one acceleration evaluation, added in the order before the sort:
// lam_x[perm[s]] += lxd[s], lam_u[perm[s]] += lvd[s] (fluid only).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_adj_accum(int n, const double* __restrict__ lxd,
                                                      const double* __restrict__ lvd,
                                                      const uint8_t* __restrict__ type,
                                                      const uint32_t* __restrict__ perm,
                                                      double* __restrict__ lam_x,
                                                      double* __restrict__ lam_u) {
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    if (type[s] != 0) return;
    const int64_t d = perm[s];
    const int64_t N = n;
    for (int k = 0; k < DIM; ++k) {
        lam_x[k * N + d] += lxd[k * N + s];
        lam_u[k * N + d] += lvd[k * N + s];
    }
}

// Adjoint seed of the objective J = scale * sum_i m_i |u_i|^2 / 2 at a state:
// lam_x = 0, lam_u = scale m u (walls carry u = 0), lam_a = 0, in the
// [lam_x | lam_u | lam_a] layout of sph_step_backward.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_ke_seed(int n, const double* __restrict__ ux,
                                                    const double* __restrict__ uy,
                                                    const double* __restrict__ uz,
                                                    const double* __restrict__ m, double scale,
                                                    double* __restrict__ lam) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t N = n;
    const double* u[3] = {ux, uy, uz};
    const double w = scale * m[i];
    for (int k = 0; k < DIM; ++k) {
        lam[k * N + i] = 0.0;
        lam[(DIM + k) * N + i] = w * u[k][i];
        lam[(2 * DIM + k) * N + i] = 0.0;
    }
}

// Fixed-order FP64 sum: per-block partials, then one block adds the total
// to *out.
static __global__ __launch_bounds__(kBlock) void k_sum_partial(int n, const double* __restrict__ v,
                                                        double* __restrict__ part) {
    __shared__ double sh[kBlock];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    sh[threadIdx.x] = i < n ? v[i] : 0.0;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

static __global__ __launch_bounds__(kBlock) void k_sum_accum(int nparts, const double* __restrict__ part,
                                                      double* __restrict__ out) {
    __shared__ double sh[kBlock];
    double v = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) v += part[b];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out += sh[0];
}

}  // namespace sph
