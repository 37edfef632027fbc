// HIP kernels of the single-component multiphase form of the Shan-Chen step
// with the evaporation boundary (the method carried over to the multiphase
// pseudopotential model, Sec. I of Hessling, Xie and Harting,
// arXiv:1701.03637): one component whose force of Eq. (sc) takes the
// component itself as the partner, F = -psi g sum_i w_i psi(x + e_i) e_i
// (g < 0 attracts), BGK towards Eq. (eqdis) with the velocity shifted by
// tau F / rho (Sec. II B), and sink nodes reset to f^eq(rho_H, 0) whose
// removed mass rho_pre - rho_H is booked as E (Sec. II C; with no partner the
// mass leaves the system).
//
// Storage: z-slab major like the two-component form, 19 planes of one
// element per node (FP64, or FP32 deviations f - w_i rho0 with the same
// exact mass bookkeeping as the two-component FP32S form). One launch per
// step; a block owns an xy tile and marches along z with a ring of three psi
// planes in LDS, the tile node's populations kept in registers from the
// density pass to the collision, halo nodes pulled for their density only.
#pragma once

#include "kernels.h"

namespace lbsc {

struct St1F64 { using T = double; using A = double; static constexpr bool kNode = false, kPair = false; };
struct St1F32S { using T = float; using A = float; static constexpr bool kNode = false, kPair = false; };
template <class S> constexpr bool kExact1 = std::is_same_v<S, St1F32S>;

// Slab elements per in-plane element of the single-component form.
constexpr int kSlabPlanes1 = kQ;

template <typename A>
struct Node1 {
    A f[kQ];
    A rho;    // rho0 + drho
    A drho;   // sum of the stored deviations
};

// Loads of the pull of node (x, y, z): f_i(x) = f*_i(x - e_i), or the
// reflected population of the node itself across a z-seam wall.
template <class S>
__device__ __forceinline__ void pull1(const typename S::T* __restrict__ src, const Inst& I, int x, int y, int z,
                                      Node1<typename S::A>& v)
{
    using T = typename S::T;
    const PullAddr<S> a(src, I, x, y, z);
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        v.f[i] = (typename S::A)bload<T>(a.rsrc(i), a.xy(i) * (uint32_t)sizeof(T),
                                         (uint32_t)a.q(i) * a.ps * (uint32_t)sizeof(T));
}

template <class S>
__device__ __forceinline__ void store1(typename S::T* __restrict__ dst, const Inst& I, int z, uint32_t xy,
                                       const Node1<typename S::A>& v)
{
    using T = typename S::T;
    const Rsrc dz = slab_rsrc(dst + (int64_t)z * I.slab);
    const uint32_t ps = (uint32_t)I.ps;
#pragma unroll
    for (int i = 0; i < kQ; ++i) bstore(narrow<T>(v.f[i]), dz, xy * (uint32_t)sizeof(T), (uint32_t)i * ps * sizeof(T));
}

template <typename A>
__device__ __forceinline__ void density1(const Inst& I, Node1<A>& v)
{
    A r = (A)0;
#pragma unroll
    for (int i = 0; i < kQ; ++i) r += v.f[i];
    v.drho = r;
    v.rho = Par<A>::shift(I, 0) + r;
}

// Evaporation boundary: f -> f^eq(rho_H, 0). Returns the mass removed,
// rho_pre - rho_H in FP64 (for FP32 storage the exact change of the stored
// mass, the new stored density being rho_H up to the rest's zero-mean
// rounding).
template <typename A, bool EX>
__device__ __forceinline__ double sink1(const Inst& I, Node1<A>& v, uint32_t key)
{
    const double rho_h = I.reset.rho_h;
    const double m = kPlain<A> ? (double)v.drho : sum64(v.f);
    A da = (A)(rho_h - I.shift[0]);
    asm volatile("" : "+v"(da));
#pragma unroll
    for (int i = 0; i < kQ; ++i) v.f[i] = (A)wgt(i) * da;
    double flux = I.shift[0] + m - rho_h;
    if constexpr (EX) {
        absorb_rest_exact(v.f, rho_h - I.shift[0], key);
        flux = m - sum64(v.f);
    }
    density1<A>(I, v);
    return flux;
}

// Neighbour sum S = sum_{i>0} w_i psi(x + e_i) e_i of Eq. (sc) from three LDS
// psi planes of footprint row stride `row` (tile column tx, row ty).
template <typename A>
__device__ __forceinline__ void force_sum1(const A* pm, const A* p0, const A* pp, int tx, int ty, int row, A S[3])
{
    A S1[3] = {0, 0, 0}, S2[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < kQ; i += 2) {
        const A* lp = ez(i) < 0 ? pm : (ez(i) > 0 ? pp : p0);
        const A* lm = ez(i) > 0 ? pm : (ez(i) < 0 ? pp : p0);
        const A d = lp[(ty + 1 + ey(i)) * row + tx + 1 + ex(i)] - lm[(ty + 1 - ey(i)) * row + tx + 1 - ex(i)];
        A(&acc)[3] = i < 7 ? S1 : S2;
        if (ex(i)) acc[0] += ex(i) > 0 ? d : -d;
        if (ey(i)) acc[1] += ey(i) > 0 ? d : -d;
        if (ez(i)) acc[2] += ez(i) > 0 ? d : -d;
    }
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) S[dd] = (A)wgt(1) * S1[dd] + (A)wgt(7) * S2[dd];
}

// BGK of one fluid node towards f^eq(rho, u + tau F / rho), F = -psi g S.
template <typename A, bool EX>
__device__ __forceinline__ void collide1(const Inst& I, Node1<A>& v, const A S[3], A psi, uint32_t key)
{
    A j[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        if (ex(i)) j[0] += ex(i) > 0 ? v.f[i] : -v.f[i];
        if (ey(i)) j[1] += ey(i) > 0 ? v.f[i] : -v.f[i];
        if (ez(i)) j[2] += ez(i) > 0 ? v.f[i] : -v.f[i];
    }
    const A rho = v.rho;
    const A inv = recip<A>(rho);
    // k = -tau g psi / rho (the shift tau F / rho = k S); zero at rho = 0
    A kc;
    if constexpr (kPlain<A>)
        kc = rho != (A)0 ? Par<A>::ntg(I, 0) * psi * inv : (A)0;
    else if (!I.psi_exp)
        kc = Par<A>::ntg(I, 0);
    else
        kc = __builtin_fabsf(rho) >= __FLT_MIN__ ? Par<A>::ntg(I, 0) * psi * inv
                                                  : (rho != (A)0 ? Par<A>::ntg(I, 0) : (A)0);
    const A u[3] = {j[0] * inv + kc * S[0], j[1] * inv + kc * S[1], j[2] * inv + kc * S[2]};
    const A uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const A drho = v.drho;
    const A omega = Par<A>::omega(I, 0);
    const A base0 = drho - (A)1.5 * rho * uu;
    const A f0 = v.f[0];
    v.f[0] = v.f[0] - (v.f[0] - (A)wgt(0) * base0) * omega;
    A dsum = (A)0;   // FP32S: the moving populations' increments (see collide_node)
#pragma unroll
    for (int i = 1; i < kQ; i += 2) {
        const A eu = (A)ex(i) * u[0] + (A)ey(i) * u[1] + (A)ez(i) * u[2];
        const A even = (A)wgt(i) * (base0 + (A)4.5 * rho * eu * eu);
        const A odd = (A)wgt(i) * (A)3 * rho * eu;
        const A a = v.f[i], b = v.f[i + 1];
        v.f[i] = a - (a - (even + odd)) * omega;
        v.f[i + 1] = b - (b - (even - odd)) * omega;
        if constexpr (EX) {
            dsum += a - v.f[i];
            dsum += b - v.f[i + 1];
        }
    }
    if constexpr (EX) v.f[0] = round_sr_sum(f0, dsum, key);
    else if constexpr (!kPlain<A>) absorb_rest(v.f, drho);
}

// psi of a plane's node: behind a solid wall the wall's constant.
template <typename A>
__device__ __forceinline__ A psi1(const Inst& I, bool wallc, A rho)
{
    return wallc ? Par<A>::psiw(I, 0) : psi_of<A>(rho, I.psi_exp);
}

// The fused single-component step: pull, sink reset, density and psi of the
// tile and its halo per plane, force and collision of the previous plane,
// aligned store.
template <class St, int NT>
__global__ __launch_bounds__(NT) void k_step1(const Inst* __restrict__ insts, const Item* __restrict__ items,
                                              int n_items, const typename St::T* __restrict__ src,
                                              typename St::T* __restrict__ dst, double* __restrict__ eacc)
{
    using T = typename St::T;
    using A = typename St::A;
    constexpr bool EX = kExact1<St>;
    constexpr int FP = Foot<NT>::kMax;
    __shared__ A psiS[3][FP];
    __shared__ double red[NT / 64];

    const int k = xcd_item(blockIdx.x, n_items);
    if (k >= n_items) return;
    const Item it = items[k];
    if (it.nzc == 0) return;  // padding of an XCD's run of items
    const Inst I = insts[it.inst];
    const T* __restrict__ s = src + I.base;
    T* __restrict__ d = dst + I.base;

    const int t = threadIdx.x;
    const int tw = it.tw, th = it.th;
    const int row = tw + 2;
    const bool own = t < tw * th;
    const int tx = own ? t % tw : 0;
    const int ty = own ? t / tw : 0;
    const int x = wrap(it.x0 + tx, I.nx);
    const int y = wrap(it.y0 + ty, I.ny);
    const int nring = 2 * row + 2 * th;
    const int z0 = it.z0, z1 = it.z0 + it.nzc;
    const bool book = I.count_reset != 0 && I.reset.kind != kSinkNone;
    double eflux = 0.0;

    Node1<A> cur, nxt;

    auto load_plane = [&](int zq, int sl, Node1<A>& keep) {
        const int zp = psi_plane(zq, I.nz, I.wall_z);
        const bool wallc = beyond_wall(I, zq);
        for (int r = t; r < nring; r += NT) {
            int fx, fy;
            ring_coord(r, tw, th, fx, fy);
            const int hx = wrap(it.x0 + fx, I.nx), hy = wrap(it.y0 + fy, I.ny);
            Node1<A> h;
            pull1<St>(s, I, hx, hy, zp, h);
            density1<A>(I, h);
            if (in_sink(I.reset, hx, hy, zp, I.nx, I.ny, I.nz)) sink1<A, EX>(I, h, node_key(I, hx, hy, zp));
            psiS[sl][(fy + 1) * row + fx + 1] = psi1<A>(I, wallc, h.rho);
        }
        if (own) {
            pull1<St>(s, I, x, y, zp, keep);
            density1<A>(I, keep);
            if (in_sink(I.reset, x, y, zp, I.nx, I.ny, I.nz)) {
                const double fl = sink1<A, EX>(I, keep, node_key(I, x, y, zp));
                if (book && zq >= z0 && zq < z1) eflux += fl;
            }
            psiS[sl][(ty + 1) * row + tx + 1] = psi1<A>(I, wallc, keep.rho);
        }
    };

    auto collide_plane = [&](int z, Node1<A>& v) {
        if (!own) return;
        const int sm = (z - z0) % 3, s0 = (z - z0 + 1) % 3, sp = (z - z0 + 2) % 3;
        const uint32_t xy = (uint32_t)y * (uint32_t)I.nx + (uint32_t)x;
        if (!in_sink(I.cur, x, y, z, I.nx, I.ny, I.nz)) {
            A S[3];
            force_sum1<A>(psiS[sm], psiS[s0], psiS[sp], tx, ty, row, S);
            collide1<A, EX>(I, v, S, psiS[s0][(ty + 1) * row + tx + 1], node_key(I, x, y, z));
        }
        store1<St>(d, I, z, xy, v);
    };

    load_plane(z0 - 1, 0, nxt);
    load_plane(z0, 1, cur);
    for (int z = z0; z < z1; z += 2) {
        load_plane(z + 1, (z - z0 + 2) % 3, nxt);
        __syncthreads();
        collide_plane(z, cur);
        __syncthreads();
        if (z + 1 < z1) {
            load_plane(z + 2, (z - z0 + 3) % 3, cur);
            __syncthreads();
            collide_plane(z + 1, nxt);
            __syncthreads();
        }
    }

    if (book) {
        double e = block_sum_wave(eflux);
        if ((t & 63) == 0) red[t >> 6] = e;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
            for (int w = 0; w < NT / 64; ++w) sum += red[w];
            eacc[k] += sum;
        }
    }
}

// ---------------------------------------------------------------------------
// Initialisation and FP64 read-outs of the single-component form.
// ---------------------------------------------------------------------------

// Writes the stored element of population i at in-plane index xy of slab z:
// the FP64 value f, or its deviation from w_i rho0 in FP32.
template <class S>
__device__ __forceinline__ void put_slot1(typename S::T* __restrict__ d, const Inst& I, int i, int z, int64_t xy,
                                          double val)
{
    using T = typename S::T;
    d[(int64_t)z * I.slab + (int64_t)i * I.ps + xy] = (T)(val - wgt(i) * I.shift[0]);
}

// f = f^eq(rho, 0) from FP64 densities (the stored buffer holds the values
// each node's pull will read; see k_init_density).
template <class S>
__global__ void k_init_density1(Inst I, const double* __restrict__ rho, typename S::T* __restrict__ dst)
{
    typename S::T* d = dst + I.base;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx), y = (int)((k / I.nx) % I.ny), z = (int)(k / ((int64_t)I.nx * I.ny));
        const int64_t xy = k - (int64_t)z * I.nx * I.ny;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int zt = z + ez(i);
            const int64_t src = (I.wall_z && (zt < 0 || zt >= I.nz))
                                    ? k : node_of(wrap(x + ex(i), I.nx), wrap(y + ey(i), I.ny), wrap(zt, I.nz), I.nx, I.ny);
            put_slot1<S>(d, I, i, z, xy, wgt(i) * rho[src]);
        }
    }
}

// From FP64 populations f[i*fstride + node].
template <class S>
__global__ void k_init_pops1(Inst I, const double* __restrict__ f, int64_t fstride, typename S::T* __restrict__ dst)
{
    typename S::T* d = dst + I.base;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx), y = (int)((k / I.nx) % I.ny), z = (int)(k / ((int64_t)I.nx * I.ny));
        const int64_t xy = k - (int64_t)z * I.nx * I.ny;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int zt = z + ez(i);
            int64_t src;
            int q;
            if (I.wall_z && (zt < 0 || zt >= I.nz)) {
                src = k;
                q = opp(i);
            } else {
                src = node_of(wrap(x + ex(i), I.nx), wrap(y + ey(i), I.ny), wrap(zt, I.nz), I.nx, I.ny);
                q = i;
            }
            put_slot1<S>(d, I, i, z, xy, f[(int64_t)q * fstride + src]);
        }
    }
}

template <class S>
__device__ __forceinline__ void state_at1(const typename S::T* s, const Inst& I, int x, int y, int z,
                                          Node1<typename S::A>& v)
{
    using A = typename S::A;
    pull1<S>(s, I, x, y, z, v);
    density1<A>(I, v);
    if (in_sink(I.reset, x, y, z, I.nx, I.ny, I.nz)) sink1<A, kExact1<S>>(I, v, node_key(I, x, y, z));
}

template <class S>
__global__ void k_read_density1(Inst I, const typename S::T* __restrict__ src, double* __restrict__ out)
{
    const typename S::T* s = src + I.base;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx), y = (int)((k / I.nx) % I.ny), z = (int)(k / ((int64_t)I.nx * I.ny));
        Node1<typename S::A> v;
        state_at1<S>(s, I, x, y, z, v);
        out[k] = I.shift[0] + (double)v.drho;
    }
}

// out[i*ostride + node].
template <class S>
__global__ void k_read_pops1(Inst I, const typename S::T* __restrict__ src, double* __restrict__ out, int64_t ostride)
{
    const typename S::T* s = src + I.base;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx), y = (int)((k / I.nx) % I.ny), z = (int)(k / ((int64_t)I.nx * I.ny));
        Node1<typename S::A> v;
        state_at1<S>(s, I, x, y, z, v);
#pragma unroll
        for (int i = 0; i < kQ; ++i) out[(int64_t)i * ostride + k] = (double)v.f[i] + wgt(i) * I.shift[0];
    }
}

// U of Eq. (velw) for one component: (j + F/2) / rho, F = -psi g S, from
// S(t) and its densities (written by k_read_density1); U[d*ustride + node].
template <class S>
__global__ void k_read_velocity1(Inst I, const typename S::T* __restrict__ src, const double* __restrict__ rho,
                                 double* __restrict__ U, int64_t ustride)
{
    const typename S::T* s = src + I.base;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < I.n; k += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(k % I.nx), y = (int)((k / I.nx) % I.ny), z = (int)(k / ((int64_t)I.nx * I.ny));
        Node1<typename S::A> v;
        state_at1<S>(s, I, x, y, z, v);
        double num[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            num[0] += (double)v.f[i] * ex(i);
            num[1] += (double)v.f[i] * ey(i);
            num[2] += (double)v.f[i] * ez(i);
        }
        if (!in_sink(I.cur, x, y, z, I.nx, I.ny, I.nz)) {
            double Sv[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                const int zn = psi_plane(z + ez(i), I.nz, I.wall_z);
                const double r = rho[node_of(wrap(x + ex(i), I.nx), wrap(y + ey(i), I.ny), zn, I.nx, I.ny)];
                const double p = beyond_wall(I, z + ez(i)) ? I.psi_w[0] : (I.psi_exp ? 1.0 - exp(-r) : r);
                Sv[0] += wgt(i) * p * ex(i);
                Sv[1] += wgt(i) * p * ey(i);
                Sv[2] += wgt(i) * p * ez(i);
            }
            const double pc = I.psi_exp ? 1.0 - exp(-rho[k]) : rho[k];
            for (int dd = 0; dd < 3; ++dd) num[dd] += 0.5 * (-pc * I.g * Sv[dd]);
        }
        for (int dd = 0; dd < 3; ++dd) U[(int64_t)dd * ustride + k] = num[dd] / rho[k];
    }
}

// Plane partials of the diagnostics (layout of k_diag_planes): mass, a
// second slot holding the phase midpoint times the plane's node count (so
// that k_diag_final's plane difference is the plane sum of rho minus the
// midpoint, whose zero is the interface), momentum, phase fraction, pending
// sink flux, non-finite and non-positive counts. The exact FP64 sum of the
// stored deviations gives the mass.
template <class S>
__global__ __launch_bounds__(256) void k_diag_planes1(Inst I, const typename S::T* __restrict__ src,
                                                      double* __restrict__ part)
{
    using A = typename S::A;
    __shared__ double lds[kDiagVals * 4];
    const typename S::T* s = src + I.base;
    const int z = blockIdx.x;
    const int area = I.nx * I.ny;
    const double mid = 0.5 * (I.phi_in + I.phi_out);
    double acc[kDiagVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = threadIdx.x; k < area; k += blockDim.x) {
        const int x = k % I.nx, y = k / I.nx;
        Node1<A> v;
        pull1<S>(s, I, x, y, z, v);
        density1<A>(I, v);
        if (in_sink(I.reset, x, y, z, I.nx, I.ny, I.nz)) acc[6] += sink1<A, kExact1<S>>(I, v, node_key(I, x, y, z));
        const double r = I.shift[0] + sum64(v.f);
        acc[0] += r;
        acc[1] += mid;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const double fi = (double)v.f[i];
            acc[2] += fi * ex(i);
            acc[3] += fi * ey(i);
            acc[4] += fi * ez(i);
        }
        double phi = (r - I.phi_out) / (I.phi_in - I.phi_out);
        phi = phi < 0.0 ? 0.0 : (phi > 1.0 ? 1.0 : phi);
        acc[5] += phi;
        if (!isfinite(r)) acc[7] += 1.0;
        if (r <= 0.0) acc[8] += 1.0;
    }
    block_sum_n<double>(acc, kDiagVals, lds);
    if (threadIdx.x < kDiagVals) part[(int64_t)z * kDiagVals + threadIdx.x] = acc[threadIdx.x];
}

}  // namespace lbsc
