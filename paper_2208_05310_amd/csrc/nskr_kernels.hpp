// nskr_kernels.hpp -- gfx950 kernels of the DGSEM right-hand side and the
// low-storage RK update for relaxation model 1 of the non-isothermal NSK
// equations with a van der Waals fluid (arXiv 2208.05310, Sec. 2.3.2, 2.4, 3).
//
// Execution model
//   One workgroup of 256 threads owns EPB = 256 / (N+1)^3 elements; each
//   thread owns one volume node.  Element tiles are staged in LDS for the 1D
//   derivative sweeps along xi, eta, zeta; face work runs as a strided loop
//   over the block's face points.  State is structure-of-arrays
//   [var][element][node]; face traces are element-major [var][element][face]
//   [point] so that each element writes its own six faces contiguously and
//   reads its neighbour's face as one contiguous run.
//
// Phases of one stage (BR1 needs three neighbour exchanges):
//   k_lift1  : U + neighbour primitive traces -> grad(rho,u,c) (15 fields), T
//              at the nodes, and own-face traces of grad c and T.
//   k_lift2  : T, grad c + neighbour traces -> grad T (3), lap c (1); then the
//              own-face flux traces (normal flux, wave speed, state) or the
//              complete wall flux on wall faces.
//   k_update : volume integral of the contravariant fluxes, surface integral
//              of the Rusanov + central viscous face flux, point-wise source,
//              Jacobian scaling, RK stage update, and the primitive face
//              traces of the new state for the next stage.
// Metric terms are per element (affine elements).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nskr {

constexpr int kBlock = 256;

struct Phys {
    double R, a, b, cv, mu, kappa, gam, alpha, beta;
    double inv_Rcv;   // 1 / (R c_v)
    double cs_fac;    // (1 + 1/c_v) R
};

struct BcDev {
    int kind;         // 1 no-slip isothermal with contact angle, 2 slip adiabatic
    double twall;
    double rv, rl;    // Maxwell densities at twall
    double gcoef;     // contact-angle flux g(c) = gcoef (c - rl)(c - rv)
};

// 1D operators for one polynomial degree (host computed, FP64).
struct Basis {
    double Dh[36];    // Dhat[i*P + l] = -(w_l / w_i) D_li
    double L[2][6];   // l_j(-1), l_j(+1)
    double Lh[2][6];  // l_j(-1)/w_j, l_j(+1)/w_j
    double w[6];      // Gauss weights
    double x[6];      // Gauss nodes
};

struct MeshDev {
    int E;
    const int *nbr;      // [E][6] neighbour element, -1 on a wall
    const int *bcid;     // [E][6] 0 interior, else 1-based wall index
    const double *emet;  // [E][10] Ja[d*3+m], J
    const double *fmet;  // [E][6][4] outward unit normal, surface element
    const double *egeo;  // [E][12] corner 0 and the three edge vectors
    const BcDev *bcs;
};

template <int P> struct Tile {
    static constexpr int n2 = P * P, n3 = P * P * P;
    static constexpr int EPB = kBlock / n3;     // elements per block
    static constexpr int NV = EPB * n3;         // active node threads
    static constexpr int NF = EPB * 6 * n2;     // face points per block
};

template <int P> __device__ __forceinline__ int line_node(int d, int l, int p, int q)
{
    return d == 0 ? l + P * (p + P * q) : (d == 1 ? p + P * (l + P * q) : p + P * (q + P * l));
}

// ---------------------------------------------------------------- physics
// Temperature recovery of eq. totalenergyalpha with eps = R c_v T - a rho
// (always FP64: it cancels large terms near the spinodal).
__device__ __forceinline__ double temperature(const Phys &ph, double rho, double m0, double m1, double m2,
                                              double E, double c, double q0, double q1, double q2)
{
    double kin = 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho;
    double rel = 0.5 * ph.alpha * (rho - c) * (rho - c);
    double grd = 0.5 * ph.gam * (q0 * q0 + q1 * q1 + q2 * q2);
    return ((E - kin - rel - grd) / rho + ph.a * rho) * ph.inv_Rcv;
}

// van der Waals pressure (eq. pressure) and isentropic sound speed squared
// (eq. speedofsound for the Helmholtz energy of Sec. 2.1), FP64.
__device__ __forceinline__ void eos(const Phys &ph, double rho, double T, double &p, double &cs2)
{
    double q = 1.0 / (1.0 - ph.b * rho);
    p = rho * ph.R * T * q - ph.a * rho * rho;
    cs2 = ph.cs_fac * T * q * q - 2.0 * ph.a * rho;
}

// Local state at a point for the flux evaluation.
template <typename T> struct Pt {
    T rho, m[3], E, c;    // conserved
    T p;                  // pressure
    T gu[3][3];           // gu[j][i] = d u_j / d x_i
    T gT[3], gc[3], lapc; // grad T, grad c, lap c
};

// (F^C - F^V) . v for an arbitrary vector v (unit normal on faces, the
// contravariant metric row Ja^d in the volume), relaxation model 1
// (eq. navierstokeskorteweg_p): F^V = (0, tau, tau u + j_e, gamma beta grad c),
// tau = mu (grad u + grad u^T - 2/3 div u I), j_e = k grad T - gamma c grad c
// div u + gamma grad c zeta, zeta = beta (gamma lap c + alpha (rho - c)).
template <typename T>
__device__ __forceinline__ void flux_dot(const Phys &ph, const Pt<T> &s, const T v[3], T out[6])
{
    const T ir = T(1) / s.rho;
    const T u0 = s.m[0] * ir, u1 = s.m[1] * ir, u2 = s.m[2] * ir;
    const T mv = s.m[0] * v[0] + s.m[1] * v[1] + s.m[2] * v[2];
    const T uv = mv * ir;
    const T div = s.gu[0][0] + s.gu[1][1] + s.gu[2][2];
    const T mu = T(ph.mu);
    const T tdiv = T(2.0 / 3.0) * div;
    // tau . v  (tau symmetric): (tau v)_j = mu sum_i (du_j/dx_i + du_i/dx_j) v_i - mu 2/3 div v_j
    T tv[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) acc += (s.gu[j][i] + s.gu[i][j]) * v[i];
        tv[j] = mu * (acc - tdiv * v[j]);
    }
    const T gcv = s.gc[0] * v[0] + s.gc[1] * v[1] + s.gc[2] * v[2];
    const T gTv = s.gT[0] * v[0] + s.gT[1] * v[1] + s.gT[2] * v[2];
    const T zeta = T(ph.beta) * (T(ph.gam) * s.lapc + T(ph.alpha) * (s.rho - s.c));
    const T jev = T(ph.kappa) * gTv - T(ph.gam) * s.c * gcv * div + T(ph.gam) * gcv * zeta;
    out[0] = mv;
    out[1] = s.m[0] * uv + s.p * v[0] - tv[0];
    out[2] = s.m[1] * uv + s.p * v[1] - tv[1];
    out[3] = s.m[2] * uv + s.p * v[2] - tv[2];
    out[4] = (s.E + s.p) * uv - (tv[0] * u0 + tv[1] * u1 + tv[2] * u2) - jev;
    out[5] = s.c * uv - T(ph.gam * ph.beta) * gcv;
}

// Non-conservative source of relaxation model 1, evaluated point-wise with the
// lifted gradients (Sec. 3.1): momentum alpha rho grad(c - rho), energy
// alpha rho grad(c - rho).u + alpha/2 (c^2 - rho^2) div u + gamma (|grad c|^2/2
// div u - grad c (x) grad c : grad u), order parameter alpha beta (rho - c).
template <typename T>
__device__ __forceinline__ void source(const Phys &ph, const Pt<T> &s, const T grho[3], T S[6])
{
    const T ir = T(1) / s.rho;
    const T u[3] = {s.m[0] * ir, s.m[1] * ir, s.m[2] * ir};
    const T div = s.gu[0][0] + s.gu[1][1] + s.gu[2][2];
    const T al = T(ph.alpha);
    T d[3], gg = T(0), cc = T(0), du = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        d[i] = s.gc[i] - grho[i];
        gg += s.gc[i] * s.gc[i];
        du += d[i] * u[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T r = T(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) r += s.gc[j] * s.gu[j][i];
        cc += s.gc[i] * r;
    }
    S[0] = T(0);
    S[1] = al * s.rho * d[0];
    S[2] = al * s.rho * d[1];
    S[3] = al * s.rho * d[2];
    S[4] = al * s.rho * du + T(0.5) * al * (s.c * s.c - s.rho * s.rho) * div +
           T(ph.gam) * (T(0.5) * gg * div - cc);
    S[5] = al * T(ph.beta) * (s.rho - s.c);
}

// Complete wall flux (F* . n), Sec. 3.2 with the relaxation-model wall
// conditions of Sec. 2.4: Rusanov against the mirrored ghost state (density,
// order parameter and total energy copied, velocity mirrored: fully on the
// no-slip wall, normal part on the slip wall), minus the wall viscous flux:
// traction tau n (no-slip) or its normal part (slip); energy k grad T . n -
// gamma c g div u on the isothermal wall, 0 on the adiabatic one; order
// parameter gamma beta g with the contact-angle flux g.
template <typename T>
__device__ __forceinline__ void wall_flux(const Phys &ph, const BcDev &bc, const Pt<T> &s, double T_face,
                                          const T n[3], T out[6])
{
    const T ir = T(1) / s.rho;
    const T mn = s.m[0] * n[0] + s.m[1] * n[1] + s.m[2] * n[2];
    const T un = mn * ir;
    double pd, cs2;
    eos(ph, (double)s.rho, T_face, pd, cs2);
    const T lam = fabs(un) + T(sqrt(fabs(cs2)));
    const T p = s.p;
    T tv[3];
    const T div = s.gu[0][0] + s.gu[1][1] + s.gu[2][2];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < 3; ++i) acc += (s.gu[j][i] + s.gu[i][j]) * n[i];
        tv[j] = T(ph.mu) * (acc - T(2.0 / 3.0) * div * n[j]);
    }
    out[0] = T(0);
    out[4] = T(0);
    out[5] = T(0);
    if (bc.kind == 1) {
        // ghost m_g = -m, so 1/2(F(U) + F(U_g)).n = m un + p n; -1/2 lam (m_g - m) = lam m
#pragma unroll
        for (int j = 0; j < 3; ++j) out[1 + j] = s.m[j] * un + p * n[j] + lam * s.m[j] - tv[j];
        const T g = T(bc.gcoef) * (s.c - T(bc.rl)) * (s.c - T(bc.rv));
        const T gTn = s.gT[0] * n[0] + s.gT[1] * n[1] + s.gT[2] * n[2];
        out[4] = -(T(ph.kappa) * gTn - T(ph.gam) * s.c * g * div);
        out[5] = -T(ph.gam * ph.beta) * g;
    } else {
        // ghost m_g = m - 2 mn n: 1/2 (F + F_g).n = mn/ rho (m - mn n) + p n ... written out:
        // 1/2 [m un + (m - 2 mn n)(-un)] + p n = mn un n + p n; dissipation lam mn n
        const T tnn = tv[0] * n[0] + tv[1] * n[1] + tv[2] * n[2];
#pragma unroll
        for (int j = 0; j < 3; ++j) out[1 + j] = (mn * un + p + lam * mn - tnn) * n[j];
    }
}

// ------------------------------------------------------------ kernel args
template <typename T> struct ProlongArgs {
    const T *U; T *TU; MeshDev mesh; Basis bas; size_t NN;
};

template <typename T> struct Lift1Args {
    const T *U; const T *TU; T *Q; T *TH; T *T2; MeshDev mesh; Phys ph; Basis bas; size_t NN;
};

template <typename T> struct Lift2Args {
    const T *U; const T *Q; const T *TH; const T *T2; T *G2; T *TF; MeshDev mesh; Phys ph; Basis bas; size_t NN;
};

template <typename T> struct UpdateArgs {
    T *U; T *R; T *Ut; const T *Q; const T *TH; const T *G2; const T *TF; T *TU;
    MeshDev mesh; Phys ph; Basis bas; size_t NN;
    int mode;        // 0: write U_t; 1: RK stage (update U, R, write traces)
    int first;       // RK: assign R at the first stage
    double A, B, dt; // RK coefficients of this stage
};

// Copy the basis into LDS (the rows each thread needs differ per lane).
template <int P>
__device__ __forceinline__ void load_basis(const Basis &b, double *sDh, double *sL, double *sLh)
{
    const int t = threadIdx.x;
    if (t < P * P) sDh[t] = b.Dh[t];
    if (t < 2 * P) {
        sL[t] = b.L[t / P][t % P];
        sLh[t] = b.Lh[t / P][t % P];
    }
}

// Face point task -> (local element, face, face point, neighbour-side info).
template <int P> struct FaceTask {
    int le, f, fp, d, s, p, q;
    __device__ __forceinline__ FaceTask(int task)
    {
        le = task / (6 * P * P);
        int r = task - le * 6 * P * P;
        f = r / (P * P);
        fp = r - f * P * P;
        d = f >> 1;
        s = f & 1;
        p = fp % P;
        q = fp / P;
    }
};

// Prolongation of an LDS field of one element to a face point.
template <int P, typename T>
__device__ __forceinline__ T prolong(const T *s, int base, const double *sL, const FaceTask<P> &ft)
{
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < P; ++l) acc += T(sL[ft.s * P + l]) * s[base + line_node<P>(ft.d, l, ft.p, ft.q)];
    return acc;
}

// ------------------------------------------------------------ k_prolong
// Primitive face traces (rho, u, v, w, c) of the state, from the prolonged
// conserved variables.
template <int P, typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(ProlongArgs<T> a)
{
    using G = Tile<P>;
    __shared__ T sU[6][G::NV];
    __shared__ double sDh[P * P], sL[2 * P], sLh[2 * P];
    load_basis<P>(a.bas, sDh, sL, sLh);
    const int e0 = blockIdx.x * G::EPB;
    const int E = a.mesh.E;
    const int t = threadIdx.x;
    if (t < G::NV && e0 + t / G::n3 < E) {
        size_t g = (size_t)e0 * G::n3 + t;
#pragma unroll
        for (int v = 0; v < 6; ++v) sU[v][t] = a.U[v * a.NN + g];
    }
    __syncthreads();
    const size_t NF = (size_t)E * 6 * G::n2;
    for (int task = t; task < G::NF; task += kBlock) {
        FaceTask<P> ft(task);
        const int e = e0 + ft.le;
        if (e >= E) continue;
        const int base = ft.le * G::n3;
        T u6[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) u6[v] = prolong<P>(sU[v], base, sL, ft);
        const size_t o = ((size_t)e * 6 + ft.f) * G::n2 + ft.fp;
        const T ir = T(1) / u6[0];
        a.TU[0 * NF + o] = u6[0];
        a.TU[1 * NF + o] = u6[1] * ir;
        a.TU[2 * NF + o] = u6[2] * ir;
        a.TU[3 * NF + o] = u6[3] * ir;
        a.TU[4 * NF + o] = u6[5];
    }
}

// ------------------------------------------------------------ k_lift1
template <int P, typename T>
__global__ __launch_bounds__(kBlock) void k_lift1(Lift1Args<T> a)
{
    using G = Tile<P>;
    __shared__ T sU[6][G::NV];
    __shared__ T sW[5][G::NV];
    __shared__ T sS[5][G::NF];
    __shared__ double sDh[P * P], sL[2 * P], sLh[2 * P];
    load_basis<P>(a.bas, sDh, sL, sLh);
    const int E = a.mesh.E;
    const int e0 = blockIdx.x * G::EPB;
    const int t = threadIdx.x;
    const int le = t / G::n3, nd = t - le * G::n3;
    const int e = e0 + le;
    const bool act = t < G::NV && e < E;
    const size_t g = (size_t)e0 * G::n3 + t;
    if (act) {
        T u6[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) { u6[v] = a.U[v * a.NN + g]; sU[v][t] = u6[v]; }
        const T ir = T(1) / u6[0];
        sW[0][t] = u6[0];
        sW[1][t] = u6[1] * ir;
        sW[2][t] = u6[2] * ir;
        sW[3][t] = u6[3] * ir;
        sW[4][t] = u6[5];
    }
    __syncthreads();
    // face values w* of the BR1 lifting
    const size_t NF = (size_t)E * 6 * G::n2;
    for (int task = t; task < G::NF; task += kBlock) {
        FaceTask<P> ft(task);
        const int ef = e0 + ft.le;
        if (ef >= E) continue;
        const int base = ft.le * G::n3;
        T u6[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) u6[v] = prolong<P>(sU[v], base, sL, ft);
        const T ir = T(1) / u6[0];
        T w[5] = {u6[0], u6[1] * ir, u6[2] * ir, u6[3] * ir, u6[5]};
        const int nb = a.mesh.nbr[ef * 6 + ft.f];
        if (nb >= 0) {
            const size_t o = ((size_t)nb * 6 + (ft.f ^ 1)) * G::n2 + ft.fp;
#pragma unroll
            for (int k = 0; k < 5; ++k) w[k] = T(0.5) * (w[k] + a.TU[k * NF + o]);
        } else {
            const BcDev bc = a.mesh.bcs[a.mesh.bcid[ef * 6 + ft.f] - 1];
            if (bc.kind == 1) {
                w[1] = w[2] = w[3] = T(0);
            } else {
                const double *fm = a.mesh.fmet + ((size_t)ef * 6 + ft.f) * 4;
                const T n0 = T(fm[0]), n1 = T(fm[1]), n2 = T(fm[2]);
                const T un = w[1] * n0 + w[2] * n1 + w[3] * n2;
                w[1] -= un * n0;
                w[2] -= un * n1;
                w[3] -= un * n2;
            }
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) sS[k][task] = w[k];
    }
    __syncthreads();
    // volume + surface: J q_m = sum_d Ja^d_m (Dhat w + lhat+ w*_+ - lhat- w*_-)
    T qc[3] = {T(0), T(0), T(0)};
    if (act) {
        const int i = nd % P, j = (nd / P) % P, k = nd / (P * P);
        const int idx[3] = {i, j, k};
        const int fpd[3] = {j + P * k, i + P * k, i + P * j};
        const double *em = a.mesh.emet + (size_t)e * 10;
        T Ja[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) Ja[r] = T(em[r]);
        const T iJ = T(1.0 / em[9]);
        const int base = le * G::n3;
        const int fbase = le * 6 * G::n2;
#pragma unroll
        for (int w = 0; w < 5; ++w) {
            T gd[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                T acc = T(0);
                const int id = idx[d];
                const int p = d == 0 ? j : i, q = d == 2 ? j : k;
#pragma unroll
                for (int l = 0; l < P; ++l) acc += T(sDh[id * P + l]) * sW[w][base + line_node<P>(d, l, p, q)];
                acc += T(sLh[P + id]) * sS[w][fbase + (2 * d + 1) * G::n2 + fpd[d]];
                acc -= T(sLh[id]) * sS[w][fbase + (2 * d) * G::n2 + fpd[d]];
                gd[d] = acc;
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const T q = iJ * (Ja[m] * gd[0] + Ja[3 + m] * gd[1] + Ja[6 + m] * gd[2]);
                a.Q[(3 * w + m) * a.NN + g] = q;
                if (w == 4) qc[m] = q;
            }
        }
        const double Tn = temperature(a.ph, (double)sU[0][t], (double)sU[1][t], (double)sU[2][t], (double)sU[3][t],
                                      (double)sU[4][t], (double)sU[5][t], (double)qc[0], (double)qc[1], (double)qc[2]);
        a.TH[g] = T(Tn);
    }
    __syncthreads();
    // reuse sW[0..2] for grad c to prolong it to the faces
    if (act) {
        sW[0][t] = qc[0];
        sW[1][t] = qc[1];
        sW[2][t] = qc[2];
    }
    __syncthreads();
    for (int task = t; task < G::NF; task += kBlock) {
        FaceTask<P> ft(task);
        const int ef = e0 + ft.le;
        if (ef >= E) continue;
        const int base = ft.le * G::n3;
        T u6[6], q3[3];
#pragma unroll
        for (int v = 0; v < 6; ++v) u6[v] = prolong<P>(sU[v], base, sL, ft);
#pragma unroll
        for (int m = 0; m < 3; ++m) q3[m] = prolong<P>(sW[m], base, sL, ft);
        const double Tf = temperature(a.ph, (double)u6[0], (double)u6[1], (double)u6[2], (double)u6[3],
                                      (double)u6[4], (double)u6[5], (double)q3[0], (double)q3[1], (double)q3[2]);
        const size_t o = ((size_t)ef * 6 + ft.f) * G::n2 + ft.fp;
        a.T2[0 * NF + o] = q3[0];
        a.T2[1 * NF + o] = q3[1];
        a.T2[2 * NF + o] = q3[2];
        a.T2[3 * NF + o] = T(Tf);
    }
}

// ------------------------------------------------------------ k_lift2
template <int P, typename T>
__global__ __launch_bounds__(kBlock) void k_lift2(Lift2Args<T> a)
{
    using G = Tile<P>;
    __shared__ T sA[5][G::NV];     // T, grad c (3); then grad T (3), lap c
    __shared__ T sU[6][G::NV];
    __shared__ T sGu[9][G::NV];
    __shared__ T sTs[G::NF], sFs[G::NF];
    __shared__ double sDh[P * P], sL[2 * P], sLh[2 * P];
    load_basis<P>(a.bas, sDh, sL, sLh);
    const int E = a.mesh.E;
    const int e0 = blockIdx.x * G::EPB;
    const int t = threadIdx.x;
    const int le = t / G::n3, nd = t - le * G::n3;
    const int e = e0 + le;
    const bool act = t < G::NV && e < E;
    const size_t g = (size_t)e0 * G::n3 + t;
    if (act) {
        sA[0][t] = a.TH[g];
#pragma unroll
        for (int m = 0; m < 3; ++m) sA[1 + m][t] = a.Q[(12 + m) * a.NN + g];
#pragma unroll
        for (int v = 0; v < 6; ++v) sU[v][t] = a.U[v * a.NN + g];
#pragma unroll
        for (int r = 0; r < 9; ++r) sGu[r][t] = a.Q[(3 + r) * a.NN + g];
    }
    __syncthreads();
    const size_t NF = (size_t)E * 6 * G::n2;
    for (int task = t; task < G::NF; task += kBlock) {
        FaceTask<P> ft(task);
        const int ef = e0 + ft.le;
        if (ef >= E) continue;
        const size_t o = ((size_t)ef * 6 + ft.f) * G::n2 + ft.fp;
        const double *fm = a.mesh.fmet + ((size_t)ef * 6 + ft.f) * 4;
        const T Tm = a.T2[3 * NF + o];
        const int nb = a.mesh.nbr[ef * 6 + ft.f];
        T Ts, Fs;
        if (nb >= 0) {
            const size_t on = ((size_t)nb * 6 + (ft.f ^ 1)) * G::n2 + ft.fp;
            Ts = T(0.5) * (Tm + a.T2[3 * NF + on]);
            T acc = T(0);
#pragma unroll
            for (int m = 0; m < 3; ++m) acc += T(0.5) * (a.T2[m * NF + o] + a.T2[m * NF + on]) * T(fm[m] * fm[3]);
            Fs = acc;
        } else {
            const BcDev bc = a.mesh.bcs[a.mesh.bcid[ef * 6 + ft.f] - 1];
            if (bc.kind == 1) {
                Ts = T(bc.twall);
                const T c = prolong<P>(sU[5], ft.le * G::n3, sL, ft);
                Fs = T(bc.gcoef) * (c - T(bc.rl)) * (c - T(bc.rv)) * T(fm[3]);
            } else {
                Ts = Tm;
                Fs = T(0);
            }
        }
        sTs[task] = Ts;
        sFs[task] = Fs;
    }
    __syncthreads();
    T gT[3] = {T(0), T(0), T(0)}, lap = T(0);
    if (act) {
        const int i = nd % P, j = (nd / P) % P, k = nd / (P * P);
        const int idx[3] = {i, j, k};
        const int fpd[3] = {j + P * k, i + P * k, i + P * j};
        const double *em = a.mesh.emet + (size_t)e * 10;
        T Ja[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) Ja[r] = T(em[r]);
        const T iJ = T(1.0 / em[9]);
        const int base = le * G::n3;
        const int fbase = le * 6 * G::n2;
        T gd[3], dl = T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int id = idx[d];
            const int p = d == 0 ? j : i, q = d == 2 ? j : k;
            T accT = T(0), a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
            for (int l = 0; l < P; ++l) {
                const int n = base + line_node<P>(d, l, p, q);
                const T D = T(sDh[id * P + l]);
                accT += D * sA[0][n];
                a0 += D * sA[1][n];
                a1 += D * sA[2][n];
                a2 += D * sA[3][n];
            }
            const int fp = fbase + (2 * d + 1) * G::n2 + fpd[d], fm_ = fbase + (2 * d) * G::n2 + fpd[d];
            accT += T(sLh[P + id]) * sTs[fp] - T(sLh[id]) * sTs[fm_];
            gd[d] = accT;
            dl += Ja[3 * d + 0] * a0 + Ja[3 * d + 1] * a1 + Ja[3 * d + 2] * a2 +
                  T(sLh[P + id]) * sFs[fp] + T(sLh[id]) * sFs[fm_];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) gT[m] = iJ * (Ja[m] * gd[0] + Ja[3 + m] * gd[1] + Ja[6 + m] * gd[2]);
        lap = iJ * dl;
        a.G2[0 * a.NN + g] = gT[0];
        a.G2[1 * a.NN + g] = gT[1];
        a.G2[2 * a.NN + g] = gT[2];
        a.G2[3 * a.NN + g] = lap;
    }
    __syncthreads();
    if (act) {
        sA[0][t] = gT[0];
        sA[1][t] = gT[1];
        sA[2][t] = gT[2];
        sA[3][t] = lap;
    }
    __syncthreads();
    // own-face flux traces: G = (F^C - F^V).n, wave speed, state; walls: the
    // complete wall flux in G.
    for (int task = t; task < G::NF; task += kBlock) {
        FaceTask<P> ft(task);
        const int ef = e0 + ft.le;
        if (ef >= E) continue;
        const int base = ft.le * G::n3;
        const size_t o = ((size_t)ef * 6 + ft.f) * G::n2 + ft.fp;
        const double *fm = a.mesh.fmet + ((size_t)ef * 6 + ft.f) * 4;
        Pt<T> s;
        s.rho = prolong<P>(sU[0], base, sL, ft);
        s.m[0] = prolong<P>(sU[1], base, sL, ft);
        s.m[1] = prolong<P>(sU[2], base, sL, ft);
        s.m[2] = prolong<P>(sU[3], base, sL, ft);
        s.E = prolong<P>(sU[4], base, sL, ft);
        s.c = prolong<P>(sU[5], base, sL, ft);
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) s.gu[jj][ii] = prolong<P>(sGu[3 * jj + ii], base, sL, ft);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            s.gT[m] = prolong<P>(sA[m], base, sL, ft);
            s.gc[m] = a.T2[m * NF + o];
        }
        s.lapc = prolong<P>(sA[3], base, sL, ft);
        const double Tf = (double)a.T2[3 * NF + o];
        double pd, cs2;
        eos(a.ph, (double)s.rho, Tf, pd, cs2);
        s.p = T(pd);
        const T n[3] = {T(fm[0]), T(fm[1]), T(fm[2])};
        T out[6];
        const int nb = a.mesh.nbr[ef * 6 + ft.f];
        if (nb >= 0) {
            flux_dot(a.ph, s, n, out);
            const T un = (s.m[0] * n[0] + s.m[1] * n[1] + s.m[2] * n[2]) / s.rho;
            a.TF[6 * NF + o] = fabs(un) + T(sqrt(fabs(cs2)));
            a.TF[7 * NF + o] = s.rho;
            a.TF[8 * NF + o] = s.m[0];
            a.TF[9 * NF + o] = s.m[1];
            a.TF[10 * NF + o] = s.m[2];
            a.TF[11 * NF + o] = s.E;
            a.TF[12 * NF + o] = s.c;
        } else {
            const BcDev bc = a.mesh.bcs[a.mesh.bcid[ef * 6 + ft.f] - 1];
            wall_flux(a.ph, bc, s, Tf, n, out);
        }
#pragma unroll
        for (int v = 0; v < 6; ++v) a.TF[v * NF + o] = out[v];
    }
}

// ------------------------------------------------------------ k_update
template <int P, typename T>
__global__ __launch_bounds__(kBlock) void k_update(UpdateArgs<T> a)
{
    using G = Tile<P>;
    __shared__ T sF[6][G::NV];
    __shared__ T sFs[6][G::NF];
    __shared__ double sDh[P * P], sL[2 * P], sLh[2 * P];
    load_basis<P>(a.bas, sDh, sL, sLh);
    const int E = a.mesh.E;
    const int e0 = blockIdx.x * G::EPB;
    const int t = threadIdx.x;
    const int le = t / G::n3, nd = t - le * G::n3;
    const int e = e0 + le;
    const bool act = t < G::NV && e < E;
    const size_t g = (size_t)e0 * G::n3 + t;
    const size_t NF = (size_t)E * 6 * G::n2;

    // surface flux (F* . n) dS per face point
    for (int task = t; task < G::NF; task += kBlock) {
        FaceTask<P> ft(task);
        const int ef = e0 + ft.le;
        if (ef >= E) continue;
        const size_t o = ((size_t)ef * 6 + ft.f) * G::n2 + ft.fp;
        const T dS = T(a.mesh.fmet[((size_t)ef * 6 + ft.f) * 4 + 3]);
        const int nb = a.mesh.nbr[ef * 6 + ft.f];
        if (nb >= 0) {
            const size_t on = ((size_t)nb * 6 + (ft.f ^ 1)) * G::n2 + ft.fp;
            const T lm = a.TF[6 * NF + o], lp = a.TF[6 * NF + on];
            const T lam = lm > lp ? lm : lp;
#pragma unroll
            for (int v = 0; v < 6; ++v) {
                const T Fn = T(0.5) * (a.TF[v * NF + o] - a.TF[v * NF + on]) -
                             T(0.5) * lam * (a.TF[(7 + v) * NF + on] - a.TF[(7 + v) * NF + o]);
                sFs[v][task] = Fn * dS;
            }
        } else {
#pragma unroll
            for (int v = 0; v < 6; ++v) sFs[v][task] = a.TF[v * NF + o] * dS;
        }
    }

    // point-wise fluxes and source
    Pt<T> s;
    T S[6], Ft[3][6], Ja[9], iJ = T(0);
    if (act) {
        s.rho = a.U[0 * a.NN + g];
        s.m[0] = a.U[1 * a.NN + g];
        s.m[1] = a.U[2 * a.NN + g];
        s.m[2] = a.U[3 * a.NN + g];
        s.E = a.U[4 * a.NN + g];
        s.c = a.U[5 * a.NN + g];
        T grho[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) grho[m] = a.Q[m * a.NN + g];
#pragma unroll
        for (int jj = 0; jj < 3; ++jj)
#pragma unroll
            for (int ii = 0; ii < 3; ++ii) s.gu[jj][ii] = a.Q[(3 + 3 * jj + ii) * a.NN + g];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            s.gc[m] = a.Q[(12 + m) * a.NN + g];
            s.gT[m] = a.G2[m * a.NN + g];
        }
        s.lapc = a.G2[3 * a.NN + g];
        double pd, cs2;
        eos(a.ph, (double)s.rho, (double)a.TH[g], pd, cs2);
        s.p = T(pd);
        const double *em = a.mesh.emet + (size_t)e * 10;
#pragma unroll
        for (int r = 0; r < 9; ++r) Ja[r] = T(em[r]);
        iJ = T(1.0 / em[9]);
#pragma unroll
        for (int d = 0; d < 3; ++d) flux_dot(a.ph, s, &Ja[3 * d], Ft[d]);
        source(a.ph, s, grho, S);
    }
    T acc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    const int i = nd % P, j = (nd / P) % P, k = nd / (P * P);
    const int base = le * G::n3;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        __syncthreads();
        if (act) {
#pragma unroll
            for (int v = 0; v < 6; ++v) sF[v][t] = Ft[d][v];
        }
        __syncthreads();
        if (act) {
            const int id = d == 0 ? i : (d == 1 ? j : k);
            const int p = d == 0 ? j : i, q = d == 2 ? j : k;
#pragma unroll
            for (int l = 0; l < P; ++l) {
                const int n = base + line_node<P>(d, l, p, q);
                const T D = T(sDh[id * P + l]);
#pragma unroll
                for (int v = 0; v < 6; ++v) acc[v] += D * sF[v][n];
            }
        }
    }
    if (act) {
        const int idx[3] = {i, j, k};
        const int fpd[3] = {j + P * k, i + P * k, i + P * j};
        const int fbase = le * 6 * G::n2;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int id = idx[d];
            const T lp = T(sLh[P + id]), lm = T(sLh[id]);
#pragma unroll
            for (int v = 0; v < 6; ++v)
                acc[v] += lp * sFs[v][fbase + (2 * d + 1) * G::n2 + fpd[d]] +
                          lm * sFs[v][fbase + (2 * d) * G::n2 + fpd[d]];
        }
    }
    T Ut[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) Ut[v] = -acc[v] * iJ + S[v];
    if (a.mode == 0) {
        if (act) {
#pragma unroll
            for (int v = 0; v < 6; ++v) a.Ut[v * a.NN + g] = Ut[v];
        }
        return;
    }
    // low-storage RK stage
    __syncthreads();
    if (act) {
        const T A = T(a.A), B = T(a.B), dt = T(a.dt);
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            T r = a.first ? dt * Ut[v] : A * a.R[v * a.NN + g] + dt * Ut[v];
            a.R[v * a.NN + g] = r;
            T u = a.U[v * a.NN + g] + B * r;
            a.U[v * a.NN + g] = u;
            sF[v][t] = u;
        }
    }
    __syncthreads();
    for (int task = t; task < G::NF; task += kBlock) {
        FaceTask<P> ft(task);
        const int ef = e0 + ft.le;
        if (ef >= E) continue;
        const int b2 = ft.le * G::n3;
        T u6[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) u6[v] = prolong<P>(sF[v], b2, sL, ft);
        const size_t o = ((size_t)ef * 6 + ft.f) * G::n2 + ft.fp;
        const T ir = T(1) / u6[0];
        a.TU[0 * NF + o] = u6[0];
        a.TU[1 * NF + o] = u6[1] * ir;
        a.TU[2 * NF + o] = u6[2] * ir;
        a.TU[3 * NF + o] = u6[3] * ir;
        a.TU[4 * NF + o] = u6[5];
    }
}

}  // namespace nskr
