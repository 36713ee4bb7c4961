// nskr_kernels.hpp -- gfx950 kernels of the DGSEM right-hand side and the
// low-storage RK update for relaxation models 1 and 2 of the non-isothermal
// NSK equations with a van der Waals fluid (arXiv 2208.05310, Sec. 2.3.2, 2.4,
// 3).
//
// Execution model
//   One workgroup of 256 (or 512) threads owns EPB = threads / (N+1)^3
//   elements; each thread owns one volume node.  Element tiles are staged in
//   LDS for the 1D derivative sweeps along xi, eta, zeta; face work runs as
//   line tasks (one thread per grid line normal to a face pair).  State is
//   structure-of-arrays [var][element][node]; face traces are face-major
//   [element][face][var][point] so that each element writes its own six faces
//   contiguously and reads all fields of a neighbour's face as one contiguous
//   run.
//
// Data flow of one stage (BR1 needs three neighbour exchanges).  Only what a
// later kernel cannot rebuild from the state goes through memory: the lifted
// gradients of the primitives are recomputed where they are needed from the
// state and the neighbours' conserved face traces, which costs a few hundred
// flops per node and saves their storage round trip.
//   k_lift1  : U + neighbour c traces -> lifted grad c; own-face traces of
//              (grad c) . n, of the face temperature and, on walls, of grad c
//              (T2).
//   k_lift2  : U + neighbour conserved traces -> lifted grad u, grad c, nodal
//              T; with the T2 traces of both sides -> grad T, lap c (G2);
//              then the own-face flux traces (normal flux, wave speed), or the
//              complete wall flux on wall faces (TF).
//   k_update : U + neighbour conserved traces -> all lifted gradients again;
//              volume integral of the contravariant fluxes, surface integral
//              of the Rusanov (model 2: HLLC) + central viscous face flux,
//              point-wise source,
//              Jacobian scaling, RK stage update, and the conserved face
//              traces of the new state for the next stage.
// The conserved traces rotate over three buffers: stage s reads buffer b(s)
// and writes b(s+1), b = 0 1 0 1 2 (0), so no kernel overwrites traces that
// a neighbouring workgroup may still read.
// Metric terms are per element (affine elements).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nskr {

constexpr int kBlock = 256;

// Global accesses of node- and element-indexed arrays through a wave-uniform
// base pointer and a 32-bit element index: the base stays in scalar
// registers (read-first-lane keeps the compiler from folding it into per-lane
// 64-bit address arithmetic) and the byte offset is one 32-bit vector
// register shared by every field at the same node, so a load or store costs
// no vector address instruction.  Every array addressed this way is below
// 4 GiB (the mesh upload checks it).  Face traces keep 64-bit addresses: one
// per face point, with the field offsets as immediates.
template <typename P> __device__ __forceinline__ P *uniform_ptr(P *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P *)(((uint64_t)hi << 32) | lo);
}
template <typename T> __device__ __forceinline__ T gld(const T *base, uint32_t i)
{
    typedef __attribute__((address_space(1))) const char gc;
    return *(__attribute__((address_space(1))) const T *)((gc *)uniform_ptr(base) + i * (uint32_t)sizeof(T));
}
template <typename T> __device__ __forceinline__ void gst(T *base, uint32_t i, T v)
{
    typedef __attribute__((address_space(1))) char gc;
    *(__attribute__((address_space(1))) T *)((gc *)uniform_ptr(base) + i * (uint32_t)sizeof(T)) = v;
}
// The same accesses with the non-temporal hint (NT), for the update
// kernel's node arrays on meshes whose node data would fill much of the
// last-level cache: they stream through it instead of displacing the face
// traces that the next kernels read again.
template <bool NT, typename T> __device__ __forceinline__ T gldn(const T *base, uint32_t i)
{
    typedef __attribute__((address_space(1))) const char gc;
    const auto *p = (__attribute__((address_space(1))) const T *)((gc *)uniform_ptr(base) + i * (uint32_t)sizeof(T));
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T> __device__ __forceinline__ void gstn(T *base, uint32_t i, T v)
{
    typedef __attribute__((address_space(1))) char gc;
    auto *p = (__attribute__((address_space(1))) T *)((gc *)uniform_ptr(base) + i * (uint32_t)sizeof(T));
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

struct Phys {
    double R, a, b, cv, mu, kappa, gam, alpha, beta;
    double inv_Rcv;   // 1 / (R c_v)
    double cs_fac;    // (1 + 1/c_v) R
    double ap;        // alpha for relaxation model 2 (p_alpha = p + ap/2 rho^2), 0 for model 1
    int model;        // 1 or 2
};

struct BcDev {
    int kind;         // 1 no-slip isothermal with contact angle (moving with uw),
                      // 2 slip adiabatic neutral, 3 generalized Navier slip
    int iso;          // 1: T* = twall in the lifting and k grad T . n (kind 1; kind 3 with gamma3 infinite)
    double twall;
    double rv, rl;    // Maxwell densities at twall
    double gcoef;     // static contact-angle flux g(c) = gcoef (c - rl)(c - rv)
    double uw[3];     // tangential wall velocity (kinds 1, 3)
    double g1, g2, g3, g4;  // gamma_1..gamma_4 (kind 3; zero otherwise)
    double g1_gam;    // gamma_1 / gamma: the dynamic part of g, times div u
    double inv_tw;    // 1 / twall
    int var;          // wall temperature twall + tg . x + rate t (table lookup per face point)
    double tg[3];
    double rate;
    double cg;        // -6 cos(theta) / gamma: gcoef = cg sigma / (rl - rv)^3
    double s2g;       // sqrt(2 gamma): sigma = s2g * (tabulated sigma / sqrt(2 gamma))
};

// Wall-temperature table (Sec. 3.2): kTabN equidistant temperatures on
// [kTabT0, kTabT1], entries (sigma / sqrt(2 gamma), rho_v, rho_l).
constexpr int kTabN = 10000;
constexpr double kTabT0 = 0.3, kTabT1 = 1.0;

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
    const int *nbr;      // [E][6] neighbour face and orientation, (6 nb + nf) 8 + o, or -1 on a wall
    const int *bcid;     // [E][6] 0 interior, else 1-based wall index
    // affine elements (the kernels' CV = false instances)
    const double *emet;  // [E][10] Ja[d*3+m], J
    const double *fmet;  // [E][6][4] outward unit normal, surface element
    const double *egeo;  // [E][12] corner 0 and the three edge vectors
    // curved elements (CV = true), in the element type of the precision
    const void *nmet;    // [10][nodes] Ja[d*3+m] and J at every node
    const void *fnrm;    // [E][6][P^2][4] outward unit normal and surface element at every face point
    const double *xnode; // [3][nodes] node coordinates (initial state)
    const BcDev *bcs;
    int dyn;             // some Navier-slip wall has gamma_1 != 0 (g needs div u at the wall)
    const double *stab;  // [kTabN][3] wall-temperature table (walls with a temperature gradient)
    int var;             // some wall has a temperature gradient or rate
};

template <int P, int BS = kBlock> struct Tile {
    static constexpr int n2 = P * P, n3 = P * P * P;
    static constexpr int EPB = BS / n3;         // elements per block
    static constexpr int NV = EPB * n3;         // active node threads
    static constexpr int NF = EPB * 6 * n2;     // face points per block
};

template <int P> __device__ __forceinline__ int line_node(int d, int l, int p, int q)
{
    return d == 0 ? l + P * (p + P * q) : (d == 1 ? p + P * (l + P * q) : p + P * (q + P * l));
}

// Face point of the neighbour that matches face point fp = p + P q of the
// own face (p, q: the two remaining node indices in increasing axis order)
// under orientation o: (a, b) = (q, p) if o & 4 else (p, q); a -> P-1-a if
// o & 1; b -> P-1-b if o & 2; the neighbour's point is a + P b.
template <int P> __device__ __forceinline__ int orient_fp(int fp, int o)
{
    int a = fp % P, b = fp / P;
    if (o & 4) {
        const int t = a;
        a = b;
        b = t;
    }
    if (o & 1) a = P - 1 - a;
    if (o & 2) b = P - 1 - b;
    return a + P * b;
}

// Face index (6 element + local face) of the neighbour across a face with
// connectivity code `code` >= 0, and the neighbour's matching point.
template <int P> __device__ __forceinline__ size_t nbr_face(int code) { return (size_t)(code >> 3); }
template <int P> __device__ __forceinline__ int nbr_point(int code, int fp) { return orient_fp<P>(fp, code & 7); }

// Outward unit normal and surface element at face point fp of face
// `face` (= 6 element + local face): per face on affine elements, per face
// point on curved ones.
template <int P, typename T, bool CV>
__device__ __forceinline__ void face_normal(const MeshDev &m, size_t face, int fp, T n[3], T &dS)
{
    if (CV) {
        const uint32_t q = ((uint32_t)face * (P * P) + fp) * 4;
        const T *fn = (const T *)m.fnrm;
        n[0] = gld(fn, q);
        n[1] = gld(fn, q + 1);
        n[2] = gld(fn, q + 2);
        dS = gld(fn, q + 3);
    } else {
        const uint32_t q = (uint32_t)face * 4;
        n[0] = T(gld(m.fmet, q));
        n[1] = T(gld(m.fmet, q + 1));
        n[2] = T(gld(m.fmet, q + 2));
        dS = T(gld(m.fmet, q + 3));
    }
}
template <int P, typename T, bool CV> __device__ __forceinline__ T face_dS(const MeshDev &m, size_t face, int fp)
{
    if (CV) return gld((const T *)m.fnrm, ((uint32_t)face * (P * P) + fp) * 4 + 3);
    return T(gld(m.fmet, (uint32_t)face * 4 + 3));
}

// ---------------------------------------------------------------- physics
// 1/x in FP64.  FAST (the FP32-mixed instances, whose inputs carry FP32
// precision): the hardware FP32 reciprocal refined by one Newton step in FP64,
// r + r (1 - x r), relative error about 1e-14 (the square of the FP32
// estimate's); else the correctly rounded division.
template <bool FAST> __device__ __forceinline__ double recip(double x)
{
    if (FAST) {
        const double r = (double)__builtin_amdgcn_rcpf((float)x);
        return fma(r, fma(-x, r, 1.0), r);
    }
    return 1.0 / x;
}

// Temperature recovery of eq. totalenergyalpha with eps = R c_v T - a rho
// (always FP64 arithmetic: it cancels large terms near the spinodal).
template <bool FAST = false>
__device__ __forceinline__ double temperature(const Phys &ph, double rho, double m0, double m1, double m2,
                                              double E, double c, double q0, double q1, double q2)
{
    const double ir = recip<FAST>(rho);
    double kin = 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) * ir;
    double rel = 0.5 * ph.alpha * (rho - c) * (rho - c);
    double grd = 0.5 * ph.gam * (q0 * q0 + q1 * q1 + q2 * q2);
    return ((E - kin - rel - grd) * ir + ph.a * rho) * ph.inv_Rcv;
}

// van der Waals pressure (eq. pressure) and isentropic sound speed squared
// (eq. speedofsound for the Helmholtz energy of Sec. 2.1), FP64.
template <bool FAST = false>
__device__ __forceinline__ void eos(const Phys &ph, double rho, double T, double &p, double &cs2)
{
    double q = recip<FAST>(1.0 - ph.b * rho);
    p = rho * ph.R * T * q - ph.a * rho * rho;
    cs2 = ph.cs_fac * T * q * q - 2.0 * ph.a * rho;
}

// The FP32-mixed instances take the refined reciprocals above.
template <typename T> constexpr bool fast_fp64() { return sizeof(T) == 4; }

// sqrt of a non-negative FP64 value into the element type: FP32 instances
// round the argument and take the FP32 square root.
template <typename T> __device__ __forceinline__ T sqrt_to(double x)
{
    if (sizeof(T) == 4) return T(sqrtf((float)x));
    return T(sqrt(x));
}

// Local state at a point for the flux evaluation.
template <typename T> struct Pt {
    T rho, m[3], E, c;    // conserved
    T ir;                 // 1 / rho
    T p;                  // pressure
    T gu[3][3];           // gu[j][i] = d u_j / d x_i
    T gT[3], gc[3], lapc; // grad T, grad c, lap c
};

// Physical flux tensor of relaxation model 1 (eq. navierstokeskorteweg_p),
// F[v][i] = (F^C - F^V)_v . e_i, so that (F^C - F^V) . w = sum_i F[v][i] w_i
// for any vector w (the contravariant metric rows in the volume integral):
// F^V = (0, tau, tau u + j_e, gamma beta grad c), tau = mu (grad u + grad u^T
// - 2/3 div u I), j_e = k grad T - gamma c grad c div u + gamma grad c zeta,
// zeta = beta (gamma lap c + alpha (rho - c)).
template <typename T>
__device__ __forceinline__ void flux_tensor(const Phys &ph, const Pt<T> &s, T F[6][3])
{
    const T ir = s.ir;
    const T u[3] = {s.m[0] * ir, s.m[1] * ir, s.m[2] * ir};
    const T div = s.gu[0][0] + s.gu[1][1] + s.gu[2][2];
    const T mu = T(ph.mu), tdiv = T(2.0 / 3.0) * div;
    T tau[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 3; ++i) tau[j][i] = mu * (s.gu[j][i] + s.gu[i][j] - (i == j ? tdiv : T(0)));
    const T zeta = T(ph.beta) * (T(ph.gam) * s.lapc + T(ph.alpha) * (s.rho - s.c));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T je = T(ph.kappa) * s.gT[i] - T(ph.gam) * s.c * s.gc[i] * div + T(ph.gam) * s.gc[i] * zeta;
        F[0][i] = s.m[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) F[1 + j][i] = s.m[j] * u[i] + (i == j ? s.p : T(0)) - tau[j][i];
        F[4][i] = (s.E + s.p) * u[i] - (tau[i][0] * u[0] + tau[i][1] * u[1] + tau[i][2] * u[2]) - je;
        F[5][i] = s.c * u[i] - T(ph.gam * ph.beta) * s.gc[i];
    }
}

// HLLC flux (Toro 2009, Sec. 10.4) of the convective part for relaxation
// model 2 along the unit normal n from the own side (left, uL) to the
// neighbour (right, uR): p is p_alpha, a = sqrt((dp_alpha/drho)_s); Davis wave
// speeds S_L = min(u_L - a_L, u_R - a_R), S_R = max(u_L + a_L, u_R + a_R);
// contact speed S*; the star state keeps its side's tangential velocity and
// c/rho (the order parameter as a passive scalar).
template <typename T>
__device__ __forceinline__ void hllc(const T uL[6], T pL, T aL, const T uR[6], T pR, T aR, const T n[3], T out[6])
{
    const T irL = T(1) / uL[0], irR = T(1) / uR[0];
    const T unL = (uL[1] * n[0] + uL[2] * n[1] + uL[3] * n[2]) * irL;
    const T unR = (uR[1] * n[0] + uR[2] * n[1] + uR[3] * n[2]) * irR;
    const T SL = fmin(unL - aL, unR - aR), SR = fmax(unL + aL, unR + aR);
    // the side whose flux (and star state) is taken
    const T Ss = (pR - pL + uL[0] * unL * (SL - unL) - uR[0] * unR * (SR - unR)) /
                 (uL[0] * (SL - unL) - uR[0] * (SR - unR));
    const bool left = SL >= T(0) || (SR > T(0) && Ss >= T(0));
    const T *u = left ? uL : uR;
    const T un = left ? unL : unR, p = left ? pL : pR, ir = left ? irL : irR;
    const T S = left ? SL : SR;
    out[0] = u[0] * un;
    out[1] = u[1] * un + p * n[0];
    out[2] = u[2] * un + p * n[1];
    out[3] = u[3] * un + p * n[2];
    out[4] = (u[4] + p) * un;
    out[5] = u[5] * un;
    if (SL >= T(0) || SR <= T(0)) return;  // supersonic: the upwind flux
    const T f = u[0] * (S - un) / (S - Ss);
    T us[6];
    us[0] = f;
#pragma unroll
    for (int m = 0; m < 3; ++m) us[1 + m] = f * (u[1 + m] * ir + (Ss - un) * n[m]);
    us[4] = f * (u[4] * ir + (Ss - un) * (Ss + p / (u[0] * (S - un))));
    us[5] = f * u[5] * ir;
#pragma unroll
    for (int v = 0; v < 6; ++v) out[v] += S * (us[v] - u[v]);
}

// Non-conservative source of relaxation model 1, evaluated point-wise with the
// lifted gradients (Sec. 3.1): momentum alpha rho grad(c - rho), energy
// alpha rho grad(c - rho).u + alpha/2 (c^2 - rho^2) div u + gamma (|grad c|^2/2
// div u - grad c (x) grad c : grad u), order parameter alpha beta (rho - c).
// Relaxation model 2 (eq. navierstokeskorteweg_palpha) drops the alpha rho
// grad rho and alpha/2 rho^2 div u parts, which its pressure p_alpha carries.
template <typename T>
__device__ __forceinline__ void source(const Phys &ph, const Pt<T> &s, const T grho[3], T S[6])
{
    const T ir = s.ir;
    const T u[3] = {s.m[0] * ir, s.m[1] * ir, s.m[2] * ir};
    const T div = s.gu[0][0] + s.gu[1][1] + s.gu[2][2];
    const T al = T(ph.alpha);
    const bool m2 = ph.model == 2;
    T d[3], gg = T(0), cc = T(0), du = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        d[i] = m2 ? s.gc[i] : s.gc[i] - grho[i];
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
    S[4] = al * s.rho * du + T(0.5) * al * (m2 ? s.c * s.c : s.c * s.c - s.rho * s.rho) * div +
           T(ph.gam) * (T(0.5) * gg * div - cc);
    S[5] = al * T(ph.beta) * (s.rho - s.c);
}

// ------------------------------------------------------------ kernel args
// One problem instance as the kernels see it: caller state, library scratch,
// mesh, physics and its own time step.
template <typename T> struct Inst {
    T *U, *R, *Ut;             // state, RK register, U_t output (rhs)
    T *Ck;                     // compensation of the state update (FP32 Kahan), or null
    T *Q, *TH;                 // grad(rho,u,c) [15] and T, for the API outputs only
    T *G2;                     // grad T + lap c [4]
    T *T2, *TF, *TU;           // face traces: grad c . n and T (+ grad c on walls) [kT2<T>()],
                               // flux + wave speed [7],
                               // conserved state [3 buffers][6]; within an array
                               // (a buffer) face-major: [face][field][point]
    MeshDev mesh;
    Phys ph;
    size_t NN;                 // nodes of the instance
    double dt;
    const int *clk;            // batch: steps taken since admission, for walls whose
                               // temperature changes in time (null otherwise)
    double t0;                 // batch: the instance's time at admission
};

// Kernel argument: a single instance by value, or (BATCH) a device table of
// instances with a block map (instance and first element of every block),
// plus what is common to the launch.
template <typename T> struct Launch {
    Inst<T> one;
    const Inst<T> *tab;
    const int *blk_inst, *blk_e0;
    const int *blk_map;  // single instance: first element of every block (null: block b, elements b EPB..)
    Basis bas;
    int mode;        // update: 0 write U_t; 1 RK stage (update U, R, write traces)
    int first;       // RK: assign R at the first stage
    int last;        // RK: the step's last stage, which does not store R (the next
                     // stage to read it is a first stage, which assigns it)
    int tb, tw;      // conserved-trace buffer read by this stage, written for the next
    int full;        // host side: launch the k_lift1 variant that also writes Q and TH
    double A, B;     // RK coefficients of this stage
    double t;        // time of this stage (walls whose temperature changes in time)
    double cs;       // batch: the stage's time fraction c_s of the step
};

// Time of RK stage s of step n from t0: (t0 + n dt) + c_s dt, rounded as the
// host rounds it for a single instance (no fused multiply-adds), so that an
// instance sees bitwise the same stage times alone and in a batch.
__device__ __forceinline__ double stage_time(double t0, int n, double dt, double cs)
{
#pragma clang fp contract(off)
    return (t0 + (double)n * dt) + cs * dt;
}

// Face traces are stored face by face: the K fields of one face's N2 points
// are contiguous ([face][field][point], face = 6 e + f). A block reading a
// neighbour's face then fetches its fields as one run of whole cache lines,
// not K runs of N2 values each that straddle line boundaries, and the field
// offsets are compile-time constants.
// Fields of the T2 face trace: (grad c) . n with the element's own outward
// normal, the face temperature, and on wall faces only the vector grad c
// (the tangential gradient of a Navier-slip wall). Interior faces need only
// the first two: the divergence lifting of grad c takes the central normal
// component, and the neighbour's outward normal is minus the own one.
// FP32 instances store the FP64 face temperature as two floats, the rounded
// value (the BR1 face value of the FP32 lifting) and the rounding error in
// the field after it, so that the pressure and sound speed at the face are
// formed from the temperature as recovered in FP64 (about 48 bits).
template <typename T> constexpr int kT2() { return sizeof(T) == 4 ? 6 : 5; }
template <typename T> constexpr int kT2gc() { return sizeof(T) == 4 ? 3 : 2; }  // first wall grad c field

template <int N2> struct FaceIx {
    size_t face;
    int fp;
    __device__ __forceinline__ FaceIx(size_t fc, int p) : face(fc), fp(p) {}
    // element of field k of a K-field trace array (64-bit: one address per
    // face point, the field offsets folded into the instructions' immediates)
    __device__ __forceinline__ size_t at(int K, int k) const { return (face * K + k) * N2 + fp; }
};


// A pointer read from ordinary device memory is generic to the compiler,
// which then emits flat loads and stores for everything addressed through it.
// The instance table is read-only while a kernel runs, so read it through the
// constant address space: pointers loaded from there are known to point to
// global memory, and accesses through them compile to global loads and stores
// exactly as for pointers passed by value in the kernel arguments.
template <typename P> __device__ __forceinline__ P load_const(const P *p, int i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(4))) P *)p)[i];
#else
    return p[i];  // host pass: the body is never run on the host
#endif
}

template <typename T, bool BATCH>
__device__ __forceinline__ void instance_of(const Launch<T> &L, Inst<T> &a, int &e0, int epb)
{
    if (BATCH) {
        const int k = load_const(L.blk_inst, blockIdx.x);
        e0 = load_const(L.blk_e0, blockIdx.x);
        a = load_const(L.tab, k);
    } else {
        a = L.one;
        e0 = L.blk_map ? load_const(L.blk_map, blockIdx.x) : blockIdx.x * epb;
    }
}

// Copy the basis into LDS (the rows each thread needs differ per lane), in
// the element type of the kernel: FP32 instances then read and multiply
// floats (the values are the FP64 host basis rounded once, as a conversion
// at every use would round them).
template <int P, typename B_>
__device__ __forceinline__ void load_basis(const Basis &b, B_ *sDh, B_ *sL, B_ *sLh)
{
    const int t = threadIdx.x;
    if (t < P * P) sDh[t] = B_(b.Dh[t]);
    if (t < 2 * P) {
        sL[t] = B_(b.L[t / P][t % P]);
        sLh[t] = B_(b.Lh[t / P][t % P]);
    }
}

// Line task: the line of P nodes through face point (p,q) along direction d
// of local element le; it carries the two face points of faces 2d (xi^d = -1)
// and 2d+1 (+1), so each LDS value of the line is read once for both faces.
template <int P> struct LineTask {
    int le, d, fp, p, q;
    int off, str;  // node l of the line is off + l * str (element-local)
    __device__ __forceinline__ LineTask(int task)
    {
        le = task / (3 * P * P);
        const int r = task - le * 3 * P * P;
        d = r / (P * P);
        fp = r - d * P * P;
        p = fp % P;
        q = fp / P;
        // d = 0: (l, p, q); d = 1: (p, l, q); d = 2: (p, q, l)
        off = d == 0 ? P * fp : (d == 1 ? p + P * P * q : fp);
        str = d == 0 ? 1 : (d == 1 ? P : P * P);
    }
};

// Prolongation of one LDS field of an element to both faces of a line.
template <int P, typename T, typename B_>
__device__ __forceinline__ void prolong2(const T *s, int base, const B_ *sL, const LineTask<P> &lt, T &vm,
                                         T &vp)
{
    T am = T(0), ap = T(0);
    const T *ln = s + base + lt.off;
#pragma unroll
    for (int l = 0; l < P; ++l) {
        const T v = ln[l * lt.str];
        am += T(sL[l]) * v;
        ap += T(sL[P + l]) * v;
    }
    vm = am;
    vp = ap;
}

// Face task: face point fp of face f of local element le, with the line of
// the element that ends on it (node l of the line is off + l * str).
template <int P> struct FaceTask {
    int le, f, fp, off, str;
    __device__ __forceinline__ FaceTask(int task)
    {
        constexpr int n2 = P * P;
        le = task / (6 * n2);
        const int r = task - le * 6 * n2;
        f = r / n2;
        fp = r - f * n2;
        const int d = f >> 1, p = fp % P, q = fp / P;
        off = d == 0 ? P * fp : (d == 1 ? p + P * P * q : fp);
        str = d == 0 ? 1 : (d == 1 ? P : P * P);
    }
};

template <int P, int BS> __device__ __forceinline__ constexpr int n_lines() { return Tile<P, BS>::EPB * 3 * P * P; }

// Line task of thread t, or -1.  The lines fill the first waves of the
// workgroup lane by lane, so waves without lines issue no instructions for
// the line phases (at N = 5, 108 lines take two waves, not 27 lanes in each
// of four: lift1 9-10 % faster on the 32^3 case in both precisions).
template <int P, int BS> __device__ __forceinline__ int line_of_thread(int t)
{
    return t < n_lines<P, BS>() ? t : -1;
}

// ------------------------------------------------------------ shared pieces
// Primitive variables (rho, u, v, w, c) of a conserved state.
template <typename T> __device__ __forceinline__ void primitives(const T u6[6], T w[5])
{
    const T ir = T(1) / u6[0];
    w[0] = u6[0];
    w[1] = u6[1] * ir;
    w[2] = u6[2] * ir;
    w[3] = u6[3] * ir;
    w[4] = u6[5];
}

// BR1 face values of the primitives on a wall face: the interior values with
// the velocity set to the wall's (no-slip) or stripped of its normal part
// (slip and Navier-slip walls).
template <typename T>
__device__ __forceinline__ void wall_primitives(const MeshDev &m, int el, int f, const T n[3], T w[5])
{
    const BcDev &bc = m.bcs[m.bcid[el * 6 + f] - 1];
    if (bc.kind == 1) {
        w[1] = T(bc.uw[0]);
        w[2] = T(bc.uw[1]);
        w[3] = T(bc.uw[2]);
    } else {
        const T un = w[1] * n[0] + w[2] * n[1] + w[3] * n[2];
        w[1] -= un * n[0];
        w[2] -= un * n[1];
        w[3] -= un * n[2];
    }
}

// Wall temperature twall + tg . x + rate t at a wall face point (x from the
// element's corner and edge vectors at the face point's reference
// coordinates: +-1 along the face's axis, the Gauss nodes of its two
// tangential indices along the others).
template <int P>
__device__ __forceinline__ double wall_temperature(const MeshDev &m, const Basis &bas, const BcDev &bc, int el, int f,
                                                   int fp, double t)
{
    const int d = f >> 1;
    const double xn = (f & 1) ? 1.0 : -1.0, xa = bas.x[fp % P], xb = bas.x[fp / P];
    const double r0 = d == 0 ? xn : xa, r1 = d == 1 ? xn : (d == 0 ? xa : xb), r2 = d == 2 ? xn : xb;
    const double *g = m.egeo + (size_t)el * 12;
    double Tw = bc.twall;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        Tw += bc.tg[k] * (g[k] + 0.5 * ((r0 + 1.0) * g[3 + k] + (r1 + 1.0) * g[6 + k] + (r2 + 1.0) * g[9 + k]));
    return Tw + bc.rate * t;
}

// Wall temperature and contact-angle constants at one wall face point: the
// wall's constants for a fixed temperature; for a temperature varying along
// the wall, sigma, rho_v, rho_l interpolated linearly in the table at T_w.
struct WallPt {
    double Tw, rv, rl, gcoef;
};
template <int P>
__device__ __forceinline__ WallPt wall_point(const MeshDev &m, const Basis &bas, const BcDev &bc, int el, int f, int fp,
                                             double t)
{
    WallPt w{bc.twall, bc.rv, bc.rl, bc.gcoef};
    if (!bc.var) return w;
    const double Tw = wall_temperature<P>(m, bas, bc, el, f, fp, t);
    const double sx = (Tw - kTabT0) / ((kTabT1 - kTabT0) / (kTabN - 1));
    int k = (int)floor(sx);
    k = k < 0 ? 0 : (k > kTabN - 2 ? kTabN - 2 : k);
    const double wt = sx - k;
    const double *t0 = m.stab + 3 * k;
    const double sig = bc.s2g * ((1.0 - wt) * t0[0] + wt * t0[3]);
    w.Tw = Tw;
    w.rv = (1.0 - wt) * t0[1] + wt * t0[4];
    w.rl = (1.0 - wt) * t0[2] + wt * t0[5];
    const double dd = w.rl - w.rv;
    w.gcoef = bc.cg * sig / (dd * dd * dd);
    return w;
}

// BR1 lifted gradient of one field at element-local node (i, j, k):
// J q_m = sum_d Ja^d_m (Dhat w + lhat(+1) w*_+ - lhat(-1) w*_-), from the node
// values fw (element starting at base) and face values fs (element's face
// points starting at fbase) in LDS.
template <int P, typename T, typename B_>
__device__ __forceinline__ void lifted_grad(const T *fw, const T *fs, int base, int fbase, int i, int j, int k,
                                            const B_ *sDh, const B_ *sLh, const T Ja[9], T iJ, T q[3])
{
    constexpr int n2 = P * P;
    const int idx[3] = {i, j, k};
    const int fpd[3] = {j + P * k, i + P * k, i + P * j};
    T gd[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T acc = T(0);
        const int id = idx[d];
        const int p = d == 0 ? j : i, r = d == 2 ? j : k;
#pragma unroll
        for (int l = 0; l < P; ++l) acc += T(sDh[id * P + l]) * fw[base + line_node<P>(d, l, p, r)];
        acc += T(sLh[P + id]) * fs[fbase + (2 * d + 1) * n2 + fpd[d]];
        acc -= T(sLh[id]) * fs[fbase + (2 * d) * n2 + fpd[d]];
        gd[d] = acc;
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) q[m] = iJ * (Ja[m] * gd[0] + Ja[3 + m] * gd[1] + Ja[6 + m] * gd[2]);
}

// The same lifted gradient for NFLD consecutive LDS fields at once, sweeping
// direction by direction so that only one row of Dhat is live: the reference
// derivatives gd[f][d] first, then the metric transform.  Each (field,
// direction) sum is formed exactly as in lifted_grad.
template <int P, int NFLD, int NVS, int NFS, typename T, typename B_>
__device__ __forceinline__ void lifted_grads(const T (*fw)[NVS], const T (*fs)[NFS], int base, int fbase, int i, int j,
                                             int k, const B_ *sDh, const B_ *sLh, T gd[NFLD][3])
{
    constexpr int n2 = P * P;
    const int idx[3] = {i, j, k};
    const int fpd[3] = {j + P * k, i + P * k, i + P * j};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int id = idx[d];
        const int p = d == 0 ? j : i, r = d == 2 ? j : k;
        T Dl[P];
#pragma unroll
        for (int l = 0; l < P; ++l) Dl[l] = T(sDh[id * P + l]);
        const T lp = T(sLh[P + id]), lm = T(sLh[id]);
#pragma unroll
        for (int f = 0; f < NFLD; ++f) {
            T acc = T(0);
#pragma unroll
            for (int l = 0; l < P; ++l) acc += Dl[l] * fw[f][base + line_node<P>(d, l, p, r)];
            acc += lp * fs[f][fbase + (2 * d + 1) * n2 + fpd[d]];
            acc -= lm * fs[f][fbase + (2 * d) * n2 + fpd[d]];
            gd[f][d] = acc;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Curved elements: the same BR1 lifting in the conservative form with the
// metrics inside the derivative, J q_m = sum_d sum_l Dhat (Ja^d_m w)_l +
// sum_faces lhat w* (n dS)_m, for NFLD consecutive LDS fields; sJa holds
// Ja^d_m (row 3d+m) at every node of the tile, sN the outward n dS at every
// face point.  Returns the physical gradients times 1/J (iJ of this node).
template <int P, int NFLD, int NVS, int NFS, typename T, typename B_>
__device__ __forceinline__ void lifted_grads_curved(const T (*fw)[NVS], const T (*fs)[NFS], const T (*sJa)[NVS],
                                                    const T (*sN)[NFS], int base, int fbase, int i, int j, int k,
                                                    const B_ *sDh, const B_ *sLh, T iJ, T q[NFLD][3])
{
    constexpr int n2 = P * P;
    const int idx[3] = {i, j, k};
    const int fpd[3] = {j + P * k, i + P * k, i + P * j};
#pragma unroll
    for (int f = 0; f < NFLD; ++f) q[f][0] = q[f][1] = q[f][2] = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int id = idx[d];
        const int p = d == 0 ? j : i, r = d == 2 ? j : k;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            const int n = base + line_node<P>(d, l, p, r);
            const T D = T(sDh[id * P + l]);
            const T a0 = D * sJa[3 * d][n], a1 = D * sJa[3 * d + 1][n], a2 = D * sJa[3 * d + 2][n];
#pragma unroll
            for (int f = 0; f < NFLD; ++f) {
                const T v = fw[f][n];
                q[f][0] += a0 * v;
                q[f][1] += a1 * v;
                q[f][2] += a2 * v;
            }
        }
        const int pp = fbase + (2 * d + 1) * n2 + fpd[d], pm = fbase + (2 * d) * n2 + fpd[d];
        const T lp = T(sLh[P + id]), lm = T(sLh[id]);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const T np_ = lp * sN[m][pp], nm_ = lm * sN[m][pm];
#pragma unroll
            for (int f = 0; f < NFLD; ++f) q[f][m] += np_ * fs[f][pp] + nm_ * fs[f][pm];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int f = 0; f < NFLD; ++f)
#pragma unroll
        for (int m = 0; m < 3; ++m) q[f][m] *= iJ;
}

// Per-node metrics of a curved element tile into LDS (nine Ja rows) and
// this node's 1/J; t is the node's thread, g its global node index.
template <typename T, int NVS>
__device__ __forceinline__ T stage_node_metrics(const MeshDev &m, size_t NN, size_t g, int t, T (*sJa)[NVS])
{
    const T *nm = (const T *)m.nmet;
#pragma unroll
    for (int r = 0; r < 9; ++r) sJa[r][t] = gld(nm + r * NN, (uint32_t)g);
    return T(1) / gld(nm + 9 * NN, (uint32_t)g);
}

template <typename T> __device__ __forceinline__ void to_physical(const T Ja[9], T iJ, const T gd[3], T q[3])
{
#pragma unroll
    for (int m = 0; m < 3; ++m) q[m] = iJ * (Ja[m] * gd[0] + Ja[3 + m] * gd[1] + Ja[6 + m] * gd[2]);
}

// The element whose per-element data (metrics, face normals) a node thread
// reads, as a wave-uniform index where it is one: with one element per
// workgroup it is the workgroup's, and with 64 nodes per element (N = 3)
// each wave holds exactly one element.  Those loads then become scalar
// loads into scalar registers, issued at once and costing no vector
// registers; otherwise the index is the thread's own.
template <int EPB, int N3> __device__ __forceinline__ int metric_element(int e0, int e)
{
    if constexpr (EPB == 1) return e0;
    if constexpr (N3 == 64) return __builtin_amdgcn_readfirstlane(e);
    return e;
}

template <typename T> __device__ __forceinline__ void element_metrics(const MeshDev &m, int e, T Ja[9], T &iJ)
{
#pragma unroll
    for (int r = 0; r < 9; ++r) Ja[r] = T(gld(m.emet, (uint32_t)e * 10 + r));
    iJ = T(1.0 / gld(m.emet, (uint32_t)e * 10 + 9));
}

// ------------------------------------------------------------ k_prolong
// Conserved face traces of the state (into trace buffer L.tw).
template <int P, typename T, int BS, bool BATCH>
__global__ __launch_bounds__(BS) void k_prolong(Launch<T> L)
{
    using G = Tile<P, BS>;
    Inst<T> a;
    int e0;
    instance_of<T, BATCH>(L, a, e0, G::EPB);
    __shared__ T sU[6][G::NV];
    __shared__ T sDh[P * P], sL[2 * P], sLh[2 * P];
    load_basis<P>(L.bas, sDh, sL, sLh);
    const int E = a.mesh.E;
    const int t = threadIdx.x;
    if (t < G::NV && e0 + t / G::n3 < E) {
        const size_t g = (size_t)e0 * G::n3 + t;
    const uint32_t g32 = (uint32_t)g;
#pragma unroll
        for (int v = 0; v < 6; ++v) sU[v][t] = gld(a.U + (v) * a.NN, g32);
    }
    __syncthreads();
    const size_t NF = (size_t)E * 6 * G::n2;
    T *TU = a.TU + (size_t)L.tw * 6 * NF;
    for (int task = t; task < n_lines<P, BS>(); task += BS) {
        LineTask<P> lt(task);
        const int e = e0 + lt.le;
        if (e >= E) continue;
        const int base = lt.le * G::n3;
        T um[6], up[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) prolong2<P>(sU[v], base, sL, lt, um[v], up[v]);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const FaceIx<G::n2> o((size_t)e * 6 + 2 * lt.d + s, lt.fp);
#pragma unroll
            for (int v = 0; v < 6; ++v) TU[o.at(6, v)] = s ? up[v] : um[v];
        }
    }
}

// ------------------------------------------------------------ k_lift1
// Lifted grad c, and the own-face traces of grad c and of the face
// temperature.  FULL: also every lifted gradient and the nodal temperature
// (Q, TH) for the API outputs.
// The per-stage instances on affine elements in 256-thread workgroups are
// latency-bound and keep as many waves per SIMD as their LDS allows without
// register spills: 7 in FP32 (8 spills; so does 7 in 448-thread
// workgroups), and in FP64 8 at N = 5 (63 registers instead of 79) and 6 at
// N = 3 (80 instead of 83).
template <int P, typename T, int BS, bool FULL, bool CV> constexpr int lift1_waves()
{
    if (BS != 256 || FULL || CV) return 1;
    if (sizeof(T) == 4) return 7;
    return P == 6 ? 8 : (P == 4 ? 6 : 1);
}

template <int P, typename T, int BS, bool BATCH, bool FULL = false, bool CV = false>
__global__ __launch_bounds__(BS, (lift1_waves<P, T, BS, FULL, CV>())) void k_lift1(Launch<T> L)
{
    using G = Tile<P, BS>;
    Inst<T> a;
    int e0;
    instance_of<T, BATCH>(L, a, e0, G::EPB);
    static_assert(n_lines<P, BS>() <= BS, "one line per thread");
    // node values of the lifted primitives (c last; slots 0..2 later hold
    // grad c) and their BR1 face values: all five with FULL, else c only
    constexpr int NW = FULL ? 5 : 4, NS = FULL ? 5 : 1;
    // curved elements: the metrics of every node and n dS of every face point
    constexpr int NJ = CV ? 9 : 1, NQ = CV ? 3 : 1, NJV = CV ? G::NV : 1, NQF = CV ? G::NF : 1;
    __shared__ T sU[6][G::NV];
    __shared__ T sW[NW][G::NV];
    __shared__ T sS[NS][G::NF];
    __shared__ T sJa[NJ][NJV];
    __shared__ T sN[NQ][NQF];
    __shared__ T sDh[P * P], sL[2 * P], sLh[2 * P];
    load_basis<P>(L.bas, sDh, sL, sLh);
    const int E = a.mesh.E;
    const int t = threadIdx.x;
    const int le = t / G::n3, nd = t - le * G::n3;
    const int e = e0 + le;
    const bool act = t < G::NV && e < E;
    const size_t g = (size_t)e0 * G::n3 + t;
    const uint32_t g32 = (uint32_t)g;
    const size_t NF = (size_t)E * 6 * G::n2;
    constexpr bool full = FULL;
    const T *TU = a.TU + (size_t)L.tb * 6 * NF;

    // early loads: own nodes, and the neighbour traces of this thread's line
    const int ltask = line_of_thread<P, BS>(t);
    const LineTask<P> lt(ltask < 0 ? 0 : ltask);
    const int el = e0 + lt.le;
    const bool lact = ltask >= 0 && el < E;
    int nbm = -1, nbp = -1;
    T wn[2][6];
    if (lact) {
        nbm = gld(a.mesh.nbr, el * 6 + 2 * lt.d);
        nbp = gld(a.mesh.nbr, el * 6 + 2 * lt.d + 1);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int nb = s ? nbp : nbm;
            if (nb >= 0) {
                const FaceIx<G::n2> o(nbr_face<P>(nb), nbr_point<P>(nb, lt.fp));
                if (full) {
#pragma unroll
                    for (int v = 0; v < 6; ++v)
                        if (v != 4) wn[s][v] = TU[o.at(6, v)];
                } else {
                    wn[s][5] = TU[o.at(6, 5)];
                }
            }
        }
    }
    T iJn = T(0);
    if (act) {
        T u6[6], w[5];
#pragma unroll
        for (int v = 0; v < 6; ++v) { u6[v] = gld(a.U + (v) * a.NN, g32); sU[v][t] = u6[v]; }
        primitives(u6, w);
        if (full) {
#pragma unroll
            for (int k = 0; k < 4; ++k) sW[k][t] = w[k];
        }
        sW[NW - 1][t] = w[4];
        if constexpr (CV) iJn = stage_node_metrics<T, NJV>(a.mesh, a.NN, g, t, sJa);
    }
    __syncthreads();
    // BR1 face values w* on both faces of the line
    if (lact) {
        const int base = lt.le * G::n3;
        T uf[2][6];
        if (full) {
#pragma unroll
            for (int v = 0; v < 6; ++v) prolong2<P>(sU[v], base, sL, lt, uf[0][v], uf[1][v]);
        } else {
            prolong2<P>(sU[5], base, sL, lt, uf[0][5], uf[1][5]);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int f = 2 * lt.d + s;
            const int nb = s ? nbp : nbm;
            const int slot = lt.le * 6 * G::n2 + f * G::n2 + lt.fp;
            if constexpr (CV) {
                T n[3], dS;
                face_normal<P, T, true>(a.mesh, (size_t)el * 6 + f, lt.fp, n, dS);
#pragma unroll
                for (int m = 0; m < 3; ++m) sN[m][slot] = n[m] * dS;
            }
            if (full) {
                T w[5];
                primitives(uf[s], w);
                if (nb >= 0) {
                    T v5[5];
                    primitives(wn[s], v5);
#pragma unroll
                    for (int k = 0; k < 5; ++k) w[k] = T(0.5) * (w[k] + v5[k]);
                } else {
                    T n[3], dS;
                    face_normal<P, T, CV>(a.mesh, (size_t)el * 6 + f, lt.fp, n, dS);
                    wall_primitives(a.mesh, el, f, n, w);
                }
#pragma unroll
                for (int k = 0; k < NS; ++k) sS[k][slot] = w[k];
            } else {
                sS[NS - 1][slot] = nb >= 0 ? T(0.5) * (uf[s][5] + wn[s][5]) : uf[s][5];
            }
        }
    }
    __syncthreads();
    T qc[3] = {T(0), T(0), T(0)};
    if (act) {
        const int i = nd % P, j = (nd / P) % P, k = nd / (P * P);
        const int base = le * G::n3, fbase = le * 6 * G::n2;
        if constexpr (CV) {
            if (full) {
                T q[5][3];
                lifted_grads_curved<P, 5, G::NV, G::NF>(sW, sS, sJa, sN, base, fbase, i, j, k, sDh, sLh, iJn, q);
#pragma unroll
                for (int w = 0; w < 4; ++w)
#pragma unroll
                    for (int m = 0; m < 3; ++m) gst(a.Q + ((3 * w + m)) * a.NN, g32, T(q[w][m]));
                qc[0] = q[4][0];
                qc[1] = q[4][1];
                qc[2] = q[4][2];
            } else {
                T q[1][3];
                lifted_grads_curved<P, 1, G::NV, G::NF>(sW + (NW - 1), sS + (NS - 1), sJa, sN, base, fbase, i, j, k,
                                                        sDh, sLh, iJn, q);
                qc[0] = q[0][0];
                qc[1] = q[0][1];
                qc[2] = q[0][2];
            }
        } else {
            T Ja[9], iJ;
            // (FP32: the scalar loads cost the one vector register that keeps 8 waves per SIMD)
            element_metrics(a.mesh, sizeof(T) == 8 ? metric_element<G::EPB, G::n3>(e0, e) : e, Ja, iJ);
            if (full) {
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    T q[3];
                    lifted_grad<P>(sW[w], sS[w], base, fbase, i, j, k, sDh, sLh, Ja, iJ, q);
#pragma unroll
                    for (int m = 0; m < 3; ++m) gst(a.Q + ((3 * w + m)) * a.NN, g32, T(q[m]));
                }
            }
            lifted_grad<P>(sW[NW - 1], sS[NS - 1], base, fbase, i, j, k, sDh, sLh, Ja, iJ, qc);
        }
        if (full) {
#pragma unroll
            for (int m = 0; m < 3; ++m) gst(a.Q + ((12 + m)) * a.NN, g32, T(qc[m]));
            const double Tn = temperature<fast_fp64<T>()>(a.ph, (double)sU[0][t], (double)sU[1][t], (double)sU[2][t], (double)sU[3][t],
                                          (double)sU[4][t], (double)sU[5][t], (double)qc[0], (double)qc[1],
                                          (double)qc[2]);
            gst(a.TH, g32, T(Tn));
        }
    }
    __syncthreads();
    // reuse sW[0..2] for grad c to prolong it to the faces
    if (act) {
        sW[0][t] = qc[0];
        sW[1][t] = qc[1];
        sW[2][t] = qc[2];
    }
    __syncthreads();
    if (lact) {
        const int base = lt.le * G::n3;
        T qf[2][3], uf[2][6];
#pragma unroll
        for (int m = 0; m < 3; ++m) prolong2<P>(sW[m], base, sL, lt, qf[0][m], qf[1][m]);
        // outward normal of each face of this line: on affine elements the -
        // face's is the exact negative of the + face's, as the mesh upload
        // forms them
        T nf[2][3];
        if constexpr (CV) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                T dS;
                face_normal<P, T, true>(a.mesh, (size_t)el * 6 + 2 * lt.d + s, lt.fp, nf[s], dS);
            }
        } else {
            const uint32_t fq = ((uint32_t)el * 6 + 2 * lt.d + 1) * 4;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                nf[1][m] = T(gld(a.mesh.fmet, fq + m));
                nf[0][m] = -nf[1][m];
            }
        }
#pragma unroll
        for (int v = 0; v < 6; ++v) prolong2<P>(sU[v], base, sL, lt, uf[0][v], uf[1][v]);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double Tf = temperature<fast_fp64<T>()>(a.ph, (double)uf[s][0], (double)uf[s][1], (double)uf[s][2], (double)uf[s][3],
                                          (double)uf[s][4], (double)uf[s][5], (double)qf[s][0], (double)qf[s][1],
                                          (double)qf[s][2]);
            const FaceIx<G::n2> o((size_t)el * 6 + 2 * lt.d + s, lt.fp);
            const T gn = qf[s][0] * nf[s][0] + qf[s][1] * nf[s][1] + qf[s][2] * nf[s][2];
            a.T2[o.at(kT2<T>(), 0)] = gn;
            const T Th = T(Tf);
            a.T2[o.at(kT2<T>(), 1)] = Th;
            if constexpr (sizeof(T) == 4) a.T2[o.at(kT2<T>(), 2)] = T(Tf - (double)Th);
        }
        // wall faces also keep the vector grad c (Navier-slip traction), in
        // a loop of its own: inside the one above the branch costs ~40 VGPRs
#pragma unroll
        for (int s = 0; s < 2; ++s)
            if ((s ? nbp : nbm) < 0) {
                const FaceIx<G::n2> o((size_t)el * 6 + 2 * lt.d + s, lt.fp);
                a.T2[o.at(kT2<T>(), kT2gc<T>())] = qf[s][0];
                a.T2[o.at(kT2<T>(), kT2gc<T>() + 1)] = qf[s][1];
                a.T2[o.at(kT2<T>(), kT2gc<T>() + 2)] = qf[s][2];
            }
    }
}

// ------------------------------------------------------------ k_lift2
template <int P, typename T, int BS, bool BATCH, bool CV = false>
__global__ __launch_bounds__(BS) void k_lift2(Launch<T> L)
{
    using G = Tile<P, BS>;
    Inst<T> a;
    int e0;
    instance_of<T, BATCH>(L, a, e0, G::EPB);
    // sX holds the primitives u, v, w, c [4][NV] and their BR1 face values
    // [4][NF] while grad u and grad c are lifted, then grad u [9][NV]
    constexpr int kX = 9 * G::NV > 4 * G::NV + 4 * G::NF ? 9 * G::NV : 4 * G::NV + 4 * G::NF;
    // curved elements: the metrics of every node and n dS of every face point
    constexpr int NJ = CV ? 9 : 1, NQ = CV ? 3 : 1, NJV = CV ? G::NV : 1, NQF = CV ? G::NF : 1;
    __shared__ T sA[4][G::NV];     // T, grad c (curved: its contravariant components); then grad T, lap c
    __shared__ T sX[kX];
    __shared__ T sTs[G::NF], sFs[G::NF];
    __shared__ T sJa[NJ][NJV];
    __shared__ T sN[NQ][NQF];
    __shared__ T sDh[P * P], sL[2 * P], sLh[2 * P];
    T(*sW)[G::NV] = reinterpret_cast<T(*)[G::NV]>(sX);
    T(*sS)[G::NF] = reinterpret_cast<T(*)[G::NF]>(sX + 4 * G::NV);
    T(*sGu)[G::NV] = reinterpret_cast<T(*)[G::NV]>(sX);
    load_basis<P>(L.bas, sDh, sL, sLh);
    const int E = a.mesh.E;
    const int t = threadIdx.x;
    const int le = t / G::n3, nd = t - le * G::n3;
    const int e = e0 + le;
    const bool act = t < G::NV && e < E;
    const size_t g = (size_t)e0 * G::n3 + t;
    const uint32_t g32 = (uint32_t)g;
    const size_t NF = (size_t)E * 6 * G::n2;
    const T *TU = a.TU + (size_t)L.tb * 6 * NF;

    // face work runs as face tasks (one face point per thread, a second round
    // where the block has more face points than threads); the first round's
    // traces are loaded before the node loads: both sides' conserved state
    // (rho, m, c; the own side's is the prolongation of the state, written by
    // the previous stage) and both sides' grad c and T
    // The own side's traces of the first round's face point (the whole
    // conserved state and (grad c) . n, T; in FP32 also T's rounding error)
    // stay in registers from this load to the flux pass at the end, instead
    // of being read again from memory there, where they mostly miss the L2
    // (where the block has more face points than threads, the second
    // round's are read again).  FP32 instances keep them only where one
    // round covers the block: with two rounds the registers cost a wave per
    // SIMD, which measured slower than the re-read.
    constexpr bool kKeep = sizeof(T) == 8 || G::NF <= BS;
    // FP64, where one round covers the block: the face point's normal and
    // surface element are loaded with its traces too (their loads otherwise
    // stall both face phases; in FP32 the registers would cost a wave per
    // SIMD)
    constexpr bool kOne = G::NF <= BS && sizeof(T) == 8;
    struct Tr {
        int nb;
        T own[3], oth[2], wn[6], uo[6];
        T n[3], dS;
    };
    auto load_tr = [&](int task, Tr &r) {
        const FaceTask<P> ft(task);
        const int el = e0 + ft.le;
        r.nb = -1;
        if (el >= E) return;
        const FaceIx<G::n2> o((size_t)el * 6 + ft.f, ft.fp);
#pragma unroll
        for (int k = 0; k < 2; ++k) r.own[k] = a.T2[o.at(kT2<T>(), k)];
        if constexpr (kKeep && sizeof(T) == 4) r.own[2] = a.T2[o.at(kT2<T>(), 2)];
#pragma unroll
        for (int v = 0; v < 6; ++v)
            if (v != 4 || kKeep) r.uo[v] = TU[o.at(6, v)];
        r.nb = gld(a.mesh.nbr, el * 6 + ft.f);
        if constexpr (kOne) face_normal<P, T, CV>(a.mesh, (size_t)el * 6 + ft.f, ft.fp, r.n, r.dS);
        if (r.nb >= 0) {
            const FaceIx<G::n2> on(nbr_face<P>(r.nb), nbr_point<P>(r.nb, ft.fp));
#pragma unroll
            for (int k = 0; k < 2; ++k) r.oth[k] = a.T2[on.at(kT2<T>(), k)];
#pragma unroll
            for (int v = 0; v < 6; ++v)
                if (v != 4) r.wn[v] = TU[on.at(6, v)];
        }
    };
    Tr tr0;
    if (t < G::NF) load_tr(t, tr0);
    T un[6];
    T iJn = T(0);
    if (act) {
        T w[5];
#pragma unroll
        for (int v = 0; v < 6; ++v) un[v] = gld(a.U + (v) * a.NN, g32);
        primitives(un, w);
#pragma unroll
        for (int k = 0; k < 4; ++k) sW[k][t] = w[1 + k];
        if constexpr (CV) iJn = stage_node_metrics<T, NJV>(a.mesh, a.NN, g, t, sJa);
    }
    __syncthreads();
    // face values: BR1 w* of u, v, w, c; T* and (grad c)* . n dS of the second lifting
    for (int task = t; task < G::NF; task += BS) {
        const FaceTask<P> ft(task);
        const int el = e0 + ft.le, f = ft.f;
        if (el >= E) continue;
        Tr tr;
        if (task == t) tr = tr0; else load_tr(task, tr);
        // the surface element always; the normal where it is used (walls,
        // and the lifting's n dS on curved elements)
        T n[3] = {T(0), T(0), T(0)}, dS;
        if constexpr (kOne) {
            n[0] = tr.n[0];
            n[1] = tr.n[1];
            n[2] = tr.n[2];
            dS = tr.dS;
        } else if (CV || tr.nb < 0) {
            face_normal<P, T, CV>(a.mesh, (size_t)el * 6 + f, ft.fp, n, dS);
        } else {
            dS = face_dS<P, T, CV>(a.mesh, (size_t)el * 6 + f, ft.fp);
        }
        const T *uf = tr.uo;
        T w[5];
        primitives(uf, w);
        T Ts, Fs;
        if (tr.nb >= 0) {
            T v5[5];
            primitives(tr.wn, v5);
#pragma unroll
            for (int k = 1; k < 5; ++k) w[k] = T(0.5) * (w[k] + v5[k]);
            Ts = T(0.5) * (tr.own[1] + tr.oth[1]);
            Fs = T(0.5) * (tr.own[0] - tr.oth[0]) * dS;
        } else {
            wall_primitives(a.mesh, el, f, n, w);
            const BcDev &bc = a.mesh.bcs[a.mesh.bcid[el * 6 + f] - 1];
            Ts = bc.iso ? T(bc.twall) : tr.own[1];
            if (bc.kind != 2) {
                // static part of the contact-angle flux (a varying wall
                // temperature is applied in the pass below; the dynamic part,
                // gamma_1 div u, once grad u is lifted)
                const T c = uf[5];
                Fs = T(bc.gcoef) * (c - T(bc.rl)) * (c - T(bc.rv)) * dS;
            } else {
                Fs = T(0);
            }
        }
        const int slot = ft.le * 6 * G::n2 + f * G::n2 + ft.fp;
#pragma unroll
        for (int k = 0; k < 4; ++k) sS[k][slot] = w[1 + k];
        sTs[slot] = Ts;
        sFs[slot] = Fs;
        if constexpr (CV) {
#pragma unroll
            for (int m = 0; m < 3; ++m) sN[m][slot] = n[m] * dS;
        }
    }
    if (a.mesh.var) {
        // walls whose temperature varies along them: T* and the static
        // contact-angle flux at the local wall temperature, through the table
        // (each thread rewrites only the face points it wrote above)
        double tb = 0.0;  // a batch instance's stage time
        if (BATCH && a.clk) tb = stage_time(a.t0, *a.clk, a.dt, L.cs);
        for (int task = t; task < G::NF; task += BS) {
            const FaceTask<P> ft(task);
            const int el = e0 + ft.le, f = ft.f;
            if (el >= E) continue;
            if (gld(a.mesh.nbr, el * 6 + f) >= 0) continue;  // interior: no wall-table entry
            const BcDev &bc = a.mesh.bcs[a.mesh.bcid[el * 6 + f] - 1];
            if (!bc.var) continue;
            const WallPt wp = wall_point<P>(a.mesh, L.bas, bc, el, f, ft.fp, BATCH ? tb : L.t);
            const int slot = ft.le * 6 * G::n2 + f * G::n2 + ft.fp;
            const FaceIx<G::n2> o((size_t)el * 6 + f, ft.fp);
            if (bc.iso) sTs[slot] = T(wp.Tw);
            else a.TF[o.at(7, 6)] = 1.0 / wp.Tw;  // 1/T_w for the heat-transfer flux below (TF[6] is free on walls)
            const T c = TU[o.at(6, 5)];
            sFs[slot] = T(wp.gcoef) * (c - T(wp.rl)) * (c - T(wp.rv)) * face_dS<P, T, CV>(a.mesh, (size_t)el * 6 + f, ft.fp);
        }
    }
    __syncthreads();
    // lifted grad u, grad c and the nodal temperature
    T gu[9], gc[3];
    double Tn = 0.0;
    const int i = nd % P, j = (nd / P) % P, k = nd / (P * P);
    T Ja[9], iJ = T(0);
    if (act) {
        if constexpr (CV) {
            T q[4][3];
            lifted_grads_curved<P, 4, G::NV, G::NF>(sW, sS, sJa, sN, le * G::n3, le * 6 * G::n2, i, j, k, sDh, sLh,
                                                    iJn, q);
#pragma unroll
            for (int w = 0; w < 3; ++w)
#pragma unroll
                for (int m = 0; m < 3; ++m) gu[3 * w + m] = q[w][m];
#pragma unroll
            for (int m = 0; m < 3; ++m) gc[m] = q[3][m];
            iJ = iJn;
        } else {
            T gd[4][3];
            lifted_grads<P, 4>(sW, sS, le * G::n3, le * 6 * G::n2, i, j, k, sDh, sLh, gd);
            element_metrics(a.mesh, metric_element<G::EPB, G::n3>(e0, e), Ja, iJ);
#pragma unroll
            for (int w = 0; w < 3; ++w) to_physical(Ja, iJ, gd[w], gu + 3 * w);
            to_physical(Ja, iJ, gd[3], gc);
        }
        Tn = temperature<fast_fp64<T>()>(a.ph, (double)un[0], (double)un[1], (double)un[2], (double)un[3], (double)un[4],
                         (double)un[5], (double)gc[0], (double)gc[1], (double)gc[2]);
    }
    __syncthreads();
    if (act) {
        sA[0][t] = T(Tn);
        if constexpr (CV) {
            // contravariant components Ja^d . grad c for the divergence lifting
#pragma unroll
            for (int d = 0; d < 3; ++d)
                sA[1 + d][t] = sJa[3 * d][t] * gc[0] + sJa[3 * d + 1][t] * gc[1] + sJa[3 * d + 2][t] * gc[2];
        } else {
#pragma unroll
            for (int m = 0; m < 3; ++m) sA[1 + m][t] = gc[m];
        }
#pragma unroll
        for (int r = 0; r < 9; ++r) sGu[r][t] = gu[r];
    }
    __syncthreads();
    if (a.mesh.dyn) {
        // Navier-slip walls with gamma_1 != 0: the contact-angle flux gains
        // (gamma_1/gamma) div u, div u the trace of the lifted velocity gradient
        for (int task = t; task < G::NF; task += BS) {
            const FaceTask<P> ft(task);
            const int el = e0 + ft.le, f = ft.f;
            if (el >= E) continue;
            if (gld(a.mesh.nbr, el * 6 + f) >= 0) continue;  // interior: no wall-table entry
            const BcDev &bc = a.mesh.bcs[a.mesh.bcid[el * 6 + f] - 1];
            if (bc.kind != 3 || bc.g1 == 0.0) continue;
            const T *Lf = sL + (f & 1) * P;
            const int lo = ft.le * G::n3 + ft.off, ls = ft.str;
            T d0 = T(0), d1 = T(0), d2 = T(0);
#pragma unroll
            for (int l = 0; l < P; ++l) {
                d0 += T(Lf[l]) * sGu[0][lo + l * ls];
                d1 += T(Lf[l]) * sGu[4][lo + l * ls];
                d2 += T(Lf[l]) * sGu[8][lo + l * ls];
            }
            const T dS = face_dS<P, T, CV>(a.mesh, (size_t)el * 6 + f, ft.fp);
            sFs[ft.le * 6 * G::n2 + f * G::n2 + ft.fp] += T(bc.g1_gam) * ((d0 + d1) + d2) * dS;
        }
        __syncthreads();
    }
    // grad T (BR1 with T*) and lap c (divergence lifting of grad c)
    T gT[3] = {T(0), T(0), T(0)}, lap = T(0);
    if (act) {
        const int idx[3] = {i, j, k};
        const int fpd[3] = {j + P * k, i + P * k, i + P * j};
        const int base = le * G::n3;
        const int fbase = le * 6 * G::n2;
        if constexpr (CV) {
            // lap c: Dhat sweeps of the contravariant components; grad T: the
            // conservative lifting with the node metrics
            T dl = T(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int id = idx[d];
                const int p = d == 0 ? j : i, q = d == 2 ? j : k;
                T ad = T(0);
#pragma unroll
                for (int l = 0; l < P; ++l) ad += T(sDh[id * P + l]) * sA[1 + d][base + line_node<P>(d, l, p, q)];
                const int fp = fbase + (2 * d + 1) * G::n2 + fpd[d], fm_ = fbase + (2 * d) * G::n2 + fpd[d];
                dl += ad + T(sLh[P + id]) * sFs[fp] + T(sLh[id]) * sFs[fm_];
            }
            T qT[1][3];
            lifted_grads_curved<P, 1, G::NV, G::NF>(sA, &sTs, sJa, sN, base, fbase, i, j, k, sDh, sLh, iJ, qT);
            gT[0] = qT[0][0];
            gT[1] = qT[0][1];
            gT[2] = qT[0][2];
            lap = iJ * dl;
        } else {
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
        }
        gst(a.G2 + (0) * a.NN, g32, T(gT[0]));
        gst(a.G2 + (1) * a.NN, g32, T(gT[1]));
        gst(a.G2 + (2) * a.NN, g32, T(gT[2]));
        gst(a.G2 + (3) * a.NN, g32, T(lap));
    }
    __syncthreads();
    if constexpr (CV) {
        // curved elements: the normal varies along the face, so the face
        // tasks prolong grad u (already in sX), grad T and lap c and take
        // their normal components at each face point: grad T in sA[1..3],
        // lap c in sTs
        if (act) {
            sA[1][t] = gT[0];
            sA[2][t] = gT[1];
            sA[3][t] = gT[2];
            sTs[t] = lap;
        }
    } else {
        // per direction d, at the nodes: tau . n_d (3) and grad T . n_d with n_d
        // the outward normal of face 2d+1 (face 2d has exactly -n_d on these
        // affine elements), plus div u and lap c.  Their face values are the
        // prolongations of these nodal values (n_d is constant on the face), so
        // a face task prolongs 12 fields instead of 19.  Layout: direction 0 in
        // sA, directions 1 and 2 and div u in sX (each thread overwrites only its
        // own node's grad u, which it has read), lap c in sTs.
        if (act) {
            T gg[9];
#pragma unroll
            for (int r = 0; r < 9; ++r) gg[r] = sGu[r][t];
            const T div = gg[0] + gg[4] + gg[8];
            const T td = T(2.0 / 3.0) * div, mu = T(a.ph.mu);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const uint32_t fq = ((uint32_t)metric_element<G::EPB, G::n3>(e0, e) * 6 + 2 * d + 1) * 4;
                const T n0 = T(gld(a.mesh.fmet, fq)), n1 = T(gld(a.mesh.fmet, fq + 1)), n2 = T(gld(a.mesh.fmet, fq + 2));
                T *out = d == 0 ? &sA[0][0] : sX + (d - 1) * 4 * G::NV;
                out[0 * G::NV + t] = mu * ((gg[0] + gg[0]) * n0 + (gg[1] + gg[3]) * n1 + (gg[2] + gg[6]) * n2 - td * n0);
                out[1 * G::NV + t] = mu * ((gg[3] + gg[1]) * n0 + (gg[4] + gg[4]) * n1 + (gg[5] + gg[7]) * n2 - td * n1);
                out[2 * G::NV + t] = mu * ((gg[6] + gg[2]) * n0 + (gg[7] + gg[5]) * n1 + (gg[8] + gg[8]) * n2 - td * n2);
                out[3 * G::NV + t] = gT[0] * n0 + gT[1] * n1 + gT[2] * n2;
            }
            sX[8 * G::NV + t] = div;
            sTs[t] = lap;
        }
    }
    __syncthreads();
    // own-face flux traces, one face point per task: G = (F^C - F^V).n and
    // the wave speed; on walls the complete wall flux in G.  Each field group
    // is folded into the six flux components as soon as it is prolonged, so
    // few values stay live.
    for (int task = t; task < G::NF; task += BS) {
        {
            const FaceTask<P> ft(task);
            const int el = e0 + ft.le, f = ft.f;
            if (el >= E) continue;
            const T *Lf = sL + (f & 1) * P;
            const int lo = ft.le * G::n3 + ft.off, ls = ft.str;
            auto pro = [&](const T *fld) {
                T acc = T(0);
#pragma unroll
                for (int l = 0; l < P; ++l) acc += T(Lf[l]) * fld[lo + l * ls];
                return acc;
            };
            const FaceIx<G::n2> o((size_t)el * 6 + f, ft.fp);
            T nrm[3], dSf;
            bool wall;
            if constexpr (kOne) {  // task == t: the values loaded with the traces
                nrm[0] = tr0.n[0];
                nrm[1] = tr0.n[1];
                nrm[2] = tr0.n[2];
                dSf = tr0.dS;
                wall = tr0.nb < 0;
            } else {
                face_normal<P, T, CV>(a.mesh, (size_t)el * 6 + f, ft.fp, nrm, dSf);
                wall = gld(a.mesh.nbr, el * 6 + f) < 0;
            }
            const T n0 = nrm[0], n1 = nrm[1], n2 = nrm[2];
            int kind = 0;  // interior faces have no wall-table entry
            if (wall) kind = a.mesh.bcs[a.mesh.bcid[el * 6 + f] - 1].kind;
            // state and convective part
            // scheduling barriers keep each field group's LDS loads next to the
            // arithmetic that consumes them (otherwise all of them are hoisted
            // and the register demand limits occupancy)
            T rho, m0, m1, m2, E, c, gcn;
            double Tf;
            if (kKeep && task == t) {
                rho = tr0.uo[0]; m0 = tr0.uo[1]; m1 = tr0.uo[2]; m2 = tr0.uo[3]; E = tr0.uo[4]; c = tr0.uo[5];
                gcn = tr0.own[0];
                Tf = (double)tr0.own[1];
                if constexpr (sizeof(T) == 4) Tf += (double)tr0.own[2];
            } else {
                rho = TU[o.at(6, 0)]; m0 = TU[o.at(6, 1)]; m1 = TU[o.at(6, 2)]; m2 = TU[o.at(6, 3)];
                E = TU[o.at(6, 4)]; c = TU[o.at(6, 5)];
                gcn = a.T2[o.at(kT2<T>(), 0)];
                // the face temperature as recovered in FP64 (FP32: value + rounding error)
                Tf = (double)a.T2[o.at(kT2<T>(), 1)];
                if constexpr (sizeof(T) == 4) Tf += (double)a.T2[o.at(kT2<T>(), 2)];
            }
            __builtin_amdgcn_sched_barrier(0);
            const T ir = T(1) / rho;
            const T u0 = m0 * ir, u1 = m1 * ir, u2 = m2 * ir;
            const T mn = m0 * n0 + m1 * n1 + m2 * n2;
            const T un = mn * ir;
            double pd, cs2;
            eos<fast_fp64<T>()>(a.ph, (double)rho, Tf, pd, cs2);
            // model 2: p_alpha and its sound speed (ap = 0 for model 1)
            const T p = T(pd + 0.5 * a.ph.ap * (double)rho * (double)rho);
            const T cw = sqrt_to<T>(fabs(cs2 + a.ph.ap * (double)rho));
            const T lam = fabs(un) + cw;
            // interior faces of model 2 store p_alpha, -F^V.n and the sound
            // speed; the HLLC flux is formed from both sides' traces later
            const bool hl = !wall && a.ph.model == 2;
            T G0, G1, G2_, G3, G4, G5;
            if (hl) {
                G0 = p;
                G1 = G2_ = G3 = G4 = G5 = T(0);
            } else if (!wall) {
                G0 = mn;
                G1 = m0 * un + p * n0;
                G2_ = m1 * un + p * n1;
                G3 = m2 * un + p * n2;
                G4 = (E + p) * un;
                G5 = c * un;
            } else if (kind == 1) {  // ghost velocity 2 u_w - u (same rho, c, T)
                const BcDev &bc = a.mesh.bcs[a.mesh.bcid[el * 6 + f] - 1];
                const T w0 = T(bc.uw[0]), w1 = T(bc.uw[1]), w2 = T(bc.uw[2]);
                const T r0 = m0 - rho * w0, r1 = m1 - rho * w1, r2 = m2 - rho * w2;
                G0 = T(0);
                G1 = r0 * un + p * n0 + lam * r0;
                G2_ = r1 * un + p * n1 + lam * r1;
                G3 = r2 * un + p * n2 + lam * r2;
                // energy: -(u.n + lam)/2 times the ghost's extra kinetic energy
                // 2 rho (|u_w|^2 - u_w . u)
                G4 = -(un + lam) * rho * (w0 * (w0 - u0) + w1 * (w1 - u1) + w2 * (w2 - u2));
                G5 = T(0);
            } else {                 // mirrored normal velocity only
                const T q = mn * un + p + lam * mn;
                G0 = T(0);
                G1 = q * n0;
                G2_ = q * n1;
                G3 = q * n2;
                G4 = T(0);
                G5 = T(0);
            }
            // viscous traction tau n = mu ((grad u + grad u^T) n - 2/3 div u n)
            __builtin_amdgcn_sched_barrier(0);
            // affine elements: the nodal normal components of direction f/2,
            // with the face's sign; curved: the normal components are taken
            // of the prolonged gradients at this face point
            const T sgn = (f & 1) ? T(1) : T(-1);
            const T *nf = (f >> 1) == 0 ? &sA[0][0] : sX + ((f >> 1) - 1) * 4 * G::NV;
            auto grad_T_n = [&]() {
                if constexpr (CV) return pro(sA[1]) * n0 + pro(sA[2]) * n1 + pro(sA[3]) * n2;
                else return sgn * pro(nf + 3 * G::NV);
            };
            T div, tn0, tn1, tn2;
            if constexpr (CV) {
                T gf[9];
#pragma unroll
                for (int r = 0; r < 9; ++r) gf[r] = pro(sGu[r]);  // gf[3 j + i] = d u_j / d x_i
                div = gf[0] + gf[4] + gf[8];
                const T td = T(2.0 / 3.0) * div, mu = T(a.ph.mu);
                tn0 = mu * ((gf[0] + gf[0]) * n0 + (gf[1] + gf[3]) * n1 + (gf[2] + gf[6]) * n2 - td * n0);
                tn1 = mu * ((gf[3] + gf[1]) * n0 + (gf[4] + gf[4]) * n1 + (gf[5] + gf[7]) * n2 - td * n1);
                tn2 = mu * ((gf[6] + gf[2]) * n0 + (gf[7] + gf[5]) * n1 + (gf[8] + gf[8]) * n2 - td * n2);
            } else {
                div = pro(sX + 8 * G::NV);
                tn0 = sgn * pro(nf);
                tn1 = sgn * pro(nf + G::NV);
                tn2 = sgn * pro(nf + 2 * G::NV);
            }
            if (!wall) {
                G1 -= tn0;
                G2_ -= tn1;
                G3 -= tn2;
                G4 -= tn0 * u0 + tn1 * u1 + tn2 * u2;
            } else if (kind == 1) {  // traction, and its work at the wall velocity
                const BcDev &bc = a.mesh.bcs[a.mesh.bcid[el * 6 + f] - 1];
                G1 -= tn0;
                G2_ -= tn1;
                G3 -= tn2;
                G4 -= tn0 * T(bc.uw[0]) + tn1 * T(bc.uw[1]) + tn2 * T(bc.uw[2]);
            } else {
                const T tnn = tn0 * n0 + tn1 * n1 + tn2 * n2;
                G1 -= tnn * n0;
                G2_ -= tnn * n1;
                G3 -= tnn * n2;
                if (kind == 3) {
                    // Navier slip: tangential traction gamma_1 div u grad_G c -
                    // gamma_2 (u_t - u_w,t), and its work on u_t
                    const BcDev &bc = a.mesh.bcs[a.mesh.bcid[el * 6 + f] - 1];
                    const T gc0 = a.T2[o.at(kT2<T>(), kT2gc<T>())], gc1 = a.T2[o.at(kT2<T>(), kT2gc<T>() + 1)],
                            gc2 = a.T2[o.at(kT2<T>(), kT2gc<T>() + 2)];
                    const T gcn = gc0 * n0 + gc1 * n1 + gc2 * n2;
                    const T w0 = T(bc.uw[0]), w1 = T(bc.uw[1]), w2 = T(bc.uw[2]);
                    const T wn = w0 * n0 + w1 * n1 + w2 * n2;
                    const T a1 = T(bc.g1) * div, a2 = T(bc.g2);
                    const T ut0 = u0 - un * n0, ut1 = u1 - un * n1, ut2 = u2 - un * n2;
                    const T t0 = a1 * (gc0 - gcn * n0) - a2 * (ut0 - (w0 - wn * n0));
                    const T t1 = a1 * (gc1 - gcn * n1) - a2 * (ut1 - (w1 - wn * n1));
                    const T t2 = a1 * (gc2 - gcn * n2) - a2 * (ut2 - (w2 - wn * n2));
                    G1 -= t0;
                    G2_ -= t1;
                    G3 -= t2;
                    G4 -= t0 * ut0 + t1 * ut1 + t2 * ut2;
                }
            }
            // heat flux
            __builtin_amdgcn_sched_barrier(0);
            // (interior faces have no wall-table entry: bcid is 0 there)
            if (!wall) {
                const T gTn = grad_T_n();
                G4 -= T(a.ph.kappa) * gTn;
            } else if (kind != 2) {
                const BcDev &bc = a.mesh.bcs[a.mesh.bcid[el * 6 + f] - 1];
                if (bc.iso) {
                    const T gTn = grad_T_n();
                    G4 -= T(a.ph.kappa) * gTn;
                } else {  // heat transfer, eq. bc_energy_alpha
                    const double itw = bc.var ? (double)a.TF[o.at(7, 6)] : bc.inv_tw;
                    G4 -= T(-bc.g3 * (itw - 1.0 / Tf));
                }
            }
            // order-parameter terms of j_e and F^V_c
            __builtin_amdgcn_sched_barrier(0);
            if (!wall) {
                const T lapc = pro(sTs);
                const T zeta = T(a.ph.beta) * (T(a.ph.gam) * lapc + T(a.ph.alpha) * (rho - c));
                G4 -= -T(a.ph.gam) * c * gcn * div + T(a.ph.gam) * gcn * zeta;
                G5 -= T(a.ph.gam * a.ph.beta) * gcn;
                a.TF[o.at(7, 6)] = hl ? cw : lam;
            } else if (kind != 2) {
                // contact-angle flux g (with gamma_1 div u on Navier-slip
                // walls), as the second lifting used it: sFs holds g dS; and
                // the wall value zeta_c = -gamma_1 gamma_4 div u
                const BcDev &bc = a.mesh.bcs[a.mesh.bcid[el * 6 + f] - 1];
                const T gw = sFs[ft.le * 6 * G::n2 + f * G::n2 + ft.fp] / dSf;
                const T zeta = -T(bc.g1 * bc.g4) * div;
                G4 -= -T(a.ph.gam) * c * gw * div + T(a.ph.gam) * gw * zeta;
                G5 -= T(a.ph.gam * a.ph.beta) * gw;
            }
            a.TF[o.at(7, 0)] = G0;
            a.TF[o.at(7, 1)] = G1;
            a.TF[o.at(7, 2)] = G2_;
            a.TF[o.at(7, 3)] = G3;
            a.TF[o.at(7, 4)] = G4;
            a.TF[o.at(7, 5)] = G5;
        }
    }
}

// ------------------------------------------------------------ k_update
template <int P, typename T, int BS, bool BATCH, bool CV = false, bool NT = false>
__global__ __launch_bounds__(BS) void k_update(Launch<T> L)
{
    using G = Tile<P, BS>;
    Inst<T> a;
    int e0;
    instance_of<T, BATCH>(L, a, e0, G::EPB);
    // sF: primitives; contravariant fluxes (even directions); new state.
    // sB: BR1 face values of the primitives [5][NF], then the contravariant
    // fluxes of the odd direction [6][NV].
    constexpr int kB = 5 * G::NF > 6 * G::NV ? 5 * G::NF : 6 * G::NV;
    __shared__ T sF[6][G::NV];
    __shared__ T sB[kB];
    __shared__ T sFs[6][G::NF];    // surface flux (F* . n) dS
    // curved elements: the metrics of every node and n dS of every face point
    constexpr int NJ = CV ? 9 : 1, NQ = CV ? 3 : 1, NJV = CV ? G::NV : 1, NQF = CV ? G::NF : 1;
    __shared__ T sJa[NJ][NJV];
    __shared__ T sN[NQ][NQF];
    T(*sS)[G::NF] = reinterpret_cast<T(*)[G::NF]>(sB);
    T(*sF2)[G::NV] = reinterpret_cast<T(*)[G::NV]>(sB);
    __shared__ T sDh[P * P], sL[2 * P], sLh[2 * P];
    load_basis<P>(L.bas, sDh, sL, sLh);
    const int E = a.mesh.E;
    const int t = threadIdx.x;
    const int le = t / G::n3, nd = t - le * G::n3;
    const int e = e0 + le;
    const bool act = t < G::NV && e < E;
    const size_t g = (size_t)e0 * G::n3 + t;
    const uint32_t g32 = (uint32_t)g;
    const size_t NF = (size_t)E * 6 * G::n2;
    const T *TUr = a.TU + (size_t)L.tb * 6 * NF;

    // face tasks (one face point per thread, a second round where the block
    // has more face points than threads); the first round's traces are
    // requested before the node loads so that both are in flight together
    struct Tr {
        int nb;
        T uo[6], un[6], G[7], Gn[7];
    };
    auto load_tr = [&](int task, Tr &r) {
        const FaceTask<P> ft(task);
        const int el = e0 + ft.le;
        r.nb = -1;
        if (el >= E) return;
        const FaceIx<G::n2> o((size_t)el * 6 + ft.f, ft.fp);
        r.nb = gld(a.mesh.nbr, el * 6 + ft.f);
#pragma unroll
        for (int v = 0; v < 6; ++v) r.uo[v] = TUr[o.at(6, v)];
#pragma unroll
        for (int v = 0; v < 6; ++v) r.G[v] = a.TF[o.at(7, v)];
        if (r.nb >= 0) {
            const FaceIx<G::n2> on(nbr_face<P>(r.nb), nbr_point<P>(r.nb, ft.fp));
            r.G[6] = a.TF[o.at(7, 6)];
#pragma unroll
            for (int v = 0; v < 7; ++v) r.Gn[v] = a.TF[on.at(7, v)];
#pragma unroll
            for (int v = 0; v < 6; ++v) r.un[v] = TUr[on.at(6, v)];
        }
    };
    // (only where one round covers the block: holding a round's traces across
    // the node loads costs too many registers otherwise)
    constexpr bool kEarly = G::NF <= BS;
    Tr tr0;
    if (kEarly && t < G::NF) load_tr(t, tr0);
    Pt<T> s;
    T iJn = T(0);
    if (act) {
        if constexpr (CV) iJn = stage_node_metrics<T, NJV>(a.mesh, a.NN, g, t, sJa);
        s.rho = gldn<NT>(a.U + (0) * a.NN, g32);
        s.m[0] = gldn<NT>(a.U + (1) * a.NN, g32);
        s.m[1] = gldn<NT>(a.U + (2) * a.NN, g32);
        s.m[2] = gldn<NT>(a.U + (3) * a.NN, g32);
        s.E = gldn<NT>(a.U + (4) * a.NN, g32);
        s.c = gldn<NT>(a.U + (5) * a.NN, g32);
        const T u6[6] = {s.rho, s.m[0], s.m[1], s.m[2], s.E, s.c};
        T w[5];
        primitives(u6, w);
#pragma unroll
        for (int k = 0; k < 5; ++k) sF[k][t] = w[k];
    }
    // per face point: BR1 face values of the primitives, and the Rusanov +
    // central viscous flux (F* . n) dS from both sides' traces (the own
    // side's conserved trace is the prolongation of the current state,
    // written by the previous stage)
    for (int task = t; task < G::NF; task += BS) {
        const FaceTask<P> ft(task);
        const int el = e0 + ft.le, f = ft.f;
        if (el >= E) continue;
        Tr tr;
        if (kEarly) tr = tr0; else load_tr(task, tr);
        // the surface element always; the normal where it is used (walls,
        // model 2's HLLC, the lifting's n dS on curved elements)
        T n[3] = {T(0), T(0), T(0)}, dS;
        if (CV || tr.nb < 0 || a.ph.model == 2)
            face_normal<P, T, CV>(a.mesh, (size_t)el * 6 + f, ft.fp, n, dS);
        else
            dS = face_dS<P, T, CV>(a.mesh, (size_t)el * 6 + f, ft.fp);
        const int slot = ft.le * 6 * G::n2 + f * G::n2 + ft.fp;
        if constexpr (CV) {
#pragma unroll
            for (int m = 0; m < 3; ++m) sN[m][slot] = n[m] * dS;
        }
        T w[5];
        primitives(tr.uo, w);
        if (tr.nb >= 0 && a.ph.model == 2) {
            // HLLC on the convective part, central viscous flux: the traces
            // hold p_alpha, -F^V.n (own normal) and the sound speed
            // (face values and the viscous part go to LDS first, so that
            // they are not held in registers across the HLLC arithmetic)
            T wn[5];
            primitives(tr.un, wn);
#pragma unroll
            for (int k = 0; k < 5; ++k) sS[k][slot] = T(0.5) * (w[k] + wn[k]);
#pragma unroll
            for (int v = 1; v < 6; ++v) sFs[v][slot] = T(0.5) * (tr.G[v] - tr.Gn[v]) * dS;
            T Fc[6];
            hllc(tr.uo, tr.G[0], tr.G[6], tr.un, tr.Gn[0], tr.Gn[6], n, Fc);
            sFs[0][slot] = Fc[0] * dS;
#pragma unroll
            for (int v = 1; v < 6; ++v) sFs[v][slot] += Fc[v] * dS;
            continue;
        } else if (tr.nb >= 0) {
            T wn[5];
            const T lam = tr.G[6] > tr.Gn[6] ? tr.G[6] : tr.Gn[6];
#pragma unroll
            for (int v = 0; v < 6; ++v) {
                const T Fn = T(0.5) * (tr.G[v] - tr.Gn[v]) - T(0.5) * lam * (tr.un[v] - tr.uo[v]);
                sFs[v][slot] = Fn * dS;
            }
            primitives(tr.un, wn);
#pragma unroll
            for (int k = 0; k < 5; ++k) w[k] = T(0.5) * (w[k] + wn[k]);
        } else {
#pragma unroll
            for (int v = 0; v < 6; ++v) sFs[v][slot] = tr.G[v] * dS;
            wall_primitives(a.mesh, el, f, n, w);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) sS[k][slot] = w[k];
    }
    __syncthreads();
    // lifted gradients, temperature, pressure and the point-wise source
    T S[6] = {T(0), T(0), T(0), T(0), T(0), T(0)}, iJ = T(0);
    T Fx[6][3];
    const int i = nd % P, j = (nd / P) % P, k = nd / (P * P);
    const int base = le * G::n3;
    if (act) {
#pragma unroll
        for (int m = 0; m < 3; ++m) s.gT[m] = gldn<NT>(a.G2 + (m) * a.NN, g32);
        s.lapc = gldn<NT>(a.G2 + (3) * a.NN, g32);
        T grho[3];
        if constexpr (CV) {
            T q[5][3];
            lifted_grads_curved<P, 5, G::NV, G::NF>(sF, sS, sJa, sN, base, le * 6 * G::n2, i, j, k, sDh, sLh, iJn, q);
            iJ = iJn;
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                grho[m] = q[0][m];
                s.gu[0][m] = q[1][m];
                s.gu[1][m] = q[2][m];
                s.gu[2][m] = q[3][m];
                s.gc[m] = q[4][m];
            }
        } else {
            T gd[5][3];
            lifted_grads<P, 5>(sF, sS, base, le * 6 * G::n2, i, j, k, sDh, sLh, gd);
            T Ja[9];
            element_metrics(a.mesh, metric_element<G::EPB, G::n3>(e0, e), Ja, iJ);
            to_physical(Ja, iJ, gd[0], grho);
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) to_physical(Ja, iJ, gd[1 + jj], s.gu[jj]);
            to_physical(Ja, iJ, gd[4], s.gc);
        }
        // the temperature stays FP64 through the pressure in both precisions
        const double Tn = temperature<fast_fp64<T>()>(a.ph, (double)s.rho, (double)s.m[0], (double)s.m[1],
                                                      (double)s.m[2], (double)s.E, (double)s.c, (double)s.gc[0],
                                                      (double)s.gc[1], (double)s.gc[2]);
        double pd, cs2;
        eos<fast_fp64<T>()>(a.ph, (double)s.rho, Tn, pd, cs2);
        s.p = T(pd + 0.5 * a.ph.ap * (double)s.rho * (double)s.rho);  // p_alpha for model 2
        s.ir = T(1) / s.rho;
        source(a.ph, s, grho, S);
        flux_tensor(a.ph, s, Fx);
    }
    // the RK register (and the compensation of an FP32 instance) of this
    // node, requested now so that the loads complete during the volume
    // integral
    T Rn[6], Cn[6];
    if (L.mode == 1 && act) {
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            Rn[v] = L.first ? T(0) : gldn<NT>(a.R + (v) * a.NN, g32);
            if constexpr (sizeof(T) == 4) Cn[v] = a.Ck ? gldn<NT>(a.Ck + (v) * a.NN, g32) : T(0);
        }
    }
    // volume integral sum_d Dhat_d (Ja^d . F): the contravariant fluxes of
    // direction d go to buffer d & 1, so direction d+1 is written while
    // direction d is read, one barrier per direction
    T acc[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
    auto put_flux = [&](int d, T (*buf)[G::NV]) {
        T Jd[3];
        if constexpr (CV) {
            Jd[0] = sJa[3 * d][t];
            Jd[1] = sJa[3 * d + 1][t];
            Jd[2] = sJa[3 * d + 2][t];
        } else {
            const uint32_t eq = (uint32_t)metric_element<G::EPB, G::n3>(e0, e) * 10 + 3 * d;
            Jd[0] = T(gld(a.mesh.emet, eq));
            Jd[1] = T(gld(a.mesh.emet, eq + 1));
            Jd[2] = T(gld(a.mesh.emet, eq + 2));
        }
#pragma unroll
        for (int v = 0; v < 6; ++v) buf[v][t] = Jd[0] * Fx[v][0] + Jd[1] * Fx[v][1] + Jd[2] * Fx[v][2];
    };
    __syncthreads();
    if (act) put_flux(0, sF);
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
        __syncthreads();
        if (act) {
            if (d < 2) put_flux(d + 1, (d & 1) ? sF : sF2);
            __builtin_amdgcn_sched_barrier(0);
            const T(*buf)[G::NV] = (d & 1) ? sF2 : sF;
            // the line through this node along d, addressed branch-free:
            // node l is lo + l * str
            const int id = d == 0 ? i : (d == 1 ? j : k);
            const int str = d == 0 ? 1 : (d == 1 ? P : P * P);
            const int lo = base + nd - id * str;
#pragma unroll
            for (int l = 0; l < P; ++l) {
                const T D = T(sDh[id * P + l]);
#pragma unroll
                for (int v = 0; v < 6; ++v) acc[v] += D * buf[v][lo + l * str];
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
    if (L.mode == 0) {
        if (act) {
#pragma unroll
            for (int v = 0; v < 6; ++v) gst(a.Ut + (v) * a.NN, g32, T(Ut[v]));
        }
        return;
    }
    // low-storage RK stage
    __syncthreads();
    if (act) {
        const T A = T(L.A), B = T(L.B), dt = T(a.dt);
        T u6[6] = {s.rho, s.m[0], s.m[1], s.m[2], s.E, s.c};
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            const T r = L.first ? dt * Ut[v] : A * Rn[v] + dt * Ut[v];
            if (!L.last) gstn<NT>(a.R + (v) * a.NN, g32, T(r));
            T u;
            if (sizeof(T) == 4 && a.Ck) {
                // compensated summation: the low-order part lost by u6 + B r is
                // kept in Ck and fed into the next stage's increment
                const T y = B * r - Cn[v];
                u = u6[v] + y;
                gstn<NT>(a.Ck + (v) * a.NN, g32, T((u - u6[v]) - y));
            } else {
                u = u6[v] + B * r;
            }
            gstn<NT>(a.U + (v) * a.NN, g32, T(u));
            sF[v][t] = u;
        }
    }
    __syncthreads();
    const int ltask = line_of_thread<P, BS>(t);
    const LineTask<P> lt(ltask < 0 ? 0 : ltask);
    const int el = e0 + lt.le;
    const bool lact = ltask >= 0 && el < E;
    if (lact) {
        T *TUw = a.TU + (size_t)L.tw * 6 * NF;
        const int b2 = lt.le * G::n3;
        T um[6], up[6];
#pragma unroll
        for (int v = 0; v < 6; ++v) prolong2<P>(sF[v], b2, sL, lt, um[v], up[v]);
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const FaceIx<G::n2> o((size_t)el * 6 + 2 * lt.d + sd, lt.fp);
#pragma unroll
            for (int v = 0; v < 6; ++v) TUw[o.at(6, v)] = sd ? up[v] : um[v];
        }
    }
}

}  // namespace nskr
