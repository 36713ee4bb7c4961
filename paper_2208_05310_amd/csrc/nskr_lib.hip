// nskr_lib.hip -- host side of the gfx950 library behind include/nskr.h:
// argument validation, mesh and metric upload, per-wall constants, launch
// sequences of the DGSEM stages, the low-storage RK loop, the FP64 time-step
// and integral reductions, and the droplet initialisation.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/nskr.h"
#include "nskr_kernels.hpp"

using namespace nskr;

// ------------------------------------------------------------------ context
struct nskr_ctx {
    nskr_params p;
    int N = 0, P = 0, device = 0;
    int bs = 256;               // threads per block of the stage kernels
    bool poisoned = false;
    std::string err;
    // mesh
    int E = 0;
    size_t NN = 0, NF = 0;
    int *d_nbr = nullptr, *d_bcid = nullptr;
    double *d_emet = nullptr, *d_fmet = nullptr, *d_egeo = nullptr;
    bool curved = false;         // some element is not affine: per-node metrics
    void *d_nmet = nullptr, *d_fnrm = nullptr;  // curved: node metrics, face-point normals (element type)
    double *d_xnode = nullptr;   // curved: node coordinates
    BcDev *d_bcs = nullptr;
    int dyn = 0;                 // a Navier-slip wall with gamma_1 != 0
    double *d_stab = nullptr;    // wall-temperature table (walls with a temperature gradient)
    int var = 0;                 // some wall has a temperature gradient or rate
    int trate = 0;               // some wall's temperature changes in time
    double time = 0.0;           // simulation time (walls whose temperature changes in time)
    std::vector<std::array<double, 3>> wall_trange;  // per wall: min, max of twall + grad . x over it; rate
    // scratch (element type of the precision)
    void *d_Q = nullptr, *d_TH = nullptr, *d_G2 = nullptr, *d_T2 = nullptr, *d_TF = nullptr, *d_TU = nullptr;
    void *d_Ck = nullptr;        // Kahan compensation of the FP32 state update
    int *d_clk = nullptr;        // batch: steps since admission (walls whose temperature changes in time)
    double *d_part = nullptr;    // reduction partials
    double *d_out = nullptr;     // final reduction values (device)
    double *d_noise = nullptr;   // init noise
    double *d_drop = nullptr;    // init droplets
    std::vector<float> cent;     // element centroids (host), for the block order
    int *d_bmap = nullptr;       // first element of every stage-kernel block, in XCD order
    int bmap_bs = 0;             // block size d_bmap was built for
    int stream_nodes = 0;        // the update kernel's node arrays stream past the last-level cache
    size_t bytes = 0;
    Basis bas;
    Phys ph;
    // optional per-kernel event timing
    bool prof = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_events;
    std::vector<hipEvent_t> event_pool;
};

// Events for per-kernel timing, reused across profile reads.
static hipEvent_t take_event(nskr_ctx *c)
{
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch one stage kernel.  With profiling on, the event pair rides on the
// dispatch itself, so the recorded interval is the kernel's own begin-to-end
// time (no dispatch gap, no marker packets between kernels).
template <typename T>
static void stage_launch(nskr_ctx *c, int kind, void (*kern)(Launch<T>), unsigned grid, unsigned block,
                         hipStream_t s, const Launch<T> &L)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->prof) {
        a = take_event(c);
        b = take_event(c);
    }
    if (a && b) {
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, a, b, 0, L);
        c->prof_events.push_back({kind, {a, b}});
        return;
    }
    if (a) c->event_pool.push_back(a);
    if (b) c->event_pool.push_back(b);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, L);
}

static const char *g_null_msg = "nskr: null context";

static int fail(nskr_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(c, x)                                                                    \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            (c)->poisoned = true;                                                       \
            return fail((c), NSKR_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
        }                                                                               \
    } while (0)

struct DeviceGuard {
    int old = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&old) != hipSuccess) old = -1;
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (old >= 0) (void)hipSetDevice(old);
    }
};

// ------------------------------------------------------------ host numerics
// Legendre-Gauss nodes/weights, Lagrange face values and the weak derivative
// matrix, computed in extended precision and rounded once.
typedef long double ld;

static void legendre_ld(int n, ld x, ld &Pn, ld &dPn)
{
    ld p0 = 1, p1 = x;
    if (n == 0) { Pn = 1; dPn = 0; return; }
    for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    Pn = p1;
    dPn = n * (x * p1 - p0) / (x * x - 1);  // derivative identity of Legendre polynomials
}

static void make_basis(int N, Basis &b)
{
    const int P = N + 1;
    ld x[8], w[8];
    for (int i = 0; i < P; ++i) {
        // Chebyshev-Gauss initial guess, Newton on P_{N+1}
        ld xi = -cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (P + 0.5L));
        for (int it = 0; it < 60; ++it) {
            ld Pn, dP;
            legendre_ld(P, xi, Pn, dP);
            ld dx = Pn / dP;
            xi -= dx;
            if (fabsl(dx) < 1e-21L) break;
        }
        ld Pn, dP;
        legendre_ld(P, xi, Pn, dP);
        x[i] = xi;
        w[i] = 2 / ((1 - xi * xi) * dP * dP);
    }
    // barycentric weights
    ld lam[8];
    for (int j = 0; j < P; ++j) {
        ld prod = 1;
        for (int k = 0; k < P; ++k)
            if (k != j) prod *= x[j] - x[k];
        lam[j] = 1 / prod;
    }
    ld D[8][8];
    for (int i = 0; i < P; ++i) {
        ld s = 0;
        for (int j = 0; j < P; ++j) {
            if (i == j) continue;
            D[i][j] = lam[j] / (lam[i] * (x[i] - x[j]));
            s += D[i][j];
        }
        D[i][i] = -s;
    }
    memset(&b, 0, sizeof(b));
    for (int i = 0; i < P; ++i)
        for (int l = 0; l < P; ++l) b.Dh[i * P + l] = (double)(-(w[l] / w[i]) * D[l][i]);
    for (int j = 0; j < P; ++j) {
        // l_j(+-1) from the barycentric form of the second kind
        for (int sgn = 0; sgn < 2; ++sgn) {
            ld xe = sgn ? 1.0L : -1.0L, num = 0, den = 0;
            for (int k = 0; k < P; ++k) {
                ld t = lam[k] / (xe - x[k]);
                den += t;
                if (k == j) num = t;
            }
            ld val = num / den;
            b.L[sgn][j] = (double)val;
            b.Lh[sgn][j] = (double)(val / w[j]);
        }
        b.w[j] = (double)w[j];
        b.x[j] = (double)x[j];
    }
}

// van der Waals thermodynamics on the host (Sec. 2.1), extended precision.
struct Vdw {
    ld R, a, b;
    ld p(ld r, ld T) const { return r * R * T / (1 - b * r) - a * r * r; }
    ld dp(ld r, ld T) const { return R * T / ((1 - b * r) * (1 - b * r)) - 2 * a * r; }
    ld mu(ld r, ld T) const { return R * T * logl(b * r / (1 - b * r)) + R * T / (1 - b * r) - 2 * a * r; }
    ld dmu(ld r, ld T) const { return dp(r, T) / r; }  // d mu / d rho = (dp/drho) / rho
    ld psi_nl(ld r, ld T) const { return r * R * T * logl(b * r / (1 - b * r)) - a * r * r; }
};

static bool maxwell_newton(const Vdw &v, ld T, ld sv, ld sl, ld &rv, ld &rl);

// Maxwell states: Newton on p(rv) = p(rl), mu(rv) = mu(rl), started from the
// two spinodal densities pushed outwards, with a step-halving guard that keeps
// both iterates on their branches.
static bool maxwell_host(const Vdw &v, ld T, ld &rv, ld &rl)
{
    // spinodal: zeros of dp/drho; bracket them by scanning
    const ld rmax = 1 / v.b;
    ld sv = -1, sl = -1, prev = v.dp(rmax * 1e-6L, T);
    const int n = 20000;
    for (int k = 1; k < n; ++k) {
        ld r = rmax * k / n, d = v.dp(r, T);
        if (prev > 0 && d <= 0 && sv < 0) sv = r;
        if (prev < 0 && d >= 0 && sv > 0 && sl < 0) sl = r;
        prev = d;
    }
    if (sv < 0 || sl < 0) return false;
    rv = 0.5L * sv;
    rl = 0.5L * (sl + rmax);
    return maxwell_newton(v, T, sv, sl, rv, rl);
}

// Newton for the Maxwell states from (rv, rl), each iterate kept inside (0, sv)
// and (sl, 1/b) by step halving.
static bool maxwell_newton(const Vdw &v, ld T, ld sv, ld sl, ld &rv, ld &rl)
{
    const ld rmax = 1 / v.b;
    for (int it = 0; it < 200; ++it) {
        ld f1 = v.p(rv, T) - v.p(rl, T), f2 = v.mu(rv, T) - v.mu(rl, T);
        ld a11 = v.dp(rv, T), a12 = -v.dp(rl, T), a21 = v.dmu(rv, T), a22 = -v.dmu(rl, T);
        ld det = a11 * a22 - a12 * a21;
        ld dv = (f1 * a22 - a12 * f2) / det, dl = (a11 * f2 - a21 * f1) / det;
        ld s = 1;
        while (s > 1e-6L && (rv - s * dv <= 0 || rv - s * dv >= sv || rl - s * dl <= sl || rl - s * dl >= rmax)) s *= 0.5L;
        rv -= s * dv;
        rl -= s * dl;
        if (fabsl(dv) < 1e-19L * rv && fabsl(dl) < 1e-19L * rl) break;
    }
    return fabsl(v.p(rv, T) - v.p(rl, T)) < 1e-14L && fabsl(v.mu(rv, T) - v.mu(rl, T)) < 1e-13L;
}

// Surface tension of eq. surftenscoef with the prefactor sqrt(2 gamma):
// composite 16-point Gauss-Legendre over 48 panels of [rv, rl].
static ld sigma_host(const Vdw &v, ld T, ld gam, ld rv, ld rl)
{
    const int m = 16;
    ld x[16], w[16];
    for (int i = 0; i < m; ++i) {
        ld xi = -cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (m + 0.5L));
        for (int it = 0; it < 60; ++it) {
            ld Pn, dP;
            legendre_ld(m, xi, Pn, dP);
            ld dx = Pn / dP;
            xi -= dx;
            if (fabsl(dx) < 1e-21L) break;
        }
        ld Pn, dP;
        legendre_ld(m, xi, Pn, dP);
        x[i] = xi;
        w[i] = 2 / ((1 - xi * xi) * dP * dP);
    }
    const ld muv = v.mu(rv, T), psiv = v.psi_nl(rv, T);
    const int panels = 48;
    const ld h = (rl - rv) / panels;
    ld I = 0;
    for (int k = 0; k < panels; ++k) {
        ld A = rv + k * h;
        for (int i = 0; i < m; ++i) {
            ld r = A + 0.5L * h * (x[i] + 1);
            ld d = v.psi_nl(r, T) - (psiv + (r - rv) * muv);
            I += 0.5L * h * w[i] * (d > 0 ? sqrtl(d) : 0);
        }
    }
    return sqrtl(2 * gam) * I;
}

// sigma_vl / sqrt(2 gamma) by the single 15-point Gauss-Legendre rule over
// [rv, rl] that the wall-temperature table of Sec. 3.2 prescribes.
static ld sigma15_host(const Vdw &v, ld T, ld rv, ld rl)
{
    const int m = 15;
    const ld muv = v.mu(rv, T), psiv = v.psi_nl(rv, T);
    ld I = 0;
    for (int i = 0; i < m; ++i) {
        ld xi = -cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (m + 0.5L));
        for (int it = 0; it < 60; ++it) {
            ld Pn, dP;
            legendre_ld(m, xi, Pn, dP);
            ld dx = Pn / dP;
            xi -= dx;
            if (fabsl(dx) < 1e-21L) break;
        }
        ld Pn, dP;
        legendre_ld(m, xi, Pn, dP);
        const ld wi = 2 / ((1 - xi * xi) * dP * dP);
        const ld r = 0.5L * (rv + rl) + 0.5L * (rl - rv) * xi;
        const ld d = v.psi_nl(r, T) - (psiv + (r - rv) * muv);
        I += 0.5L * (rl - rv) * wi * (d > 0 ? sqrtl(d) : 0);
    }
    return I;
}

// The wall-temperature table: kTabN temperatures T_k = 0.3 + k (0.7/(kTabN-1))
// with (sigma / sqrt(2 gamma), rho_v, rho_l); Maxwell states by Newton
// continued from the previous temperature (a full solve where that fails);
// the last entry is the critical point.  Built once per van der Waals fluid.
static const std::vector<double> &wall_table_host(const Vdw &v)
{
    static std::mutex mtx;
    static std::map<std::array<double, 3>, std::vector<double>> cache;
    std::lock_guard<std::mutex> lock(mtx);
    const std::array<double, 3> key{(double)v.R, (double)v.a, (double)v.b};
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    std::vector<double> tab(3 * kTabN);
    ld rv = 0, rl = 0;
    bool have = false;
    const ld rc = 1 / (3 * v.b);
    for (int k = 0; k < kTabN; ++k) {
        const double Tk = kTabT0 + k * ((kTabT1 - kTabT0) / (kTabN - 1));
        bool ok = false;
        if (k < kTabN - 1) {
            if (have) {
                ld a = rv, b = rl;
                ok = maxwell_newton(v, Tk, rc, rc, a, b) && a < rc && b > rc;
                if (ok) { rv = a; rl = b; }
            }
            if (!ok) ok = maxwell_host(v, Tk, rv, rl);
        }
        if (ok) {
            tab[3 * k] = (double)sigma15_host(v, Tk, rv, rl);
            tab[3 * k + 1] = (double)rv;
            tab[3 * k + 2] = (double)rl;
        } else {
            tab[3 * k] = 0.0;
            tab[3 * k + 1] = tab[3 * k + 2] = (double)rc;
        }
        have = ok;
    }
    return cache.emplace(key, std::move(tab)).first->second;
}

// ------------------------------------------------- RK and time-step constants
// 5-stage 2N-storage RK4(3)5, Carpenter & Kennedy (1994).
static const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                               -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
// stage times c_s of the same scheme (stage s is evaluated at t + c_s dt)
static const double kRkC[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                               2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};
static const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                               1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                               2277821191437.0 / 14882151754819.0};
// Conserved face-trace buffer read by stage s and written for stage s+1: three
// buffers so that no stage overwrites the buffer it reads, and the last stage
// writes the buffer the next step's first stage reads (k_prolong fills 0).
static const int kTraceBuf[6] = {0, 1, 0, 1, 2, 0};
// 1D stability constants (periodic Gauss DGSEM spectra under the scheme's
// stability polynomial), index N: advective dt a / h and diffusive spectral
// radius at h = 1; stability interval on the negative real axis.
static const double kTN[6] = {0, 0, 0.3521, 0.2200, 0.1523, 0.1126};
static const double kRhoN[6] = {0, 0, 64.8, 176.2, 387.0, 745.2};
static const double kRkReal = 4.6567;
// Wall limit of Navier-slip walls with gamma_1 > 0: spectral radius of the
// BR1 lifted first derivative on the reference element (Bloch spectrum of
// the periodic Gauss DGSEM), index N; stability interval on the imaginary axis.
static const double kSigN[6] = {0, 0, 4.0406, 6.6385, 9.8386, 13.6629};
static const double kRkImag = 3.3407;

// ------------------------------------------------------------ extra kernels
// Reduction operations: 0 sum, 1 min, 2 max.
__device__ __forceinline__ double combine(int kd, double x, double y)
{
    return kd == 0 ? x + y : (kd == 1 ? fmin(x, y) : fmax(x, y));
}

// Reduce over the 64 lanes of a wave by xor shuffles (every lane ends with
// the result; the pairing is fixed, so sums do not depend on timing).
__device__ __forceinline__ double wave_reduce(int kd, double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = combine(kd, v, __shfl_xor(v, off, 64));
    return v;
}

struct RateArgs {
    MeshDev mesh; Phys ph; size_t NN; double *part; int nblk;
    double sig;  // spectral radius of the lifted first derivative (wall limit)
};

// Number of time-step rates reduced by k_dt_rates: the advective rate, the
// mesh factor, the diffusivity and the wall rate.
constexpr int kNRates = 4;

// Wall rate of one node of element e (gamma_1 terms of the generalized
// Navier-slip condition, Sec. 2.4): for each Navier-slip face with gamma_1 > 0
// and face direction n, with Lambda = (N+1)^2/2 the Gauss surface-lifting
// weight, a = |Ja^n|/J and the tangential directions d,
//   sig (Lambda a gamma_1 sum_d |grad c . Ja^d|/(J rho)
//        + sqrt(alpha beta gamma_1 Lambda a sum_d (|Ja^d|/J)^2)),
// the traction gamma_1 div u grad_G c acting as a wall viscosity, and the
// c-flux beta gamma_1 div u closed through the alpha grad c source.
template <int P>
__device__ double wall_rate(const RateArgs &a, int e, const double *em, double rho, const double gc[3])
{
    const double lam = 0.5 * P * P, iJ = 1.0 / em[9];
    double r = 0.0;
    for (int f = 0; f < 6; ++f) {
        const int b = a.mesh.bcid[(size_t)e * 6 + f];
        if (!b) continue;
        const BcDev &bc = a.mesh.bcs[b - 1];
        if (bc.kind != 3 || !(bc.g1 > 0.0)) continue;
        const int dn = f >> 1;
        const double *An = em + 3 * dn;
        const double an = sqrt(An[0] * An[0] + An[1] * An[1] + An[2] * An[2]) * iJ;
        double st = 0.0, gt = 0.0;
        for (int d = 0; d < 3; ++d) {
            if (d == dn) continue;
            const double *Ad = em + 3 * d;
            const double nd = sqrt(Ad[0] * Ad[0] + Ad[1] * Ad[1] + Ad[2] * Ad[2]) * iJ;
            st += nd * nd;
            gt += fabs(gc[0] * Ad[0] + gc[1] * Ad[1] + gc[2] * Ad[2]) * iJ;
        }
        r += a.sig * (lam * an * bc.g1 * gt / rho + sqrt(a.ph.alpha * a.ph.beta * bc.g1 * lam * an * st));
    }
    return r;
}

template <int P, typename T, bool CV>
__global__ __launch_bounds__(kBlock) void k_dt_rates(const T *U, const T *Q, RateArgs a)
{
    using G = Tile<P>;
    __shared__ double sr[kNRates][kBlock / 64];
    const int t = threadIdx.x;
    const int e0 = blockIdx.x * G::EPB, le = t / G::n3, e = e0 + le;
    const size_t g = (size_t)e0 * G::n3 + t;
    double r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    if (t < G::NV && e < a.mesh.E) {
        double rho = U[g], m0 = U[a.NN + g], m1 = U[2 * a.NN + g], m2 = U[3 * a.NN + g];
        double E = U[4 * a.NN + g], c = U[5 * a.NN + g];
        double Tn = temperature(a.ph, rho, m0, m1, m2, E, c, Q[12 * a.NN + g], Q[13 * a.NN + g], Q[14 * a.NN + g]);
        double p, cs2;
        eos(a.ph, rho, Tn, p, cs2);
        double cs = sqrt(fabs(cs2 + a.ph.ap * rho));  // sound speed of the convective flux
        double em[10];
        if (CV) {
            const T *nm = (const T *)a.mesh.nmet;
            for (int r = 0; r < 10; ++r) em[r] = (double)nm[r * a.NN + g];
        } else {
            for (int r = 0; r < 10; ++r) em[r] = a.mesh.emet[(size_t)e * 10 + r];
        }
        double iJ = 1.0 / em[9];
        for (int d = 0; d < 3; ++d) {
            const double *Ja = em + 3 * d;
            double nJ = sqrt(Ja[0] * Ja[0] + Ja[1] * Ja[1] + Ja[2] * Ja[2]);
            r0 += (fabs(m0 * Ja[0] + m1 * Ja[1] + m2 * Ja[2]) / rho + cs * nJ) * iJ;
            double h = 0.5 * nJ * iJ;
            r1 += h * h;
        }
        r2 = fmax(fmax(4.0 * a.ph.mu / (3.0 * rho), a.ph.kappa / (rho * a.ph.R * a.ph.cv)), a.ph.gam * a.ph.beta);
        if (a.mesh.dyn) {
            const double gc[3] = {(double)Q[12 * a.NN + g], (double)Q[13 * a.NN + g], (double)Q[14 * a.NN + g]};
            r3 = wall_rate<P>(a, e, em, rho, gc);
        }
        if (!isfinite(r0) || !isfinite(r2) || !isfinite(r3)) r0 = r2 = INFINITY;
    }
    const double rv[kNRates] = {r0, r1, r2, r3};
    const int w = t >> 6, lane = t & 63;
#pragma unroll
    for (int k = 0; k < kNRates; ++k) {
        const double m = wave_reduce(2, rv[k]);
        if (lane == 0) sr[k][w] = m;
    }
    __syncthreads();
    if (t < kNRates) {
        double m = sr[t][0];
        for (int q = 1; q < kBlock / 64; ++q) m = fmax(m, sr[t][q]);
        a.part[(size_t)t * a.nblk + blockIdx.x] = m;
    }
}

// Final pass of a two-level reduction: workgroup k reduces partials
// part[k][0..nblk) with the operation of kind(k) (0 sum, 1 min, 2 max): each
// thread over a fixed stride, then the wave shuffles and the waves in order,
// so that the result does not depend on timing.
template <typename KindF>
__device__ __forceinline__ void reduce_final(const double *part, int nblk, double *out, KindF kind)
{
    __shared__ double s[kBlock / 64];
    const int k = blockIdx.x, kd = kind(k);
    double m = kd == 0 ? 0.0 : (kd == 1 ? INFINITY : -INFINITY);
    for (int b = threadIdx.x; b < nblk; b += kBlock) m = combine(kd, m, part[(size_t)k * nblk + b]);
    m = wave_reduce(kd, m);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = s[0];
        for (int q = 1; q < kBlock / 64; ++q) r = combine(kd, r, s[q]);
        out[k] = r;
    }
}

// maxima of the time-step rates: one workgroup per value
__global__ __launch_bounds__(kBlock) void k_max_final(const double *part, int nblk, double *out)
{
    reduce_final(part, nblk, out, [](int) { return 2; });
}

// Integrals: kinds 0 = sum, 1 = min, 2 = max for the NSKR_SUM_* slots.
__device__ __forceinline__ int sum_kind(int k) { return k == 10 || k == 12 ? 1 : (k == 11 || k == 13 ? 2 : 0); }

template <int P, typename T, bool CV>
__global__ __launch_bounds__(kBlock) void k_integrals(const T *U, const T *Q, RateArgs a, Basis bas)
{
    using G = Tile<P>;
    __shared__ double sr[NSKR_NSUMS][kBlock / 64];
    const int t = threadIdx.x;
    const int e0 = blockIdx.x * G::EPB, le = t / G::n3, e = e0 + le, nd = t - le * G::n3;
    const size_t g = (size_t)e0 * G::n3 + t;
    double v[NSKR_NSUMS];
    for (int k = 0; k < NSKR_NSUMS; ++k) v[k] = 0.0;
    v[10] = v[12] = INFINITY;
    v[11] = v[13] = -INFINITY;
    if (t < G::NV && e < a.mesh.E) {
        const int i = nd % P, j = (nd / P) % P, k = nd / (P * P);
        const double Jn = CV ? (double)((const T *)a.mesh.nmet)[9 * a.NN + g] : a.mesh.emet[(size_t)e * 10 + 9];
        const double wJ = bas.w[i] * bas.w[j] * bas.w[k] * Jn;
        double u[6];
        bool bad = false;
        for (int q = 0; q < 6; ++q) {
            u[q] = (double)U[q * a.NN + g];
            if (!isfinite(u[q])) bad = true;
        }
        if (bad) {
            v[14] = 1.0;
        } else {
            const double q0 = Q[12 * a.NN + g], q1 = Q[13 * a.NN + g], q2 = Q[14 * a.NN + g];
            const double rho = u[0];
            const double Tn = temperature(a.ph, rho, u[1], u[2], u[3], u[4], u[5], q0, q1, q2);
            double p, cs2;
            eos(a.ph, rho, Tn, p, cs2);
            if (!(rho > 0.0 && rho * a.ph.b < 1.0)) v[15] = 1.0;
            if (!(Tn > 0.0)) v[16] = 1.0;
            if (cs2 < 0.0) v[17] = 1.0;
            const double g2 = q0 * q0 + q1 * q1 + q2 * q2;
            v[0] = wJ * rho;
            v[1] = wJ * u[1];
            v[2] = wJ * u[2];
            v[3] = wJ * u[3];
            v[4] = wJ * u[4];
            v[5] = wJ * u[5];
            v[6] = wJ * 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / rho;
            v[7] = wJ * 0.5 * a.ph.gam * g2;
            v[8] = wJ * 0.5 * a.ph.alpha * (rho - u[5]) * (rho - u[5]);
            v[9] = wJ * (rho - u[5]) * (rho - u[5]);
            v[10] = v[11] = rho;
            v[12] = v[13] = Tn;
            if (a.ph.b > 0.0 && Tn > 0.0 && rho > 0.0 && rho * a.ph.b < 1.0)
                v[18] = -wJ * rho * (a.ph.R * a.ph.cv * log(Tn) - a.ph.R * log(a.ph.b * rho / (1.0 - a.ph.b * rho)));
            v[19] = wJ;
        }
    }
    const int w = t >> 6, lane = t & 63;
#pragma unroll
    for (int k = 0; k < NSKR_NSUMS; ++k) {
        const double m = wave_reduce(sum_kind(k), v[k]);
        if (lane == 0) sr[k][w] = m;
    }
    __syncthreads();
    if (t < NSKR_NSUMS) {
        const int kd = sum_kind(t);
        double m = sr[t][0];
        for (int q = 1; q < kBlock / 64; ++q) m = combine(kd, m, sr[t][q]);
        a.part[(size_t)t * a.nblk + blockIdx.x] = m;
    }
}

// integrals: one workgroup per NSKR_SUM_* slot
__global__ __launch_bounds__(kBlock) void k_integrals_final(const double *part, int nblk, double *out)
{
    reduce_final(part, nblk, out, [](int k) { return sum_kind(k); });
}

struct InitArgs {
    MeshDev mesh; Basis bas; size_t NN; const double *drop; int ndrop; double width, rv, rl;
    double len[3]; int per[3]; const double *noise;
    double wax[3];  // 1 for the axes the droplet distance spans, 0 for a cylinder's axis
};

template <int P, typename T, bool CV>
__global__ __launch_bounds__(kBlock) void k_init_rho(T *U, InitArgs a)
{
    using G = Tile<P>;
    const int t = threadIdx.x;
    const int e0 = blockIdx.x * G::EPB, le = t / G::n3, e = e0 + le, nd = t - le * G::n3;
    if (t >= G::NV || e >= a.mesh.E) return;
    const size_t g = (size_t)e0 * G::n3 + t;
    const int idx[3] = {nd % P, (nd / P) % P, nd / (P * P)};
    double x[3];
    if (CV) {
        for (int m = 0; m < 3; ++m) x[m] = a.mesh.xnode[m * a.NN + g];
    } else {
        const double *eg = a.mesh.egeo + (size_t)e * 12;
        for (int m = 0; m < 3; ++m) {
            double s = eg[m];
            for (int d = 0; d < 3; ++d) s += eg[3 + 3 * d + m] * 0.5 * (a.bas.x[idx[d]] + 1.0);
            x[m] = s;
        }
    }
    double rho = a.rv, u[3] = {0.0, 0.0, 0.0};
    for (int jd = 0; jd < a.ndrop; ++jd) {
        const double *dj = a.drop + 7 * jd;
        double d2 = 0;
        for (int m = 0; m < 3; ++m) {
            double dx = x[m] - dj[m];
            if (a.per[m]) dx -= a.len[m] * rint(dx / a.len[m]);
            d2 += a.wax[m] * (dx * dx);
        }
        const double th = 1.0 + tanh((dj[3] - sqrt(d2)) / a.width);
        rho += 0.5 * (a.rl - a.rv) * th;
        for (int m = 0; m < 3; ++m) u[m] += dj[4 + m] * (0.5 * th);  // v_j times the droplet indicator
    }
    if (a.noise) rho += a.noise[g];
    U[g] = T(rho);
    U[a.NN + g] = T(rho * u[0]);
    U[2 * a.NN + g] = T(rho * u[1]);
    U[3 * a.NN + g] = T(rho * u[2]);
    U[4 * a.NN + g] = T(0);
    U[5 * a.NN + g] = T(rho);
}

template <int P, typename T>
__global__ __launch_bounds__(kBlock) void k_init_energy(T *U, const T *Q, int E, size_t NN, Phys ph, double T0)
{
    using G = Tile<P>;
    const int t = threadIdx.x;
    const int e0 = blockIdx.x * G::EPB, le = t / G::n3, e = e0 + le;
    if (t >= G::NV || e >= E) return;
    const size_t g = (size_t)e0 * G::n3 + t;
    const double rho = U[g], m0 = U[NN + g], m1 = U[2 * NN + g], m2 = U[3 * NN + g];
    const double q0 = Q[12 * NN + g], q1 = Q[13 * NN + g], q2 = Q[14 * NN + g];
    U[4 * NN + g] = T(rho * (ph.R * ph.cv * T0 - ph.a * rho) + 0.5 * ph.gam * (q0 * q0 + q1 * q1 + q2 * q2) +
                      0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho);
}

// Zero fill (used instead of a memset so that it can sit in captured graphs).
template <typename T> __global__ __launch_bounds__(kBlock) void k_zero(T *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) p[i] = T(0);
}

// One step taken by every batch instance whose walls change in time: advance
// its step counter (read by the next step's stages for their times).
__global__ __launch_bounds__(64) void k_tick(int *const *clk, int n)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i < n) *clk[i] += 1;
}

// ------------------------------------------------------------ launch layer
template <int P, typename T, int BS, bool CV> struct Impl {
    static constexpr int kP = P, kBS = BS;
    static constexpr bool kCV = CV;
    using Real = T;
    using G = Tile<P, BS>;
    using G256 = Tile<P, kBlock>;
    static int nblk(const nskr_ctx *c) { return (c->E + G::EPB - 1) / G::EPB; }
    static int nblk256(const nskr_ctx *c) { return (c->E + G256::EPB - 1) / G256::EPB; }

    static MeshDev mesh(const nskr_ctx *c)
    {
        MeshDev m;
        m.E = c->E; m.nbr = c->d_nbr; m.bcid = c->d_bcid; m.emet = c->d_emet; m.fmet = c->d_fmet;
        m.egeo = c->d_egeo; m.bcs = c->d_bcs; m.dyn = c->dyn; m.stab = c->d_stab; m.var = c->var;
        m.nmet = c->d_nmet; m.fnrm = c->d_fnrm; m.xnode = c->d_xnode;
        return m;
    }
    static Inst<T> inst(const nskr_ctx *c, const void *U, void *R, void *Ut, double dt)
    {
        Inst<T> I;
        I.U = (T *)U; I.R = (T *)R; I.Ut = (T *)Ut;
        I.Ck = (T *)c->d_Ck;
        I.Q = (T *)c->d_Q; I.TH = (T *)c->d_TH; I.G2 = (T *)c->d_G2;
        I.T2 = (T *)c->d_T2; I.TF = (T *)c->d_TF; I.TU = (T *)c->d_TU;
        I.mesh = mesh(c); I.ph = c->ph; I.NN = c->NN; I.dt = dt;
        I.clk = nullptr; I.t0 = 0.0;
        return I;
    }
    static Launch<T> launch(const nskr_ctx *c, const Inst<T> &I)
    {
        Launch<T> L;
        memset(&L, 0, sizeof(L));
        L.one = I;
        L.bas = c->bas;
        L.t = c->time;
        L.blk_map = c->d_bmap;
        return L;
    }
    // every stage kernel's static LDS fits the device's per-block limit
    static int fits(int maxlds)
    {
        const void *fns[] = {reinterpret_cast<const void *>(&k_prolong<P, T, BS, false>),
                             reinterpret_cast<const void *>(&k_lift1<P, T, BS, false, false, CV>),
                             reinterpret_cast<const void *>(&k_lift1<P, T, BS, false, true, CV>),
                             reinterpret_cast<const void *>(&k_lift2<P, T, BS, false, CV>),
                             reinterpret_cast<const void *>(&k_update<P, T, BS, false, CV, false>),
                             reinterpret_cast<const void *>(&k_update<P, T, BS, false, CV, true>)};
        for (const void *f : fns) {
            hipFuncAttributes at;
            if (hipFuncGetAttributes(&at, f) != hipSuccess) return 0;
            if ((int)at.sharedSizeBytes > maxlds || at.maxThreadsPerBlock < BS) return 0;
        }
        return 1;
    }
    // single-instance launches
    static void prolong(nskr_ctx *c, const Launch<T> &L, hipStream_t s)
    {
        stage_launch<T>(c, 0, &k_prolong<P, T, BS, false>, nblk(c), BS, s, L);
    }
    static void lift1(nskr_ctx *c, const Launch<T> &L, hipStream_t s)
    {
        if (L.full)
            stage_launch<T>(c, 1, &k_lift1<P, T, BS, false, true, CV>, nblk(c), BS, s, L);
        else
            stage_launch<T>(c, 1, &k_lift1<P, T, BS, false, false, CV>, nblk(c), BS, s, L);
    }
    static void lift2(nskr_ctx *c, const Launch<T> &L, hipStream_t s)
    {
        stage_launch<T>(c, 2, &k_lift2<P, T, BS, false, CV>, nblk(c), BS, s, L);
    }
    static void update(nskr_ctx *c, const Launch<T> &L, hipStream_t s)
    {
        if (c->stream_nodes)
            stage_launch<T>(c, 3, &k_update<P, T, BS, false, CV, true>, nblk(c), BS, s, L);
        else
            stage_launch<T>(c, 3, &k_update<P, T, BS, false, CV, false>, nblk(c), BS, s, L);
    }
    // batched launches over a group table
    // one RK step of every instance of a group; the face traces of the first
    // stage come from the previous step's last update (or from prime())
    static void step_batched(const Launch<T> &L0, int nblocks, hipStream_t s)
    {
        Launch<T> L = L0;
        for (int st = 0; st < 5; ++st) {
            L.mode = 1;
            L.first = st == 0;
            L.last = st == 4;
            L.A = kRkA[st];
            L.B = kRkB[st];
            L.tb = kTraceBuf[st];
            L.tw = kTraceBuf[st + 1];
            L.cs = kRkC[st];
            hipLaunchKernelGGL((k_lift1<P, T, BS, true, false, CV>), dim3(nblocks), dim3(BS), 0, s, L);
            hipLaunchKernelGGL((k_lift2<P, T, BS, true, CV>), dim3(nblocks), dim3(BS), 0, s, L);
            hipLaunchKernelGGL((k_update<P, T, BS, true, CV>), dim3(nblocks), dim3(BS), 0, s, L);
        }
    }

    // traces of a newly admitted batch instance (once, as at the start of rk())
    static int prime(nskr_ctx *c, void *U, void *R, double dt, hipStream_t s)
    {
        Launch<T> L = launch(c, inst(c, U, R, nullptr, dt));
        prolong(c, L, s);
        return NSKR_OK;
    }
    static int rhs(nskr_ctx *c, const void *U, void *Ut, hipStream_t s)
    {
        Launch<T> L = launch(c, inst(c, U, nullptr, Ut, 0.0));
        L.mode = 0;
        prolong(c, L, s);
        lift1(c, L, s);
        lift2(c, L, s);
        update(c, L, s);
        HIPCHK(c, hipGetLastError());
        return NSKR_OK;
    }
    static void zero_comp(nskr_ctx *c, hipStream_t s)
    {
        if (!c->d_Ck) return;
        const size_t n = 6 * c->NN;
        const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock < 4096 ? (n + kBlock - 1) / kBlock : 4096);
        hipLaunchKernelGGL((k_zero<T>), dim3(grid), dim3(kBlock), 0, s, (T *)c->d_Ck, n);
    }
    static int rk(nskr_ctx *c, void *U, void *R, double dt, int nsteps, hipStream_t s)
    {
        if (nsteps == 0) return NSKR_OK;
        Launch<T> L = launch(c, inst(c, U, R, nullptr, dt));
        zero_comp(c, s);
        prolong(c, L, s);
        const double t0 = c->time;
        for (int n = 0; n < nsteps; ++n)
            for (int st = 0; st < 5; ++st) {
                L.mode = 1;
                L.first = st == 0;
                L.last = st == 4;
                L.A = kRkA[st];
                L.B = kRkB[st];
                L.tb = kTraceBuf[st];
                L.tw = kTraceBuf[st + 1];
                L.t = (t0 + n * dt) + kRkC[st] * dt;
                lift1(c, L, s);
                lift2(c, L, s);
                update(c, L, s);
            }
        c->time = t0 + nsteps * dt;
        HIPCHK(c, hipGetLastError());
        return NSKR_OK;
    }
    static int lift1_out(nskr_ctx *c, const void *U, void *q, hipStream_t s)
    {
        Launch<T> L = launch(c, inst(c, U, nullptr, nullptr, 0.0));
        L.full = 1;  // every lifted gradient and the nodal temperature
        prolong(c, L, s);
        lift1(c, L, s);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(q, c->d_Q, sizeof(T) * 15 * c->NN, hipMemcpyDeviceToDevice, s));
        return NSKR_OK;
    }
    static int lift2_out(nskr_ctx *c, const void *U, void *o, hipStream_t s)
    {
        Launch<T> L = launch(c, inst(c, U, nullptr, nullptr, 0.0));
        L.full = 1;  // every lifted gradient and the nodal temperature
        prolong(c, L, s);
        lift1(c, L, s);
        lift2(c, L, s);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(o, c->d_TH, sizeof(T) * c->NN, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync((T *)o + c->NN, c->d_G2, sizeof(T) * 4 * c->NN, hipMemcpyDeviceToDevice, s));
        return NSKR_OK;
    }
    // the largest wave speed, mesh factor, diffusivity and wall rate over the
    // nodes; part holds kNRates partial maxima per tile, dout the results (device)
    static int dt(nskr_ctx *c, const void *U, double *rates, hipStream_t s, double *part, double *dout)
    {
        Launch<T> L = launch(c, inst(c, U, nullptr, nullptr, 0.0));
        L.full = 1;  // every lifted gradient and the nodal temperature
        prolong(c, L, s);
        lift1(c, L, s);
        RateArgs a{mesh(c), c->ph, c->NN, part, nblk256(c), kSigN[P - 1]};
        hipLaunchKernelGGL((k_dt_rates<P, T, CV>), dim3(nblk256(c)), dim3(kBlock), 0, s, (const T *)U,
                           (const T *)c->d_Q, a);
        hipLaunchKernelGGL(k_max_final, dim3(kNRates), dim3(kBlock), 0, s, (const double *)part, nblk256(c), dout);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(rates, dout, kNRates * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return NSKR_OK;
    }
    static int reduce(nskr_ctx *c, const void *U, double *out, hipStream_t s)
    {
        Launch<T> L = launch(c, inst(c, U, nullptr, nullptr, 0.0));
        L.full = 1;  // every lifted gradient and the nodal temperature
        prolong(c, L, s);
        lift1(c, L, s);
        RateArgs a{mesh(c), c->ph, c->NN, c->d_part, nblk256(c), 0.0};
        hipLaunchKernelGGL((k_integrals<P, T, CV>), dim3(nblk256(c)), dim3(kBlock), 0, s, (const T *)U,
                           (const T *)c->d_Q, a, c->bas);
        hipLaunchKernelGGL(k_integrals_final, dim3(NSKR_NSUMS), dim3(kBlock), 0, s, (const double *)c->d_part,
                           nblk256(c), c->d_out);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(out, c->d_out, NSKR_NSUMS * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        return NSKR_OK;
    }
    static int init(nskr_ctx *c, const InitArgs &ia, double T0, void *Uv, hipStream_t s)
    {
        T *U = (T *)Uv;
        hipLaunchKernelGGL((k_init_rho<P, T, CV>), dim3(nblk256(c)), dim3(kBlock), 0, s, U, ia);
        Launch<T> L = launch(c, inst(c, U, nullptr, nullptr, 0.0));
        L.full = 1;
        prolong(c, L, s);
        lift1(c, L, s);
        hipLaunchKernelGGL((k_init_energy<P, T>), dim3(nblk256(c)), dim3(kBlock), 0, s, U, (const T *)c->d_Q, c->E,
                           c->NN, c->ph, T0);
        HIPCHK(c, hipGetLastError());
        return NSKR_OK;
    }
};

// Workgroup sizes built for each degree: 256 and 512 threads, and one size
// that packs whole elements into waves more tightly than 256 does (N = 2:
// 7 elements of 27 nodes in 192 threads; N = 3, 4: one wave pair, 2 and 1
// elements; N = 5: 2 elements of 216 nodes in 448 threads, against 1 in 256).
static int tight_block(int N) { return N == 2 ? 192 : (N == 5 ? 448 : 128); }
// Default threads per workgroup: 128 at N = 3 (two elements per workgroup,
// the same occupancy in finer workgroups: 3.4 % faster in FP64 and 0.7 % in
// FP32-mixed than 256 on the 48x48x24 and 50^3 meshes), else 256 (at N = 4
// the two measure the same; at N = 5 and N = 2 the tight sizes are slower).
static int default_block(int N) { return N == 3 ? 128 : 256; }

// Valid block sizes per degree: one of the built sizes, holding at least one
// element and one line task per thread.
static bool block_ok(int N, int bs)
{
    const int P = N + 1, n3 = P * P * P;
    if (N < 2 || N > 5) return false;
    if (bs != 256 && bs != 512 && bs != tight_block(N)) return false;
    const int epb = bs / n3;
    return epb >= 1 && epb * 3 * P * P <= bs;
}

template <int PP, int BS, typename F> static int impl_prec(bool dbl, F &&f)
{
    return dbl ? f(Impl<PP, double, BS, false>()) : f(Impl<PP, float, BS, false>());
}

// The kernel instance set of a (degree, precision, block size, curved) choice.
// Curved meshes run 256-thread workgroups only (their per-node metrics do
// not fit the LDS of larger tiles at every degree).
template <typename F> static int impl_dispatch(int N, int prec, int bs, bool curved, F &&f)
{
    const bool dbl = prec == 0;
#define NSKR_CASE(NN, PP, TB)                                                                           \
    case NN:                                                                                            \
        if (curved) {                                                                                   \
            if (bs != 256) return NSKR_E_UNSUPPORTED;                                                   \
            return dbl ? f(Impl<PP, double, 256, true>()) : f(Impl<PP, float, 256, true>());            \
        }                                                                                               \
        if (bs == 512) return impl_prec<PP, 512>(dbl, f);                                               \
        if (bs == TB) return impl_prec<PP, TB>(dbl, f);                                                 \
        return impl_prec<PP, 256>(dbl, f);
    switch (N) {
        NSKR_CASE(2, 3, 192)
        NSKR_CASE(3, 4, 128)
        NSKR_CASE(4, 5, 128)
        NSKR_CASE(5, 6, 448)
    }
#undef NSKR_CASE
    return NSKR_E_ARG;
}

template <typename F> static int dispatch(const nskr_ctx *c, F &&f)
{
    return impl_dispatch(c->N, c->p.precision, c->bs, c->curved, f);
}

static int elem_per_block(int N)
{
    const int n3 = (N + 1) * (N + 1) * (N + 1);
    return kBlock / n3;
}

// Order of the stage kernels' blocks across the XCDs.  Workgroups go to the
// 8 XCDs round robin (block b to XCD b mod 8), each with its own L2, and an
// element's face traces are read by its own block and by its neighbours'.
// The groups of elements that share a block are split into 8 slabs of equal
// count along the longest extent of the mesh (by their centroids), slab k
// going to the blocks b = k mod 8 in the elements' own order, so most
// neighbours of an element are processed on the same XCD at about the same
// time and read its traces from that L2.  Concurrent XCDs still work on
// nearby addresses (neighbouring slabs at the same position in their own
// order).
constexpr int kXcds = 8;
// Node data of the update kernel (U, R and grad T + lap c: 16 values per
// node) beyond which its node accesses carry the non-temporal hint: half the
// 256 MiB last-level cache.  Measured: 0.5-1.3 % faster in FP64 on the
// 32^3 N = 5, 48x48x24 N = 3 and 50^3 N = 3 meshes, 3-5 % in FP32-mixed on the
// N = 3 meshes; 1-8 % slower on the 16^3 N = 4 mesh, whose arrays stay cached.
constexpr double kStreamBytes = 134217728.0;

static int build_block_map(nskr_ctx *c)
{
    const int epb = c->bs / ((c->N + 1) * (c->N + 1) * (c->N + 1));
    const int E = c->E, G = (E + epb - 1) / epb;
    std::vector<double> gc((size_t)G * 3, 0.0);
    for (int e = 0; e < E; ++e)
        for (int m = 0; m < 3; ++m) gc[(size_t)(e / epb) * 3 + m] += c->cent[(size_t)e * 3 + m];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int g = 0; g < G; ++g) {
        const int n = std::min(epb, E - g * epb);
        for (int m = 0; m < 3; ++m) {
            gc[(size_t)g * 3 + m] /= n;
            lo[m] = std::min(lo[m], gc[(size_t)g * 3 + m]);
            hi[m] = std::max(hi[m], gc[(size_t)g * 3 + m]);
        }
    }
    int ax = 0;
    for (int m = 1; m < 3; ++m)
        if (hi[m] - lo[m] > (hi[ax] - lo[ax]) * (1 + 1e-12)) ax = m;
    std::vector<int> by(G);
    for (int g = 0; g < G; ++g) by[g] = g;
    std::stable_sort(by.begin(), by.end(), [&](int a, int b) { return gc[(size_t)a * 3 + ax] < gc[(size_t)b * 3 + ax]; });
    // slab k holds q + (k < r) groups; within a slab the groups keep their order
    const int q = G / kXcds, r = G % kXcds;
    std::vector<int> map(G);
    int start = 0;
    for (int k = 0; k < kXcds; ++k) {
        const int cnt = q + (k < r ? 1 : 0);
        std::vector<int> slab(by.begin() + start, by.begin() + start + cnt);
        std::sort(slab.begin(), slab.end());
        for (int j = 0; j < cnt; ++j) map[(size_t)j * kXcds + k] = slab[j] * epb;
        start += cnt;
    }
    // every group exactly once
    std::vector<char> seen(G, 0);
    for (int b = 0; b < G; ++b) {
        const int g = map[b] / epb;
        if (map[b] % epb != 0 || g < 0 || g >= G || seen[g]) return fail(c, NSKR_E_STATE, "block order is not a permutation");
        seen[g] = 1;
    }
    if (c->d_bmap) {
        (void)hipFree(c->d_bmap);
        c->d_bmap = nullptr;
        c->bmap_bs = 0;
    }
    HIPCHK(c, hipMalloc((void **)&c->d_bmap, sizeof(int) * (size_t)G));
    HIPCHK(c, hipMemcpy(c->d_bmap, map.data(), sizeof(int) * (size_t)G, hipMemcpyHostToDevice));
    c->bmap_bs = c->bs;
    return NSKR_OK;
}

// Reduction scratch of nskr_dt_noalloc, for callers that cannot allocate:
// kNRates partial maxima per element tile of the 256-thread reduction kernel,
// then the kNRates results.  Each device holds its own copy for the life of the
// process; its address on each device is looked up once, at the first
// nskr_create on that device, and only that address is handed to kernels.
// Every partial is written before it is read, so nothing needs clearing.
constexpr int kStaticTiles = 131072;
static __device__ __align__(256) double scratch[kNRates * (kStaticTiles + 1)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mtx;
static double *g_scratch[kMaxDevices];

// Look up the array's address on `device` (the caller has made it current).
static bool setup_static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return false;
    std::lock_guard<std::mutex> lock(g_scratch_mtx);
    if (g_scratch[device]) return true;
    double *ptr = nullptr;
    if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return false;
    g_scratch[device] = ptr;
    return true;
}

static double *static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mtx);
    return g_scratch[device];
}

// ------------------------------------------------------------ mesh geometry
// Elements are given by their geometry nodes on the Gauss-Lobatto points of
// degree ngeo <= N (Sec. 3.1: curved elements of geometry degree N_geo); the
// library interpolates them to the degree-N Gauss-Lobatto points and forms
// the metric terms Ja^d_m = J d xi^d / d x_m in the conservative curl form
// (Kopriva 2006): Ja^i_n = -(curl_xi (X_l grad_xi X_m))_i, (n, m, l)
// cyclic, evaluated at the Gauss-Lobatto points, then interpolated to the
// Gauss nodes (volume) and to the Gauss points of each face (xi^d = +-1 is a
// Gauss-Lobatto layer).  Extended precision, rounded once.

// Gauss-Lobatto points of degree n: the ends and the roots of P_{n+1} -
// P_{n-1}, which vanish exactly where P_n' does, by Newton from the
// Chebyshev-Lobatto points.
static void lobatto_host(int n, ld *x)
{
    x[0] = -1;
    x[n] = 1;
    for (int i = 1; i < n; ++i) {
        ld xi = -cosl(3.14159265358979323846264338327950288L * i / n);
        for (int it = 0; it < 100; ++it) {
            ld pm, dpm, pp, dpp;
            legendre_ld(n - 1, xi, pm, dpm);
            legendre_ld(n + 1, xi, pp, dpp);
            const ld dx = (pp - pm) / (dpp - dpm);
            xi -= dx;
            if (fabsl(dx) < 1e-21L) break;
        }
        x[i] = xi;
    }
}

// M[a][b] = l_b(y_a), the Lagrange basis of the nodes xs[0..nx) at ys[0..ny).
static std::vector<ld> interp_matrix(int nx, const ld *xs, int ny, const ld *ys)
{
    std::vector<ld> M((size_t)ny * nx, 1.0L);
    for (int a = 0; a < ny; ++a)
        for (int b = 0; b < nx; ++b)
            for (int k = 0; k < nx; ++k)
                if (k != b) M[(size_t)a * nx + b] *= (ys[a] - xs[k]) / (xs[b] - xs[k]);
    return M;
}

// Apply the (nout x nin) matrix M along direction d of a tensor array with
// extents n[3] (index a + n0 (b + n1 c)); the result has n[d] = nout.
static std::vector<ld> tensor_apply(const std::vector<ld> &in, const int n[3], int d, const ld *M, int nout)
{
    int m[3] = {n[0], n[1], n[2]};
    m[d] = nout;
    std::vector<ld> out((size_t)m[0] * m[1] * m[2], 0.0L);
    for (int c = 0; c < m[2]; ++c)
        for (int b = 0; b < m[1]; ++b)
            for (int a = 0; a < m[0]; ++a) {
                const int o[3] = {a, b, c};
                ld acc = 0;
                for (int l = 0; l < n[d]; ++l) {
                    int ii[3] = {a, b, c};
                    ii[d] = l;
                    acc += M[(size_t)o[d] * n[d] + l] * in[ii[0] + (size_t)n[0] * (ii[1] + (size_t)n[1] * ii[2])];
                }
                out[a + (size_t)m[0] * (b + (size_t)m[1] * c)] = acc;
            }
    return out;
}

struct GeomOps {
    int N, P, ng;
    ld xs[8];                     // Gauss nodes
    std::vector<ld> Vg, Dl, Vs;   // GL(ngeo) -> GL(N), derivative on GL(N), GL(N) -> Gauss
    GeomOps(int N_, int ng_, const Basis &b) : N(N_), P(N_ + 1), ng(ng_)
    {
        ld xg[8], xl[8];
        lobatto_host(ng, xg);
        lobatto_host(N, xl);
        Vg = interp_matrix(ng + 1, xg, P, xl);
        for (int i = 0; i < P; ++i) xs[i] = (ld)b.x[i];
        Vs = interp_matrix(P, xl, P, xs);
        // barycentric derivative matrix on the Gauss-Lobatto points
        ld lam[8];
        for (int j = 0; j < P; ++j) {
            ld pr = 1;
            for (int k = 0; k < P; ++k)
                if (k != j) pr *= xl[j] - xl[k];
            lam[j] = 1 / pr;
        }
        Dl.assign((size_t)P * P, 0.0L);
        for (int i = 0; i < P; ++i) {
            ld sum = 0;
            for (int j = 0; j < P; ++j)
                if (j != i) {
                    Dl[(size_t)i * P + j] = lam[j] / (lam[i] * (xl[i] - xl[j]));
                    sum += Dl[(size_t)i * P + j];
                }
            Dl[(size_t)i * P + i] = -sum;
        }
    }
    // the element's coordinates (3 arrays) at the degree-N Gauss-Lobatto points
    void geometry(const double *xg, std::vector<ld> X[3]) const
    {
        const int g1 = ng + 1;
        for (int m = 0; m < 3; ++m) {
            std::vector<ld> v((size_t)g1 * g1 * g1);
            for (size_t q = 0; q < v.size(); ++q) v[q] = xg[3 * q + m];
            int n[3] = {g1, g1, g1};
            for (int d = 0; d < 3; ++d) {
                v = tensor_apply(v, n, d, Vg.data(), P);
                n[d] = P;
            }
            X[m].swap(v);
        }
    }
    std::vector<ld> to_gauss(const std::vector<ld> &v) const
    {
        int n[3] = {P, P, P};
        std::vector<ld> w = v;
        for (int d = 0; d < 3; ++d) w = tensor_apply(w, n, d, Vs.data(), P);
        return w;
    }
    std::vector<ld> deriv(const std::vector<ld> &v, int d) const
    {
        int n[3] = {P, P, P};
        return tensor_apply(v, n, d, Dl.data(), P);
    }
    // the Gauss-Lobatto layer xi^d = -1 (s = 0) or +1 (s = 1) of v, interpolated
    // to the face's Gauss points: out[p + P q], (p, q) the two remaining axes
    // in increasing order
    void face(const std::vector<ld> &v, int d, int s, ld *out) const
    {
        const int lay = s ? N : 0;
        const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
        for (int q = 0; q < P; ++q)
            for (int p = 0; p < P; ++p) {
                ld acc = 0;
                for (int b2 = 0; b2 < P; ++b2)
                    for (int b1 = 0; b1 < P; ++b1) {
                        int ii[3];
                        ii[d] = lay;
                        ii[d1] = b1;
                        ii[d2] = b2;
                        acc += Vs[(size_t)p * P + b1] * Vs[(size_t)q * P + b2] * v[ii[0] + P * (ii[1] + P * ii[2])];
                    }
                out[p + P * q] = acc;
            }
    }
};

// Orientation map of face points (see nskr.h): own point fp -> neighbour's.
static int orient_host(int P, int fp, int o)
{
    int a = fp % P, b = fp / P;
    if (o & 4) std::swap(a, b);
    if (o & 1) a = P - 1 - a;
    if (o & 2) b = P - 1 - b;
    return a + P * b;
}

// ------------------------------------------------------------------ ABI
extern "C" {

int nskr_version(void) { return NSKR_ABI_VERSION; }

int nskr_create(const nskr_params *p, int N, int device, nskr_ctx **out)
{
    if (!out || !p) return NSKR_E_ARG;
    *out = nullptr;
    if (N < 2 || N > 5) return NSKR_E_ARG;
    if (!(p->mu >= 0) || !(p->kappa >= 0) || !(p->gam >= 0) || !(p->alpha >= 0) || !(p->beta >= 0) ||
        !(p->b >= 0) || !(p->cv > 0) || !(p->R > 0) || !(p->cfl > 0) || !(p->a >= 0))
        return NSKR_E_ARG;
    if (p->precision != 0 && p->precision != 1) return NSKR_E_ARG;
    if (p->kahan != 0 && p->kahan != 1) return NSKR_E_ARG;
    if (p->model < 0 || p->model > 2) return NSKR_E_UNSUPPORTED;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return NSKR_E_HIP;
    // make sure the device code for this GPU is present
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, reinterpret_cast<const void *>(&k_update<4, double, 256, false>)) != hipSuccess)
        return NSKR_E_HIP;
    {
        DeviceGuard guard(device);
        if (!setup_static_scratch(device)) return NSKR_E_HIP;
    }
    nskr_ctx *c = new nskr_ctx();
    c->p = *p;
    c->N = N;
    c->P = N + 1;
    c->bs = default_block(N);
    c->device = device;
    make_basis(N, c->bas);
    c->ph.R = p->R; c->ph.a = p->a; c->ph.b = p->b; c->ph.cv = p->cv; c->ph.mu = p->mu;
    c->ph.kappa = p->kappa; c->ph.gam = p->gam; c->ph.alpha = p->alpha; c->ph.beta = p->beta;
    c->ph.inv_Rcv = 1.0 / (p->R * p->cv);
    c->ph.cs_fac = (1.0 + 1.0 / p->cv) * p->R;
    c->ph.model = p->model == 2 ? 2 : 1;
    c->ph.ap = p->model == 2 ? p->alpha : 0.0;
    *out = c;
    return NSKR_OK;
}

static void free_mesh(nskr_ctx *c)
{
    void *ptrs[] = {c->d_nbr, c->d_bcid, c->d_emet, c->d_fmet, c->d_egeo, c->d_bcs, c->d_Q, c->d_TH,
                    c->d_G2, c->d_T2, c->d_TF, c->d_TU, c->d_part, c->d_out, c->d_noise, c->d_drop, c->d_Ck,
                    c->d_stab, c->d_clk, c->d_nmet, c->d_fnrm, c->d_xnode, c->d_bmap};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    c->d_nbr = c->d_bcid = nullptr;
    c->d_emet = c->d_fmet = c->d_egeo = nullptr;
    c->d_nmet = c->d_fnrm = nullptr;
    c->d_xnode = nullptr;
    c->curved = false;
    c->d_bcs = nullptr;
    c->d_stab = nullptr;
    c->d_clk = nullptr;
    c->d_Q = c->d_TH = c->d_G2 = c->d_T2 = c->d_TF = c->d_TU = c->d_Ck = nullptr;
    c->d_part = c->d_out = c->d_noise = c->d_drop = nullptr;
    c->d_bmap = nullptr;
    c->bmap_bs = 0;
    std::vector<float>().swap(c->cent);
    c->E = 0;
    c->NN = c->NF = 0;
    c->bytes = 0;
}

int nskr_destroy(nskr_ctx *c)
{
    if (!c) return NSKR_OK;
    {
        DeviceGuard g(c->device);
        free_mesh(c);
        for (auto &pe : c->prof_events) {
            (void)hipEventDestroy(pe.second.first);
            (void)hipEventDestroy(pe.second.second);
        }
        for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    }
    delete c;
    return NSKR_OK;
}

static int dalloc(nskr_ctx *c, void **p, size_t bytes)
{
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        return fail(c, NSKR_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    c->bytes += bytes;
    return NSKR_OK;
}

int nskr_mesh_upload(nskr_ctx *c, const nskr_mesh *m, nskr_stream sv)
{
    if (!c) return NSKR_E_ARG;
    if (c->poisoned) return fail(c, NSKR_E_STATE, "context poisoned by an earlier HIP error");
    if (!m || m->nelems <= 0 || !m->xgeo || !m->nbr || !m->nbr_face || !m->bc)
        return fail(c, NSKR_E_ARG, "mesh arrays missing or nelems <= 0");
    if (m->ngeo < 1 || m->ngeo > c->N) return fail(c, NSKR_E_ARG, "geometry degree ngeo must be in 1..N");
    if (m->nbcs < 0 || (m->nbcs > 0 && !m->bcs)) return fail(c, NSKR_E_ARG, "bad wall table");
    const int E = m->nelems;
    if ((long long)E * 48 > 2147483647LL) return fail(c, NSKR_E_ARG, "too many elements for the connectivity codes");
    const int P = c->P, n2 = P * P, n3 = n2 * P, ng = m->ngeo, g3 = (ng + 1) * (ng + 1) * (ng + 1);
    auto orient = [&](int e, int f) { return m->nbr_orient ? m->nbr_orient[e * 6 + f] : 0; };
    // connectivity: reciprocal neighbours, inverse orientations, wall indices
    for (int e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            const int nb = m->nbr[e * 6 + f], bc = m->bc[e * 6 + f];
            if (nb >= E || nb < -1) return fail(c, NSKR_E_ARG, "neighbour index out of range");
            if (nb >= 0) {
                const int nf = m->nbr_face[e * 6 + f], o = orient(e, f);
                if (nf < 0 || nf > 5 || o < 0 || o > 7) return fail(c, NSKR_E_ARG, "neighbour face or orientation out of range");
                if (nb == e && nf == f) return fail(c, NSKR_E_ARG, "a face cannot be its own neighbour");
                if (m->nbr[nb * 6 + nf] != e || m->nbr_face[nb * 6 + nf] != f)
                    return fail(c, NSKR_E_ARG, "connectivity not reciprocal");
                const int ob = orient(nb, nf);
                for (int fp = 0; fp < n2; ++fp)
                    if (orient_host(P, orient_host(P, fp, o), ob) != fp)
                        return fail(c, NSKR_E_ARG, "the two orientations of a face are not inverse to each other");
                if (bc != 0) return fail(c, NSKR_E_ARG, "interior face with a wall index");
            } else {
                if (bc < 1 || bc > m->nbcs) return fail(c, NSKR_E_ARG, "wall face without a valid wall index");
                const nskr_bc &w = m->bcs[bc - 1];
                if (w.kind != 1 && w.kind != 2 && w.kind != 3) return fail(c, NSKR_E_ARG, "wall kind must be 1, 2 or 3");
                if (w.kind == 3 && !(w.gamma1 >= 0 && w.gamma2 >= 0 && w.gamma3 >= 0 && w.gamma4 >= 0))
                    return fail(c, NSKR_E_ARG, "Navier-slip wall coefficients must be non-negative");
                if (w.kind != 2 && !(std::isfinite(w.uwall[0]) && std::isfinite(w.uwall[1]) && std::isfinite(w.uwall[2])))
                    return fail(c, NSKR_E_ARG, "wall velocity must be finite");
            }
        }
    // the kernels address node- and element-indexed arrays with 32-bit byte
    // offsets from a per-field base: every such array stays below 4 GiB
    {
        const double tsz = c->p.precision == 0 ? 8.0 : 4.0, nn = (double)E * n3;
        const double worst = fmax(fmax(nn * 8.0, (double)E * 24 * 8), (double)E * 6 * n2 * 4 * tsz);
        if (worst >= 4294967296.0)
            return fail(c, NSKR_E_UNSUPPORTED, "mesh too large for one context (a node or face-point array exceeds "
                                               "4 GiB); split it into several instances");
    }
    // pass 1: every element's geometry at the degree-N Gauss-Lobatto points;
    // is it affine (a parallelepiped)? its corner and edge vectors, its size,
    // and the coordinates of its face points
    GeomOps ops(c->N, ng, c->bas);
    ld xl[8];
    lobatto_host(c->N, xl);
    std::vector<double> egeo((size_t)E * 12), fpos((size_t)E * 6 * n2 * 3), escale(E);
    bool curved = false;
    // The common case first: elements given by their 8 corners that are all
    // parallelepipeds.  Corner, edge vectors and face points then follow from
    // the corners in FP64 (the map is affine), without interpolating the
    // geometry; any other element sends the whole mesh through the general
    // pass below.  (A trilinear map deviates most from the affine one at the
    // corners, so the corner test is the general pass's test.)
    bool affine_corners = ng == 1;
    for (int e = 0; e < E && affine_corners; ++e) {
        const double *v = m->xgeo + (size_t)e * 24;
        for (int q = 0; q < 24; ++q)
            if (!std::isfinite(v[q])) return fail(c, NSKR_E_ARG, "non-finite geometry node");
        double a[3][3], scale = 0;
        for (int mm = 0; mm < 3; ++mm) {
            a[0][mm] = v[3 + mm] - v[mm];
            a[1][mm] = v[6 + mm] - v[mm];
            a[2][mm] = v[12 + mm] - v[mm];
            for (int d = 0; d < 3; ++d) scale = fmax(scale, fabs(a[d][mm]));
        }
        if (!(scale > 0)) return fail(c, NSKR_E_ARG, "element " + std::to_string(e) + " is degenerate");
        for (int cn = 0; cn < 8 && affine_corners; ++cn)
            for (int mm = 0; mm < 3; ++mm) {
                const double lin = v[mm] + (cn & 1) * a[0][mm] + ((cn >> 1) & 1) * a[1][mm] + (cn >> 2) * a[2][mm];
                if (fabs(lin - v[3 * cn + mm]) > 1e-12 * scale) affine_corners = false;
            }
        escale[e] = scale;
        for (int mm = 0; mm < 3; ++mm) egeo[(size_t)e * 12 + mm] = v[mm];
        for (int d = 0; d < 3; ++d)
            for (int mm = 0; mm < 3; ++mm) egeo[(size_t)e * 12 + 3 + 3 * d + mm] = a[d][mm];
        for (int f = 0; f < 6; ++f) {
            const int d = f >> 1;
            const double xn = (f & 1) ? 1.0 : -1.0;
            for (int fp = 0; fp < n2; ++fp) {
                const double xa = c->bas.x[fp % P], xb = c->bas.x[fp / P];
                const double r[3] = {d == 0 ? xn : xa, d == 1 ? xn : (d == 0 ? xa : xb), d == 2 ? xn : xb};
                for (int mm = 0; mm < 3; ++mm)
                    fpos[(((size_t)e * 6 + f) * n2 + fp) * 3 + mm] =
                        v[mm] + 0.5 * ((r[0] + 1.0) * a[0][mm] + (r[1] + 1.0) * a[1][mm] + (r[2] + 1.0) * a[2][mm]);
            }
        }
    }
    for (int e = 0; e < E && !affine_corners; ++e) {
        const double *xe = m->xgeo + (size_t)e * g3 * 3;
        for (int q = 0; q < 3 * g3; ++q)
            if (!std::isfinite(xe[q])) return fail(c, NSKR_E_ARG, "non-finite geometry node");
        std::vector<ld> X[3];
        ops.geometry(xe, X);
        auto at = [&](int mm, int i, int j, int k) { return X[mm][i + P * (j + P * k)]; };
        ld x0[3], a[3][3];
        double scale = 0;
        for (int mm = 0; mm < 3; ++mm) {
            x0[mm] = at(mm, 0, 0, 0);
            a[0][mm] = at(mm, c->N, 0, 0) - x0[mm];
            a[1][mm] = at(mm, 0, c->N, 0) - x0[mm];
            a[2][mm] = at(mm, 0, 0, c->N) - x0[mm];
        }
        for (int d = 0; d < 3; ++d)
            for (int mm = 0; mm < 3; ++mm) scale = fmax(scale, (double)fabsl(a[d][mm]));
        if (!(scale > 0)) return fail(c, NSKR_E_ARG, "element " + std::to_string(e) + " is degenerate");
        escale[e] = scale;
        for (int k = 0; k < P && !curved; ++k)
            for (int j = 0; j < P && !curved; ++j)
                for (int i = 0; i < P && !curved; ++i)
                    for (int mm = 0; mm < 3; ++mm) {
                        const ld lin = x0[mm] + 0.5L * ((xl[i] + 1) * a[0][mm] + (xl[j] + 1) * a[1][mm] +
                                                        (xl[k] + 1) * a[2][mm]);
                        if (fabsl(lin - at(mm, i, j, k)) > 1e-12L * scale) curved = true;
                    }
        for (int mm = 0; mm < 3; ++mm) egeo[(size_t)e * 12 + mm] = (double)x0[mm];
        for (int d = 0; d < 3; ++d)
            for (int mm = 0; mm < 3; ++mm) egeo[(size_t)e * 12 + 3 + 3 * d + mm] = (double)a[d][mm];
        for (int f = 0; f < 6; ++f) {
            ld fv[64];
            for (int mm = 0; mm < 3; ++mm) {
                ops.face(X[mm], f >> 1, f & 1, fv);
                for (int fp = 0; fp < n2; ++fp) fpos[(((size_t)e * 6 + f) * n2 + fp) * 3 + mm] = (double)fv[fp];
            }
        }
    }
    // the two sides of every interior face are the same surface: the
    // neighbour's matching points (through the orientation) differ from the
    // own ones by one translation (zero, or a period of the domain)
    for (int e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            const int nb = m->nbr[e * 6 + f];
            if (nb < 0) continue;
            const int nf = m->nbr_face[e * 6 + f], o = orient(e, f);
            const double tol = 1e-10 * fmax(escale[e], escale[nb]);
            double t0[3];
            for (int fp = 0; fp < n2; ++fp) {
                const double *xo = &fpos[(((size_t)e * 6 + f) * n2 + fp) * 3];
                const double *xn = &fpos[(((size_t)nb * 6 + nf) * n2 + orient_host(P, fp, o)) * 3];
                for (int mm = 0; mm < 3; ++mm) {
                    const double dv = xn[mm] - xo[mm];
                    if (fp == 0) t0[mm] = dv;
                    else if (fabs(dv - t0[mm]) > tol)
                        return fail(c, NSKR_E_ARG, "face " + std::to_string(f) + " of element " + std::to_string(e) +
                                                       " does not match its neighbour's face under the given orientation");
                }
            }
        }
    std::vector<double>().swap(fpos);
    if (curved) {
        for (int k = 0; k < m->nbcs; ++k) {
            const double *tg = m->bcs[k].twall_grad;
            if (m->bcs[k].kind != 2 && (tg[0] != 0.0 || tg[1] != 0.0 || tg[2] != 0.0 || m->bcs[k].twall_rate != 0.0))
                return fail(c, NSKR_E_UNSUPPORTED, "walls whose temperature varies need affine elements");
        }
    }
    // metric terms: per element on affine meshes; per node and face point
    // (curl form) on curved ones.  Face vectors: outward unit normal and
    // surface element.
    std::vector<double> emet, fmet, nmet, fnrm, xnode;
    const size_t NN = (size_t)E * n3;
    if (!curved) {
        emet.resize((size_t)E * 10);
        fmet.resize((size_t)E * 24);
        for (int e = 0; e < E; ++e) {
            double a[3][3];
            for (int d = 0; d < 3; ++d)
                for (int k = 0; k < 3; ++k) a[d][k] = egeo[(size_t)e * 12 + 3 + 3 * d + k];
            // dx/dxi^d = a_d / 2; Ja^1 = (a_2 x a_3)/4, Ja^2 = (a_3 x a_1)/4, Ja^3 = (a_1 x a_2)/4
            for (int d = 0; d < 3; ++d) {
                const double *u = a[(d + 1) % 3], *w = a[(d + 2) % 3];
                emet[(size_t)e * 10 + 3 * d + 0] = 0.25 * (u[1] * w[2] - u[2] * w[1]);
                emet[(size_t)e * 10 + 3 * d + 1] = 0.25 * (u[2] * w[0] - u[0] * w[2]);
                emet[(size_t)e * 10 + 3 * d + 2] = 0.25 * (u[0] * w[1] - u[1] * w[0]);
            }
            const double J = 0.125 * (a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                                      a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                                      a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]));
            if (!(J > 0)) return fail(c, NSKR_E_ARG, "element " + std::to_string(e) + " has J <= 0");
            emet[(size_t)e * 10 + 9] = J;
            for (int d = 0; d < 3; ++d) {
                const double *Ja = &emet[(size_t)e * 10 + 3 * d];
                const double nrm = sqrt(Ja[0] * Ja[0] + Ja[1] * Ja[1] + Ja[2] * Ja[2]);
                for (int s = 0; s < 2; ++s) {
                    double *fm = &fmet[((size_t)e * 6 + 2 * d + s) * 4];
                    const double sg = s ? 1.0 : -1.0;
                    for (int k = 0; k < 3; ++k) fm[k] = sg * Ja[k] / nrm;
                    fm[3] = nrm;
                }
            }
        }
    } else {
        nmet.resize(10 * NN);
        fnrm.resize((size_t)E * 6 * n2 * 4);
        xnode.resize(3 * NN);
        for (int e = 0; e < E; ++e) {
            std::vector<ld> X[3], dX[3][3], Ja[3][3];
            ops.geometry(m->xgeo + (size_t)e * g3 * 3, X);
            for (int mm = 0; mm < 3; ++mm)
                for (int d = 0; d < 3; ++d) dX[mm][d] = ops.deriv(X[mm], d);
            for (int n = 0; n < 3; ++n) {
                const int mm = (n + 1) % 3, l = (n + 2) % 3;
                // R_j = X_l d X_m / d xi^j, X_l relative to the element's first
                // point (a constant shift leaves the curl unchanged)
                std::vector<ld> Rv[3];
                for (int j = 0; j < 3; ++j) {
                    Rv[j].resize(n3);
                    for (int q = 0; q < n3; ++q) Rv[j][q] = (X[l][q] - X[l][0]) * dX[mm][j][q];
                }
                for (int i = 0; i < 3; ++i) {
                    const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
                    std::vector<ld> c1 = ops.deriv(Rv[i2], i1), c2 = ops.deriv(Rv[i1], i2);
                    Ja[i][n].resize(n3);
                    for (int q = 0; q < n3; ++q) Ja[i][n][q] = -(c1[q] - c2[q]);
                }
            }
            // volume: Ja and J at the Gauss nodes
            std::vector<ld> JaG[3][3], dXG[3][3], XG[3];
            for (int i = 0; i < 3; ++i)
                for (int n = 0; n < 3; ++n) {
                    JaG[i][n] = ops.to_gauss(Ja[i][n]);
                    dXG[i][n] = ops.to_gauss(dX[i][n]);
                }
            for (int mm = 0; mm < 3; ++mm) XG[mm] = ops.to_gauss(X[mm]);
            for (int q = 0; q < n3; ++q) {
                const size_t gq = (size_t)e * n3 + q;
                for (int i = 0; i < 3; ++i)
                    for (int n = 0; n < 3; ++n) nmet[(size_t)(3 * i + n) * NN + gq] = (double)JaG[i][n][q];
                const ld J = dXG[0][0][q] * (dXG[1][1][q] * dXG[2][2][q] - dXG[1][2][q] * dXG[2][1][q]) -
                             dXG[0][1][q] * (dXG[1][0][q] * dXG[2][2][q] - dXG[1][2][q] * dXG[2][0][q]) +
                             dXG[0][2][q] * (dXG[1][0][q] * dXG[2][1][q] - dXG[1][1][q] * dXG[2][0][q]);
                if (!(J > 0)) return fail(c, NSKR_E_ARG, "element " + std::to_string(e) + " has J <= 0");
                nmet[9 * NN + gq] = (double)J;
                for (int mm = 0; mm < 3; ++mm) xnode[mm * NN + gq] = (double)XG[mm][q];
            }
            // faces: outward n dS = +-Ja^d on the layer xi^d = +-1
            for (int f = 0; f < 6; ++f) {
                const int d = f >> 1;
                ld v[3][64];
                for (int mm = 0; mm < 3; ++mm) ops.face(Ja[d][mm], d, f & 1, v[mm]);
                for (int fp = 0; fp < n2; ++fp) {
                    const ld sg = (f & 1) ? 1.0L : -1.0L;
                    const ld nx = sg * v[0][fp], ny = sg * v[1][fp], nz = sg * v[2][fp];
                    const ld dS = sqrtl(nx * nx + ny * ny + nz * nz);
                    double *fo = &fnrm[(((size_t)e * 6 + f) * n2 + fp) * 4];
                    fo[0] = (double)(nx / dS);
                    fo[1] = (double)(ny / dS);
                    fo[2] = (double)(nz / dS);
                    fo[3] = (double)dS;
                }
            }
        }
    }
    // the two sides of an interior face use exactly opposite normals and the
    // same surface element (conservation): one side (the master: the face on
    // the element's + side, else the lower element and face) keeps its own,
    // the other takes the master's negated, after checking that they agree
    auto master = [&](int e, int f, int nb, int nf) {
        if ((f & 1) != (nf & 1)) return (f & 1) == 1;
        return e < nb || (e == nb && f < nf);
    };
    for (int e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            const int nb = m->nbr[e * 6 + f];
            if (nb < 0) continue;
            const int nf = m->nbr_face[e * 6 + f], o = orient(e, f);
            if (!master(e, f, nb, nf)) continue;
            const int npts = curved ? n2 : 1;
            for (int fp = 0; fp < npts; ++fp) {
                double *mo = curved ? &fnrm[(((size_t)e * 6 + f) * n2 + fp) * 4] : &fmet[((size_t)e * 6 + f) * 4];
                double *sl = curved ? &fnrm[(((size_t)nb * 6 + nf) * n2 + orient_host(P, fp, o)) * 4]
                                    : &fmet[((size_t)nb * 6 + nf) * 4];
                double dn = 0;
                for (int k = 0; k < 3; ++k) dn = fmax(dn, fabs(sl[k] + mo[k]));
                if (dn > 1e-8 || fabs(sl[3] - mo[3]) > 1e-8 * mo[3])
                    return fail(c, NSKR_E_ARG, "face " + std::to_string(f) + " of element " + std::to_string(e) +
                                                   ": the neighbour's normal or surface element does not match");
                for (int k = 0; k < 3; ++k) sl[k] = -mo[k];
                sl[3] = mo[3];
            }
        }
    // per wall: extremes of twall + grad . x over its faces, and the rate; a
    // moving wall moves within its own plane at every face point
    std::vector<std::array<double, 3>> trange(m->nbcs > 0 ? m->nbcs : 1,
                                              std::array<double, 3>{INFINITY, -INFINITY, 0.0});
    for (int e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            const int bc = m->bc[e * 6 + f];
            if (m->nbr[e * 6 + f] >= 0 || m->bcs[bc - 1].kind == 2) continue;
            const double *uw = m->bcs[bc - 1].uwall;
            const int npts = curved ? n2 : 1;
            for (int fp = 0; fp < npts; ++fp) {
                const double *fm = curved ? &fnrm[(((size_t)e * 6 + f) * n2 + fp) * 4] : &fmet[((size_t)e * 6 + f) * 4];
                const double un = uw[0] * fm[0] + uw[1] * fm[1] + uw[2] * fm[2];
                if (fabs(un) > 1e-12 * (fabs(uw[0]) + fabs(uw[1]) + fabs(uw[2])))
                    return fail(c, NSKR_E_ARG, "wall velocity must be tangential to the wall");
            }
            const double *tg = m->bcs[bc - 1].twall_grad;
            const double rate = m->bcs[bc - 1].twall_rate;
            if (!(std::isfinite(tg[0]) && std::isfinite(tg[1]) && std::isfinite(tg[2]) && std::isfinite(rate)))
                return fail(c, NSKR_E_ARG, "wall temperature gradient and rate must be finite");
            if (tg[0] == 0.0 && tg[1] == 0.0 && tg[2] == 0.0 && rate == 0.0) continue;
            // affine here: the temperature is linear on the face, so its
            // extremes are at the face's corners
            const int d = f >> 1, sd = f & 1;
            auto &tr = trange[bc - 1];
            for (int v = 0; v < 8; ++v) {
                if (((v >> d) & 1) != sd) continue;
                double T = m->bcs[bc - 1].twall;
                for (int k = 0; k < 3; ++k) {
                    double x = egeo[(size_t)e * 12 + k];
                    for (int dd = 0; dd < 3; ++dd) x += ((v >> dd) & 1) * egeo[(size_t)e * 12 + 3 + 3 * dd + k];
                    T += tg[k] * x;
                }
                if (!(T >= 0.3 && T <= 0.99))
                    return fail(c, NSKR_E_ARG, "wall temperature must stay in [0.3, 0.99] along the wall");
                tr[0] = T < tr[0] ? T : tr[0];
                tr[1] = T > tr[1] ? T : tr[1];
                tr[2] = rate;
            }
        }
    // connectivity codes: (6 nb + nf) 8 + orientation, -1 on walls
    std::vector<int> code((size_t)E * 6);
    for (int e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            const int nb = m->nbr[e * 6 + f];
            code[(size_t)e * 6 + f] = nb < 0 ? -1 : ((nb * 6 + m->nbr_face[e * 6 + f]) << 3) | orient(e, f);
        }
    // wall constants
    std::vector<BcDev> bcs(m->nbcs > 0 ? m->nbcs : 1);
    int dyn = 0, var = 0, trate = 0;
    Vdw vdw{(ld)c->p.R, (ld)c->p.a, (ld)c->p.b};
    for (int k = 0; k < m->nbcs; ++k) {
        BcDev &b = bcs[k];
        memset(&b, 0, sizeof(b));
        b.kind = m->bcs[k].kind;
        b.twall = m->bcs[k].twall;
        b.iso = b.kind == 1 || (b.kind == 3 && std::isinf(m->bcs[k].gamma3));
        if (b.kind != 2)
            for (int d = 0; d < 3; ++d) b.uw[d] = m->bcs[k].uwall[d];
        if (b.kind == 3) {
            b.g1 = m->bcs[k].gamma1;
            b.g2 = m->bcs[k].gamma2;
            b.g3 = b.iso ? 0.0 : m->bcs[k].gamma3;
            b.g4 = m->bcs[k].gamma4;
            b.g1_gam = c->p.gam > 0 ? b.g1 / c->p.gam : 0.0;
            if (b.g1 != 0.0) dyn = 1;
        }
        if (b.kind != 2) {
            ld rv, rl;
            if (!(m->bcs[k].twall > 0) || !maxwell_host(vdw, (ld)m->bcs[k].twall, rv, rl))
                return fail(c, NSKR_E_ARG, "wall temperature must be subcritical and positive");
            ld sig = sigma_host(vdw, (ld)m->bcs[k].twall, (ld)c->p.gam, rv, rl);
            ld d = rl - rv;
            ld ct = cosl((ld)m->bcs[k].theta_deg * 3.14159265358979323846264338327950288L / 180);
            b.rv = (double)rv;
            b.rl = (double)rl;
            // g = -(1/gamma) dpsi_Gamma/dc = -6 sigma cos(theta) / (gamma (rl - rv)^3) (c - rl)(c - rv)
            b.gcoef = c->p.gam > 0 ? (double)(-6 * sig * ct / ((ld)c->p.gam * d * d * d)) : 0.0;
            b.inv_tw = 1.0 / b.twall;
            const double *tg = m->bcs[k].twall_grad;
            b.var = tg[0] != 0.0 || tg[1] != 0.0 || tg[2] != 0.0;
            for (int q = 0; q < 3; ++q) b.tg[q] = tg[q];
            b.cg = c->p.gam > 0 ? (double)(-6 * ct / (ld)c->p.gam) : 0.0;
            b.s2g = (double)sqrtl(2 * (ld)c->p.gam);
            b.rate = m->bcs[k].twall_rate;
            if (b.rate != 0.0) { b.var = 1; trate = 1; }
            if (b.var) var = 1;
        }
    }
    DeviceGuard guard(c->device);
    hipStream_t s = (hipStream_t)sv;
    const std::vector<double> *tab = var ? &wall_table_host(vdw) : nullptr;
    free_mesh(c);
    c->E = E;
    c->dyn = dyn;
    c->var = var;
    c->trate = trate;
    c->wall_trange.swap(trange);
    // (n3, n2: nodes and face points per element, as above)
    c->NN = (size_t)E * n3;
    c->NF = (size_t)E * 6 * n2;
    const size_t ts = c->p.precision == 0 ? sizeof(double) : sizeof(float);
    const int nblk = (E + elem_per_block(c->N) - 1) / elem_per_block(c->N);
    c->stream_nodes = (double)ts * 16.0 * (double)c->NN > kStreamBytes;
    c->curved = curved;
    if (curved) c->bs = 256;  // the only workgroup size built for curved elements
    int rc = NSKR_OK;
    const size_t n_emet = curved ? 0 : emet.size(), n_fmet = curved ? 0 : fmet.size();
    if ((rc = dalloc(c, (void **)&c->d_nbr, sizeof(int) * E * 6)) ||
        (rc = dalloc(c, (void **)&c->d_bcid, sizeof(int) * E * 6)) ||
        (!curved && (rc = dalloc(c, (void **)&c->d_emet, sizeof(double) * n_emet))) ||
        (!curved && (rc = dalloc(c, (void **)&c->d_fmet, sizeof(double) * n_fmet))) ||
        (rc = dalloc(c, (void **)&c->d_egeo, sizeof(double) * egeo.size())) ||
        (curved && (rc = dalloc(c, &c->d_nmet, ts * nmet.size()))) ||
        (curved && (rc = dalloc(c, &c->d_fnrm, ts * fnrm.size()))) ||
        (curved && (rc = dalloc(c, (void **)&c->d_xnode, sizeof(double) * xnode.size()))) ||
        (rc = dalloc(c, (void **)&c->d_bcs, sizeof(BcDev) * bcs.size())) ||
        (rc = dalloc(c, &c->d_Q, ts * 15 * c->NN)) || (rc = dalloc(c, &c->d_TH, ts * c->NN)) ||
        (rc = dalloc(c, &c->d_G2, ts * 4 * c->NN)) || (rc = dalloc(c, &c->d_T2, ts * (ts == 4 ? kT2<float>() : kT2<double>()) * c->NF)) ||
        (rc = dalloc(c, &c->d_TF, ts * 7 * c->NF)) || (rc = dalloc(c, &c->d_TU, ts * 3 * 6 * c->NF)) ||
        (rc = dalloc(c, (void **)&c->d_part, sizeof(double) * NSKR_NSUMS * (size_t)nblk)) ||
        (rc = dalloc(c, (void **)&c->d_out, sizeof(double) * NSKR_NSUMS)) ||
        (c->p.precision == 1 && c->p.kahan && (rc = dalloc(c, &c->d_Ck, ts * 6 * c->NN))) ||
        (tab && (rc = dalloc(c, (void **)&c->d_stab, sizeof(double) * tab->size()))) ||
        (trate && (rc = dalloc(c, (void **)&c->d_clk, sizeof(int))))) {
        free_mesh(c);
        return rc;
    }
    // curved metrics in the element type of the precision
    auto upload_real = [&](void *dst, const std::vector<double> &v) -> hipError_t {
        if (c->p.precision == 0) return hipMemcpy(dst, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice);
        std::vector<float> f(v.size());
        for (size_t q = 0; q < v.size(); ++q) f[q] = (float)v[q];
        return hipMemcpy(dst, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice);
    };
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipMemcpy(c->d_nbr, code.data(), sizeof(int) * E * 6, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_bcid, m->bc, sizeof(int) * E * 6, hipMemcpyHostToDevice));
    if (!curved) {
        HIPCHK(c, hipMemcpy(c->d_emet, emet.data(), sizeof(double) * emet.size(), hipMemcpyHostToDevice));
        HIPCHK(c, hipMemcpy(c->d_fmet, fmet.data(), sizeof(double) * fmet.size(), hipMemcpyHostToDevice));
    } else {
        HIPCHK(c, upload_real(c->d_nmet, nmet));
        HIPCHK(c, upload_real(c->d_fnrm, fnrm));
        HIPCHK(c, hipMemcpy(c->d_xnode, xnode.data(), sizeof(double) * xnode.size(), hipMemcpyHostToDevice));
    }
    HIPCHK(c, hipMemcpy(c->d_egeo, egeo.data(), sizeof(double) * egeo.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_bcs, bcs.data(), sizeof(BcDev) * bcs.size(), hipMemcpyHostToDevice));
    if (tab) HIPCHK(c, hipMemcpy(c->d_stab, tab->data(), sizeof(double) * tab->size(), hipMemcpyHostToDevice));
    c->cent.resize((size_t)E * 3);
    for (int e = 0; e < E; ++e)
        for (int mm = 0; mm < 3; ++mm) {
            const double *g = &egeo[(size_t)e * 12];
            c->cent[(size_t)e * 3 + mm] = (float)(g[mm] + 0.5 * (g[3 + mm] + g[6 + mm] + g[9 + mm]));
        }
    return build_block_map(c);
}

int nskr_state_size(const nskr_ctx *c, size_t *n)
{
    if (!c || !n) return NSKR_E_ARG;
    if (c->E == 0) return NSKR_E_STATE;
    *n = 6 * c->NN;
    return NSKR_OK;
}

int nskr_device_bytes(const nskr_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return NSKR_E_ARG;
    *bytes = c->bytes;
    return NSKR_OK;
}

static int ready(nskr_ctx *c)
{
    if (!c) return NSKR_E_ARG;
    if (c->poisoned) return fail(c, NSKR_E_STATE, "context poisoned by an earlier HIP error");
    if (c->E == 0) return fail(c, NSKR_E_STATE, "no mesh uploaded");
    return NSKR_OK;
}

int nskr_init_droplets(nskr_ctx *c, const nskr_init *ic, const double *noise, void *U, nskr_stream sv)
{
    int rc = ready(c);
    if (rc) return rc;
    if (!ic || !U || ic->ndrop < 0 || !(ic->width > 0) || (ic->ndrop > 0 && (!ic->centres || !ic->radii)))
        return fail(c, NSKR_E_ARG, "bad initial condition");
    for (int k = 0; k < 3; ++k)
        if (ic->periodic[k] && !(ic->length[k] > 0)) return fail(c, NSKR_E_ARG, "periodic axis needs a length");
    Vdw vdw{(ld)c->p.R, (ld)c->p.a, (ld)c->p.b};
    ld rv, rl;
    if (!(ic->T0 > 0)) return fail(c, NSKR_E_ARG, "T0 must be positive");
    if (ic->cylinder_axis < -1 || ic->cylinder_axis > 2) return fail(c, NSKR_E_ARG, "cylinder_axis must be -1, 0, 1 or 2");
    if (ic->rho_v > 0 && ic->rho_l > 0) {
        rv = ic->rho_v;
        rl = ic->rho_l;
        if (!(rl > rv) || (c->p.b > 0 && !(rl * c->p.b < 1)))
            return fail(c, NSKR_E_ARG, "bulk densities must satisfy 0 < rho_v < rho_l < 1/b");
    } else if (!maxwell_host(vdw, (ld)ic->T0, rv, rl)) {
        return fail(c, NSKR_E_ARG, "T0 must be subcritical for the Maxwell densities");
    }
    DeviceGuard guard(c->device);
    hipStream_t s = (hipStream_t)sv;
    if (c->d_drop) { (void)hipFree(c->d_drop); c->d_drop = nullptr; }
    if (c->d_noise) { (void)hipFree(c->d_noise); c->d_noise = nullptr; }
    // per droplet: centre (3), radius, velocity (3)
    std::vector<double> drop(7 * (size_t)(ic->ndrop > 0 ? ic->ndrop : 1), 0.0);
    for (int j = 0; j < ic->ndrop; ++j) {
        for (int k = 0; k < 3; ++k) drop[7 * j + k] = ic->centres[3 * j + k];
        drop[7 * j + 3] = ic->radii[j];
        for (int k = 0; k < 3; ++k) drop[7 * j + 4 + k] = ic->velocities ? ic->velocities[3 * j + k] : 0.0;
    }
    if (hipMalloc((void **)&c->d_drop, sizeof(double) * drop.size()) != hipSuccess)
        return fail(c, NSKR_E_NOMEM, "droplet table allocation failed");
    HIPCHK(c, hipMemcpyAsync(c->d_drop, drop.data(), sizeof(double) * drop.size(), hipMemcpyHostToDevice, s));
    if (noise) {
        if (hipMalloc((void **)&c->d_noise, sizeof(double) * c->NN) != hipSuccess)
            return fail(c, NSKR_E_NOMEM, "noise allocation failed");
        HIPCHK(c, hipMemcpyAsync(c->d_noise, noise, sizeof(double) * c->NN, hipMemcpyHostToDevice, s));
    }
    InitArgs ia;
    ia.mesh = Impl<4, double, 256, false>::mesh(c);
    ia.bas = c->bas;
    ia.NN = c->NN;
    ia.drop = c->d_drop;
    ia.ndrop = ic->ndrop;
    ia.width = ic->width;
    ia.rv = (double)rv;
    ia.rl = (double)rl;
    for (int k = 0; k < 3; ++k) { ia.len[k] = ic->length[k]; ia.per[k] = ic->periodic[k]; }
    for (int k = 0; k < 3; ++k) ia.wax[k] = k == ic->cylinder_axis ? 0.0 : 1.0;
    ia.noise = c->d_noise;
    rc = dispatch(c, [&](auto impl) { return decltype(impl)::init(c, ia, ic->T0, U, s); });
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(s));  // the host-side tables are freed on the next call
    return NSKR_OK;
}

// walls whose temperature changes in time stay inside the table's range over
// [t0, t1] (linear in t, so the ends suffice)
static int check_wall_time(nskr_ctx *c, double t0, double t1)
{
    if (!c->trate) return NSKR_OK;
    for (const auto &r : c->wall_trange) {
        if (r[2] == 0.0) continue;
        for (double t : {t0, t1})
            if (!(r[0] + r[2] * t >= 0.3 && r[1] + r[2] * t <= 0.99))
                return fail(c, NSKR_E_ARG, "wall temperature leaves [0.3, 0.99] during this call");
    }
    return NSKR_OK;
}

int nskr_set_time(nskr_ctx *c, double t)
{
    if (!c || !isfinite(t)) return NSKR_E_ARG;
    c->time = t;
    return NSKR_OK;
}

int nskr_get_time(const nskr_ctx *c, double *t)
{
    if (!c || !t) return NSKR_E_ARG;
    *t = c->time;
    return NSKR_OK;
}

int nskr_rhs(nskr_ctx *c, const void *U, void *Ut, nskr_stream sv)
{
    int rc = ready(c);
    if (rc) return rc;
    if (!U || !Ut || U == Ut) return fail(c, NSKR_E_ARG, "null or aliasing state buffers");
    if ((rc = check_wall_time(c, c->time, c->time))) return rc;
    DeviceGuard guard(c->device);
    return dispatch(c, [&](auto impl) { return decltype(impl)::rhs(c, U, Ut, (hipStream_t)sv); });
}

int nskr_lift1(nskr_ctx *c, const void *U, void *q, nskr_stream sv)
{
    int rc = ready(c);
    if (rc) return rc;
    if (!U || !q || U == q) return fail(c, NSKR_E_ARG, "null or aliasing buffers");
    if ((rc = check_wall_time(c, c->time, c->time))) return rc;
    DeviceGuard guard(c->device);
    return dispatch(c, [&](auto impl) { return decltype(impl)::lift1_out(c, U, q, (hipStream_t)sv); });
}

int nskr_lift2(nskr_ctx *c, const void *U, void *o, nskr_stream sv)
{
    int rc = ready(c);
    if (rc) return rc;
    if (!U || !o || U == o) return fail(c, NSKR_E_ARG, "null or aliasing buffers");
    if ((rc = check_wall_time(c, c->time, c->time))) return rc;
    DeviceGuard guard(c->device);
    return dispatch(c, [&](auto impl) { return decltype(impl)::lift2_out(c, U, o, (hipStream_t)sv); });
}

// dt from the maxima (advective rate, mesh factor, diffusivity, wall rate)
static int dt_from_rates(nskr_ctx *c, const double r[kNRates], double *dt)
{
    if (!isfinite(r[0]) || !isfinite(r[1]) || !isfinite(r[2]) || !isfinite(r[3]) || !(r[0] > 0))
        return fail(c, NSKR_E_NONFINITE, "non-finite wave speed or diffusivity");
    const double dt_adv = c->p.cfl * kTN[c->N] * 2.0 / r[0];
    const double den = c->p.alpha * c->p.beta + kRhoN[c->N] * r[2] * r[1];
    const double dt_par = den > 0 ? c->p.cfl * kRkReal / den : INFINITY;
    const double dt_wall = r[3] > 0 ? c->p.cfl * kRkImag / r[3] : INFINITY;
    *dt = fmin(fmin(dt_adv, dt_par), dt_wall);
    return NSKR_OK;
}

int nskr_dt(nskr_ctx *c, const void *U, double *dt, nskr_stream sv)
{
    int rc = ready(c);
    if (rc) return rc;
    if (!U || !dt) return fail(c, NSKR_E_ARG, "null argument");
    DeviceGuard guard(c->device);
    double r[kNRates];
    rc = dispatch(c, [&](auto impl) { return decltype(impl)::dt(c, U, r, (hipStream_t)sv, c->d_part, c->d_out); });
    if (rc) return rc;
    return dt_from_rates(c, r, dt);
}

int nskr_dt_noalloc(nskr_ctx *c, const void *U, double *dt, nskr_stream sv)
{
    int rc = ready(c);
    if (rc) return rc;
    if (!U || !dt) return fail(c, NSKR_E_ARG, "null argument");
    const int tiles = (c->E + elem_per_block(c->N) - 1) / elem_per_block(c->N);
    if (tiles > kStaticTiles)
        return fail(c, NSKR_E_ARG, "mesh has " + std::to_string(tiles) + " element tiles; the static reduction "
                    "scratch of nskr_dt_noalloc holds " + std::to_string(kStaticTiles));
    double *ptr = static_scratch(c->device);
    if (!ptr) return fail(c, NSKR_E_STATE, "static reduction scratch not set up on this device");
    DeviceGuard guard(c->device);
    double r[kNRates];
    rc = dispatch(c, [&](auto impl) {
        return decltype(impl)::dt(c, U, r, (hipStream_t)sv, ptr, ptr + kNRates * (size_t)kStaticTiles);
    });
    if (rc) return rc;
    return dt_from_rates(c, r, dt);
}

int nskr_rk_steps(nskr_ctx *c, void *U, void *R, double dt, int nsteps, nskr_stream sv)
{
    int rc = ready(c);
    if (rc) return rc;
    if (!U || !R || U == R) return fail(c, NSKR_E_ARG, "null or aliasing state buffers");
    if (!(dt > 0) || !isfinite(dt) || nsteps < 0) return fail(c, NSKR_E_ARG, "dt must be positive and finite");
    if ((rc = check_wall_time(c, c->time, c->time + nsteps * dt))) return rc;
    DeviceGuard guard(c->device);
    return dispatch(c, [&](auto impl) { return decltype(impl)::rk(c, U, R, dt, nsteps, (hipStream_t)sv); });
}

int nskr_reduce(nskr_ctx *c, const void *U, double *out, nskr_stream sv)
{
    int rc = ready(c);
    if (rc) return rc;
    if (!U || !out) return fail(c, NSKR_E_ARG, "null argument");
    DeviceGuard guard(c->device);
    rc = dispatch(c, [&](auto impl) { return decltype(impl)::reduce(c, U, out, (hipStream_t)sv); });
    if (rc) return rc;
    if (out[NSKR_CNT_NONFINITE] > 0 || out[NSKR_CNT_RHO_RANGE] > 0 || out[NSKR_CNT_T_NONPOS] > 0)
        return fail(c, NSKR_E_NONFINITE, "non-finite or out-of-range state");
    return NSKR_OK;
}

int nskr_set_block(nskr_ctx *c, int threads)
{
    if (!c) return NSKR_E_ARG;
    if (!block_ok(c->N, threads))
        return fail(c, NSKR_E_ARG, "block size must be 256, 512 or the degree's tight size (N=2: 192, N=3, 4: 128, "
                                   "N=5: 448) and hold an element");
    if (c->curved && threads != 256) return fail(c, NSKR_E_UNSUPPORTED, "meshes with curved elements run 256 threads");
    DeviceGuard guard(c->device);
    int maxlds = 0;
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess)
        return fail(c, NSKR_E_HIP, "cannot query the LDS limit");
    const int old = c->bs;
    c->bs = threads;
    const int ok = dispatch(c, [&](auto impl) { return decltype(impl)::fits(maxlds); });
    if (!ok) {
        c->bs = old;
        return fail(c, NSKR_E_UNSUPPORTED, "kernels of this block size exceed the device's LDS per block");
    }
    if (c->E > 0 && c->bmap_bs != c->bs) return build_block_map(c);
    return NSKR_OK;
}

int nskr_get_block(const nskr_ctx *c, int *threads)
{
    if (!c || !threads) return NSKR_E_ARG;
    *threads = c->bs;
    return NSKR_OK;
}

int nskr_set_profiling(nskr_ctx *c, int on)
{
    if (!c) return NSKR_E_ARG;
    c->prof = on != 0;
    return NSKR_OK;
}

int nskr_profile(nskr_ctx *c, double *ms, long *count, nskr_stream sv)
{
    if (!c || !ms || !count) return NSKR_E_ARG;
    DeviceGuard guard(c->device);
    for (int k = 0; k < NSKR_NKINDS; ++k) { ms[k] = 0.0; count[k] = 0; }
    HIPCHK(c, hipStreamSynchronize((hipStream_t)sv));
    for (auto &pe : c->prof_events) {
        float t = 0.0f;
        HIPCHK(c, hipEventSynchronize(pe.second.second));
        HIPCHK(c, hipEventElapsedTime(&t, pe.second.first, pe.second.second));
        ms[pe.first] += t;
        count[pe.first] += 1;
        c->event_pool.push_back(pe.second.first);
        c->event_pool.push_back(pe.second.second);
    }
    c->prof_events.clear();
    return NSKR_OK;
}

const char *nskr_last_error(const nskr_ctx *c)
{
    if (!c) return g_null_msg;
    return c->err.c_str();
}

// ------------------------------------------------------------------ batches
}  // extern "C"

struct BatchSlot {
    nskr_ctx *c = nullptr;
    void *U = nullptr, *R = nullptr;
    double dt = 0.0;
    int nsteps = 0, done = 0;
    int state = 0;  // 0 free, 1 active, 2 last step queued (finished once `last` has completed)
    bool fresh = true;  // face traces not yet prolonged (and compensation not yet cleared)
    double t0 = 0.0;    // instance time at admission
    size_t bytes = 0;
    hipEvent_t last = nullptr;  // recorded after the step that completes the instance
};

struct BatchGroup {
    int N = 0, prec = 0, bs = 0, nblocks = 0;
    bool curved = false;
    void *d_tab = nullptr;
    int *d_bi = nullptr, *d_be = nullptr;
    Basis bas;
};

struct nskr_batch {
    int device = 0;
    size_t budget = 0, used = 0;
    std::vector<BatchSlot> slots;
    std::vector<BatchGroup> groups;
    bool dirty = true, use_graph = true, poisoned = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int **d_ticks = nullptr;  // step counters of the active instances whose walls change in time
    int nticks = 0;
    long steps = 0;
    hipEvent_t queued = nullptr;  // recorded after every step: all work queued so far
    std::vector<hipEvent_t> event_pool;
    std::string err;
};

static hipEvent_t batch_event(nskr_batch *b)
{
    if (!b->event_pool.empty()) {
        hipEvent_t e = b->event_pool.back();
        b->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

static int bfail(nskr_batch *b, int code, const std::string &msg)
{
    b->err = msg;
    return code;
}

#define BHIPCHK(b, x)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            (b)->poisoned = true;                                                        \
            return bfail((b), NSKR_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
        }                                                                                \
    } while (0)

static void batch_free_groups(nskr_batch *b)
{
    for (auto &g : b->groups) {
        if (g.d_tab) (void)hipFree(g.d_tab);
        if (g.d_bi) (void)hipFree(g.d_bi);
        if (g.d_be) (void)hipFree(g.d_be);
    }
    b->groups.clear();
    if (b->d_ticks) { (void)hipFree(b->d_ticks); b->d_ticks = nullptr; }
    b->nticks = 0;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
}

template <int P, typename T, int BS, bool CV>
static int build_group(nskr_batch *b, BatchGroup &g, const std::vector<int> &members)
{
    using G = Tile<P, BS>;
    std::vector<Inst<T>> tab;
    std::vector<int> bi, be;
    for (size_t k = 0; k < members.size(); ++k) {
        BatchSlot &sl = b->slots[members[k]];
        tab.push_back(Impl<P, T, BS, CV>::inst(sl.c, sl.U, sl.R, nullptr, sl.dt));
        tab.back().clk = sl.c->trate ? sl.c->d_clk : nullptr;
        tab.back().t0 = sl.t0;
        const int nb = (sl.c->E + G::EPB - 1) / G::EPB;
        for (int j = 0; j < nb; ++j) {
            bi.push_back((int)k);
            be.push_back(j * G::EPB);
        }
    }
    g.nblocks = (int)bi.size();
    g.bas = b->slots[members[0]].c->bas;
    BHIPCHK(b, hipMalloc(&g.d_tab, sizeof(Inst<T>) * tab.size()));
    BHIPCHK(b, hipMalloc((void **)&g.d_bi, sizeof(int) * bi.size()));
    BHIPCHK(b, hipMalloc((void **)&g.d_be, sizeof(int) * be.size()));
    BHIPCHK(b, hipMemcpy(g.d_tab, tab.data(), sizeof(Inst<T>) * tab.size(), hipMemcpyHostToDevice));
    BHIPCHK(b, hipMemcpy(g.d_bi, bi.data(), sizeof(int) * bi.size(), hipMemcpyHostToDevice));
    BHIPCHK(b, hipMemcpy(g.d_be, be.data(), sizeof(int) * be.size(), hipMemcpyHostToDevice));
    return NSKR_OK;
}

template <int P, typename T, int BS, bool CV> static void launch_group(const BatchGroup &g, hipStream_t s)
{
    Launch<T> L;
    memset(&L, 0, sizeof(L));
    L.tab = (const Inst<T> *)g.d_tab;
    L.blk_inst = g.d_bi;
    L.blk_e0 = g.d_be;
    L.bas = g.bas;
    Impl<P, T, BS, CV>::step_batched(L, g.nblocks, s);
}

template <typename F> static int group_dispatch(const BatchGroup &g, F &&f)
{
    return impl_dispatch(g.N, g.prec, g.bs, g.curved, f);
}

static int batch_rebuild(nskr_batch *b)
{
    batch_free_groups(b);
    // group active instances by (degree, precision, block size)
    std::vector<std::vector<int>> members;
    std::vector<BatchGroup> groups;
    for (int i = 0; i < (int)b->slots.size(); ++i) {
        const BatchSlot &sl = b->slots[i];
        if (sl.state != 1) continue;
        int gi = -1;
        for (int k = 0; k < (int)groups.size(); ++k)
            if (groups[k].N == sl.c->N && groups[k].prec == sl.c->p.precision && groups[k].bs == sl.c->bs &&
                groups[k].curved == sl.c->curved)
                gi = k;
        if (gi < 0) {
            BatchGroup g;
            g.N = sl.c->N;
            g.prec = sl.c->p.precision;
            g.bs = sl.c->bs;
            g.curved = sl.c->curved;
            groups.push_back(g);
            members.emplace_back();
            gi = (int)groups.size() - 1;
        }
        members[gi].push_back(i);
    }
    for (size_t k = 0; k < groups.size(); ++k) {
        BatchGroup &g = groups[k];
        int rc = group_dispatch(g, [&](auto impl) {
            using I = decltype(impl);
            return build_group<I::kP, typename I::Real, I::kBS, I::kCV>(b, g, members[k]);
        });
        b->groups.push_back(g);
        if (rc) return rc;
    }
    std::vector<int *> ticks;
    for (const auto &sl : b->slots)
        if (sl.state == 1 && sl.c->trate) ticks.push_back(sl.c->d_clk);
    if (!ticks.empty()) {
        BHIPCHK(b, hipMalloc((void **)&b->d_ticks, sizeof(int *) * ticks.size()));
        BHIPCHK(b, hipMemcpy(b->d_ticks, ticks.data(), sizeof(int *) * ticks.size(), hipMemcpyHostToDevice));
        b->nticks = (int)ticks.size();
    }
    b->dirty = false;
    return NSKR_OK;
}

extern "C" {

int nskr_batch_create(int device, size_t budget_bytes, nskr_batch **out)
{
    if (!out) return NSKR_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return NSKR_E_HIP;
    nskr_batch *b = new nskr_batch();
    b->device = device;
    b->budget = budget_bytes;
    *out = b;
    return NSKR_OK;
}

int nskr_batch_destroy(nskr_batch *b)
{
    if (!b) return NSKR_OK;
    {
        DeviceGuard g(b->device);
        if (b->queued) (void)hipEventSynchronize(b->queued);
        batch_free_groups(b);
        for (auto &sl : b->slots)
            if (sl.last) (void)hipEventDestroy(sl.last);
        for (hipEvent_t e : b->event_pool) (void)hipEventDestroy(e);
        if (b->queued) (void)hipEventDestroy(b->queued);
    }
    delete b;
    return NSKR_OK;
}

int nskr_batch_set_graph(nskr_batch *b, int on)
{
    if (!b) return NSKR_E_ARG;
    if ((on != 0) != b->use_graph) {
        b->use_graph = on != 0;
        b->dirty = true;
    }
    return NSKR_OK;
}

int nskr_batch_admit(nskr_batch *b, nskr_ctx *c, void *U, void *R, double dt, int nsteps, int *slot)
{
    if (!b || !c || !slot) return NSKR_E_ARG;
    if (b->poisoned) return bfail(b, NSKR_E_STATE, "batch poisoned by an earlier HIP error");
    if (c->poisoned || c->E == 0) return bfail(b, NSKR_E_STATE, "instance has no mesh or is poisoned");
    if (c->device != b->device) return bfail(b, NSKR_E_ARG, "instance lives on another device");
    if (!U || !R || U == R) return bfail(b, NSKR_E_ARG, "null or aliasing state buffers");
    if (!(dt > 0) || !isfinite(dt) || nsteps < 1) return bfail(b, NSKR_E_ARG, "dt must be positive, nsteps >= 1");
    for (const auto &sl : b->slots)
        if (sl.state != 0 && sl.c == c) return bfail(b, NSKR_E_ARG, "instance already admitted");
    if (check_wall_time(c, c->time, c->time + nsteps * dt))
        return bfail(b, NSKR_E_ARG, "wall temperature leaves [0.3, 0.99] during the admitted steps");
    const size_t ts = c->p.precision == 0 ? sizeof(double) : sizeof(float);
    const size_t need = c->bytes + 2 * 6 * c->NN * ts;
    if (b->used + need > b->budget) return bfail(b, NSKR_E_NOMEM, "no room in the memory budget now");
    int k = -1;
    for (int i = 0; i < (int)b->slots.size(); ++i)
        if (b->slots[i].state == 0) { k = i; break; }
    if (k < 0) {
        b->slots.emplace_back();
        k = (int)b->slots.size() - 1;
    }
    BatchSlot &sl = b->slots[k];
    sl.c = c; sl.U = U; sl.R = R; sl.dt = dt; sl.nsteps = nsteps; sl.done = 0; sl.state = 1; sl.bytes = need;
    sl.fresh = true;
    sl.t0 = c->time;
    b->used += need;
    b->dirty = true;
    *slot = k;
    return NSKR_OK;
}

int nskr_batch_retire(nskr_batch *b, int slot)
{
    if (!b || slot < 0 || slot >= (int)b->slots.size() || b->slots[slot].state == 0) return NSKR_E_ARG;
    BatchSlot &sl = b->slots[slot];
    {
        // the buffers go back to the caller: wait until no queued step of the
        // batch can still touch them
        DeviceGuard guard(b->device);
        if (b->queued) BHIPCHK(b, hipEventSynchronize(b->queued));
    }
    if (sl.state == 1) {
        b->dirty = true;
        sl.c->time = sl.t0 + sl.done * sl.dt;
    }
    if (sl.last) b->event_pool.push_back(sl.last);
    b->used -= sl.bytes;
    sl = BatchSlot();
    return NSKR_OK;
}

int nskr_batch_step(nskr_batch *b, nskr_stream sv)
{
    if (!b) return NSKR_E_ARG;
    if (b->poisoned) return bfail(b, NSKR_E_STATE, "batch poisoned by an earlier HIP error");
    DeviceGuard guard(b->device);
    hipStream_t s = (hipStream_t)sv;
    int nact = 0;
    for (const auto &sl : b->slots) nact += sl.state == 1;
    if (nact == 0) return NSKR_OK;
    if (b->dirty) {
        BHIPCHK(b, hipStreamSynchronize(s));  // earlier replays may still read the old tables
        int rc = batch_rebuild(b);
        if (rc) return rc;
    }
    for (auto &sl : b->slots)
        if (sl.state == 1 && sl.fresh) {
            // on the step stream, ahead of the instance's first step: its
            // compensation cleared and its face traces prolonged
            dispatch(sl.c, [&](auto impl) {
                decltype(impl)::zero_comp(sl.c, s);
                return decltype(impl)::prime(sl.c, sl.U, sl.R, sl.dt, s);
            });
            if (sl.c->trate) hipLaunchKernelGGL((k_zero<int>), dim3(1), dim3(kBlock), 0, s, sl.c->d_clk, (size_t)1);
            sl.fresh = false;
        }
    if (b->use_graph) {
        if (!b->exec) {
            BHIPCHK(b, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            for (const auto &g : b->groups)
                group_dispatch(g, [&](auto impl) {
                    using I = decltype(impl);
                    launch_group<I::kP, typename I::Real, I::kBS, I::kCV>(g, s);
                    return 0;
                });
            if (b->nticks)
                hipLaunchKernelGGL(k_tick, dim3((b->nticks + 63) / 64), dim3(64), 0, s, b->d_ticks, b->nticks);
            BHIPCHK(b, hipStreamEndCapture(s, &b->graph));
            BHIPCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        }
        BHIPCHK(b, hipGraphLaunch(b->exec, s));
    } else {
        for (const auto &g : b->groups)
            group_dispatch(g, [&](auto impl) {
                using I = decltype(impl);
                launch_group<I::kP, typename I::Real, I::kBS, I::kCV>(g, s);
                return 0;
            });
        if (b->nticks)
            hipLaunchKernelGGL(k_tick, dim3((b->nticks + 63) / 64), dim3(64), 0, s, b->d_ticks, b->nticks);
        BHIPCHK(b, hipGetLastError());
    }
    b->steps++;
    if (!b->queued) {
        b->queued = batch_event(b);
        if (!b->queued) return bfail(b, NSKR_E_HIP, "event creation failed");
    }
    BHIPCHK(b, hipEventRecord(b->queued, s));
    for (auto &sl : b->slots)
        if (sl.state == 1 && ++sl.done >= sl.nsteps) {
            sl.state = 2;
            sl.c->time = sl.t0 + sl.nsteps * sl.dt;
            b->dirty = true;
            if (!sl.last) sl.last = batch_event(b);
            if (!sl.last) return bfail(b, NSKR_E_HIP, "event creation failed");
            BHIPCHK(b, hipEventRecord(sl.last, s));
        }
    return NSKR_OK;
}

int nskr_batch_poll(nskr_batch *b, int *slots, int cap, int *n)
{
    if (!b || !n || (cap > 0 && !slots)) return NSKR_E_ARG;
    DeviceGuard guard(b->device);
    int k = 0;
    for (int i = 0; i < (int)b->slots.size(); ++i) {
        const BatchSlot &sl = b->slots[i];
        if (sl.state != 2) continue;
        if (sl.last) {
            const hipError_t q = hipEventQuery(sl.last);
            if (q == hipErrorNotReady) continue;  // its last step has not run yet
            if (q != hipSuccess) {
                b->poisoned = true;
                return bfail(b, NSKR_E_HIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
            }
        }
        if (k < cap) slots[k] = i;
        ++k;
    }
    *n = k;
    return NSKR_OK;
}

int nskr_batch_info(const nskr_batch *b, size_t *used_bytes, int *active, long *steps)
{
    if (!b) return NSKR_E_ARG;
    int nact = 0;
    for (const auto &sl : b->slots) nact += sl.state == 1;
    if (used_bytes) *used_bytes = b->used;
    if (active) *active = nact;
    if (steps) *steps = b->steps;
    return NSKR_OK;
}

const char *nskr_batch_last_error(const nskr_batch *b)
{
    if (!b) return "nskr: null batch";
    return b->err.c_str();
}

}  // extern "C"
