// kernels.h -- HIP kernels of the non-LTE library (gfx950, wave64).
//
// Data layout: structure of arrays, C order [q][z][y][x] with x fastest.  A voxel index
// is v = (k*ny + y)*nx + x; a plane point index is g = y*nx + x.  Populations and rate
// data are FP64; sweep inputs/outputs are of the sweep precision R (float or double).
#pragma once
#include "devmath.h"

namespace nlte {

constexpr int kMaxLevels = 8;
constexpr int kMaxLines = 16;
constexpr int kNDir = 24;
constexpr int kNHemi = 12;

// A4 directions (unit vectors), 12 upward then their reflections; weights are 1/24.
__constant__ double c_mu[kNDir * 3];

struct LineInfo {
    int lower, upper, fstart, nfreq, gauss;
    double nu0, A, Bij, Bji, hnu4pi, gamma_rad, gamma_vdw;
};

struct AtomInfo {
    int N, nline, ncont, ncoll, eps_mode;
    int cont_active;     // 1: continua are transitions of the formal solution, 0: fixed rates
    double mass, xi, eps;
    double E[kMaxLevels], g[kMaxLevels];
    int stage[kMaxLevels];
    LineInfo line[kMaxLines];
    int cont_lower[kMaxLevels], cont_upper[kMaxLevels];
    double cont_alpha0[kMaxLevels];
    int cont_nup;                   // active continua: distinct upper levels,
    int cont_ulev[kMaxLevels];      // in order of first appearance,
    int cont_uidx[kMaxLevels];      // and each continuum's index among them
    int coll_lower[kMaxLevels * kMaxLevels], coll_upper[kMaxLevels * kMaxLevels];
    double coll_cul[kMaxLevels * kMaxLevels], coll_Tref[kMaxLevels * kMaxLevels],
        coll_beta[kMaxLevels * kMaxLevels];
};

// ------------------------------------------------------------------ level setup
// Primitive field order in the FP64 primitive block.
enum { P_T = 0, P_NE, P_NH, P_NTOT, P_VX, P_VY, P_VZ, P_CHIC };

// Sweep-constant block (precision R): [SC_*][nline][nvox] then [SV_*][nvox].
enum { SC_CHIC = 0, SC_ETAC, SC_ADAMP, SC_PN, SC_PW, SC_B, SC_NQ };
enum { SV_INVVD = 0, SV_VX, SV_VY, SV_VZ, SV_NQ };

template <typename R>
struct SetupArgs {
    const AtomInfo* atom;
    const double* prim;      // [7 + nline][nvox]
    int has_chic;
    size_t nvox;
    R* sc;                   // [SC_NQ][nline][nvox]
    R* sv;                   // [SV_NQ][nvox]
    double* nstar;           // [N][nvox]
    double* pfix;            // [N*N][nvox], rate i -> j at (i*N + j)
    double* ntot;            // [nvox]
};

// Per-voxel local physics: Doppler width, damping, Planck, background, LTE
// populations and the fixed (collisional + bound-free) rates.  FP64 throughout.
template <typename R>
__global__ void setup_level_kernel(SetupArgs<R> a) {
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= a.nvox) return;
    const AtomInfo& at = *a.atom;
    const size_t nv = a.nvox;
    const double T = a.prim[P_T * nv + v];
    const double ne = a.prim[P_NE * nv + v];
    const double nH = a.prim[P_NH * nv + v];
    const double nt = a.prim[P_NTOT * nv + v];
    const double vD = sqrt(2.0 * kKB * T / (at.mass * kAMU) + at.xi * at.xi);
    const double ivD = 1.0 / vD;
    a.sv[SV_INVVD * nv + v] = R(ivD);
    a.sv[SV_VX * nv + v] = R(a.prim[P_VX * nv + v] * ivD);
    a.sv[SV_VY * nv + v] = R(a.prim[P_VY * nv + v] * ivD);
    a.sv[SV_VZ * nv + v] = R(a.prim[P_VZ * nv + v] * ivD);
    a.ntot[v] = nt;
    const int L = at.nline;
    for (int l = 0; l < L; ++l) {
        const LineInfo& ln = at.line[l];
        const double B = planck(ln.nu0, T);
        const double dnuD = ln.nu0 * vD / kC;
        const double gam = ln.gamma_rad + ln.gamma_vdw * nH * pow(T / 5000.0, 0.3);
        const double chic = a.has_chic ? a.prim[(P_CHIC + l) * nv + v] : 0.0;
        a.sc[(SC_CHIC * L + l) * nv + v] = R(chic);
        a.sc[(SC_ETAC * L + l) * nv + v] = R(chic * B);
        a.sc[(SC_ADAMP * L + l) * nv + v] = R(gam / (4.0 * kPI * dnuD));
        a.sc[(SC_PN * L + l) * nv + v] = R(1.0 / (kSQRTPI * dnuD));
        a.sc[(SC_B * L + l) * nv + v] = R(B);
    }
    // Saha-Boltzmann: n_i* ~ g_i exp(-hcE_i/kT) Phi^(s_i - s_min), Phi = 2(2 pi m kT/h^2)^1.5/n_e
    const int N = at.N;
    int smin = at.stage[0];
    for (int i = 1; i < N; ++i) smin = min(smin, at.stage[i]);
    double lw[kMaxLevels], mx = -1e300;
    const double hc_kT = kH * kC / (kKB * T);
    for (int i = 0; i < N; ++i) {
        double w = log(at.g[i]) - hc_kT * at.E[i];
        if (at.stage[i] != smin) {
            const double phi = 2.0 * pow(2.0 * kPI * kME * kKB * T / (kH * kH), 1.5) / ne;
            w += (at.stage[i] - smin) * log(phi);
        }
        lw[i] = w;
        mx = fmax(mx, w);
    }
    double ws[kMaxLevels], tot = 0.0;
    for (int i = 0; i < N; ++i) { ws[i] = exp(lw[i] - mx); tot += ws[i]; }
    double ns[kMaxLevels];
    for (int i = 0; i < N; ++i) { ns[i] = nt * ws[i] / tot; a.nstar[i * nv + v] = ns[i]; }
    double P[kMaxLevels * kMaxLevels];
    for (int i = 0; i < N * N; ++i) P[i] = 0.0;
    if (at.eps_mode) {
        for (int l = 0; l < L; ++l) {
            const LineInfo& ln = at.line[l];
            const double c21 = at.eps * ln.A / ((1.0 - at.eps) * (-expm1(-kH * ln.nu0 / (kKB * T))));
            P[ln.upper * N + ln.lower] += c21;
            P[ln.lower * N + ln.upper] += c21 * ws[ln.upper] / ws[ln.lower];
        }
    } else {
        for (int c = 0; c < at.ncoll; ++c) {
            const int lo = at.coll_lower[c], up = at.coll_upper[c];
            const double cul = ne * at.coll_cul[c] * pow(T / at.coll_Tref[c], at.coll_beta[c]);
            P[up * N + lo] += cul;
            P[lo * N + up] += cul * ws[up] / ws[lo];
        }
    }
    for (int c = 0; c < (at.cont_active ? 0 : at.ncont); ++c) {
        const int i = at.cont_lower[c], j = at.cont_upper[c];
        const double nue = kC * (at.E[j] - at.E[i]);
        const double x = kH * nue / (kKB * T);
        const double ric = 8.0 * kPI * at.cont_alpha0[c] * nue * nue * nue / (kC * kC) * bf_planck_integral(x);
        P[i * N + j] += ric;
        P[j * N + i] += ric * ws[i] / ws[j];
    }
    for (int i = 0; i < N * N; ++i) a.pfix[size_t(i) * nv + v] = P[i];
}

// Profile normalisation phi~ = phi / sum_d sum_m w_d w_m phi per (line, voxel), using
// the same profile evaluation as the sweep.  Writes pw = pn * N_l.
template <typename R>
__global__ void profile_norm_kernel(const AtomInfo* atom, const R* qf, const R* wf, R* sc,
                                   const R* sv, size_t nvox) {
    // the small-damping Voigt table (FP32 profiles), staged in LDS as in the sweep
    __shared__ float4 dawg[kDawIntervals];
    if (sizeof(R) == 4) {
        for (int i = int(threadIdx.x); i < kDawIntervals; i += int(blockDim.x)) dawg[i] = c_dawg[i];
        __syncthreads();
    }
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    const AtomInfo& at = *atom;
    const int L = at.nline;
    const R ivD = sv[SV_INVVD * nvox + v];
    const R vx = sv[SV_VX * nvox + v], vy = sv[SV_VY * nvox + v], vz = sv[SV_VZ * nvox + v];
    for (int l = 0; l < L; ++l) {
        const LineInfo& ln = at.line[l];
        const R a = sc[(SC_ADAMP * L + l) * nvox + v];
        const R pn = sc[(SC_PN * L + l) * nvox + v];
        double acc = 0.0;
        for (int d = 0; d < kNDir; ++d) {
            const R vn = vx * R(c_mu[3 * d]) + vy * R(c_mu[3 * d + 1]) + vz * R(c_mu[3 * d + 2]);
            double accd = 0.0;
            for (int m = 0; m < ln.nfreq; ++m) {
                const int f = ln.fstart + m;
                const R u = qf[f] * ivD - vn;
                const R H = profile_H<R>(a, u, ln.gauss != 0, dawg);
                accd += double(wf[f]) * double(H * pn);
            }
            acc += accd / kNDir;
        }
        sc[(SC_PW * L + l) * nvox + v] = R(double(pn) / acc);
    }
}

// The line profile shape H(a, u) of the sweeps (damped lines) at n points, evaluated in
// precision R from FP64 inputs (rounded to R first).
template <typename R>
__global__ void voigt_eval_kernel(const double* a, const double* u, double* H, int n) {
    const int i = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) H[i] = double(profile_H<R>(R(a[i]), R(u[i]), false, c_dawg));
}

// ------------------------------------------------------------------ line coefficients
// k_l^+ = max((h nu0/4pi)(n_i^+ B_ij - n_j^+ B_ji), 0), e_l = (h nu0/4pi) n_j^+ A_ji.
template <typename R>
__global__ void line_coef_kernel(const AtomInfo* atom, const double* n, R* lc, size_t nvox) {
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    const AtomInfo& at = *atom;
    const int L = at.nline;
    for (int l = 0; l < L; ++l) {
        const LineInfo& ln = at.line[l];
        const double ni = fmax(n[size_t(ln.lower) * nvox + v], 0.0);
        const double nj = fmax(n[size_t(ln.upper) * nvox + v], 0.0);
        lc[size_t(l) * nvox + v] = R(fmax(ln.hnu4pi * (ni * ln.Bij - nj * ln.Bji), 0.0));
        lc[size_t(L + l) * nvox + v] = R(ln.hnu4pi * nj * ln.A);
    }
}

// ------------------------------------------------------------------ sweep
// Plane state of one (direction, frequency, point).  FP32 stores the intensity and the
// profile value phi (8 bytes): a reader rebuilds an upwind corner's opacity and source
// function from phi and that voxel's line constants with the writer's own expressions
// (corner_SC), so it sees exactly the values the writer computed while a third less state
// moves through HBM.  FP64, bound by its arithmetic, where the rebuild's divisions would
// cost more than the bytes save, stores the intensity, source function and opacity.
template <typename R>
struct Cell;
template <>
struct Cell<float> {
    float I, P;
};
template <>
struct Cell<double> {
    double I, S, C;
};
template <typename R>
constexpr bool kPhiCell = sizeof(R) == 4;

// Everything one update produces at a point: intensity, source function, opacity, phi.
template <typename R>
struct CellVals {
    R I, S, C, P;
};
__device__ inline Cell<float> make_cell(const CellVals<float>& v) { return Cell<float>{v.I, v.P}; }
__device__ inline Cell<double> make_cell(const CellVals<double>& v) { return Cell<double>{v.I, v.S, v.C}; }

// Cells move through raw buffer instructions: the resource holds the wave-uniform base
// of one (direction, line) column and its size, the lane supplies a fixed byte offset
// within a frequency row and the scalar offset selects the row, so addressing costs no
// vector instructions.  Accesses past the resource size read 0 and write nothing.
// Word 3 is the raw-buffer format of the gfx9 family.
__device__ inline __amdgpu_buffer_rsrc_t cell_rsrc(const void* base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, int(bytes), 0x00020000);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ inline Cell<float> cell_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    const f32x2 x = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    return Cell<float>{x.x, x.y};
}
__device__ inline Cell<double> cell_load_d(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    const f64x2 a = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    const double c = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff + 16u, soff, 0));
    return Cell<double>{a.x, a.y, c};
}
template <typename R> __device__ inline Cell<R> cell_get(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <> __device__ inline Cell<float> cell_get<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return cell_load(r, voff, soff);
}
template <> __device__ inline Cell<double> cell_get<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    return cell_load_d(r, voff, soff);
}
// FP32 cells are stored non-temporally (cache-policy bit 1, `nt`): a plane step's cells are
// read back only by the next plane step's launch, long after they have left L2, so they
// should not displace the upwind rows that neighbouring tiles of the same launch re-read
// (measured on 504x504 planes: 3.6 % less time per launch; the values are unchanged).
constexpr int kStoreNonTemporal = 2;
__device__ inline void cell_put(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, const Cell<float>& c) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, f32x2{c.I, c.P}), r, voff, soff,
                                          kStoreNonTemporal);
}
__device__ inline void cell_put(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, const Cell<double>& c) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned,
                                                              f64x2{c.I, c.S}), r, voff, soff, 0);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, c.C),
                                          r, voff + 16u, soff, 0);
}

// Read-only tables read through the constant address space, so that loads at a
// wave-uniform index become scalar loads.
template <typename R>
using const_as = __attribute__((address_space(4))) const R;

// Partial sums of the sweep.  Every thread sums one direction's contributions over
// its frequencies in order; directions are then combined by one fixed tree, whatever
// the block shape:  g_i = (d_3i + d_3i+1) + d_3i+2  (8 groups of 3),
// hemisphere = (g_0 + g_1) + (g_2 + g_3), total = up + down.  A block of DB directions
// evaluates the part of the tree it holds and stores one slot per block; the readers
// finish the tree over the 24/DB slots with tree_slots().
constexpr int kMaxSlots = 8;

template <typename R>
__device__ __host__ inline R tree_slots(const R* x, size_t stride, int nslot) {
    if (nslot == 2) return x[0] + x[stride];
    if (nslot == 4) return (x[0] + x[stride]) + (x[2 * stride] + x[3 * stride]);
    return ((x[0] + x[stride]) + (x[2 * stride] + x[3 * stride])) +
           ((x[4 * stride] + x[5 * stride]) + (x[6 * stride] + x[7 * stride]));
}

// One plane step of the short-characteristics formal solution for all 24 directions.
// Step s: upward directions solve plane s from plane s-1, downward directions plane
// nz-1-s from nz-s; s = 0 sets the boundary planes (I = B below, I = 0 or prescribed
// above).  Block: DB x FC waves; wave (c, w) takes direction grp*DB + w and the c-th of
// FC contiguous chunks of the line's frequencies over 64 consecutive plane points.
// Grid: (plane tiles of 64 points, lines, 24/DB direction groups), dealt to the XCDs
// so that all tiles of a (line, direction group) share one L2.  Direction and frequency
// are uniform across a wave, so the frequency tables are scalar loads and every cell
// access is a scalar base plus a fixed 32-bit lane offset.  A wave sums its chunk in
// frequency order; chunks are added in order, then directions by the fixed tree.  FC
// changes the rounding of the frequency sum, so it is fixed by the level shape alone.
// One short-characteristics update of a cell for one direction and frequency, shared by
// every sweep kernel so that they compute bit-identical cells and sums: the local opacity
// and source function from the profile, the segment from the (already interpolated)
// upwind values, the new cell, and the two positive accumulation terms.
template <typename R>
struct PointConst {
    R chic, etac, adamp, pn, pw, kpl, el, ivD, vn;
};

template <typename R>
__device__ inline PointConst<R> point_const(const R* sc, const R* sv, const R* lc, int L, int l, size_t nv,
                                            size_t v, double mux, double muy, double muz) {
    PointConst<R> c;
    c.chic = sc[(SC_CHIC * L + l) * nv + v];
    c.etac = sc[(SC_ETAC * L + l) * nv + v];
    c.adamp = sc[(SC_ADAMP * L + l) * nv + v];
    c.pn = sc[(SC_PN * L + l) * nv + v];
    c.pw = sc[(SC_PW * L + l) * nv + v] * R(1.0 / kNDir);
    c.kpl = lc[size_t(l) * nv + v];
    c.el = lc[size_t(L + l) * nv + v];
    c.ivD = sv[SV_INVVD * nv + v];
    c.vn = sv[SV_VX * nv + v] * R(mux) + sv[SV_VY * nv + v] * R(muy) + sv[SV_VZ * nv + v] * R(muz);
    return c;
}

template <typename R>
__device__ inline R interp4(R w00, R w01, R w10, R w11, R a00, R a01, R a10, R a11) {
    return fma(w00, a00, fma(w01, a01, fma(w10, a10, w11 * a11)));
}

// Line constants of an upwind corner voxel, to rebuild its opacity and source function
// from a stored phi; sfb is the source function where the opacity is negligible, which
// does not depend on phi.
template <typename R>
struct CornerConst {
    R kpl, chic, el, etac, sfb;
};
template <typename R>
struct Corners {
    CornerConst<R> q00, q01, q10, q11;
};

template <typename R>
__device__ inline CornerConst<R> corner_const(const R* sc, const R* lc, int L, int l, size_t nv, size_t v) {
    CornerConst<R> q;
    q.chic = sc[(SC_CHIC * L + l) * nv + v];
    q.etac = sc[(SC_ETAC * L + l) * nv + v];
    q.kpl = lc[size_t(l) * nv + v];
    q.el = lc[size_t(L + l) * nv + v];
    q.sfb = source_limit(q.chic, q.etac, q.kpl, q.el);
    return q;
}

// The corners' constants where cells carry phi (FP32); nothing to load otherwise.
template <typename R>
__device__ inline Corners<R> corners_at(const R* sc, const R* lc, int L, int l, size_t nv, size_t v00, size_t v01,
                                        size_t v10, size_t v11) {
    Corners<R> q{};
    if constexpr (kPhiCell<R>) {
        q.q00 = corner_const<R>(sc, lc, L, l, nv, v00);
        q.q01 = corner_const<R>(sc, lc, L, l, nv, v01);
        q.q10 = corner_const<R>(sc, lc, L, l, nv, v10);
        q.q11 = corner_const<R>(sc, lc, L, l, nv, v11);
    }
    return q;
}

// Opacity and source function of a point from phi: the expressions of sc_point.
template <typename R>
__device__ inline void corner_SC(const CornerConst<R>& q, R phi, R& S, R& chi) {
    chi = fma(q.kpl, phi, q.chic);
    S = opaque(chi) ? fma(q.el, phi, q.etac) * dev_rcp(chi) : q.sfb;
}

// Upwind intensity, source function and opacity: bilinear in the four corner cells.
__device__ inline void upwind_values(const Corners<float>& q, float w00, float w01, float w10, float w11,
                                     const Cell<float>& c00, const Cell<float>& c01, const Cell<float>& c10,
                                     const Cell<float>& c11, float& Iu, float& Su, float& Cu) {
    float S00, S01, S10, S11, X00, X01, X10, X11;
    corner_SC(q.q00, c00.P, S00, X00);
    corner_SC(q.q01, c01.P, S01, X01);
    corner_SC(q.q10, c10.P, S10, X10);
    corner_SC(q.q11, c11.P, S11, X11);
    Iu = interp4(w00, w01, w10, w11, c00.I, c01.I, c10.I, c11.I);
    Su = interp4(w00, w01, w10, w11, S00, S01, S10, S11);
    Cu = interp4(w00, w01, w10, w11, X00, X01, X10, X11);
}
__device__ inline void upwind_values(const Corners<double>&, double w00, double w01, double w10, double w11,
                                     const Cell<double>& c00, const Cell<double>& c01, const Cell<double>& c10,
                                     const Cell<double>& c11, double& Iu, double& Su, double& Cu) {
    Iu = interp4(w00, w01, w10, w11, c00.I, c01.I, c10.I, c11.I);
    Su = interp4(w00, w01, w10, w11, c00.S, c01.S, c10.S, c11.S);
    Cu = interp4(w00, w01, w10, w11, c00.C, c01.C, c10.C, c11.C);
}

// Monotone cubic Hermite interpolation between v1 and v2 (unit spacing) at fraction t,
// with the Fritsch-Butland slopes: the harmonic mean of the adjacent differences, zero
// where they differ in sign.  The result stays within [v1, v2].
template <typename R>
__device__ inline R mono_slope(R sl, R sr) {
    return (sl * sr > R(0)) ? sl * sr / (R(0.5) * sr + R(0.5) * sl) : R(0);
}
template <typename R>
__device__ inline R hermite_between(R v0, R v1, R v2, R v3, R t) {
    const R d1 = mono_slope(v1 - v0, v2 - v1), d2 = mono_slope(v2 - v1, v3 - v2);
    const R t2 = t * t, t3 = t * t * t;
    return ((R(2) * t3 - R(3) * t2 + R(1)) * v1 + (t3 - R(2) * t2 + t) * d1) + (R(-2) * t3 + R(3) * t2) * v2 +
           (t3 - t2) * d2;
}

// I, S and chi of a stored cell (FP32 cells rebuild S and chi from phi).
__device__ inline void cell_values(const Cell<float>& c, const CornerConst<float>& q, float& I, float& S, float& X) {
    I = c.I;
    corner_SC(q, c.P, S, X);
}
__device__ inline void cell_values(const Cell<double>& c, const CornerConst<double>&, double& I, double& S,
                                   double& X) {
    I = c.I;
    S = c.S;
    X = c.C;
}

template <typename R>
__device__ inline void sc_point(const PointConst<R>& c, R q, R w, bool gauss, const float4* tab, R Iu, R Su,
                                R Cu, R rds, CellVals<R>& cell, R& jacc, R& lacc) {
    const R u = q * c.ivD - c.vn;
    const R H = profile_H<R>(c.adamp, u, gauss, tab);
    const R phi = H * c.pn;
    const R chi = fma(c.kpl, phi, c.chic);
    R rchi;
    const R S = source_fn(chi, c.chic, c.etac, c.kpl, c.el, phi, rchi);
    const R dtau = R(0.5) * (Cu + chi) * rds;
    R ex, pu, po, omp;
    sc_coeffs(dtau, ex, pu, po, omp);
    const R Ith = fma(Iu, ex, pu * Su);
    cell.I = fma(po, S, Ith);
    cell.S = S;
    cell.C = chi;
    cell.P = phi;
    const R wphi = w * H * c.pw;
    const R por = po * rchi;
    jacc = fma(wphi, fma(por, c.etac, Ith), jacc);
    lacc = fma(wphi, fma(por, c.chic, omp), lacc);
}

template <typename R>
struct SweepArgs {
    const AtomInfo* atom;
    int nx, ny, nz, nf;
    unsigned nxy;
    size_t nvox;
    double dx, dy;
    const double* z;
    const R* sc;         // [SC_NQ][nline][nvox]
    const R* sv;         // [SV_NQ][nvox]
    const R* lc;         // [2][nline][nvox]: k+, e
    const R* qf;         // [nf] velocity offsets
    const R* wf;         // [nf] frequency weights (Hz)
    const R* topI;       // [nf][nxy] or null
    Cell<R>* state;      // [2 slots][24][nline * Q][nxy]
    R* acc;              // [2 qty][24/DB slots][nline][nvox]
    int m0, Q;           // this pass covers frequencies m0 .. m0+Q-1 of every line
    int add;             // 1: add this pass's sums to acc; 0: overwrite
    int nstate;          // plane-state slots (2), used by step % nstate
    int fc;              // frequency chunks per (direction, tile) of this level (work-list launches)
};

constexpr int kMaxSweepWaves = 12;
// FP32: at most 80 VGPRs, so six waves share each SIMD (the sweep hides its HBM latency
// with waves); FP64 needs its ~175 registers.
constexpr int kSweepWavesPerSimdF32 = 6;

// HERM: upwind values by monotone bicubic Hermite interpolation on the 4x4 surrounding
// points (x along the four rows, then y) instead of bilinear; one frequency chunk per
// wave, three directions per block.
// XCD-aware order: the dispatcher deals consecutive blocks round-robin to the 8 XCDs;
// when the block count divides by 8, XCD x takes the x-th contiguous eighth of the work
// list, so the tiles that read each other's upwind rows (same line and directions) share
// an L2.
__device__ inline unsigned xcd_work(unsigned lin, unsigned nb) {
    return (nb % 8u == 0u) ? (lin % 8u) * (nb / 8u) + lin / 8u : lin;
}

// The plane step of one block: tile bx (64 plane points) of line l for direction group
// grp, with FC frequency chunks per direction; the block holds DB x FCW waves, and waves
// of chunk c >= FC (when one launch serves levels with different FC) have no frequencies.
template <typename R, int DB, bool HERM>
__device__ __forceinline__ void sweep_step_body(const SweepArgs<R>& a, int s, unsigned bx, int l, int grp, int FC) {
    static_assert(DB == 3 || DB == 6 || DB == 12, "direction groups follow the fixed tree");
    static_assert(!HERM || DB == 3, "the Hermite variant runs three directions per block");
    constexpr int kW = 64;
    const int lane = int(threadIdx.x) & (kW - 1);
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kW);
    const int w = wv % DB, c = wv / DB;
    const int d = grp * DB + w;
    const int h = (grp * DB) / kNHemi;
    const AtomInfo& at = *a.atom;
    const LineInfo& ln = at.line[l];
    const int L = at.nline;
    const unsigned nxy = a.nxy;
    const unsigned graw = bx * kW + unsigned(lane);
    const bool valid = graw < nxy;
    const unsigned g = valid ? graw : nxy - 1;   // lanes past the plane compute a copy, store nothing
    const int k = (h == 0) ? s : a.nz - 1 - s;
    const size_t nv = a.nvox;
    const size_t v = size_t(k) * nxy + g;
    const size_t dstride = size_t(L) * a.Q * nxy;            // one direction's planes in this pass
    const size_t slot_stride = size_t(kNDir) * dstride;
    const int mend = min(ln.nfreq, a.m0 + a.Q);
    const int clen = (mend - a.m0 + FC - 1) / FC;
    const int mb = min(mend, a.m0 + c * clen), me = min(mend, mb + clen);   // this wave's chunk
    const double mux = c_mu[3 * d], muy = c_mu[3 * d + 1], muz = c_mu[3 * d + 2];
    const PointConst<R> pc = point_const<R>(a.sc, a.sv, a.lc, L, l, nv, v, mux, muy, muz);
    const bool gauss = ln.gauss != 0;
    const const_as<R>* qf = (const const_as<R>*)(a.qf + ln.fstart);
    const const_as<R>* wf = (const const_as<R>*)(a.wf + ln.fstart);
    const size_t col = size_t(d) * dstride + size_t(l) * a.Q * nxy;   // this (direction, line) column
    const unsigned csz = sizeof(Cell<R>);
    const unsigned rowb = nxy * csz;                                  // bytes per frequency row
    const unsigned colb = unsigned(mend - a.m0) * rowb;
    const auto rcur = cell_rsrc(a.state + size_t(s % a.nstate) * slot_stride + col, colb);
    // the small-damping Voigt table (FP32 profiles), staged in LDS
    __shared__ float4 dawg[kDawIntervals];
    if (sizeof(R) == 4) {
        for (int i = int(threadIdx.x); i < kDawIntervals; i += int(blockDim.x)) dawg[i] = c_dawg[i];
        __syncthreads();
    }
    R jacc = R(0), lacc = R(0);
    const unsigned oc = g * csz;
    if (s == 0) {
        const R Bb = a.sc[(SC_B * L + l) * nv + v];
        const R* top = a.topI ? a.topI + size_t(ln.fstart) * nxy + g : nullptr;
        for (int m = mb; m < me; ++m) {
            const R u = qf[m] * pc.ivD - pc.vn;
            const R H = profile_H<R>(pc.adamp, u, gauss, dawg);
            const R phi = H * pc.pn;
            const R chi = fma(pc.kpl, phi, pc.chic);
            R rchi_b;
            const R S = source_fn(chi, pc.chic, pc.etac, pc.kpl, pc.el, phi, rchi_b);
            const R I = (h == 0) ? Bb : (top ? top[size_t(m) * nxy] : R(0));
            if (valid) cell_put(rcur, oc, unsigned(m - a.m0) * rowb, make_cell(CellVals<R>{I, S, chi, phi}));
            const R wphi = wf[m] * H * pc.pw;
            jacc += wphi * I;
            lacc += wphi;
        }
    } else {
        const int kp = (h == 0) ? s - 1 : a.nz - s;
        const double ds = fabs(a.z[k] - a.z[kp]) / fabs(muz);
        const double sx = -ds * mux / a.dx, sy = -ds * muy / a.dy;
        const double fsx = floor(sx), fsy = floor(sy);
        const R fx = R(sx - fsx), fy = R(sy - fsy);
        const int x = int(g % unsigned(a.nx)), y = int(g / unsigned(a.nx));
        int x0 = int((long long)(x + (long long)fsx) % a.nx); if (x0 < 0) x0 += a.nx;
        int y0 = int((long long)(y + (long long)fsy) % a.ny); if (y0 < 0) y0 += a.ny;
        const int x1 = (x0 + 1 == a.nx) ? 0 : x0 + 1;
        const int y1 = (y0 + 1 == a.ny) ? 0 : y0 + 1;
        const unsigned o00 = unsigned(y0 * a.nx + x0) * csz, o01 = unsigned(y0 * a.nx + x1) * csz;
        const unsigned o10 = unsigned(y1 * a.nx + x0) * csz, o11 = unsigned(y1 * a.nx + x1) * csz;
        const size_t vp = size_t(kp) * nxy;
        const Corners<R> qc = corners_at<R>(a.sc, a.lc, L, l, nv, vp + o00 / csz, vp + o01 / csz,
                                            vp + o10 / csz, vp + o11 / csz);
        const R w00 = (R(1) - fx) * (R(1) - fy), w01 = fx * (R(1) - fy);
        const R w10 = (R(1) - fx) * fy, w11 = fx * fy;
        const R rds = R(ds);
        const auto rprv = cell_rsrc(a.state + size_t((s - 1) % a.nstate) * slot_stride + col, colb);
        if constexpr (HERM) {
            // the 4x4 stencil: columns x0-1 .. x0+2 and rows y0-1 .. y0+2, periodic
            const int xs[4] = {x0 == 0 ? a.nx - 1 : x0 - 1, x0, x1, x1 + 1 == a.nx ? 0 : x1 + 1};
            const int ys[4] = {y0 == 0 ? a.ny - 1 : y0 - 1, y0, y1, y1 + 1 == a.ny ? 0 : y1 + 1};
            unsigned ho[4][4];
            CornerConst<R> hq[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    ho[r][c] = unsigned(ys[r] * a.nx + xs[c]) * csz;
                    if constexpr (kPhiCell<R>) hq[r][c] = corner_const<R>(a.sc, a.lc, L, l, nv, vp + ho[r][c] / csz);
                }
            for (int m = mb; m < me; ++m) {
                const unsigned so = unsigned(m - a.m0) * rowb;
                R gI[4], gS[4], gX[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    R vI[4], vS[4], vX[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) cell_values(cell_get<R>(rprv, ho[r][c], so), hq[r][c], vI[c], vS[c], vX[c]);
                    gI[r] = hermite_between(vI[0], vI[1], vI[2], vI[3], fx);
                    gS[r] = hermite_between(vS[0], vS[1], vS[2], vS[3], fx);
                    gX[r] = hermite_between(vX[0], vX[1], vX[2], vX[3], fx);
                }
                const R Iu = hermite_between(gI[0], gI[1], gI[2], gI[3], fy);
                const R Su = hermite_between(gS[0], gS[1], gS[2], gS[3], fy);
                const R Cu = hermite_between(gX[0], gX[1], gX[2], gX[3], fy);
                CellVals<R> cell;
                sc_point(pc, R(qf[m]), R(wf[m]), gauss, dawg, Iu, Su, Cu, rds, cell, jacc, lacc);
                if (valid) cell_put(rcur, oc, so, make_cell(cell));
            }
        } else {
            for (int m = mb; m < me; ++m) {
                const unsigned so = unsigned(m - a.m0) * rowb;
                const Cell<R> c00 = cell_get<R>(rprv, o00, so), c01 = cell_get<R>(rprv, o01, so);
                const Cell<R> c10 = cell_get<R>(rprv, o10, so), c11 = cell_get<R>(rprv, o11, so);
                R Iu, Su, Cu;
                upwind_values(qc, w00, w01, w10, w11, c00, c01, c10, c11, Iu, Su, Cu);
                CellVals<R> cell;
                sc_point(pc, R(qf[m]), R(wf[m]), gauss, dawg, Iu, Su, Cu, rds, cell, jacc, lacc);
                if (valid) cell_put(rcur, oc, so, make_cell(cell));
            }
        }
    }
    __shared__ R sj[kMaxSweepWaves * kW];
    __shared__ R sl[kMaxSweepWaves * kW];
    sj[threadIdx.x] = jacc;
    sl[threadIdx.x] = lacc;
    __syncthreads();
    if (int(threadIdx.x) < kW && valid) {
        // frequency chunks in order, per direction
        R dj[DB], dl[DB];
#pragma unroll
        for (int q = 0; q < DB; ++q) {
            dj[q] = sj[q * kW + lane];
            dl[q] = sl[q * kW + lane];
            for (int cc = 1; cc < FC; ++cc) {
                dj[q] += sj[(cc * DB + q) * kW + lane];
                dl[q] += sl[(cc * DB + q) * kW + lane];
            }
        }
        // groups of three directions, then pairs of groups (the fixed tree)
        R gj[DB / 3], gl[DB / 3];
#pragma unroll
        for (int q = 0; q < DB / 3; ++q) {
            gj[q] = (dj[3 * q] + dj[3 * q + 1]) + dj[3 * q + 2];
            gl[q] = (dl[3 * q] + dl[3 * q + 1]) + dl[3 * q + 2];
        }
        R jt, lt;
        if constexpr (DB == 3) {
            jt = gj[0]; lt = gl[0];
        } else if constexpr (DB == 6) {
            jt = gj[0] + gj[1]; lt = gl[0] + gl[1];
        } else {
            jt = (gj[0] + gj[1]) + (gj[2] + gj[3]);
            lt = (gl[0] + gl[1]) + (gl[2] + gl[3]);
        }
        constexpr int nslot = kNDir / DB;
        R* aj = a.acc + ((size_t(0) * nslot + grp) * L + l) * nv + v;
        R* al = a.acc + ((size_t(1) * nslot + grp) * L + l) * nv + v;
        if (a.add) { jt += *aj; lt += *al; }
        *aj = jt;
        *al = lt;
    }
}


template <typename R, int DB, bool HERM = false>
__global__ __launch_bounds__((sizeof(R) == 4 && !HERM ? kMaxSweepWaves : DB) * 64)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 && !HERM ? kSweepWavesPerSimdF32 : 1))) void sweep_step_kernel(
    SweepArgs<R> a, int s) {
    const unsigned T = gridDim.x;
    const unsigned work = xcd_work(blockIdx.x + T * (blockIdx.y + gridDim.y * blockIdx.z), T * gridDim.y * gridDim.z);
    const unsigned bx = work % T;
    const int l = int((work / T) % gridDim.y);
    const int grp = int(work / (T * gridDim.y));
    sweep_step_body<R, DB, HERM>(a, s, bx, l, grp, int(blockDim.x) / (64 * DB));
}

// One plane step for several grids in one launch (a work list): grid j (its level's sweep
// arguments jobs[j]) owns blocks first[j] .. first[j+1]-1, (tile, line, direction group)
// in the order of the one-grid launch.  Grids are sorted by plane count, most first, and
// the launch covers the first nact of them (those with a plane at step s).  Every block
// computes exactly what the one-grid launch computes for that tile, with that grid's own
// frequency chunks, so the results do not depend on the other grids of the list.
template <typename R, int DB>
__global__ __launch_bounds__((sizeof(R) == 4 ? kMaxSweepWaves : DB) * 64)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? kSweepWavesPerSimdF32 : 1))) void sweep_list_kernel(
    const SweepArgs<R>* __restrict__ jobs, const unsigned* __restrict__ first, int nact, int s) {
    // The list is read through the constant address space with a wave-uniform index: the
    // compiler then copies the job's arguments with scalar loads into scalar registers, as
    // it does a kernel's own arguments (read as ordinary global data they would occupy
    // vector registers and spill).  The host compilation pass, which never runs this code,
    // has no such address space and reads plain memory.
#if defined(__HIP_DEVICE_COMPILE__)
    const auto* jl = (const __attribute__((address_space(4))) SweepArgs<R>*)(jobs);
    const auto* fl = (const __attribute__((address_space(4))) unsigned*)(first);
#else
    const SweepArgs<R>* jl = jobs;
    const unsigned* fl = first;
#endif
    const unsigned work = xcd_work(blockIdx.x, gridDim.x);
    int j = 0;
    while (j + 1 < nact && fl[j + 1] <= work) ++j;
    j = __builtin_amdgcn_readfirstlane(j);
    const SweepArgs<R> a = jl[j];
    const unsigned local = work - fl[j];
    const unsigned T = (a.nxy + 63u) / 64u;
    const unsigned L = unsigned(a.atom->nline);
    sweep_step_body<R, DB, false>(a, s, local % T, int((local / T) % L), int(local / (T * L)), a.fc);
}

// Emergent intensity: one plane step of an upward sweep for a single direction (thread
// per (frequency, plane point)); the last step writes I at the top plane.  The level
// constants are read in their storage precision R; the solve itself is always FP64.
template <typename R>
struct EmergentArgs {
    const AtomInfo* atom;
    int nx, ny, nz, nf;
    size_t nxy, nvox;
    double dx, dy, mux, muy, muz;
    const double* z;
    const R* sc;
    const R* sv;
    const R* lc;
    const R* qf;
    const int* line_of;  // [nf]
    double* state;       // [2][3][fn][nxy]: this chunk's plane state
    float* out;          // [nf][nxy]
    int herm;            // 1: monotone bicubic Hermite upwind interpolation
    int f0, fn;          // the launch covers frequencies f0 .. f0+fn-1 (each independent of the others)
};

template <typename R>
__global__ void emergent_step_kernel(EmergentArgs<R> a, int k) {
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= size_t(a.fn) * a.nxy) return;
    const int fl = int(idx / a.nxy);   // frequency within the chunk (state index)
    const int f = a.f0 + fl;
    const size_t g = idx % a.nxy;
    const AtomInfo& at = *a.atom;
    const int l = a.line_of[f];
    const int L = at.nline;
    const LineInfo& ln = at.line[l];
    const size_t nv = a.nvox, v = size_t(k) * a.nxy + g;
    const double chic = a.sc[(SC_CHIC * L + l) * nv + v];
    const double etac = a.sc[(SC_ETAC * L + l) * nv + v];
    const double adamp = a.sc[(SC_ADAMP * L + l) * nv + v];
    const double pn = a.sc[(SC_PN * L + l) * nv + v];
    const double kpl = a.lc[size_t(l) * nv + v];
    const double el = a.lc[size_t(L + l) * nv + v];
    const double ivD = a.sv[SV_INVVD * nv + v];
    const double vn = double(a.sv[SV_VX * nv + v]) * a.mux + double(a.sv[SV_VY * nv + v]) * a.muy +
                      double(a.sv[SV_VZ * nv + v]) * a.muz;
    const double u = double(a.qf[f]) * ivD - vn;
    const double H = profile_H<double>(adamp, u, ln.gauss != 0, nullptr);
    const double phi = H * pn;
    const double chi = chic + kpl * phi;
    double rchi_e;
    const double S = source_fn(chi, chic, etac, kpl, el, phi, rchi_e);
    const size_t ps = size_t(a.fn) * a.nxy;
    double* cur = a.state + size_t(k & 1) * 3 * ps;
    double I;
    if (k == 0) {
        I = a.sc[(SC_B * L + l) * nv + v];
    } else {
        const double* prv = a.state + size_t((k - 1) & 1) * 3 * ps;
        const double ds = (a.z[k] - a.z[k - 1]) / a.muz;
        const double sx = -ds * a.mux / a.dx, sy = -ds * a.muy / a.dy;
        const double fsx = floor(sx), fsy = floor(sy);
        const double fx = sx - fsx, fy = sy - fsy;
        const int x = int(g % a.nx), y = int(g / a.nx);
        int x0 = int((long long)(x + (long long)fsx) % a.nx); if (x0 < 0) x0 += a.nx;
        int y0 = int((long long)(y + (long long)fsy) % a.ny); if (y0 < 0) y0 += a.ny;
        const int x1 = (x0 + 1 == a.nx) ? 0 : x0 + 1;
        const int y1 = (y0 + 1 == a.ny) ? 0 : y0 + 1;
        const size_t fo = size_t(fl) * a.nxy;
        const size_t g00 = fo + size_t(y0) * a.nx + x0, g01 = fo + size_t(y0) * a.nx + x1;
        const size_t g10 = fo + size_t(y1) * a.nx + x0, g11 = fo + size_t(y1) * a.nx + x1;
        const double w00 = (1.0 - fx) * (1.0 - fy), w01 = fx * (1.0 - fy);
        const double w10 = (1.0 - fx) * fy, w11 = fx * fy;
        double Iu, Su, Cu;
        if (a.herm) {
            const int xs[4] = {x0 == 0 ? a.nx - 1 : x0 - 1, x0, x1, x1 + 1 == a.nx ? 0 : x1 + 1};
            const int ys[4] = {y0 == 0 ? a.ny - 1 : y0 - 1, y0, y1, y1 + 1 == a.ny ? 0 : y1 + 1};
            double q[3][4];
            for (int r = 0; r < 4; ++r) {
                const size_t rowo = fo + size_t(ys[r]) * a.nx;
                for (int f3 = 0; f3 < 3; ++f3) {
                    const double* p3 = prv + size_t(f3) * ps + rowo;
                    q[f3][r] = hermite_between(p3[xs[0]], p3[xs[1]], p3[xs[2]], p3[xs[3]], fx);
                }
            }
            Iu = hermite_between(q[0][0], q[0][1], q[0][2], q[0][3], fy);
            Su = hermite_between(q[1][0], q[1][1], q[1][2], q[1][3], fy);
            Cu = hermite_between(q[2][0], q[2][1], q[2][2], q[2][3], fy);
        } else {
            Iu = w00 * prv[g00] + w01 * prv[g01] + w10 * prv[g10] + w11 * prv[g11];
            Su = w00 * prv[ps + g00] + w01 * prv[ps + g01] + w10 * prv[ps + g10] + w11 * prv[ps + g11];
            Cu = w00 * prv[2 * ps + g00] + w01 * prv[2 * ps + g01] + w10 * prv[2 * ps + g10] + w11 * prv[2 * ps + g11];
        }
        const double dtau = 0.5 * (Cu + chi) * ds;
        double ex, pu, po, omp;
        sc_coeffs(dtau, ex, pu, po, omp);
        I = Iu * ex + pu * Su + po * S;
    }
    cur[size_t(fl) * a.nxy + g] = I;
    cur[ps + size_t(fl) * a.nxy + g] = S;
    cur[2 * ps + size_t(fl) * a.nxy + g] = chi;
    if (k == a.nz - 1) a.out[size_t(f) * a.nxy + g] = float(I);
}

// ------------------------------------------------------------------ active continua
// Continua as transitions of the formal solution (on request).  Per voxel: the LTE ratio
// n_l*/n_c* of every continuum, h/kT, and the spontaneous part of the downward rate,
// F_t = sum_k (4 pi w_tk / h nu_k) alpha_tk g_tk 2 h nu_k^3/c^2 with g = (n_l*/n_c*) e^{-h nu/kT}.
constexpr int kMaxCont = 8;
constexpr int kMaxContUp = 4;   // distinct upper levels of the active continua

template <typename R>
__global__ void cont_setup_kernel(const AtomInfo* atom, const double* prim, const double* nstar, const double* cnu,
                                  const double* ce, const double* cfw, const double* calpha, int nfc, R* cr, R* hkT,
                                  double* cF, size_t nvox) {
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    const AtomInfo& at = *atom;
    const double T = prim[P_T * nvox + v];
    const double hk = kH / (kKB * T);
    hkT[v] = R(hk);
    for (int t = 0; t < at.ncont; ++t) {
        const double ratio = nstar[size_t(at.cont_lower[t]) * nvox + v] / nstar[size_t(at.cont_upper[t]) * nvox + v];
        cr[size_t(t) * nvox + v] = R(ratio);
        double F = 0.0;
        for (int k = 0; k < nfc; ++k)
            F += cfw[size_t(t) * nfc + k] * calpha[size_t(t) * nfc + k] * ratio * exp(-hk * cnu[k]) * ce[k];
        cF[size_t(t) * nvox + v] = F;
    }
}

// Plane state of the continuum sweep: intensity, source function and opacity, moved by
// raw buffer instructions like the line sweep's cells (lane offset fixed, frequency row in
// the scalar offset).
template <typename R>
struct CCell {
    R I, S, C;
};
typedef float f32x3c __attribute__((ext_vector_type(3)));
__device__ inline CCell<float> ccell_get(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float) {
    const f32x3c x = __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, 0);
    return CCell<float>{x.x, x.y, x.z};
}
__device__ inline CCell<double> ccell_get(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double) {
    const Cell<double> c = cell_load_d(r, voff, soff);
    return CCell<double>{c.I, c.S, c.C};
}
__device__ inline void ccell_put(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, const CCell<float>& c) {
    __builtin_amdgcn_raw_buffer_store_b96(f32x3c{c.I, c.S, c.C}, r, voff, soff, 0);
}
__device__ inline void ccell_put(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, const CCell<double>& c) {
    cell_put(r, voff, soff, Cell<double>{c.I, c.S, c.C});
}

constexpr int kContRow = 2 + 2 * kMaxCont + 2;   // one frequency's table row (20 values)

template <typename R>
struct ContArgs {
    const AtomInfo* atom;
    int nx, ny, nz, nfc;
    unsigned nxy;
    size_t nvox;
    double dx, dy;
    const double* z;
    const double* n;      // [N][nvox] populations
    const R* cr;          // [ncont][nvox] n_l*/n_c*
    const R* hkT;         // [nvox] h/kT
    const R* ctab;        // [nfc][kContRow]: nu, 2 h nu^3/c^2, alpha_t (8), 4 pi w_t/(h nu) (8), pad
    CCell<R>* state;      // [2][24][nfc][nxy]
    R* acc;               // [(2 + nup) ncont][8 slots][nvox]: U_t, G_t, then L_t,u (t major)
};

// One plane step of the formal solution at the continuum frequencies, for three
// directions per block over 64 plane points, the frequencies split into FC contiguous
// chunks (block = 3 x FC waves, FC = blockDim / 192).  Opacity and emissivity at a point
// sum over the continua open at the frequency, the emissivity as sum_u n_u E_u over the
// NUP distinct upper levels (E_u: alpha g 2 h nu^3/c^2 summed over the continua ending on
// u).  The sums per continuum t (U: alpha Jeff, G: alpha g Jeff, and per upper level u
// the preconditioned local part L_t,u: (chi_t/chi) Psi_o E_u, each times 4 pi w / h nu and
// the direction weight 1/24) are added over the chunks in order, then over the block's
// three directions as (d0 + d1) + d2, and stored per direction group; the rate kernel
// finishes the fixed tree.
// FP64 keeps to two chunks (six waves per block), which leaves it 256 registers per lane.
constexpr int kContMaxChunks = 4;
template <typename R>
constexpr int cont_max_chunks() { return sizeof(R) == 8 ? 2 : kContMaxChunks; }

template <typename R, int NUP>
__global__ __launch_bounds__(3 * cont_max_chunks<R>() * 64) void sweep_cont_kernel(ContArgs<R> a, int s) {
    constexpr int kW = 64;
    const int lane = int(threadIdx.x) & (kW - 1);
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / kW);
    const int FC = int(blockDim.x) / (3 * kW);
    const int w = wv % 3, cch = wv / 3;
    // XCD-aware order, as in the line sweep: with the block count a multiple of 8, XCD x
    // takes the x-th contiguous eighth of the (tile, direction group) list, so the tiles
    // whose upwind rows overlap share an L2.
    const unsigned T = gridDim.x;
    const unsigned nb = T * gridDim.z;
    const unsigned lin = blockIdx.x + T * blockIdx.z;
    const unsigned work = (nb % 8u == 0u) ? (lin % 8u) * (nb / 8u) + lin / 8u : lin;
    const unsigned bx = work % T;
    const int grp = int(work / T);
    const int d = grp * 3 + w;
    const int h = (grp * 3) / kNHemi;
    const AtomInfo& at = *a.atom;
    const int nct = at.ncont;
    const unsigned nxy = a.nxy;
    const unsigned graw = bx * kW + unsigned(lane);
    const bool valid = graw < nxy;
    const unsigned g = valid ? graw : nxy - 1;
    const int k = (h == 0) ? s : a.nz - 1 - s;
    const size_t nv = a.nvox;
    const size_t v = size_t(k) * nxy + g;
    const int nfc = a.nfc;
    const size_t dstride = size_t(nfc) * nxy;
    const size_t slot_stride = size_t(kNDir) * dstride;
    constexpr unsigned csz = sizeof(CCell<R>);
    const unsigned rowb = nxy * csz;                  // bytes per frequency row
    const auto rcur = cell_rsrc(a.state + size_t(s & 1) * slot_stride + size_t(d) * dstride, unsigned(nfc) * rowb);
    R ncu[NUP];
#pragma unroll
    for (int u = 0; u < NUP; ++u) ncu[u] = R(fmax(a.n[size_t(at.cont_ulev[u]) * nv + v], 0.0));
    R nl[kMaxCont], ratio[kMaxCont], nc[kMaxCont];
#pragma unroll
    for (int t = 0; t < kMaxCont; ++t) {
        nl[t] = t < nct ? R(fmax(a.n[size_t(at.cont_lower[t]) * nv + v], 0.0)) : R(0);
        ratio[t] = t < nct ? a.cr[size_t(t) * nv + v] : R(0);
        nc[t] = ncu[0];   // the population of t's upper level
#pragma unroll
        for (int u = 1; u < NUP; ++u)
            if (at.cont_uidx[t] == u) nc[t] = ncu[u];
    }
    const R hk = a.hkT[v];
    const R wd = R(1.0 / kNDir);
    R aU[kMaxCont], aG[kMaxCont], aL[kMaxCont][NUP];
#pragma unroll
    for (int t = 0; t < kMaxCont; ++t) {
        aU[t] = aG[t] = R(0);
#pragma unroll
        for (int u = 0; u < NUP; ++u) aL[t][u] = R(0);
    }
    // upwind geometry (planes after the boundary)
    unsigned o00 = 0, o01 = 0, o10 = 0, o11 = 0;
    R w00 = R(0), w01 = R(0), w10 = R(0), w11 = R(0), rds = R(0);
    auto rprv = rcur;
    if (s > 0) {
        const double mux = c_mu[3 * d], muy = c_mu[3 * d + 1], muz = c_mu[3 * d + 2];
        const int kp = (h == 0) ? s - 1 : a.nz - s;
        const double ds = fabs(a.z[k] - a.z[kp]) / fabs(muz);
        const double sx = -ds * mux / a.dx, sy = -ds * muy / a.dy;
        const double fsx = floor(sx), fsy = floor(sy);
        const R fx = R(sx - fsx), fy = R(sy - fsy);
        const int x = int(g % unsigned(a.nx)), y = int(g / unsigned(a.nx));
        int x0 = int((long long)(x + (long long)fsx) % a.nx); if (x0 < 0) x0 += a.nx;
        int y0 = int((long long)(y + (long long)fsy) % a.ny); if (y0 < 0) y0 += a.ny;
        const int x1 = (x0 + 1 == a.nx) ? 0 : x0 + 1;
        const int y1 = (y0 + 1 == a.ny) ? 0 : y0 + 1;
        o00 = unsigned(y0 * a.nx + x0) * csz; o01 = unsigned(y0 * a.nx + x1) * csz;
        o10 = unsigned(y1 * a.nx + x0) * csz; o11 = unsigned(y1 * a.nx + x1) * csz;
        w00 = (R(1) - fx) * (R(1) - fy); w01 = fx * (R(1) - fy);
        w10 = (R(1) - fx) * fy; w11 = fx * fy;
        rds = R(ds);
        rprv = cell_rsrc(a.state + size_t((s - 1) & 1) * slot_stride + size_t(d) * dstride, unsigned(nfc) * rowb);
    }
    const int clen = (nfc + FC - 1) / FC;
    const int mb = min(nfc, cch * clen), me = min(nfc, mb + clen);
    for (int m = mb; m < me; ++m) {
        // the frequency's table row, wave-uniform: scalar loads
        const const_as<R>* row = (const const_as<R>*)(a.ctab + size_t(m) * kContRow);
        const R x = dev_exp_neg(hk * row[0]);
        const R e = row[1];
        R chis[kMaxCont], gg[kMaxCont];
        R chi = R(0), E[NUP];
#pragma unroll
        for (int u = 0; u < NUP; ++u) E[u] = R(0);
#pragma unroll
        for (int t = 0; t < kMaxCont; ++t) {
            const R al = row[2 + t];   // 0 for absent continua and below the edge
            gg[t] = ratio[t] * x;
            chis[t] = al * fmax(nl[t] - nc[t] * gg[t], R(0));
            chi += chis[t];
#pragma unroll
            for (int u = 0; u < NUP; ++u)
                if (NUP == 1 || at.cont_uidx[t] == u) E[u] = fma(al, gg[t], E[u]);
        }
        R eta = R(0);
#pragma unroll
        for (int u = 0; u < NUP; ++u) {
            E[u] *= e;
            eta = u == 0 ? ncu[0] * E[0] : fma(ncu[u], E[u], eta);
        }
        const R rchi = chi > R(0) ? dev_rcp(chi) : R(0);
        const R S = eta * rchi;
        R Jd, Io, po = R(0);
        if (s == 0) {
            Io = (h == 0) ? e * x / (R(1) - x) : R(0);
            Jd = Io;
        } else {
            const unsigned so = unsigned(m) * rowb;
            const CCell<R> c00 = ccell_get(rprv, o00, so, R(0)), c01 = ccell_get(rprv, o01, so, R(0));
            const CCell<R> c10 = ccell_get(rprv, o10, so, R(0)), c11 = ccell_get(rprv, o11, so, R(0));
            const R Iu = interp4(w00, w01, w10, w11, c00.I, c01.I, c10.I, c11.I);
            const R Su = interp4(w00, w01, w10, w11, c00.S, c01.S, c10.S, c11.S);
            const R Cu = interp4(w00, w01, w10, w11, c00.C, c01.C, c10.C, c11.C);
            const R dtau = R(0.5) * (Cu + chi) * rds;
            R ex, pu, omp;
            sc_coeffs(dtau, ex, pu, po, omp);
            Jd = fma(Iu, ex, pu * Su);
            Io = fma(po, S, Jd);
        }
        if (valid) ccell_put(rcur, g * csz, unsigned(m) * rowb, CCell<R>{Io, S, chi});
#pragma unroll
        for (int t = 0; t < kMaxCont; ++t) {
            if (t < nct) {
                const R fw = row[2 + kMaxCont + t];
                const R wa = wd * fw * row[2 + t];
                aU[t] = fma(wa, Jd, aU[t]);
                aG[t] = fma(wa * gg[t], Jd, aG[t]);
#pragma unroll
                for (int u = 0; u < NUP; ++u) aL[t][u] = fma(wd * fw, chis[t] * rchi * po * E[u], aL[t][u]);
            }
        }
    }
    // per quantity and continuum: chunks in order, then (d0 + d1) + d2
    __shared__ R red[3 * kContMaxChunks * kW];
    auto store = [&](R val, int q) {
        red[threadIdx.x] = val;
        __syncthreads();
        if (wv == 0 && valid) {
            R dsum[3];
            for (int dd = 0; dd < 3; ++dd) {
                R c = red[dd * kW + lane];
                for (int ch = 1; ch < FC; ++ch) c += red[(ch * 3 + dd) * kW + lane];
                dsum[dd] = c;
            }
            a.acc[(size_t(q) * kMaxSlots + grp) * nv + v] = (dsum[0] + dsum[1]) + dsum[2];
        }
        __syncthreads();
    };
#pragma unroll
    for (int t = 0; t < kMaxCont; ++t)
        if (t < nct) store(aU[t], t);
#pragma unroll
    for (int t = 0; t < kMaxCont; ++t)
        if (t < nct) store(aG[t], nct + t);
#pragma unroll
    for (int t = 0; t < kMaxCont; ++t)
        if (t < nct) {
#pragma unroll
            for (int u = 0; u < NUP; ++u) store(aL[t][u], 2 * nct + t * NUP + u);
        }
}

// Emergent intensity at the continuum frequencies: one upward plane step for every
// (continuum frequency, plane point) of one direction, FP64 throughout from the
// populations, the LTE populations and T (opacity sum_t alpha_t (n_l - n_c g_t)^+,
// emissivity sum_t n_c alpha_t g_t 2 h nu^3/c^2, g_t = (n_l*/n_c*) e^{-h nu/kT}), B_nu(T)
// at the lower boundary, bilinear upwind interpolation.
struct EmergentContArgs {
    const AtomInfo* atom;
    int nx, ny, nz, nfc;
    size_t nxy, nvox;
    double dx, dy, mux, muy, muz;
    const double* z;
    const double* prim;      // FP64 primitive fields (T)
    const double* nstar;     // [N][nvox]
    const double* n;         // [N][nvox]
    const double* cnu;       // [nfc]
    const double* ce;        // [nfc] 2 h nu^3 / c^2
    const double* calpha;    // [ncont][nfc], 0 below the edge
    double* state;           // [2][3][nfc][nxy]
    float* out;              // [nfc][nxy]
};

__global__ void emergent_cont_step_kernel(EmergentContArgs a, int k) {
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= size_t(a.nfc) * a.nxy) return;
    const int f = int(idx / a.nxy);
    const size_t g = idx % a.nxy;
    const AtomInfo& at = *a.atom;
    const size_t nv = a.nvox, v = size_t(k) * a.nxy + g;
    const double x = exp(-kH / (kKB * a.prim[P_T * nv + v]) * a.cnu[f]);
    const double e = a.ce[f];
    double chi = 0.0, eta = 0.0;
    for (int t = 0; t < at.ncont; ++t) {
        const double al = a.calpha[size_t(t) * a.nfc + f];
        const int lo = at.cont_lower[t], up = at.cont_upper[t];
        const double gg = a.nstar[size_t(lo) * nv + v] / a.nstar[size_t(up) * nv + v] * x;
        const double nl = fmax(a.n[size_t(lo) * nv + v], 0.0), nc = fmax(a.n[size_t(up) * nv + v], 0.0);
        chi += al * fmax(nl - nc * gg, 0.0);
        eta += nc * al * gg * e;
    }
    const double S = chi > 0.0 ? eta / chi : 0.0;
    const size_t ps = size_t(a.nfc) * a.nxy;
    double* cur = a.state + size_t(k & 1) * 3 * ps;
    double I;
    if (k == 0) {
        I = e * x / (1.0 - x);
    } else {
        const double* prv = a.state + size_t((k - 1) & 1) * 3 * ps;
        const double ds = (a.z[k] - a.z[k - 1]) / a.muz;
        const double sx = -ds * a.mux / a.dx, sy = -ds * a.muy / a.dy;
        const double fsx = floor(sx), fsy = floor(sy);
        const double fx = sx - fsx, fy = sy - fsy;
        const int xx = int(g % a.nx), yy = int(g / a.nx);
        int x0 = int((long long)(xx + (long long)fsx) % a.nx); if (x0 < 0) x0 += a.nx;
        int y0 = int((long long)(yy + (long long)fsy) % a.ny); if (y0 < 0) y0 += a.ny;
        const int x1 = (x0 + 1 == a.nx) ? 0 : x0 + 1;
        const int y1 = (y0 + 1 == a.ny) ? 0 : y0 + 1;
        const size_t fo = size_t(f) * a.nxy;
        const size_t g00 = fo + size_t(y0) * a.nx + x0, g01 = fo + size_t(y0) * a.nx + x1;
        const size_t g10 = fo + size_t(y1) * a.nx + x0, g11 = fo + size_t(y1) * a.nx + x1;
        const double w00 = (1.0 - fx) * (1.0 - fy), w01 = fx * (1.0 - fy);
        const double w10 = (1.0 - fx) * fy, w11 = fx * fy;
        const double Iu = w00 * prv[g00] + w01 * prv[g01] + w10 * prv[g10] + w11 * prv[g11];
        const double Su = w00 * prv[ps + g00] + w01 * prv[ps + g01] + w10 * prv[ps + g10] + w11 * prv[ps + g11];
        const double Cu = w00 * prv[2 * ps + g00] + w01 * prv[2 * ps + g01] + w10 * prv[2 * ps + g10] +
                          w11 * prv[2 * ps + g11];
        const double dtau = 0.5 * (Cu + chi) * ds;
        double ex, pu, po, omp;
        sc_coeffs(dtau, ex, pu, po, omp);
        I = Iu * ex + pu * Su + po * S;
    }
    cur[size_t(f) * a.nxy + g] = I;
    cur[ps + size_t(f) * a.nxy + g] = S;
    cur[2 * ps + size_t(f) * a.nxy + g] = chi;
    if (k == a.nz - 1) a.out[size_t(f) * a.nxy + g] = float(I);
}

// ------------------------------------------------------------------ rate equations
// Rate matrix from the fixed rates and the preconditioned radiative rates of
// Rybicki & Hummer (1991): upward B_ij Jeff, downward A_ji (1 - L*) + B_ji Jeff.
// System matrix A[i][i] = sum_{j != i} P_ij, A[i][j] = -P_ji, row 0 = particle
// conservation.  mode: 0 = solve A n' = f (MALI update), 1 = zero-radiation solve
// (Jeff = 0, 1 - L* = 1), 2 = out = base + sign * (A n) (W(n) at the current
// accumulators: residual and coarse-grid right-hand side).
template <typename R>
struct RateArgs {
    const AtomInfo* atom;
    size_t nvox;
    const double* pfix;   // [N*N][nvox]
    const R* acc;         // [2][nslot][nline][nvox]
    int nslot;            // 2, 4 or 8 direction-group slots per quantity
    double* n;            // [N][nvox]  (mode 0/1: updated in place)
    const double* f;      // [N][nvox]
    const double* base;   // mode 2
    double* out;          // mode 2
    double sign;
    int mode;
    double* partial;      // [gridDim.x] max relative change (modes 0/1)
    const R* cacc;        // active continua: [(2 + nup) ncont][8 slots][nvox] (U, G, L), else null
    const double* cF;     // active continua: [ncont][nvox] spontaneous recombination
};

template <int N>
__device__ inline void build_matrix(const AtomInfo& at, const double* pfix, size_t nv, size_t v,
                                    const double* Jeff, const double* omL, const double* cup,
                                    const double* cdn, double (&A)[N][N]) {
    double P[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) P[i][j] = pfix[size_t(i * N + j) * nv + v];
    // active continua: upward U_t, downward G_t + F_t - L_t
    for (int t = 0; t < (at.cont_active ? at.ncont : 0); ++t) {
        const int lo = at.cont_lower[t], up = at.cont_upper[t];
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j) {
                if (i == lo && j == up) P[i][j] += cup[t];
                if (i == up && j == lo) P[i][j] += cdn[t];
            }
    }
    for (int l = 0; l < at.nline; ++l) {
        const LineInfo& ln = at.line[l];
        const double up = ln.Bij * Jeff[l];
        const double dn = ln.A * omL[l] + ln.Bji * Jeff[l];
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int j = 0; j < N; ++j) {
                if (i == ln.lower && j == ln.upper) P[i][j] += up;
                if (i == ln.upper && j == ln.lower) P[i][j] += dn;
            }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double out = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j)
            if (j != i) out += P[i][j];
#pragma unroll
        for (int j = 0; j < N; ++j) A[i][j] = (i == j) ? out : -P[j][i];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) A[0][j] = 1.0;
}

// Gaussian elimination with partial pivoting, fully unrolled (row swaps by selects).
template <int N>
__device__ inline void lu_solve(double (&A)[N][N], double (&b)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int p = k;
        double best = fabs(A[k][k]);
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const double vr = fabs(A[r][k]);
            if (vr > best) { best = vr; p = r; }
        }
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            if (r == p) {
#pragma unroll
                for (int j = 0; j < N; ++j) { const double tmp = A[k][j]; A[k][j] = A[r][j]; A[r][j] = tmp; }
                const double tb = b[k]; b[k] = b[r]; b[r] = tb;
            }
        }
        const double inv = 1.0 / A[k][k];
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const double fct = A[r][k] * inv;
#pragma unroll
            for (int j = k; j < N; ++j) A[r][j] -= fct * A[k][j];
            b[r] -= fct * b[k];
        }
    }
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
        double sacc = b[k];
#pragma unroll
        for (int j = k + 1; j < N; ++j) sacc -= A[k][j] * b[j];
        b[k] = sacc / A[k][k];
    }
}

// One continuum sum (index q of the [(2 + nup) ncont] quantities) over its 8 slots.
template <typename R>
__device__ inline double cont_sum(const R* cacc, int q, size_t nv, size_t v) {
    return double(tree_slots(cacc + (size_t(q) * kMaxSlots) * nv + v, nv, kMaxSlots));
}

template <typename R, int N>
__global__ __launch_bounds__(256) void rate_kernel(RateArgs<R> a) {
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double cmax = 0.0;
    if (v < a.nvox) {
        const AtomInfo& at = *a.atom;
        const int L = at.nline;
        const size_t nv = a.nvox;
        double Jeff[kMaxLines], omL[kMaxLines];
        for (int l = 0; l < L; ++l) {
            if (a.mode == 1) {
                Jeff[l] = 0.0;
                omL[l] = 1.0;
            } else {
                const size_t ss = size_t(L) * nv;
                Jeff[l] = double(tree_slots(a.acc + (size_t(0) * a.nslot * L + l) * nv + v, ss, a.nslot));
                omL[l] = double(tree_slots(a.acc + (size_t(1) * a.nslot * L + l) * nv + v, ss, a.nslot));
            }
        }
        double cup[kMaxCont], cdn[kMaxCont];
        for (int t = 0; t < (at.cont_active ? at.ncont : 0); ++t) {
            const double F = a.cF[size_t(t) * nv + v];
            if (a.mode == 1) {
                cup[t] = 0.0;
                cdn[t] = F;
            } else {
                const int nc3 = at.ncont;
                cup[t] = cont_sum(a.cacc, t, nv, v);
                cdn[t] = cont_sum(a.cacc, nc3 + t, nv, v) + F -
                         cont_sum(a.cacc, 2 * nc3 + t * at.cont_nup + at.cont_uidx[t], nv, v);
            }
        }
        double A[N][N];
        build_matrix<N>(at, a.pfix, nv, v, Jeff, omL, cup, cdn, A);
        // active continua ending on several upper levels: the net upward rate of continuum
        // t (l -> c) also holds n_u L_t,u for the other upper levels u, a flux out of l
        // (A[l][u] += L) into c (A[c][u] -= L); row 0 stays the conservation row
        if (a.mode != 1 && at.cont_active && at.cont_nup > 1) {
            const int nc3 = at.ncont, nup = at.cont_nup;
            for (int t = 0; t < nc3; ++t)
                for (int u = 0; u < nup; ++u) {
                    if (u == at.cont_uidx[t]) continue;
                    const double x = cont_sum(a.cacc, 2 * nc3 + t * nup + u, nv, v);
                    const int lo = at.cont_lower[t], up = at.cont_upper[t], ul = at.cont_ulev[u];
#pragma unroll
                    for (int i = 1; i < N; ++i)
#pragma unroll
                        for (int j = 0; j < N; ++j)
                            if (j == ul) {
                                if (i == lo) A[i][j] += x;
                                if (i == up) A[i][j] -= x;
                            }
                }
        }
        double nold[N];
#pragma unroll
        for (int i = 0; i < N; ++i) nold[i] = a.n[size_t(i) * nv + v];
        if (a.mode == 2) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double w = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) w += A[i][j] * nold[j];
                a.out[size_t(i) * nv + v] = a.base[size_t(i) * nv + v] + a.sign * w;
            }
        } else {
            double b[N];
#pragma unroll
            for (int i = 0; i < N; ++i) b[i] = a.f[size_t(i) * nv + v];
            const double f0 = b[0];
            lu_solve<N>(A, b);
            double tot = 0.0;
#pragma unroll
            for (int i = 0; i < N; ++i) tot += b[i];
            const double sc = f0 / tot;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const double nn = b[i] * sc;
                cmax = fmax(cmax, fabs((nn - nold[i]) / nn));
                a.n[size_t(i) * nv + v] = nn;
            }
        }
    }
    if (a.partial) {
        __shared__ double red[256];
        red[threadIdx.x] = cmax;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0) a.partial[blockIdx.x] = red[0];
    }
}

// max over partials (single block) -> out[0]
__global__ void reduce_max_kernel(const double* partial, int n, double* out) {
    __shared__ double red[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, partial[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// max |(a - b) / a| over nq*nvox elements -> partial per block
__global__ void rel_change_kernel(const double* anew, const double* bold, size_t n, double* partial) {
    __shared__ double red[256];
    double m = 0.0;
    for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += size_t(gridDim.x) * 256)
        m = fmax(m, fabs((anew[i] - bold[i]) / anew[i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// S_l = n_j A_ji / (n_i B_ij - n_j B_ji), NaN where the denominator is <= 0.
__global__ void source_function_kernel(const AtomInfo* atom, const double* n, double* S, size_t nvox) {
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    const AtomInfo& at = *atom;
    for (int l = 0; l < at.nline; ++l) {
        const LineInfo& ln = at.line[l];
        const double ni = n[size_t(ln.lower) * nvox + v], nj = n[size_t(ln.upper) * nvox + v];
        const double k = ni * ln.Bij - nj * ln.Bji;
        S[size_t(l) * nvox + v] = k > 0.0 ? nj * ln.A / k : __builtin_nan("");
    }
}

// ------------------------------------------------------------------ grid transfer
// Restriction from the fine grid to the coarse grid (coarse point = fine index 2c),
// periodic in x and y:
//  * full weighting: 27-point tensor product of [1/4, 1/2, 1/4], [1/2, 1/2] at the
//    vertical boundary planes;
//  * half weighting: 1/2 for the point and 1/12 for each of its six axis neighbours;
//    at a vertical boundary plane the missing outward neighbour is replaced by the
//    inward one (the stencil mirrored);
//  * injection: the fine value at the coarse point.
__global__ void restrict_kernel(const double* src, double* dst, int nq, int nxf, int nyf, int nzf, int op) {
    const int nxc = nxf / 2, nyc = nyf / 2, nzc = (nzf - 1) / 2 + 1;
    const size_t ncv = size_t(nxc) * nyc * nzc;
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= ncv * nq) return;
    const int q = int(idx / ncv);
    const size_t r = idx % ncv;
    const int xc = int(r % nxc), yc = int((r / nxc) % nyc), zc = int(r / (size_t(nxc) * nyc));
    const size_t nfv = size_t(nxf) * nyf * nzf;
    const double* s = src + size_t(q) * nfv;
    const size_t pxy = size_t(nxf) * nyf;
    if (op == NLTE_RESTRICT_INJECT) {
        dst[idx] = s[size_t(2 * zc) * pxy + size_t(2 * yc) * nxf + 2 * xc];
        return;
    }
    if (op == NLTE_RESTRICT_HALF) {
        const int k = 2 * zc, y = 2 * yc, x = 2 * xc;
        const int kd = k > 0 ? k - 1 : k + 1, ku = k < nzf - 1 ? k + 1 : k - 1;
        const int xm = x > 0 ? x - 1 : nxf - 1, xp = x + 1 < nxf ? x + 1 : 0;
        const int ym = y > 0 ? y - 1 : nyf - 1, yp = y + 1 < nyf ? y + 1 : 0;
        const double nb = ((s[size_t(k) * pxy + size_t(y) * nxf + xm] + s[size_t(k) * pxy + size_t(y) * nxf + xp]) +
                           (s[size_t(k) * pxy + size_t(ym) * nxf + x] + s[size_t(k) * pxy + size_t(yp) * nxf + x])) +
                          (s[size_t(kd) * pxy + size_t(y) * nxf + x] + s[size_t(ku) * pxy + size_t(y) * nxf + x]);
        dst[idx] = 0.5 * s[size_t(k) * pxy + size_t(y) * nxf + x] + nb / 12.0;
        return;
    }
    double wz[3];
    int kz[3];
    const int kc = 2 * zc;
    if (zc == 0) { kz[0] = 0; kz[1] = 0; kz[2] = 1; wz[0] = 0.0; wz[1] = 0.5; wz[2] = 0.5; }
    else if (zc == nzc - 1) { kz[0] = nzf - 2; kz[1] = nzf - 1; kz[2] = nzf - 1; wz[0] = 0.5; wz[1] = 0.5; wz[2] = 0.0; }
    else { kz[0] = kc - 1; kz[1] = kc; kz[2] = kc + 1; wz[0] = 0.25; wz[1] = 0.5; wz[2] = 0.25; }
    const double w1[3] = {0.25, 0.5, 0.25};
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (wz[a] == 0.0) continue;
        double accy = 0.0;
        for (int b = 0; b < 3; ++b) {
            const int y = (2 * yc + b - 1 + nyf) % nyf;
            double accx = 0.0;
            for (int c = 0; c < 3; ++c) {
                const int x = (2 * xc + c - 1 + nxf) % nxf;
                accx += w1[c] * s[(size_t(kz[a]) * nyf + y) * nxf + x];
            }
            accy += w1[b] * accx;
        }
        acc += wz[a] * accy;
    }
    dst[idx] = acc;
}

// Trilinear interpolation weights of fine point (x, y, k) on the coarse grid.
struct Tri {
    int x0, x1, y0, y1, k0, k1;
    double wx, wy, wz;
};
__device__ inline Tri tri_weights(int x, int y, int k, int nxc, int nyc, const double* zf) {
    Tri t;
    t.x0 = x >> 1; t.x1 = (x & 1) ? ((t.x0 + 1) % nxc) : t.x0; t.wx = (x & 1) ? 0.5 : 0.0;
    t.y0 = y >> 1; t.y1 = (y & 1) ? ((t.y0 + 1) % nyc) : t.y0; t.wy = (y & 1) ? 0.5 : 0.0;
    t.k0 = k >> 1;
    if (k & 1) {
        t.k1 = t.k0 + 1;
        t.wz = (zf[k] - zf[k - 1]) / (zf[k + 1] - zf[k - 1]);
    } else {
        t.k1 = t.k0;
        t.wz = 0.0;
    }
    return t;
}
__device__ inline double tri_eval(const double* c, const Tri& t, int nxc, int nyc) {
    auto at = [&](int k, int y, int x) { return c[(size_t(k) * nyc + y) * nxc + x]; };
    const double a0 = (1.0 - t.wx) * at(t.k0, t.y0, t.x0) + t.wx * at(t.k0, t.y0, t.x1);
    const double a1 = (1.0 - t.wx) * at(t.k0, t.y1, t.x0) + t.wx * at(t.k0, t.y1, t.x1);
    const double b0 = (1.0 - t.wx) * at(t.k1, t.y0, t.x0) + t.wx * at(t.k1, t.y0, t.x1);
    const double b1 = (1.0 - t.wx) * at(t.k1, t.y1, t.x0) + t.wx * at(t.k1, t.y1, t.x1);
    const double a = (1.0 - t.wy) * a0 + t.wy * a1;
    const double b = (1.0 - t.wy) * b0 + t.wy * b1;
    return (1.0 - t.wz) * a + t.wz * b;
}

// Monotone cubic Hermite prolongation on the 4x4x4 coarse stencil, one axis at a time
// (x, then y, then z).  Along an axis a fine point between coarse nodes i and i+1 takes
// the cubic Hermite interpolant of the values and derivatives at those nodes; the
// derivatives are Fritsch & Butland's: zero unless the two adjacent slopes s_l, s_r
// have one sign, else s_l s_r / (a s_r + (1 - a) s_l), a = (1 + h_r / (h_l + h_r)) / 3.
// x and y are periodic with unit spacing (a = 1/2); z uses the physical heights, and
// its two boundary nodes take the slope of their one interval.
__device__ inline double fb_derivative(double sl, double sr, double a) {
    return (sl * sr > 0.0) ? sl * sr / (a * sr + (1.0 - a) * sl) : 0.0;
}
__device__ inline double hermite(double y0, double y1, double d0, double d1, double h, double t) {
    const double t2 = t * t, t3 = t * t * t;
    return ((2 * t3 - 3 * t2 + 1) * y0 + (t3 - 2 * t2 + t) * h * d0) + (-2 * t3 + 3 * t2) * y1 + (t3 - t2) * h * d1;
}
// midpoint between v1 and v2 of a periodic unit-spaced window v0..v3
__device__ inline double hermite_mid(double v0, double v1, double v2, double v3) {
    const double s0 = v1 - v0, s1 = v2 - v1, s2 = v3 - v2;
    return hermite(v1, v2, fb_derivative(s0, s1, 0.5), fb_derivative(s1, s2, 0.5), 1.0, 0.5);
}
__device__ inline double hermite_at(const double* c, int x, int y, int k, int nxc, int nyc, int nzc,
                                    const double* zf) {
    auto gx = [&](int K, int J) -> double {   // x pass at fine x on coarse row (K, J)
        const double* row = c + (size_t(K) * nyc + J) * nxc;
        const int I = x >> 1;
        if (!(x & 1)) return row[I];
        return hermite_mid(row[I == 0 ? nxc - 1 : I - 1], row[I], row[(I + 1) % nxc], row[(I + 2) % nxc]);
    };
    auto gy = [&](int K) -> double {          // then y at fine y on coarse plane K
        const int J = y >> 1;
        if (!(y & 1)) return gx(K, J);
        return hermite_mid(gx(K, J == 0 ? nyc - 1 : J - 1), gx(K, J), gx(K, (J + 1) % nyc), gx(K, (J + 2) % nyc));
    };
    const int K = k >> 1;                      // then z at fine plane k
    if (!(k & 1)) return gy(K);
    const double z0 = zf[2 * K], z1 = zf[2 * K + 2];
    const double h0 = gy(K), h1 = gy(K + 1);
    const double hm = z1 - z0, sm = (h1 - h0) / hm;
    double d0 = sm, d1 = sm;
    if (K > 0) {
        const double hl = z0 - zf[2 * K - 2];
        d0 = fb_derivative((h0 - gy(K - 1)) / hl, sm, (1.0 + hm / (hl + hm)) / 3.0);
    }
    if (K + 1 < nzc - 1) {
        const double hr = zf[2 * K + 4] - z1;
        d1 = fb_derivative(sm, (gy(K + 2) - h1) / hr, (1.0 + hr / (hm + hr)) / 3.0);
    }
    return hermite(h0, h1, d0, d1, hm, (zf[k] - z0) / hm);
}

__global__ void prolong_kernel(const double* src, double* dst, int nq, int nxf, int nyf, int nzf,
                               const double* zf, int op) {
    const size_t nfv = size_t(nxf) * nyf * nzf;
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= nfv * nq) return;
    const int q = int(idx / nfv);
    const size_t r = idx % nfv;
    const int x = int(r % nxf), y = int((r / nxf) % nyf), k = int(r / (size_t(nxf) * nyf));
    const int nxc = nxf / 2, nyc = nyf / 2, nzc = (nzf - 1) / 2 + 1;
    const double* c = src + size_t(q) * nxc * nyc * nzc;
    if (op == NLTE_INTERP_HERMITE) {
        dst[idx] = hermite_at(c, x, y, k, nxc, nyc, nzc, zf);
        return;
    }
    const Tri t = tri_weights(x, y, k, nxc, nyc, zf);
    dst[idx] = tri_eval(c, t, nxc, nyc);
}

// Coarse relative correction e = (n_after - n_before) / n_before (Eq. 11).
__global__ void rel_correction_kernel(const double* na, const double* nb, double* e, size_t n) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) e[i] = (na[i] - nb[i]) / nb[i];
}

// Relative coarse-grid correction (Eqs. 11, 12) with the negative-population repair:
// e = (n_after - n_before) / n_before on the coarse grid, interpolated trilinearly;
// n <- n (1 + I e), and n <- frac * n where that is <= 0.  Repairs counted per block.
// With Hermite interpolation the coarse e comes precomputed in ec (na, nb unused).
__global__ void correct_kernel(double* n, const double* na, const double* nb, int nq, int nxf, int nyf,
                               int nzf, const double* zf, double frac, unsigned long long* repairs,
                               const double* ec, int op) {
    const size_t nfv = size_t(nxf) * nyf * nzf;
    const size_t idx = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int rep = 0;
    if (idx < nfv * nq) {
        const int q = int(idx / nfv);
        const size_t r = idx % nfv;
        const int x = int(r % nxf), y = int((r / nxf) % nyf), k = int(r / (size_t(nxf) * nyf));
        const int nxc = nxf / 2, nyc = nyf / 2, nzc = (nzf - 1) / 2 + 1;
        const size_t ncv = size_t(nxc) * nyc * nzc;
        double ie;
        if (op == NLTE_INTERP_HERMITE) {
            ie = hermite_at(ec + size_t(q) * ncv, x, y, k, nxc, nyc, nzc, zf);
        } else {
            const Tri t = tri_weights(x, y, k, nxc, nyc, zf);
            const double* A = na + size_t(q) * ncv;
            const double* B = nb + size_t(q) * ncv;
            auto e = [&](int kk, int yy, int xx) {
                const size_t o = (size_t(kk) * nyc + yy) * nxc + xx;
                return (A[o] - B[o]) / B[o];
            };
            const double a0 = (1.0 - t.wx) * e(t.k0, t.y0, t.x0) + t.wx * e(t.k0, t.y0, t.x1);
            const double a1 = (1.0 - t.wx) * e(t.k0, t.y1, t.x0) + t.wx * e(t.k0, t.y1, t.x1);
            const double b0 = (1.0 - t.wx) * e(t.k1, t.y0, t.x0) + t.wx * e(t.k1, t.y0, t.x1);
            const double b1 = (1.0 - t.wx) * e(t.k1, t.y1, t.x0) + t.wx * e(t.k1, t.y1, t.x1);
            ie = (1.0 - t.wz) * ((1.0 - t.wy) * a0 + t.wy * a1) + t.wz * ((1.0 - t.wy) * b0 + t.wy * b1);
        }
        const double nold = n[idx];
        double nn = nold * (1.0 + ie);
        if (!(nn > 0.0)) {
            nn = frac * nold;
            rep = 1;
        }
        n[idx] = nn;
    }
    __shared__ int cnt[256];
    cnt[threadIdx.x] = rep;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && cnt[0] > 0) atomicAdd(repairs, (unsigned long long)cnt[0]);
}

// dst = src (FP64), a kernel so that graph-captured work holds no copy nodes.
__global__ void copy_kernel(const double* src, double* dst, size_t n) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

// Right-hand side f = [n_tot, 0, ..., 0].
__global__ void fine_rhs_kernel(double* f, const double* ntot, int N, size_t nvox) {
    const size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    f[v] = ntot[v];
    for (int i = 1; i < N; ++i) f[size_t(i) * nvox + v] = 0.0;
}

// Non-finite check: flag[0] = 1 if any element is NaN or Inf.
__global__ void finite_check_kernel(const double* x, size_t n, int* flag) {
    const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(x[i])) flag[0] = 1;
}

}  // namespace nlte
