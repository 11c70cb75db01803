// Device-side arithmetic of the DDF lattice Boltzmann step for gfx950.
//
// Populations are handled as offsets from the rest equilibrium (df = f - f_eq(rho0, 0),
// dg = g - g_eq(phi0, 0)) so that FP32 and 16-bit storage keep the small
// non-equilibrium parts that the vorticity extraction needs.  Every moment relation
// below is the paper's, rewritten for offsets: the rest state contributes
// rho0 (1, 0, 0, 2 c^2, 0, 0, 0, 0, c^4) to the natural raw moments, so only
// moments 0, 3 and 8 of the equilibria change form (delta-rho replaces rho there).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddf {

// D2Q9 velocities in the paper's order (Sec. 2, eq. particlevelocities1/2) and the
// opposite of each direction.
__host__ __device__ constexpr int ex(int a) { return a == 1 || a == 5 || a == 8 ? 1 : (a == 3 || a == 6 || a == 7 ? -1 : 0); }
__host__ __device__ constexpr int ey(int a) { return a == 2 || a == 5 || a == 6 ? 1 : (a == 4 || a == 7 || a == 8 ? -1 : 0); }
__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : (a <= 4 ? ((a + 1) & 3) + 1 : ((a - 3) & 3) + 5); }

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "axis opposites");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "diagonal opposites");

// ---------------------------------------------------------------------------
// Storage codecs.  Stored value = encode(offset * scale); scale is a power of two.
// enc takes 16 uniform random bits (the low half of its argument); only the
// stochastically rounded format uses them.
// ---------------------------------------------------------------------------
struct bf16 { uint16_t bits; };     // bfloat16, round to nearest even
struct bf16sr { uint16_t bits; };   // bfloat16, stochastic rounding

// 32-bit integer finaliser (xorshift-multiply rounds; the "lowbias32" constants of
// C. Wellons' hash prospector): a counter-based source of uniform bits.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Uniform bits for one stored population (of each lattice) at one time step: a hash
// of (key, step), the key naming the node and direction of the stored population.  The
// f and g stores take its low and high 16 bits, so distinct (node, direction, step,
// lattice) get independent rounding decisions and the same ones the same decisions
// (runs and checkpoint resumes are reproducible).
__device__ __forceinline__ uint32_t sr_step_salt(int64_t t) { return mix32((uint32_t)t + 0x51ed27u); }
__device__ __forceinline__ uint32_t sr_bits(int64_t key, uint32_t step_salt)
{
    return mix32(((uint32_t)key * 0x9e3779b1u) ^ (uint32_t)(key >> 32) ^ step_salt);
}

template <class S> struct Codec;
template <> struct Codec<double> {
    using R = double;
    __device__ static double dec(double v) { return v; }
    __device__ static double enc(double v, uint32_t) { return v; }
};
template <> struct Codec<float> {
    using R = float;
    __device__ static float dec(float v) { return v; }
    __device__ static float enc(float v, uint32_t) { return v; }
};
template <> struct Codec<_Float16> {
    using R = float;
    __device__ static float dec(_Float16 v) { return (float)v; }
    __device__ static _Float16 enc(float v, uint32_t) { return (_Float16)v; }   // round to nearest even
};
template <> struct Codec<bf16> {
    using R = float;
    __device__ static float dec(bf16 v) { return __uint_as_float(((uint32_t)v.bits) << 16); }
    // Round to nearest even (NaN stays NaN): the conversion instruction of gfx950.
    __device__ static bf16 enc(float v, uint32_t)
    {
        bf16 r;
        r.bits = __builtin_bit_cast(uint16_t, (__bf16)v);
        return r;
    }
};
// Stochastic rounding: the magnitude rounds up with probability equal to the dropped
// fraction of a bfloat16 ulp, so the stored value is unbiased and slow changes smaller
// than half an ulp accumulate in expectation instead of being rounded away.
template <> struct Codec<bf16sr> {
    using R = float;
    __device__ static float dec(bf16sr v) { return __uint_as_float(((uint32_t)v.bits) << 16); }
    // The low 16 bits of `bits` are added below the kept mantissa and the sum is
    // truncated (infinities stay infinite; NaN stays a quiet NaN).  gfx950's
    // stochastic-rounding conversion does exactly this with the upper half of its seed
    // operand, so the seed is bits << 16.
    __device__ static bf16sr enc(float v, uint32_t bits)
    {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        bf16sr r;
        if (v != v) {
            r.bits = (uint16_t)((__float_as_uint(v) >> 16) | 0x40u);
        } else {
            const bf16x2 o = __builtin_amdgcn_cvt_sr_bf16_f32(bf16x2{}, v, bits << 16, false);
            r.bits = (uint16_t)__builtin_bit_cast(uint32_t, o);
        }
        return r;
    }
};

// ---------------------------------------------------------------------------
// Natural raw moments m = T f (Sec. 2, eqs. basisvectors, transformationmatrix) and
// the inverse, both as sparse sums (T^-1 derived from the basis: it is 1/36 times an
// integer matrix).
// ---------------------------------------------------------------------------
template <class R>
__host__ __device__ __forceinline__ void moments(const R f[9], R m[9])
{
    const R a = f[5] - f[7], b = f[6] - f[8];
    const R c = f[5] + f[7], d = f[6] + f[8];
    m[6] = a + b;                       // e_x^2 e_y
    m[7] = a - b;                       // e_x e_y^2
    m[5] = c - d;                       // e_x e_y
    m[8] = c + d;                       // e_x^2 e_y^2
    const R sx = f[1] + f[3], sy = f[2] + f[4];
    m[0] = f[0] + sx + sy + m[8];
    m[1] = (f[1] - f[3]) + m[7];
    m[2] = (f[2] - f[4]) + m[6];
    m[3] = sx + sy + (R)2 * m[8];       // e_x^2 + e_y^2
    m[4] = sx - sy;                     // e_x^2 - e_y^2
}

template <class R>
__host__ __device__ __forceinline__ void populations(const R m[9], R f[9])
{
    const R h = (R)0.5, q = (R)0.25;
    f[0] = m[0] - m[3] + m[8];
    const R sp = q * (m[3] + m[4]), sm = q * (m[3] - m[4]);
    f[1] = h * m[1] + sp - h * (m[7] + m[8]);
    f[3] = -h * m[1] + sp + h * (m[7] - m[8]);
    f[2] = h * m[2] + sm - h * (m[6] + m[8]);
    f[4] = -h * m[2] + sm + h * (m[6] - m[8]);
    const R p = m[8] + m[6], r = m[8] - m[6];
    f[5] = q * (p + m[5] + m[7]);
    f[6] = q * (p - m[5] - m[7]);
    f[7] = q * (r + m[5] - m[7]);
    f[8] = q * (r - m[5] + m[7]);
}

// Parameters of the collision, in the compute type R.
template <class R>
struct Phys {
    R om[9];          // fluid rates (0,0,0,w3..w8)
    R omp[9];         // scalar rates (0,w1..w8)
    R b1, b2, c2, cp2;
    R rho0, phi0;
    R scale, inv_scale;
    R wall_f[4][9];   // fluid wall term per unit density for each side: f_eq_a(1,u_w) - f_eq_abar(1,u_w)
    R wall_g[4][9];   // scalar Dirichlet term (offset form): g_eq_a + g_eq_abar - 2 g_rest_a
    int wall_dirichlet[4];
    R rest_f[9];      // f_eq(1, 0) (rest populations per unit density)
    R rest_g[9];      // g_eq(1, 0)
    int force_kind;
    R F0x, F0y, fk, fom;
    R phi_min;
};

__device__ __forceinline__ void sincos_r(double v, double *s, double *c) { sincos(v, s, c); }
__device__ __forceinline__ void sincos_r(float v, float *s, float *c) { sincosf(v, s, c); }

// Body force at node (i, j), time t (Sec. 5.2 four-rolls mill, Sec. 5.3 pulsatile).
template <class R>
__device__ __forceinline__ void body_force(const Phys<R> &P, int i, int j, int64_t t, R &Fx, R &Fy)
{
    if (P.force_kind == 1) {
        Fx = P.F0x; Fy = P.F0y;
    } else if (P.force_kind == 2) {
        R sx, cx, sy, cy;
        sincos_r(P.fk * (R)i, &sx, &cx);
        sincos_r(P.fk * (R)j, &sy, &cy);
        Fx = P.F0x * sx * sy;
        Fy = P.F0x * cx * cy;
    } else if (P.force_kind == 3) {
        const double c = cos(P.fom * (double)t);
        Fx = P.F0x * (R)c; Fy = P.F0y * (R)c;
    } else {
        Fx = (R)0; Fy = (R)0;
    }
}

// Macroscopic state of one node from offset moments (Sec. 2, eq. hydrodynamic_fields).
template <class R>
struct Macro {
    R drho, rho, ux, uy, dphi, phi;
};

// Offset equilibrium moments m_eq(rho, u) - m_eq(rho0, 0) of the fluid (Sec. 2, eq. eqmrawmoment).
template <class R>
__device__ __forceinline__ void fluid_eq(const Phys<R> &P, const Macro<R> &M, R e[9])
{
    const R ux2 = M.ux * M.ux, uy2 = M.uy * M.uy, uxy = M.ux * M.uy, u2 = ux2 + uy2;
    e[0] = M.drho;
    e[1] = M.rho * M.ux;
    e[2] = M.rho * M.uy;
    e[3] = (R)2 * P.c2 * M.drho + M.rho * u2;
    e[4] = M.rho * (ux2 - uy2);
    e[5] = M.rho * uxy;
    e[6] = M.rho * M.uy * (P.c2 + ux2);
    e[7] = M.rho * M.ux * (P.c2 + uy2);
    e[8] = P.c2 * P.c2 * M.drho + M.rho * (P.c2 * u2 + ux2 * uy2);
}

// Offset equilibrium moments of the scalar with the anisotropic third-order terms
// (Sec. 3, eq. eqmrawmoment_CDE).
template <class R>
__device__ __forceinline__ void scalar_eq(const Phys<R> &P, const Macro<R> &M, R e[9])
{
    const R ux2 = M.ux * M.ux, uy2 = M.uy * M.uy, uxy = M.ux * M.uy, u2 = ux2 + uy2;
    e[0] = M.dphi;
    e[1] = M.phi * M.ux;
    e[2] = M.phi * M.uy;
    e[3] = (R)2 * P.cp2 * M.dphi + M.phi * u2;
    e[4] = M.phi * (ux2 - uy2);
    e[5] = M.phi * uxy;
    e[6] = M.phi * M.uy * (P.b1 * P.cp2 + ux2);
    e[7] = M.phi * M.ux * (P.b2 * P.cp2 + uy2);
    e[8] = P.cp2 * P.cp2 * M.dphi + M.phi * (P.cp2 * u2 + ux2 * uy2);
}

// Raw moments of the source term (Sec. 2, the sigma' list).
template <class R>
__device__ __forceinline__ void source(R Fx, R Fy, R ux, R uy, R S[9])
{
    const R fxu = Fx * ux, fyv = Fy * uy;
    S[0] = (R)0;
    S[1] = Fx;
    S[2] = Fy;
    S[3] = (R)2 * (fxu + fyv);
    S[4] = (R)2 * (fxu - fyv);
    S[5] = Fx * uy + Fy * ux;
    S[6] = ux * (Fy * ux + (R)2 * Fx * uy);
    S[7] = uy * (Fx * uy + (R)2 * Fy * ux);
    S[8] = (R)2 * ux * uy * (Fx * uy + Fy * ux);
}

template <class R>
__device__ __forceinline__ Macro<R> macro(const Phys<R> &P, const R m[9], const R n[9], R Fx, R Fy)
{
    Macro<R> M;
    M.drho = m[0];
    M.rho = P.rho0 + m[0];
    const R inv = (R)1 / M.rho;
    M.ux = (m[1] + (R)0.5 * Fx) * inv;
    M.uy = (m[2] + (R)0.5 * Fy) * inv;
    M.dphi = n[0];
    M.phi = P.phi0 + n[0];
    return M;
}

// Fluid collision in moment space (Sec. 2, eq. MRT-LBEfluidmotion_transformed):
// m* = m - Lambda (m - m_eq) + (I - Lambda/2) S, then f* = T^-1 m*.
template <class R, bool FORCE>
__device__ __forceinline__ void collide_fluid(const Phys<R> &P, const Macro<R> &M, const R m[9], R Fx, R Fy, R fo[9])
{
    R e[9], ms[9];
    fluid_eq(P, M, e);
    if (FORCE) {
        R S[9];
        source(Fx, Fy, M.ux, M.uy, S);
        ms[0] = m[0];
        ms[1] = m[1] + S[1];
        ms[2] = m[2] + S[2];
#pragma unroll
        for (int k = 3; k < 9; ++k) ms[k] = m[k] - P.om[k] * (m[k] - e[k]) + ((R)1 - (R)0.5 * P.om[k]) * S[k];
    } else {
        ms[0] = m[0];
        ms[1] = m[1];
        ms[2] = m[2];
#pragma unroll
        for (int k = 3; k < 9; ++k) ms[k] = m[k] - P.om[k] * (m[k] - e[k]);
    }
    populations(ms, fo);
}

// Scalar MRT collision (Sec. 3, eq. MRT-LBECDE).
template <class R>
__device__ __forceinline__ void collide_scalar_mrt(const Phys<R> &P, const Macro<R> &M, const R n[9], R go[9])
{
    R e[9], ns[9];
    scalar_eq(P, M, e);
    ns[0] = n[0];
#pragma unroll
    for (int k = 1; k < 9; ++k) ns[k] = n[k] - P.omp[k] * (n[k] - e[k]);
    populations(ns, go);
}

// Scalar SRT collision (App. B): g* = g - (g - g_eq) / tau_phi with g_eq built from
// the bare raw-moment equilibria through the printed inverse of the bare basis P.
template <class R>
__device__ __forceinline__ void collide_scalar_srt(const Phys<R> &P, const Macro<R> &M, const R g[9], R go[9])
{
    const R ux2 = M.ux * M.ux, uy2 = M.uy * M.uy;
    // bare equilibrium moments minus those of the rest state phi0
    const R q0 = M.dphi, qx = M.phi * M.ux, qy = M.phi * M.uy;
    const R qxx = P.cp2 * M.dphi + M.phi * ux2, qyy = P.cp2 * M.dphi + M.phi * uy2;
    const R qxy = M.phi * M.ux * M.uy;
    const R qxxy = M.phi * M.uy * (P.b1 * P.cp2 + ux2), qxyy = M.phi * M.ux * (P.b2 * P.cp2 + uy2);
    const R qxxyy = P.cp2 * P.cp2 * M.dphi + M.phi * (P.cp2 * (ux2 + uy2) + ux2 * uy2);
    const R h = (R)0.5, q = (R)0.25;
    R geq[9];
    geq[0] = q0 - qxx - qyy + qxxyy;
    geq[1] = h * (qx + qxx - qxyy - qxxyy);
    geq[2] = h * (qy + qyy - qxxy - qxxyy);
    geq[3] = h * (-qx + qxx + qxyy - qxxyy);
    geq[4] = h * (-qy + qyy + qxxy - qxxyy);
    geq[5] = q * (qxy + qxxy + qxyy + qxxyy);
    geq[6] = q * (-qxy + qxxy - qxyy + qxxyy);
    geq[7] = q * (qxy - qxxy - qxyy + qxxyy);
    geq[8] = q * (-qxy - qxxy + qxyy + qxxyy);
    const R w = P.omp[1];
#pragma unroll
    for (int a = 0; a < 9; ++a) go[a] = g[a] - w * (g[a] - geq[a]);
}

// Scalar central-moment collision (App. D; App. C relaxes the same central moments at
// the same rates and gives the same post-collision state).  Works on changes: the
// central moments of the offsets and the equilibrium-minus-rest central moments are
// both small, so FP32 keeps the non-equilibrium parts.
template <class R>
__device__ __forceinline__ void collide_scalar_central(const Phys<R> &P, const Macro<R> &M, const R g[9], R go[9])
{
    const R ux = M.ux, uy = M.uy, ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
    const R c2 = P.cp2, p0 = P.phi0;
    // bare raw moments of the offsets
    const R s = g[5] + g[6] + g[7] + g[8];
    const R q0 = g[0] + g[1] + g[2] + g[3] + g[4] + s;
    const R qx = g[1] - g[3] + g[5] - g[6] - g[7] + g[8];
    const R qy = g[2] - g[4] + g[5] + g[6] - g[7] - g[8];
    const R qxx = g[1] + g[3] + s, qyy = g[2] + g[4] + s;
    const R qxy = g[5] - g[6] + g[7] - g[8];
    const R qxxy = g[5] + g[6] - g[7] - g[8];
    const R qxyy = g[5] - g[6] - g[7] + g[8];
    const R qxxyy = s;
    // their central moments about u (binomial frame change, App. D step (b))
    const R cx = qx - ux * q0, cy = qy - uy * q0;
    const R cxx = qxx - (R)2 * ux * qx + ux2 * q0;
    const R cyy = qyy - (R)2 * uy * qy + uy2 * q0;
    const R cxy = qxy - uy * qx - ux * qy + uxy * q0;
    const R cxxy = qxxy - (R)2 * ux * qxy + ux2 * qy - uy * qxx + (R)2 * uxy * qx - ux2 * uy * q0;
    const R cxyy = qxyy - (R)2 * uy * qxy + uy2 * qx - ux * qyy + (R)2 * uxy * qy - ux * uy2 * q0;
    const R cxxyy = qxxyy - (R)2 * ux * qxyy - (R)2 * uy * qxxy + ux2 * qyy + uy2 * qxx + (R)4 * uxy * qxy
                    - (R)2 * ux2 * uy * qy - (R)2 * ux * uy2 * qx + ux2 * uy2 * q0;
    // equilibrium central moments (App. C, eq. eqmcentralmoment_CDE) minus the central
    // moments of the rest state phi0 (1, 0, 0, c^2, c^2, 0, 0, 0, c^4)
    const R dphi = M.dphi, phi = M.phi;
    const R Dx = ux * p0, Dy = uy * p0;
    const R Dxx = c2 * dphi - p0 * ux2, Dyy = c2 * dphi - p0 * uy2;
    const R Dxy = -p0 * uxy;
    const R Dxxy = (P.b1 - (R)1) * c2 * phi * uy + p0 * uy * (c2 + ux2);
    const R Dxyy = (P.b2 - (R)1) * c2 * phi * ux + p0 * ux * (c2 + uy2);
    const R Dxxyy = c2 * c2 * dphi - p0 * (c2 * (ux2 + uy2) + ux2 * uy2);
    // relaxation changes (App. D step (c))
    const R hx = P.omp[1] * (Dx - cx);
    const R hy = P.omp[2] * (Dy - cy);
    const R hs = P.omp[3] * ((Dxx + Dyy) - (cxx + cyy));
    const R hd = P.omp[4] * ((Dxx - Dyy) - (cxx - cyy));
    const R hxx = (R)0.5 * (hs + hd), hyy = (R)0.5 * (hs - hd);
    const R hxy = P.omp[5] * (Dxy - cxy);
    const R hxxy = P.omp[6] * (Dxxy - cxxy);
    const R hxyy = P.omp[7] * (Dxyy - cxyy);
    const R hxxyy = P.omp[8] * (Dxxyy - cxxyy);
    // raw changes (App. D step (d), zeroth-order change is zero)
    const R rx = hx, ry = hy;
    const R rxx = hxx + (R)2 * ux * hx;
    const R ryy = hyy + (R)2 * uy * hy;
    const R rxy = hxy + uy * hx + ux * hy;
    const R rxxy = hxxy + (R)2 * ux * hxy + ux2 * hy + uy * hxx + (R)2 * uxy * hx;
    const R rxyy = hxyy + (R)2 * uy * hxy + uy2 * hx + ux * hyy + (R)2 * uxy * hy;
    const R rxxyy = hxxyy + (R)2 * ux * hxyy + (R)2 * uy * hxxy + ux2 * hyy + uy2 * hxx + (R)4 * uxy * hxy
                    + (R)2 * ux2 * uy * hy + (R)2 * ux * uy2 * hx;
    // population changes through the inverse of the bare basis (App. D step (e))
    const R h = (R)0.5, q = (R)0.25;
    go[0] = g[0] + (-rxx - ryy + rxxyy);
    go[1] = g[1] + h * (rx + rxx - rxyy - rxxyy);
    go[2] = g[2] + h * (ry + ryy - rxxy - rxxyy);
    go[3] = g[3] + h * (-rx + rxx + rxyy - rxxyy);
    go[4] = g[4] + h * (-ry + ryy + rxxy - rxxyy);
    go[5] = g[5] + q * (rxy + rxxy + rxyy + rxxyy);
    go[6] = g[6] + q * (-rxy + rxxy - rxyy + rxxyy);
    go[7] = g[7] + q * (rxy - rxxy - rxyy + rxxyy);
    go[8] = g[8] + q * (-rxy - rxxy + rxyy + rxxyy);
}

// Local kinematics of one node from its pre-collision offset moments (Sec. 4).
// The fluid non-equilibrium moments include S/2 because the scheme evolves
// f_bar = f - S/2 (Sec. 2) while the Chapman-Enskog relations hold for f.
template <class R>
struct Kin {
    R Sxx, Syy, Sxy, wz, dxuy, dyux, dxphi, dyphi, Q, Rinv, Lx, Ly;
};

template <class R>
__device__ __forceinline__ Kin<R> kinematics(const Phys<R> &P, const Macro<R> &M, const R m[9], const R n[9],
                                            R Fx, R Fy, int scalar_model)
{
    const R ux2 = M.ux * M.ux, uy2 = M.uy * M.uy, uxy = M.ux * M.uy;
    R S3 = (R)0, S4 = (R)0, S5 = (R)0;
    if (P.force_kind != 0) {
        S3 = (R)2 * (Fx * M.ux + Fy * M.uy);
        S4 = (R)2 * (Fx * M.ux - Fy * M.uy);
        S5 = Fx * M.uy + Fy * M.ux;
    }
    const R m3 = m[3] - ((R)2 * P.c2 * M.drho + M.rho * (ux2 + uy2)) + (R)0.5 * S3;
    const R m4 = m[4] - M.rho * (ux2 - uy2) + (R)0.5 * S4;
    const R m5 = m[5] - M.rho * uxy + (R)0.5 * S5;
    const R inv4 = (R)1 / ((R)4 * P.c2 * M.rho);
    Kin<R> K;
    K.Sxx = -(P.om[3] * m3 + P.om[4] * m4) * inv4;
    K.Syy = -(P.om[3] * m3 - P.om[4] * m4) * inv4;
    const R N = -P.om[5] * m5 / (M.rho * P.c2);
    K.Sxy = (R)0.5 * N;
    const R n1 = n[1] - M.phi * M.ux, n2 = n[2] - M.phi * M.uy;
    K.dxphi = -(P.omp[1] / P.cp2) * n1;
    K.dyphi = -(P.omp[2] / P.cp2) * n2;
    R Nphi;
    if (scalar_model >= 2) {
        // central-moment schemes relax the central xy moment; its non-equilibrium part
        // carries (beta - 1) in the scalar-gradient terms
        const R c5 = (n[5] - M.phi * uxy) - M.uy * n1 - M.ux * n2;
        Nphi = -P.omp[5] * c5 / (M.phi * P.cp2)
               - ((P.b1 - (R)1) * M.uy * K.dxphi + (P.b2 - (R)1) * M.ux * K.dyphi) / M.phi;
    } else {
        const R n5 = n[5] - M.phi * uxy;
        Nphi = -P.omp[5] * n5 / (M.phi * P.cp2) - (P.b1 * M.uy * K.dxphi + P.b2 * M.ux * K.dyphi) / M.phi;
    }
    const R idb = (R)1 / (P.b1 - P.b2);
    K.dxuy = (Nphi - P.b2 * N) * idb;
    K.dyux = (P.b1 * N - Nphi) * idb;
    K.wz = ((R)2 * Nphi - (P.b1 + P.b2) * N) * idb;
    if (!(fabs(M.phi) >= P.phi_min)) {
        const R nan = (R)__builtin_nan("");
        K.dxuy = nan; K.dyux = nan; K.wz = nan;
    }
    const R SS = K.Sxx * K.Sxx + K.Syy * K.Syy + (R)2 * K.Sxy * K.Sxy;
    K.Q = (R)-0.5 * SS + (R)0.25 * K.wz * K.wz;
    // tr(S^3) of the symmetric 2x2 block
    const R tr3 = K.Sxx * K.Sxx * K.Sxx + K.Syy * K.Syy * K.Syy
                  + (R)3 * K.Sxy * K.Sxy * (K.Sxx + K.Syy);
    K.Rinv = tr3 / (R)3;
    K.Lx = -K.wz * M.uy;
    K.Ly = K.wz * M.ux;
    return K;
}

}  // namespace ddf
