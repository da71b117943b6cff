// Stage kernels of the eta-based, well-balanced central-upwind scheme
// (Brodtkorb & Holm, arXiv 1912.02457) for gfx950.
//
// Work decomposition: one wavefront owns a strip of 64 consecutive columns
// (60 output columns plus a 2-column halo on each side) and marches down a
// block of rows with a sliding register window.  Neighbours along x come from
// the adjacent lanes (cross-lane shuffles), neighbours along y from the rows
// kept in registers, so every face flux is evaluated once and reused by the
// two cells that share the face, and no LDS is needed.  Global loads are
// 64-float (256 B) row segments.  Ghost cells sit in a 2-cell frame around
// every plane, written by the stage that produces the state (swe_device.h).
//
// Arithmetic follows the paper in float32 with two exact rewritings:
//   * the rest-state pressure g R_f^2/2 with R_f = max(H_f, 0) is taken out
//     of the pressure flux g h_f^2/2 and out of the bathymetry source
//     (g/2dx)(h^E + h^W)(H_E - H_W); the two parts cancel exactly, so M is
//     unchanged, but the float32 flux difference no longer carries the
//     cancellation of g H^2/2 ~ 4e7 at 3000 m (section "Accuracy, precision
//     and GPUs" motivates eta for the same reason).  The source then reads
//     (g/2dx)[(eta^E + eta^W)(H_E - H_W) + min(H_E,0)^2 - min(H_W,0)^2]:
//     below the datum only the eta part remains, above it (dry land, H < 0)
//     nothing is subtracted and a dry cell stays exactly at rest;
//   * the north-vector projection of the Coriolis term (section "Coriolis
//     force") returns f (hv, -hu) for every angle; the default variant uses
//     that identity, PROJ = true evaluates the projection literally.
#include <hip/hip_ext.h>

#include "swe_device.h"
#include "swe_maps.h"

namespace swe {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Plane accesses by 32-bit element offset.  The byte offset is formed in 32
// bits (every plane is below 4 GiB, checked at init), so the access uses the
// scalar-base + 32-bit vector-offset addressing form and needs no 64-bit
// address arithmetic per lane.
__device__ __forceinline__ float ld(const float *__restrict__ base, uint32_t off)
{
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + (off << 2));
}
__device__ __forceinline__ void st(float *__restrict__ base, uint32_t off, float v)
{
    *reinterpret_cast<float *>(reinterpret_cast<char *>(base) + (off << 2)) = v;
}
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// The same value, opaque to the compiler (an empty asm on a VGPR, no
// instruction).  A store whose offset comes from another basic block gets
// that offset as a 64-bit value and a 64-bit address add per plane; an
// offset made opaque in the store's own block is widened there, so the
// stores take the scalar-base form like the loads.
__device__ __forceinline__ uint32_t local_off(uint32_t v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Rounding errors of the compensated state are stored in 16 bits: the upper
// half of the float32 error, rounded to nearest (ties away from zero), i.e. a
// bfloat16.  An error is at most half an ulp of its value, so the pair keeps
// the value to about 2^-10 of a float32 ulp.  A load takes two more bits of
// address arithmetic and one shift; a store one add.
__device__ __forceinline__ float ld_lo(const uint16_t *__restrict__ base, uint32_t off)
{
    const uint32_t b = *reinterpret_cast<const uint16_t *>(reinterpret_cast<const char *>(base) + (off << 1));
    return __uint_as_float(b << 16);
}
__device__ __forceinline__ void st_lo(uint16_t *__restrict__ base, uint32_t off, float v)
{
    *reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(base) + (off << 1)) =
        (uint16_t)((__float_as_uint(v) + 0x8000u) >> 16);
}

// a + b = s + err exactly (Knuth's TwoSum, no assumption on the magnitudes)
__device__ __forceinline__ float two_sum(float a, float b, float &err)
{
    const float s = a + b, bp = s - a, ap = s - bp;
    err = (a - ap) + (b - bp);
    return s;
}

constexpr uint32_t kSign = 0x80000000u;
__device__ __forceinline__ float flip_sign(float x, uint32_t s) { return __uint_as_float(__float_as_uint(x) ^ s); }

// rounding errors of the own cell's stored Q^n (0) and Q* (1) values
struct Lo {
    float e0, u0, v0, e1, u1, v1;
};

// Value held by lane-1 / lane+1 through a whole-wave DPP shift (wave_shr:1
// and wave_shl:1 of the GFX9 DPP controls; a VALU operand modifier, no LDS
// round trip).  Lane 0 / lane 63 receive 0 (bound_ctrl: the lane without a
// source reads zero, so no old value has to be set up first); they are halo
// lanes whose results are never stored.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;
__device__ __forceinline__ int from_left(int v) { return __builtin_amdgcn_update_dpp(0, v, kDppWaveShr1, 0xF, 0xF, true); }
__device__ __forceinline__ int from_right(int v) { return __builtin_amdgcn_update_dpp(0, v, kDppWaveShl1, 0xF, 0xF, true); }
__device__ __forceinline__ float from_left(float v) { return __int_as_float(from_left(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(from_right(__float_as_int(v))); }

// eq. desing_ours; h^2/(2 kappa) + kappa/2 is formed as (h h + kappa^2) /
// (2 kappa), one uniform operand per instruction.  That value q is never
// below |h| (equal only at |h| = kappa) and is below kappa exactly when |h|
// is, so max(|h|, min(q, kappa)) is the median of |h|, q and kappa.
__device__ __forceinline__ float desing(float h, const Dom &d)
{
    const float q = fmaf(h, h, d.kappa_sq) * d.inv2kappa;
    const float m = __builtin_amdgcn_fmed3f(fabsf(h), q, d.kappa);
    // sign(h) with sign(0) = +1: adding +0 turns a -0 into +0
    return copysignf(m, h + 0.f);
}

// TWICE the generalized minmod of theta*backward, central, theta*forward
// differences dm, dp: minmod(2 theta dm, dm + dp, 2 theta dp), given as its
// three candidates a = 2 theta dm, b = dm + dp, c = 2 theta dp (scaling by
// two is exact, so callers take a quarter of it where the slope's half is
// used, bitwise the same as halving the minmod).  minmod of three numbers
// is the median of (their minimum, 0, their maximum): the minimum if all
// are positive, the maximum if all are negative, else 0.  Along y each
// row's 2 theta multiple serves the faces below and above it.
__device__ __forceinline__ float limited2(float a, float b, float c)
{
    return __builtin_amdgcn_fmed3f(fminf(a, fminf(b, c)), 0.f, fmaxf(a, fmaxf(b, c)));
}

// limited2 along x, the forward difference being the right neighbour's
// backward one: its 2 theta multiple is the neighbour's product, moved by
// one lane (the same bits as multiplying the moved difference)
__device__ __forceinline__ float limited2_x(float dm, float th2)
{
    const float a = th2 * dm;
    return limited2(a, dm + from_right(dm), from_right(a));
}

__device__ __forceinline__ void time_weights(int n, const double *ts, double tau, int &k, double &s)
{
    if (n <= 1 || tau <= ts[0]) { k = 0; s = 0.0; return; }
    if (tau >= ts[n - 1]) { k = n - 2; s = 1.0; return; }
    int a = 0;
    while (a < n - 2 && ts[a + 1] <= tau) ++a;
    k = a;
    s = (tau - ts[a]) / (ts[a + 1] - ts[a]);
}

// wave-wide maximum of a float (every lane gets the result)
__device__ __forceinline__ float wave_max(float v)
{
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
    return v;
}

// CFL accumulator of one parity: maximum over the slots (all lanes get it)
__device__ __forceinline__ uint32_t read_wmax(const Ctrl *c, int parity, int lane)
{
    uint32_t v = c->wslot[parity][lane & (kCflSlots - 1)][0];
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, kWave));
    return v;
}


__device__ __forceinline__ void wind_at(const Dom &d, double tau, float &wx, float &wy)
{
    if (d.nw <= 0) { wx = wy = 0.f; return; }
    int k; double s;
    time_weights(d.nw, d.wind_t, tau, k, s);
    double ax = d.wind[2 * k], ay = d.wind[2 * k + 1];
    if (d.nw > 1) {
        ax = (1.0 - s) * ax + s * (double)d.wind[2 * k + 2];
        ay = (1.0 - s) * ay + s * (double)d.wind[2 * k + 3];
    }
    wx = (float)(ax * d.inv_rho_w);
    wy = (float)(ay * d.inv_rho_w);
}



struct F3 { float e, p, q; };

// eq. numerical_flux for a face with depth Hf between a left state (eL,pL,qL)
// and a right state; p is the momentum normal to the face, q the transverse
// one.  Desingularised velocities, face momenta recomputed as h u, wave
// speeds a+ >= 0 >= a-, transverse momentum upwinded on the mass flux.
// Written with the weights alpha = a+/(a+ - a-), 1 - alpha and
// gamma = a+ a-/(a+ - a-); when a+ = a- = 0 (both sides dry and at rest)
// alpha = 1/2, gamma = 0 give the average of the two physical fluxes.  No
// branches, so the flux of a face can be interleaved with other work.
// The pressure uses the perturbation form (see the file header).
__device__ __forceinline__ F3 cu_flux(float eL, float pL0, float qL0, float eR, float pR0, float qR0,
                                      float Hf, const Dom &d)
{
    float hL = eL + Hf, hR = eR + Hf;
    float rL = rcp(desing(hL, d)), rR = rcp(desing(hR, d));
    float uL = pL0 * rL, vL = qL0 * rL, uR = pR0 * rR, vR = qR0 * rR;
    float pL = hL * uL, pR = hR * uR;
    float cL = fsqrt(d.g * fmaxf(hL, 0.f)), cR = fsqrt(d.g * fmaxf(hR, 0.f));
    float ap = fmaxf(fmaxf(uL + cL, uR + cR), 0.f);
    float am = fminf(fminf(uL - cL, uR - cR), 0.f);
    // g (h_f^2 - R_f^2) / 2 = g/2 (eta_f + min(H_f,0)) (eta_f + H_f + max(H_f,0))
    float Hn = fminf(Hf, 0.f), Hs2 = Hf + fmaxf(Hf, 0.f);
    float PL = 0.5f * d.g * (eL + Hn) * (eL + Hs2), PR = 0.5f * d.g * (eR + Hn) * (eR + Hs2);
    float FL = fmaf(pL, uL, PL), FR = fmaf(pR, uR, PR);
    // a+ - a- below 2^-100 m/s counts as a+ = a- = 0: its FP32 reciprocal
    // would overflow (a denormal momentum on a dry face gives such speeds)
    // and turn the weights into inf * 0.  Only faces with h_f <= 1e-61 m on
    // both sides fall in the gap, where both branches agree to O(g h_f^2).
    float den = ap - am;
    bool wet = den > 0x1p-100f;
    float w = wet ? rcp(den) : 0.f;
    const float apw = ap * w;
    float al = wet ? apw : 0.5f;
    float ga = am * apw;
    // alpha F_L + (1 - alpha) F_R as F_R + alpha (F_L - F_R): one operation
    // less, and exactly F_R where the two physical fluxes are equal (a lake
    // at rest)
    const float dp = pL - pR;
    F3 r;
    r.e = fmaf(al, dp, fmaf(ga, eR - eL, pR));
    r.p = fmaf(al, FL - FR, fmaf(ga, -dp, FR));
    r.q = r.e * (r.e >= 0.f ? vL : vR);
    return r;
}

// face with the land rule: a face touching land carries the reflective-wall
// flux of its wet side; a face between two land cells carries nothing.
// `anyland` is uniform over the wave (some lane of the rows involved is
// land); without it the land selects are skipped, which gives bitwise the
// same flux.
__device__ __forceinline__ F3 face_flux(float eL, float pL, float qL, float eR, float pR, float qR,
                                        bool lL, bool lR, bool anyland, float Hf, const Dom &d)
{
    if (anyland) {
        const float e2R = lR ? eL : eR, p2R = lR ? -pL : pR, q2R = lR ? qL : qR;
        const float e2L = lL ? eR : eL, p2L = lL ? -pR : pL, q2L = lL ? qR : qL;
        eL = e2L; pL = p2L; qL = q2L;
        eR = e2R; pR = p2R; qR = q2R;
    }
    F3 r = cu_flux(eL, pL, qL, eR, pR, qR, Hf, d);
    if (anyland && lL && lR) r.e = r.p = r.q = 0.f;
    return r;
}

// bathymetry source times 2 dx / g (x) or 2 dy / g (y): (h^E + h^W)(H_E - H_W)
// minus (R_E^2 - R_W^2), R = max(H, 0), matching the pressure flux of
// cu_flux.  With h = eta + H and H^2 - max(H,0)^2 = min(H,0)^2 this is
//   (eta^E + eta^W)(H_E - H_W) + min(H_E,0)^2 - min(H_W,0)^2,
// one formula for wet and dry faces with no cancellation of large terms;
// the caller scales it by g / (2 dx) or g / (2 dy).
__device__ __forceinline__ float bathy_source(float eE, float eW, float HE, float HW)
{
    float mE = fminf(HE, 0.f), mW = fminf(HW, 0.f);
    float dry = fmaf(mE, mE, -(mW * mW));
    return fmaf(eE + eW, HE - HW, dry);
}

// bed shear stress coefficient S >= 0, the source being -S (hu, hv), from the
// cell's reciprocal desingularised depth ri = 1/h*
__device__ __forceinline__ float friction_coeff(const Dom &d, float ri, float hu, float hv)
{
    if (d.friction == FR_NONE) return 0.f;
    float ra = fabsf(ri);
    if (d.friction == FR_LINEAR) return d.fric_c * ra;
    float speed = fsqrt(hu * hu + hv * hv) * ra;
    if (d.friction == FR_QUADRATIC) return d.fric_c * speed * ra * ra;
    // Manning: g n^2 |u| / a^(4/3) = g n^2 |u| ra^(4/3)
    float ra43 = __builtin_amdgcn_exp2f((4.0f / 3.0f) * __builtin_amdgcn_logf(ra));
    return d.fric_c * speed * ra43;
}

// Face values eta +/- rho of a cell with the wet-dry fix of eq. KxE_adjust:
// a face value below the bottom (eta_f + H_f < 0) is set to the bottom and
// the other face takes 2 eta - eta_f, keeping the cell average; first the
// face on the + side, then the one on the - side.  As max/min: raising
// the + face to -H_+ is a max, and then the - face (2 eta - that) is the
// min of itself and 2 eta + H_+ -- exact when the fix applies, and equal
// to the unfixed value otherwise (up to one rounding when the two are
// within an ulp).
__device__ __forceinline__ void positivity_fix(float e, float rho, float Hp, float Hm, float &ep, float &em)
{
    ep = e + rho;
    em = e - rho;
    ep = fmaxf(ep, -Hp);
    em = fminf(em, fmaf(2.f, e, Hp));
    em = fmaxf(em, -Hm);
    ep = fminf(ep, fmaf(2.f, e, Hm));
}

// One row of the sliding window (per lane: column i).
struct Row {
    float e, u, v, f;      // state and Coriolis parameter (NaN: land)
    float cx, cy;          // Coriolis terms of the reconstruction (f v, -f u)
    float Hw, He, Hs, Hn, Hb;
    float ri;              // 1 / h* of the cell
    int land;
    bool anyland;          // some lane of the row is land (uniform over the wave)
    float dmL, dmU, dmV;   // y backward differences (this row minus the row below)
    float tmL, tmU, tmV;   // the same times 2 theta
    float eN, eS, uN, vN;  // north/south face values once the row was the middle row
};

// face depths, mean depth, land flag and Coriolis terms of a row from its
// four corner depths (south corners cs*, north corners cn*); the south face
// depth hs is the north face depth of the row below, 0.5 (cs0 + cs1)
template <bool PROJ>
__device__ __forceinline__ void row_terms(Row &R, float cs0, float cs1, float cn0, float cn1, float hs, float th,
                                          const Dom &d)
{
    R.Hw = 0.5f * (cs0 + cn0);
    R.He = 0.5f * (cs1 + cn1);
    R.Hs = hs;
    R.Hn = 0.5f * (cn0 + cn1);
    R.Hb = 0.25f * ((cs0 + cn0) + (cs1 + cn1));
    float h = R.e + R.Hb;
    float ri = rcp(desing(h, d));
    R.ri = ri;
    float uu = R.u * ri, vv = R.v * ri;
    R.land = isnan(R.f) ? 1 : 0;
    R.anyland = __ballot(R.land) != 0;
    if (PROJ) {
        float c = __cosf(th), s = __sinf(th);
        float ue = c * uu - s * vv, vn = s * uu + c * vv;
        R.cx = R.f * (c * vn - s * ue);
        R.cy = R.f * (-s * vn - c * ue);
    } else {
        R.cx = R.f * vv;
        R.cy = -R.f * uu;
    }
}

// backward differences along y of row C against the row B below it; the
// K-type difference of eq. Kbackwards in its y form (L = g(eta + U))
__device__ __forceinline__ void y_diff(Row &C, const Row &B, const Dom &d)
{
    C.dmL = C.e - B.e - d.ky * (B.cy + C.cy);
    C.dmU = C.u - B.u;
    C.dmV = C.v - B.v;
    C.tmL = d.theta2 * C.dmL;
    C.tmU = d.theta2 * C.dmU;
    C.tmV = d.theta2 * C.dmV;
}

// limited y-slopes and N/S face values of row B (eq. hE in its N/S form with
// the wet-dry fix of eq. KxE_adjust); stores the N values and eS in B and
// returns the S momenta for the face below B
__device__ __forceinline__ void y_faces(Row &B, const Row &C, int landA, bool anylandA, const Dom &d, float &uS,
                                        float &vS)
{
    // twice the limited slopes (limited2)
    float sL = limited2(B.tmL, B.dmL + C.dmL, C.tmL);
    float sU = limited2(B.tmU, B.dmU + C.dmU, C.tmU);
    float sV = limited2(B.tmV, B.dmV + C.dmV, C.tmV);
    // first order next to land (skipped for rows without land nearby)
    if ((anylandA || C.anyland) && (landA || C.land)) sL = sU = sV = 0.f;
    float rho = 0.25f * sL + d.ky * B.cy;
    float eN, eS;
    positivity_fix(B.e, rho, B.Hn, B.Hs, eN, eS);
    B.eN = eN;
    B.eS = eS;
    B.uN = B.u + 0.25f * sU;
    B.vN = B.v + 0.25f * sV;
    uS = B.u - 0.25f * sU;
    vS = B.v - 0.25f * sV;
}

// flux through the face between row A (below, its N values) and row B
// (above, its S values): normal momentum hv, transverse hu
__device__ __forceinline__ F3 y_flux(const Row &A, const Row &B, float uS, float vS, const Dom &d)
{
    return face_flux(A.eN, A.vN, A.uN, B.eS, vS, uS, A.land != 0, B.land != 0, A.anyland || B.anyland, B.Hs, d);
}

struct TileCtx {
    int i, o;        // column of this lane, output row
    bool out_lane;   // lane owns an output cell
    float dt, wx, wy;
    int bk;          // boundary snapshot interval and weight at the stage time
    double bs;
    int fbk;         // the same at the time of the stage that reads this stage's output
    double fbs;
    bool edge;       // the tile writes ghost cells (output cells within two cells of a side)
    int fca, fcb;    // ghost columns that copy this lane's cells (frame_copy_cols)
    int wk;          // wind-field snapshot interval and weight at the stage time
    float ws;
};

// Wind at 10 m from its own grid at cell (i, o): samples at the centres of a
// w10nx x w10ny partition of the domain, bilinear in space (clamped at the
// edges, as a texture fetch with linear filtering) and linear in time between
// the snapshots around the stage time (eq. windstress_interpol); then the
// stress of Large and Pond, rho_a/rho_w C_D |W| W with C_D = 1.2e-3 below
// 11 m/s and (0.49 + 0.065 |W|) 1e-3 above, as the kinematic source.
__device__ __forceinline__ void w10_stress(const Dom &d, const TileCtx &c, float &sx, float &sy)
{
    float gx = fminf(fmaxf(((float)c.i + 0.5f) * d.w10sx - 0.5f, 0.f), (float)(d.w10nx - 1));
    float gy = fminf(fmaxf(((float)c.o + 0.5f) * d.w10sy - 0.5f, 0.f), (float)(d.w10ny - 1));
    const int i0 = (int)gx, j0 = (int)gy;
    const int i1 = min(i0 + 1, d.w10nx - 1), j1 = min(j0 + 1, d.w10ny - 1);
    const float fx = gx - (float)i0, fy = gy - (float)j0;
    const uint32_t plane = (uint32_t)d.w10nx * (uint32_t)d.w10ny * 2u;
    const float *Wa = d.w10 + (uint32_t)c.wk * plane;
    const float *Wb = d.w10n > 1 ? Wa + plane : Wa;
    float W[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        auto at = [&](const float *P, int i, int j) { return P[((uint32_t)j * (uint32_t)d.w10nx + (uint32_t)i) * 2u + q]; };
        float a = (1.f - fy) * ((1.f - fx) * at(Wa, i0, j0) + fx * at(Wa, i1, j0)) +
                  fy * ((1.f - fx) * at(Wa, i0, j1) + fx * at(Wa, i1, j1));
        float b = (1.f - fy) * ((1.f - fx) * at(Wb, i0, j0) + fx * at(Wb, i1, j0)) +
                  fy * ((1.f - fx) * at(Wb, i0, j1) + fx * at(Wb, i1, j1));
        W[q] = (1.f - c.ws) * a + c.ws * b;
    }
    if (d.w10_kind) {  // a stress field, interpolated as it is
        sx = d.w10q * W[0];
        sy = d.w10q * W[1];
        return;
    }
    const float sp = fsqrt(W[0] * W[0] + W[1] * W[1]);
    const float cd = sp < 11.f ? 1.2e-3f : (0.49f + 0.065f * sp) * 1e-3f;
    const float k = d.w10q * cd * sp;
    sx = k * W[0];
    sy = k * W[1];
}

// Flow relaxation (eq. frs) of one output cell: whether it lies in a zone,
// the nearest nested side within the zone (ties W, E, S, N), its weight
// alpha = 1 - tanh(d/d0) and the two boundary snapshots around the stage
// time.  The row loop only tests the zone at the start of a row; the loads
// are issued where the update uses them (held across the row, they raised
// the register count of the whole stage-2 kernel to three waves per SIMD).
struct FrsPre {
    bool zone;
    float al;
    float a[3], b[3];
};

__device__ __forceinline__ FrsPre frs_prefetch(const Dom &d, const TileCtx &c)
{
    FrsPre f;
    const int nx = d.nx, ny = d.ny, i = c.i, o = c.o;
    // boundary-table entries on the four sides (frs_candidates in swe_maps.h)
    int idxs[4] = {o, ny + o, 2 * ny + i, 2 * ny + nx + i};
    int best, dd;
    frs_side(d, i, o, best, dd);
    f.zone = c.out_lane && best >= 0 && dd < d.frs_w;
    f.al = 0.f;
    f.a[0] = f.a[1] = f.a[2] = f.b[0] = f.b[1] = f.b[2] = 0.f;
    if (f.zone) {
        int idx = best == 0 ? idxs[0] : best == 1 ? idxs[1] : best == 2 ? idxs[2] : idxs[3];
        f.al = d.frs_alpha[dd];
        const uint32_t P = (uint32_t)d.P;
        const float *pa = d.bnd + (uint32_t)c.bk * 3u * P + (uint32_t)idx;
        const float *pb = d.nb > 1 ? pa + 3u * P : pa;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            f.a[q] = pa[q * P];
            f.b[q] = pb[q * P];
        }
    }
    return f;
}

// x-direction reconstruction and flux of the output row A, the update of
// eq. rk2_semiimp and (stage 2) the flow relaxation and CFL reduction.
// Every lane takes part in the cross-lane exchanges; only output lanes store.
// Ghost cells of the state this stage writes (Q* in stage 1, Q^{n+1} in
// stage 2) for the stage that reads it next, by edge tiles: the wall and
// periodic copies of a water cell's new values (frame_copy_cols / _rows;
// the lane's target columns are fixed for the tile, the row targets are
// uniform), stored from the registers that hold them.  A land cell keeps
// its state, and its ghosts their values.
template <int STAGE>
__device__ __forceinline__ void write_frame_copies(const Dom &d, const TileCtx &c, float e, float u, float v)
{
    float *__restrict__ E = STAGE == 1 ? d.eta1 : d.eta;
    float *__restrict__ U = STAGE == 1 ? d.hu1 : d.hu;
    float *__restrict__ V = STAGE == 1 ? d.hv1 : d.hv;
    auto put = [&](int x, int y, float uu, float vv) {
        const uint32_t o = cell_off(d, y, x);
        st(E, o, e);
        st(U, o, uu);
        st(V, o, vv);
    };
    if (c.fca != kNoFrame) put(c.fca, c.o, d.bc[0] == BC_WALL ? -u : u, v);
    if (c.fcb != kNoFrame) put(c.fcb, c.o, d.bc[1] == BC_WALL ? -u : u, v);
    int ra, rb;
    frame_copy_rows(d, c.o, ra, rb);
    if (ra != kNoFrame) put(c.i, ra, u, d.bc[2] == BC_WALL ? -v : v);
    if (rb != kNoFrame) put(c.i, rb, u, d.bc[3] == BC_WALL ? -v : v);
}

// Nested ghosts take the boundary data at the reading stage's time (the
// interpolation of the boundary loads), independent of the state: written
// after the row loop by the tiles next to a nested side, four rows at a
// time so that their loads overlap.
template <int STAGE>
__device__ __forceinline__ void write_frame_nested(const Dom &d, const TileCtx &c, int y0, int y1)
{
    float *__restrict__ E = STAGE == 1 ? d.eta1 : d.eta;
    float *__restrict__ U = STAGE == 1 ? d.hu1 : d.hu;
    float *__restrict__ V = STAGE == 1 ? d.hv1 : d.hv;
    const int nx = d.nx, ny = d.ny, x = c.i;
    const uint32_t P = (uint32_t)d.P;
    const float *__restrict__ ba = d.bnd + (uint32_t)c.fbk * 3u * P;
    const float *__restrict__ bb = d.nb > 1 ? ba + 3u * P : ba;
    const double t = c.fbs;
    auto put = [&](int idx, int xa, int ya, int xb, int yb) {
        const float e = (float)((1.0 - t) * (double)ba[idx] + t * (double)bb[idx]);
        const float u = (float)((1.0 - t) * (double)ba[P + idx] + t * (double)bb[P + idx]);
        const float v = (float)((1.0 - t) * (double)ba[2u * P + idx] + t * (double)bb[2u * P + idx]);
        const uint32_t oa = cell_off(d, ya, xa), ob = cell_off(d, yb, xb);
        st(E, oa, e); st(U, oa, u); st(V, oa, v);
        st(E, ob, e); st(U, ob, u); st(V, ob, v);
    };
    // west / east: the lane of column 0 / nx-1, every row of the tile
    const bool w = d.bc[0] == BC_NESTED && x == 0 && c.out_lane;
    const bool e = d.bc[1] == BC_NESTED && x == nx - 1 && c.out_lane;
    if (__ballot(w || e) != 0) {
        for (int y = y0; y < y1; y += 4) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int yy = y + k;
                if (yy < y1) {
                    if (w) put(yy, -1, yy, -2, yy);
                    if (e) put(ny + yy, nx, yy, nx + 1, yy);
                }
            }
        }
    }
    // south / north: every output lane of row 0 / ny-1
    if (d.bc[2] == BC_NESTED && y0 == 0 && c.out_lane) put(2 * ny + x, x, -1, x, -2);
    if (d.bc[3] == BC_NESTED && y1 == ny && c.out_lane) put(2 * ny + nx + x, x, ny, x, ny + 1);
}

// lanes of a wave that stored a non-finite state, or a water depth below
// -kappa (ballot masks, the same in every lane)
struct BadLanes {
    uint64_t nonfinite, negative;
};

template <int STAGE, bool PROJ, bool W10, bool COMP>
__device__ __forceinline__ void finish_row(const Row &A, const F3 &Gs, const F3 &Gn, const TileCtx &c,
                                           float e0, float u0, float v0, const FrsPre &fp,
                                           const Dom &d, float &wmax_loc, BadLanes &bad)
{
    const float th2 = d.theta2;
    float eL = from_left(A.e), cxL = from_left(A.cx);
    float uL = from_left(A.u), vL = from_left(A.v);
    float dmK = A.e - eL - d.kx * (cxL + A.cx);
    float dmU = A.u - uL, dmV = A.v - vL;
    // twice the limited slopes (limited2)
    float sK = limited2_x(dmK, th2);
    float sUx = limited2_x(dmU, th2);
    float sVx = limited2_x(dmV, th2);
    int landR = 0;
    if (A.anyland) {  // first order next to land (rows with land only)
        const int landL = from_left(A.land);
        landR = from_right(A.land);
        if (landL || landR) sK = sUx = sVx = 0.f;
    }
    float rx = 0.25f * sK + d.kx * A.cx;
    float eE, eW;
    positivity_fix(A.e, rx, A.He, A.Hw, eE, eW);
    float uE = A.u + 0.25f * sUx, uW = A.u - 0.25f * sUx;
    float vE = A.v + 0.25f * sVx, vW = A.v - 0.25f * sVx;
    F3 Fe = face_flux(eE, uE, vE, from_right(eW), from_right(uW), from_right(vW), A.land != 0, landR != 0,
                      A.anyland, A.He, d);
    float Fwe = from_left(Fe.e), Fwp = from_left(Fe.p), Fwq = from_left(Fe.q);
    // every lane computes; only output lanes over water store (no early exit,
    // so the x and y work of neighbouring rows can be interleaved)
    const bool store = c.out_lane && !A.land;

    float Cx, Cy;
    if (PROJ) {
        float ang = store ? ld(d.north, cell_off(d, c.o, c.i)) : 0.f;
        float cc = __cosf(ang), ss = __sinf(ang);
        float hue = cc * A.u - ss * A.v, hvn = ss * A.u + cc * A.v;
        Cx = A.f * (cc * hvn - ss * hue);
        Cy = A.f * (-ss * hvn - cc * hue);
    } else {
        Cx = A.f * A.v;
        Cy = -A.f * A.u;
    }
    float wx = c.wx, wy = c.wy;
    if (W10 && d.w10n > 0) {
        float sx, sy;
        w10_stress(d, c, sx, sy);
        wx += sx;
        wy += sy;
    }
    float Me = -(Fe.e - Fwe) * d.rdx - (Gn.e - Gs.e) * d.rdy;
    float Mu = -(Fe.p - Fwp) * d.rdx - (Gn.q - Gs.q) * d.rdy + bathy_source(eE, eW, A.He, A.Hw) * d.grdx2 +
               Cx + wx;
    float Mv = -(Fe.q - Fwq) * d.rdx - (Gn.p - Gs.p) * d.rdy + bathy_source(A.eN, A.eS, A.Hn, A.Hs) * d.grdy2 +
               Cy + wy;
    const uint32_t oo = cell_off(d, c.o, c.i);
    const float dt = c.dt;
    float S = friction_coeff(d, A.ri, A.u, A.v);
    // compensated: the stored rounding errors of the cell, loaded where they
    // are used (held across the row they would raise the register count)
    Lo lo{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (COMP) {
        lo.e0 = ld_lo(d.eta_lo, oo);
        lo.u0 = ld_lo(d.hu_lo, oo);
        lo.v0 = ld_lo(d.hv_lo, oo);
        if (STAGE == 2) {
            lo.e1 = ld_lo(d.eta1_lo, oo);
            lo.u1 = ld_lo(d.hu1_lo, oo);
            lo.v1 = ld_lo(d.hv1_lo, oo);
        }
    }
    if (STAGE == 1) {
        float den = rcp(1.f + dt * S);
        if (COMP) {
            // compensated: the increment of each field, added to the stored
            // value plus its rounding error without losing the new error
            float le, lu, lv;
            const float en = two_sum(A.e, dt * Me + lo.e0, le);
            const float un = two_sum(A.u, (dt * Mu - dt * S * A.u) * den + lo.u0, lu);
            const float vn = two_sum(A.v, (dt * Mv - dt * S * A.v) * den + lo.v0, lv);
            if (store) {
                st(d.eta1, oo, en);
                st(d.hu1, oo, un);
                st(d.hv1, oo, vn);
                st_lo(d.eta1_lo, oo, le);
                st_lo(d.hu1_lo, oo, lu);
                st_lo(d.hv1_lo, oo, lv);
                if (c.edge) write_frame_copies<1>(d, c, en, un, vn);
            }
        } else {
            float en = A.e + dt * Me;
            float un = (A.u + dt * Mu) * den;
            float vn = (A.v + dt * Mv) * den;
            if (store) {
                st(d.eta1, oo, en);
                st(d.hu1, oo, un);
                st(d.hv1, oo, vn);
                if (c.edge) write_frame_copies<1>(d, c, en, un, vn);
            }
        }
    } else {
        float den = rcp(1.f + 0.5f * dt * S);
        float en, un, vn, le = 0.f, lu = 0.f, lv = 0.f;
        if (COMP) {
            // Q^{n+1} = Q^n + (Q* - Q^n + dt M(Q*))/2 (momenta with the
            // friction factor), the differences taken with both errors
            const float de = (A.e - e0) + (lo.e1 - lo.e0);
            const float du = (A.u - u0) + (lo.u1 - lo.u0);
            const float dv = (A.v - v0) + (lo.v1 - lo.v0);
            en = two_sum(e0, 0.5f * (de + dt * Me) + lo.e0, le);
            un = two_sum(u0, (0.5f * (du + dt * Mu) - 0.5f * dt * S * u0) * den + lo.u0, lu);
            vn = two_sum(v0, (0.5f * (dv + dt * Mv) - 0.5f * dt * S * v0) * den + lo.v0, lv);
        } else {
            en = 0.5f * (e0 + (A.e + dt * Me));
            un = 0.5f * (u0 + (A.u + dt * Mu)) * den;
            vn = 0.5f * (v0 + (A.v + dt * Mv)) * den;
        }
        if (fp.zone) {
            // the boundary values are loaded here, where they are used, not
            // at the start of the row: held across the row they would raise
            // the register count of every tile's kernel
            const FrsPre fl = frs_prefetch(d, c);
            const float al = fl.al;
            const double t = c.bs;
            float ex[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) ex[q] = (float)((1.0 - t) * (double)fl.a[q] + t * (double)fl.b[q]);
            if (COMP) {
                en = two_sum(en, le + al * ((ex[0] - en) - le), le);
                un = two_sum(un, lu + al * ((ex[1] - un) - lu), lu);
                vn = two_sum(vn, lv + al * ((ex[2] - vn) - lv), lv);
            } else {
                en = (1.f - al) * en + al * ex[0];
                un = (1.f - al) * un + al * ex[1];
                vn = (1.f - al) * vn + al * ex[2];
            }
        }
        if (store) {
            const uint32_t so = local_off(oo);
            st(d.eta, so, en);
            st(d.hu, so, un);
            st(d.hv, so, vn);
            if (COMP) {
                st_lo(d.eta_lo, so, le);
                st_lo(d.hu_lo, so, lu);
                st_lo(d.hv_lo, so, lv);
            }
            if (c.edge) write_frame_copies<2>(d, c, en, un, vn);
        }

        // eq. cfl on the new state
        float h = en + A.Hb;
        float ri = rcp(desing(h, d));
        float cw = fsqrt(d.g * fmaxf(h, 0.f));
        float w = fmaxf((fabsf(un * ri) + cw) * d.rdx, (fabsf(vn * ri) + cw) * d.rdy);
        wmax_loc = store ? fmaxf(wmax_loc, w) : wmax_loc;
        // bit 0: a non-finite state; bit 1: a water depth below -kappa (the
        // scheme keeps h >= 0 under its CFL bound, so this means breakdown);
        // gathered over the wave by ballot, so the bits are scalar values
        const uint64_t m_st = __builtin_amdgcn_ballot_w64(store);
        bad.nonfinite |= m_st & (__builtin_amdgcn_ballot_w64(!isfinite(en)) | __builtin_amdgcn_ballot_w64(!isfinite(un)) |
                                 __builtin_amdgcn_ballot_w64(!isfinite(vn)));
        bad.negative |= m_st & __builtin_amdgcn_ballot_w64(h < -d.kappa);
    }
}

// ---- one tile: a wavefront's 64 columns over rows y0..y1-1 ------------------
// The window of three rows rotates by unrolling (no register moves, no
// per-row branches) and the next row is prefetched while the current one is
// processed.  Every load is a plain 32-bit offset into a framed plane: the
// ghost cells sit in the frame (filled by the stage that wrote the state),
// so edge tiles load exactly as interior ones.  frs: the tile has output
// cells inside a relaxation zone; edge: it has output cells within two
// cells of a side, whose values it also writes into the frame afterwards.
struct RawRow {
    float e, u, v, f, cn0, cn1, th;
};

template <bool PROJ>
__device__ __forceinline__ RawRow load_row(const Dom &d, const float *__restrict__ E, const float *__restrict__ U,
                                           const float *__restrict__ V, int il, int r)
{
    RawRow w;
    const uint32_t off = cell_off(d, r, il);
    const uint32_t cof = corner_off(d, r + 1, il);
    w.e = ld(E, off);
    w.u = ld(U, off);
    w.v = ld(V, off);
    w.f = ld(d.f, off);
    w.cn0 = ld(d.Hc, cof);
    w.cn1 = ld(d.Hc, cof + 1);
    w.th = PROJ ? ld(d.north, off) : 0.f;
    return w;
}

template <int STAGE, bool PROJ, bool W10, bool COMP>
__device__ __forceinline__ void run_tile(const Dom &d, TileCtx c, int y0, int y1, bool frs, bool edge, float &wmax_loc,
                                         BadLanes &bad)
{
    const float *__restrict__ E = STAGE == 1 ? d.eta : d.eta1;
    const float *__restrict__ U = STAGE == 1 ? d.hu : d.hu1;
    const float *__restrict__ V = STAGE == 1 ? d.hv : d.hv1;
    const int il = c.i;
    float cs0, cs1;  // south corners of the row loaded next
    {
        const uint32_t cof = corner_off(d, y0 - 2, il);
        cs0 = ld(d.Hc, cof);
        cs1 = ld(d.Hc, cof + 1);
    }
    const int klast = y1 + 1;
    RawRow nxt = load_row<PROJ>(d, E, U, V, il, y0 - 2);

    // B: the row below C, whose north face depth is C's south one
    auto load = [&](Row &C, const Row &B, int k) {
        RawRow cur = nxt;
        // unconditional (the last row reloads itself), so that the memory
        // counter is the same on every path and a wait for this row's own
        // loads never has to drain the prefetch of the next one
        nxt = load_row<PROJ>(d, E, U, V, il, min(k + 1, klast));
        C.e = cur.e; C.u = cur.u; C.v = cur.v; C.f = cur.f;
        row_terms<PROJ>(C, cs0, cs1, cur.cn0, cur.cn1, B.Hn, cur.th, d);
        cs0 = cur.cn0;
        cs1 = cur.cn1;
    };

    Row R0, R1, R2;
    float uS, vS;
    R2.Hn = 0.5f * (cs0 + cs1);  // the face below the first row
    load(R0, R2, y0 - 2);
    load(R1, R0, y0 - 1);
    y_diff(R1, R0, d);
    load(R2, R1, y0);
    y_diff(R2, R1, d);
    y_faces(R1, R2, R0.land, R0.anyland, d, uS, vS);
    load(R0, R2, y0 + 1);
    y_diff(R0, R2, d);
    y_faces(R2, R0, R1.land, R1.anyland, d, uS, vS);
    F3 Gs = y_flux(R1, R2, uS, vS, d);

    // steady state: A = row k-2 (output), B = row k-1, C = row k
    auto step = [&](Row &A, Row &B, Row &C, int k) {
        c.o = k - 2;
        float e0 = 0.f, u0 = 0.f, v0 = 0.f;
        if (STAGE == 2) {
            const uint32_t oq = cell_off(d, c.o, c.i);
            e0 = ld(d.eta, oq);
            u0 = ld(d.hu, oq);
            v0 = ld(d.hv, oq);
        }
        FrsPre fp;
        fp.zone = false;
        if (STAGE == 2 && frs) {
            int best, dd;
            frs_side(d, c.i, c.o, best, dd);
            fp.zone = c.out_lane && best >= 0 && dd < d.frs_w;
        }
        load(C, B, k);
        y_diff(C, B, d);
        float us, vs;
        y_faces(B, C, A.land, A.anyland, d, us, vs);
        F3 Gn = y_flux(A, B, us, vs, d);
        // a row whose output cells are all land has nothing to update
        if (__ballot(c.out_lane && !A.land) != 0)
            finish_row<STAGE, PROJ, W10, COMP>(A, Gs, Gn, c, e0, u0, v0, fp, d, wmax_loc, bad);
        Gs = Gn;
    };
    for (int k = y0 + 2;;) {
        step(R2, R0, R1, k);
        if (++k > klast) break;
        step(R0, R1, R2, k);
        if (++k > klast) break;
        step(R1, R2, R0, k);
        if (++k > klast) break;
    }
    if (edge) write_frame_nested<STAGE>(d, c, y0, y1);
}

// ---------------------------------------------------------------------------
// time step of one domain (the same in both stage kernels of a step and in
// every wave): dt from the CFL accumulator of the step's parity (eq. cfl) or a
// given dt, clamped to land on t_end, or the step skipped once t_end is reached
// ---------------------------------------------------------------------------
struct StepTime {
    double tn, dtd;
    double tnext;       // time at the start of the next step
    double hold, tupd;  // dt update policy state after this step
    uint32_t wbits;
    bool skip, last;
};

__device__ __forceinline__ StepTime step_time(const Dom &d, int parity, double dt_fixed, int lane)
{
    const Ctrl *ctrl = d.ctrl;
    StepTime s;
    s.tn = ctrl->t[parity];
    s.wbits = read_wmax(ctrl, parity, lane);
    const double te = ctrl->t_end;
    s.dtd = dt_fixed > 0.0 ? dt_fixed : (double)(d.courant_q / __uint_as_float(s.wbits));
    // dt update policy: keep the dt of the last update until the update time
    // is reached, then take the CFL dt and move the update time on by one
    // interval (to one interval past t^n if that is not enough)
    s.hold = ctrl->dt_hold[parity];
    s.tupd = ctrl->t_upd[parity];
    if (dt_fixed <= 0.0 && d.dt_interval > 0.0) {
        if (s.hold > 0.0 && s.tn < s.tupd) {
            s.dtd = s.hold;
        } else {
            s.hold = s.dtd;
            s.tupd += d.dt_interval;
            if (s.tupd <= s.tn) s.tupd = s.tn + d.dt_interval;
        }
    }
    s.skip = false;
    s.last = false;
    if (te > 0.0) {
        if (s.tn >= te) s.skip = true;
        else if (s.dtd >= te - s.tn) { s.dtd = te - s.tn; s.last = true; }
    }
    s.tnext = s.last ? te : s.tn + s.dtd;
    return s;
}

// Done by one wavefront per domain in stage 1: the slots of the next parity
// are cleared for stage 2 to accumulate into (or, for a step past t_end, get
// the current maximum), and the next time is published.
__device__ __forceinline__ void advance_ctrl(Ctrl *ctrl, const StepTime &s, int parity, int lane)
{
    if (lane < kCflSlots) ctrl->wslot[parity ^ 1][lane][0] = s.skip ? s.wbits : 0u;
    if (lane == 0) {
        // a skipped step keeps the policy state; a step clamped to t_end
        // records the dt it would have taken
        ctrl->dt_hold[parity ^ 1] = s.skip ? ctrl->dt_hold[parity] : s.hold;
        ctrl->t_upd[parity ^ 1] = s.skip ? ctrl->t_upd[parity] : s.tupd;
        if (s.skip) {
            ctrl->t[parity ^ 1] = s.tn;
        } else {
            ctrl->t[parity ^ 1] = s.tnext;
            ctrl->dt_last = (float)s.dtd;
            ctrl->steps += 1;
        }
    }
}

// One tile (wavefront) of one stage:
//   STAGE 1: Q* = (Q^n + dt M(Q^n)) / (1 + dt S(Q^n))               (momenta)
//   STAGE 2: Q^{n+1} = (Q^n + Q* + dt M(Q*)) / 2 / (1 + dt/2 S(Q*))  (momenta)
//            then flow relaxation (eq. frs) and the CFL reduction for the
//            next step (eq. cfl)
// eq. rk2_semiimp; M is eq. sw_semidiscrete with the sources of eq. swe.
template <int STAGE, bool PROJ, bool W10, bool COMP>
__device__ __forceinline__ void process_tile(const Dom &d, const Tiling &T, int tile, int parity, const StepTime &st,
                                             int lane)
{
    const double tau = STAGE == 1 ? st.tn : st.tn + st.dtd;
    TileCtx c;
    c.dt = (float)st.dtd;
    c.bk = 0;
    c.bs = 0.0;
    if (d.nb > 0) time_weights(d.nb, d.bnd_t, tau, c.bk, c.bs);
    wind_at(d, tau, c.wx, c.wy);
    c.wk = 0;
    c.ws = 0.f;
    if (d.w10n > 0) {
        double s;
        time_weights(d.w10n, d.w10_t, tau, c.wk, s);
        c.ws = (float)s;
    }

    const int nx = d.nx, ny = d.ny;
    int strip, y0, y1;
    tile_place(T, tile, ny, strip, y0, y1);
    const int x0 = strip * kStrip;
    c.i = x0 - kHalo + lane;
    c.o = y0;
    c.out_lane = lane >= kHalo && lane < kWave - kHalo && c.i < nx;

    // edge: some output cell lies within two cells of a side (its values go
    // into the frame too).  frs: some output cell lies within the relaxation
    // zone of a nested side.
    const bool edge = x0 < kHalo || x0 + kStrip > nx - kHalo || y0 < kHalo || y1 > ny - kHalo;
    const int W = d.frs_w;
    bool frs = false;
    if (W > 0) {
        frs |= d.bc[0] == BC_NESTED && x0 < W;
        frs |= d.bc[1] == BC_NESTED && x0 + kStrip > nx - W;
        frs |= d.bc[2] == BC_NESTED && y0 < W;
        frs |= d.bc[3] == BC_NESTED && y1 > ny - W;
    }
    // nested frame cells are written for the time of the stage that reads
    // them: stage 2 of this step, or stage 1 of the next
    c.fbk = 0;
    c.fbs = 0.0;
    c.edge = edge;
    frame_copy_cols(d, c.i, c.fca, c.fcb);
    if (edge && d.nb > 0) time_weights(d.nb, d.bnd_t, STAGE == 1 ? st.tn + st.dtd : st.tnext, c.fbk, c.fbs);
    float wmax_loc = 0.f;
    BadLanes bad{0, 0};
    // one row loop for every tile (a second variant of it in the same kernel
    // raised the register count of both by ~25 VGPRs): the relaxation zone
    // and the frame writes are uniform branches
    run_tile<STAGE, PROJ, W10, COMP>(d, c, y0, y1, frs, edge, wmax_loc, bad);

    if (STAGE == 2) {
        wmax_loc = wave_max(wmax_loc);
        const uint32_t fl = (bad.nonfinite ? 1u : 0u) | (bad.negative ? 2u : 0u);
        if (lane == 0) {
            atomicMax(&d.ctrl->wslot[parity ^ 1][tile & (kCflSlots - 1)][0], __float_as_uint(wmax_loc));
            if (fl) atomicOr(&d.ctrl->flags, fl);
        }
    }
}

// ---------------------------------------------------------------------------
// single-domain stage kernel: one wavefront per tile
// ---------------------------------------------------------------------------
template <int STAGE, bool PROJ, bool W10, bool COMP>
__global__ __launch_bounds__(kWave * kWavesPerBlock) void stage_kernel(Dom d, Tiling T, int parity,
                                                                      double dt_fixed)
{
    const int lane = threadIdx.x & (kWave - 1);
    // the same in every lane of the wave: read as a scalar, so that the tile's
    // rows and columns, and with them the row offsets, are scalar values
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    // tile of this wave: head blocks before tail blocks, each part grouped
    // per XCD (neighbouring tiles, which share halo rows, meet in one L2)
    const int b = blockIdx.x;
    const int tile = block_tile(T, b, wid);

    const StepTime st = step_time(d, parity, dt_fixed, lane);
    if (STAGE == 1 && b == 0 && wid == 0) advance_ctrl(d.ctrl, st, parity, lane);
    if (st.skip || tile < 0) return;
    process_tile<STAGE, PROJ, W10, COMP>(d, T, tile, parity, st, lane);
}

// ---------------------------------------------------------------------------
// ensemble stage kernel: many domains of uneven sizes in one persistent
// launch.  The work items (member, tile) sit in a device queue split into 8
// partitions; the waves of the blocks b with b % 8 == k drain partition k in
// chunks taken with one atomicAdd each, until the partition is exhausted.
// Every member has its own parameters, time, dt slot and CFL accumulator.
// ---------------------------------------------------------------------------
// Four waves per SIMD for the plain variant (128 VGPRs); the others keep
// the compiler's choice: capped at four, the compensated stage 1 ran 23 %
// slower with the frame copies of its edge items (A/B on the 256-member
// workload at fixed tiles), and the literal-projection and gridded-wind
// variants would spill.
template <int STAGE, bool PROJ, bool W10, bool COMP>
__global__ __launch_bounds__(kWave * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu((PROJ || W10 || COMP) ? 1 : 4)))
void ensemble_kernel(const EnsMember *__restrict__ mem,
                                                                         const EnsItem *__restrict__ items,
                                                                         EnsCtrl *ec, int parity, int chunk)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int part = blockIdx.x & (kEnsParts - 1);
    // reset the queue heads the next kernel of the step sequence will use:
    // stage 1 of parity p clears stage 2 of parity p, stage 2 clears stage 1
    // of parity p^1 (neither is in use while this kernel runs)
    if (blockIdx.x == 0 && threadIdx.x < kEnsParts) {
        if (STAGE == 1) ec->head[1][parity][threadIdx.x][0] = 0u;
        else ec->head[0][parity ^ 1][threadIdx.x][0] = 0u;
    }
    const uint32_t begin = ec->part_begin[part], len = ec->part_len[part];
    uint32_t *head = &ec->head[STAGE - 1][parity][part][0];
    while (true) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(head, (uint32_t)chunk);
        base = __builtin_amdgcn_readfirstlane(base);
        if (base >= len) break;
        const uint32_t end = min(base + (uint32_t)chunk, len);
        for (uint32_t j = base; j < end; ++j) {
            const EnsItem it = items[begin + j];
            const EnsMember &M = mem[it.member];
            const int p = parity ^ M.pflip;
            const StepTime st = step_time(M.d, p, 0.0, lane);
            if (STAGE == 1 && it.tile == 0) advance_ctrl(M.d.ctrl, st, p, lane);
            if (!st.skip) process_tile<STAGE, PROJ, W10, COMP>(M.d, M.T, it.tile, p, st, lane);
        }
    }
}

// ---------------------------------------------------------------------------
// CFL reduction of a given state into the slots of parity `slot` (used at init and
// after a state change); one thread per cell.
// ---------------------------------------------------------------------------
__global__ void cfl_kernel(Dom d, int slot)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    float w = 0.f;
    int bad = 0;
    if (i < d.nx && j < d.ny) {
        const size_t o = cell_off(d, j, i);
        if (!isnan(d.f[o])) {
            const float *H0 = d.Hc + corner_off(d, j, 0), *H1 = H0 + d.cpitch;
            float Hb = 0.25f * ((H0[i] + H1[i]) + (H0[i + 1] + H1[i + 1]));
            float e = d.eta[o], u = d.hu[o], v = d.hv[o];
            float h = e + Hb;
            float ri = rcp(desing(h, d));
            float c = fsqrt(d.g * fmaxf(h, 0.f));
            w = fmaxf((fabsf(u * ri) + c) * d.rdx, (fabsf(v * ri) + c) * d.rdy);
            if (!(isfinite(e) && isfinite(u) && isfinite(v))) bad |= 1;
            if (h < -d.kappa) bad |= 2;
        }
    }
    w = wave_max(w);
    const uint32_t fl = (__ballot(bad & 1) ? 1u : 0u) | (__ballot(bad & 2) ? 2u : 0u);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        int k = (blockIdx.x + blockIdx.y * gridDim.x + (threadIdx.x / kWave)) & (kCflSlots - 1);
        atomicMax(&d.ctrl->wslot[slot][k][0], __float_as_uint(w));
        if (fl) atomicOr(&d.ctrl->flags, fl);
    }
}

// ---------------------------------------------------------------------------
// Frames filled on the host side of the library's calls (init, a new state,
// new boundary data): the static planes (f, north angle, corner depths), and
// the frame of Q^n for the time of the step of a parity.  Afterwards the
// stage kernels keep the state frames current.  Every source is an interior
// cell or corner (col_map / row_map / map_corner), every target a frame cell,
// so no thread reads what another writes.
// ---------------------------------------------------------------------------
__global__ void frame_static_kernel(Dom d)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncell = frame_cells(d);
    float *f = const_cast<float *>(d.f), *north = const_cast<float *>(d.north), *Hc = const_cast<float *>(d.Hc);
    if (k < ncell) {
        int x, y;
        frame_cell(d, k, x, y);
        const GhostSrc g = ghost_src(d, col_map(d, x), x, y);
        float fv, th = 0.f;
        if (g.side >= 0) {
            const uint32_t q = (uint32_t)g.layer * (uint32_t)d.P + (uint32_t)g.idx;
            fv = d.fghost[q];
            if (north) th = d.nghost[q];
        } else {
            fv = flip_sign(f[g.off], (g.flip << 2) & kSign);
            if (north) th = north[g.off];
        }
        const uint32_t o = cell_off(d, y, x);
        f[o] = fv;
        if (north) north[o] = th;
    } else if (k < ncell + frame_corners(d)) {
        int x, y;
        frame_corner(d, k - ncell, x, y);
        const int cx = map_corner(x, d.nx, d.bc[0], d.bc[1]), cy = map_corner(y, d.ny, d.bc[2], d.bc[3]);
        Hc[corner_off(d, y, x)] = Hc[corner_off(d, cy, cx)];
    }
}

__global__ void frame_state_kernel(Dom d, int parity)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= frame_cells(d)) return;
    int x, y;
    frame_cell(d, k, x, y);
    const GhostSrc g = ghost_src(d, col_map(d, x), x, y);
    float e = 0.f, u = 0.f, v = 0.f;
    if (g.side >= 0) {
        if (d.nb > 0) {  // the interpolation of the stage kernels' boundary loads
            int bk;
            double t;
            time_weights(d.nb, d.bnd_t, d.ctrl->t[parity], bk, t);
            const uint32_t P = (uint32_t)d.P;
            const float *pa = d.bnd + (uint32_t)bk * 3u * P + (uint32_t)g.idx;
            const float *pb = d.nb > 1 ? pa + 3u * P : pa;
            e = (float)((1.0 - t) * (double)pa[0] + t * (double)pb[0]);
            u = (float)((1.0 - t) * (double)pa[P] + t * (double)pb[P]);
            v = (float)((1.0 - t) * (double)pa[2u * P] + t * (double)pb[2u * P]);
        }
    } else {
        e = d.eta[g.off];
        u = flip_sign(d.hu[g.off], g.flip & kSign);
        v = flip_sign(d.hv[g.off], (g.flip << 1) & kSign);
    }
    const uint32_t o = cell_off(d, y, x);
    d.eta[o] = e;
    d.hu[o] = u;
    d.hv[o] = v;
}

// control block set-up: time, CFL slot cleared, flags cleared
__global__ void ctrl_reset_kernel(Ctrl *c, double t, int slot)
{
    if (blockIdx.x == 0 && threadIdx.x < kCflSlots) {
        c->wslot[0][threadIdx.x][0] = 0u;
        c->wslot[1][threadIdx.x][0] = 0u;
        if (threadIdx.x == 0) {
            c->t[slot] = t;
            c->t[slot ^ 1] = t;
            c->flags = 0u;
            c->dt_last = 0.f;
            c->t_end = 0.0;
            c->dt_hold[0] = c->dt_hold[1] = 0.0;
            c->t_upd[0] = c->t_upd[1] = t;
        }
    }
}

// dt update policy restarted at the current time of the given parity
__global__ void ctrl_policy_reset_kernel(Ctrl *c, int parity)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->dt_hold[0] = c->dt_hold[1] = 0.0;
        c->t_upd[0] = c->t_upd[1] = c->t[parity];
    }
}

__global__ void ctrl_set_t_end_kernel(Ctrl *c, double te)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) c->t_end = te;
}

// ---------------------------------------------------------------------------
// float64 diagnostics: per-block partial sums in a fixed order, then one
// block adds the partials in order (deterministic).
// ---------------------------------------------------------------------------
constexpr int kDiagThreads = 256;

__global__ __launch_bounds__(kDiagThreads) void diag_partial_kernel(Dom d)
{
    __shared__ double sm[2][kDiagThreads];
    const int j = blockIdx.x;  // one block per row
    double m = 0.0, en = 0.0;
    const double area = d.dx64 * d.dy64;
    for (int i = threadIdx.x; i < d.nx; i += kDiagThreads) {
        const size_t o = cell_off(d, j, i);
        if (isnan(d.f[o])) continue;
        const float *H0 = d.Hc + corner_off(d, j, 0), *H1 = H0 + d.cpitch;
        double Hb = 0.25 * ((double)H0[i] + (double)H0[i + 1] + (double)H1[i] + (double)H1[i + 1]);
        double e = d.eta[o], u = d.hu[o], v = d.hv[o];
        double h = e + Hb;
        double a = fabs(h), kap = d.kappa64;
        double hs = fmax(a, fmin(h * h / (2.0 * kap) + 0.5 * kap, kap));
        hs = h < 0.0 ? -hs : hs;
        m += h * area;
        en += (0.5 * (u * u + v * v) / hs + 0.5 * d.g64 * e * e) * area;
    }
    sm[0][threadIdx.x] = m;
    sm[1][threadIdx.x] = en;
    __syncthreads();
    for (int s = kDiagThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sm[0][threadIdx.x] += sm[0][threadIdx.x + s];
            sm[1][threadIdx.x] += sm[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d.partials[2 * j] = sm[0][0];
        d.partials[2 * j + 1] = sm[1][0];
    }
}

__global__ __launch_bounds__(kDiagThreads) void diag_final_kernel(Dom d)
{
    __shared__ double sm[2][kDiagThreads];
    double m = 0.0, en = 0.0;
    for (int j = threadIdx.x; j < d.ny; j += kDiagThreads) {
        m += d.partials[2 * j];
        en += d.partials[2 * j + 1];
    }
    sm[0][threadIdx.x] = m;
    sm[1][threadIdx.x] = en;
    __syncthreads();
    for (int s = kDiagThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sm[0][threadIdx.x] += sm[0][threadIdx.x + s];
            sm[1][threadIdx.x] += sm[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d.ctrl->mass = sm[0][0];
        d.ctrl->energy = sm[1][0];
    }
}

// ---------------------------------------------------------------------------
// launch wrappers (host side)
// ---------------------------------------------------------------------------
// Kernel variants: stage (1, 2) x literal north projection x gridded wind x
// compensated state.  The wind-field and compensated-state code is compiled
// only into their own variants (it would otherwise raise the register count
// of every launch).
template <int S, bool P, bool W, bool C>
hipError_t launch_stage_v(const Dom &d, const Tiling &T, int parity, double dt_fixed, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1)
{
    dim3 grid(T.nblocks), block(kWave * kWavesPerBlock);
    if (ev0) hipExtLaunchKernelGGL(stage_kernel<S, P, W, C>, grid, block, 0, s, ev0, ev1, 0, d, T, parity, dt_fixed);
    else stage_kernel<S, P, W, C><<<grid, block, 0, s>>>(d, T, parity, dt_fixed);
    return hipGetLastError();
}

template <int S, bool P>
hipError_t launch_stage_pc(bool w, bool c, const Dom &d, const Tiling &T, int parity, double dt_fixed,
                           hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (c) return w ? launch_stage_v<S, P, true, true>(d, T, parity, dt_fixed, s, ev0, ev1)
                    : launch_stage_v<S, P, false, true>(d, T, parity, dt_fixed, s, ev0, ev1);
    return w ? launch_stage_v<S, P, true, false>(d, T, parity, dt_fixed, s, ev0, ev1)
             : launch_stage_v<S, P, false, false>(d, T, parity, dt_fixed, s, ev0, ev1);
}

hipError_t launch_stage(int stage, bool proj, const Dom &d, const Tiling &T, int parity, double dt_fixed,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    const bool w = d.w10n > 0, c = d.eta_lo != nullptr;
    if (stage == 1) return proj ? launch_stage_pc<1, true>(w, c, d, T, parity, dt_fixed, s, ev0, ev1)
                                : launch_stage_pc<1, false>(w, c, d, T, parity, dt_fixed, s, ev0, ev1);
    return proj ? launch_stage_pc<2, true>(w, c, d, T, parity, dt_fixed, s, ev0, ev1)
                : launch_stage_pc<2, false>(w, c, d, T, parity, dt_fixed, s, ev0, ev1);
}

// waves per SIMD that one stage kernel variant can keep resident, from its
// register usage (512 VGPRs per SIMD lane on gfx950, 8-register granules)
int waves_of(const void *f)
{
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, f) != hipSuccess || a.numRegs <= 0) return 3;
    int regs = (a.numRegs + 7) / 8 * 8;
    int w = 512 / regs;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

int stage_waves_per_simd(int stage, bool proj, bool comp)
{
    const void *f;
    if (stage == 1) f = proj ? (comp ? (const void *)stage_kernel<1, true, false, true> : (const void *)stage_kernel<1, true, false, false>)
                             : (comp ? (const void *)stage_kernel<1, false, false, true> : (const void *)stage_kernel<1, false, false, false>);
    else f = proj ? (comp ? (const void *)stage_kernel<2, true, false, true> : (const void *)stage_kernel<2, true, false, false>)
                  : (comp ? (const void *)stage_kernel<2, false, false, true> : (const void *)stage_kernel<2, false, false, false>);
    return waves_of(f);
}

template <int S, bool P, bool W, bool C>
hipError_t launch_ensemble_v(const EnsMember *mem, const EnsItem *items, EnsCtrl *ec, int parity, int chunk,
                             int nblocks, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    dim3 grid(nblocks), block(kWave * kWavesPerBlock);
    if (ev0)
        hipExtLaunchKernelGGL(ensemble_kernel<S, P, W, C>, grid, block, 0, s, ev0, ev1, 0, mem, items, ec, parity, chunk);
    else ensemble_kernel<S, P, W, C><<<grid, block, 0, s>>>(mem, items, ec, parity, chunk);
    return hipGetLastError();
}

template <int S, bool P>
hipError_t launch_ensemble_pc(bool w, bool c, const EnsMember *mem, const EnsItem *items, EnsCtrl *ec, int parity,
                              int chunk, int nblocks, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (c) return w ? launch_ensemble_v<S, P, true, true>(mem, items, ec, parity, chunk, nblocks, s, ev0, ev1)
                    : launch_ensemble_v<S, P, false, true>(mem, items, ec, parity, chunk, nblocks, s, ev0, ev1);
    return w ? launch_ensemble_v<S, P, true, false>(mem, items, ec, parity, chunk, nblocks, s, ev0, ev1)
             : launch_ensemble_v<S, P, false, false>(mem, items, ec, parity, chunk, nblocks, s, ev0, ev1);
}

hipError_t launch_ensemble(int stage, bool proj, bool w10, bool comp, const EnsMember *mem, const EnsItem *items,
                           EnsCtrl *ec, int parity, int chunk, int nblocks, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1)
{
    if (stage == 1)
        return proj ? launch_ensemble_pc<1, true>(w10, comp, mem, items, ec, parity, chunk, nblocks, s, ev0, ev1)
                    : launch_ensemble_pc<1, false>(w10, comp, mem, items, ec, parity, chunk, nblocks, s, ev0, ev1);
    return proj ? launch_ensemble_pc<2, true>(w10, comp, mem, items, ec, parity, chunk, nblocks, s, ev0, ev1)
                : launch_ensemble_pc<2, false>(w10, comp, mem, items, ec, parity, chunk, nblocks, s, ev0, ev1);
}

int ensemble_waves_per_simd(int stage, bool proj, bool comp)
{
    const void *f;
    if (stage == 1) f = proj ? (comp ? (const void *)ensemble_kernel<1, true, false, true> : (const void *)ensemble_kernel<1, true, false, false>)
                             : (comp ? (const void *)ensemble_kernel<1, false, false, true> : (const void *)ensemble_kernel<1, false, false, false>);
    else f = proj ? (comp ? (const void *)ensemble_kernel<2, true, false, true> : (const void *)ensemble_kernel<2, true, false, false>)
                  : (comp ? (const void *)ensemble_kernel<2, false, false, true> : (const void *)ensemble_kernel<2, false, false, false>);
    return waves_of(f);
}

hipError_t launch_cfl(const Dom &d, int slot, hipStream_t s)
{
    dim3 grid((d.nx + 255) / 256, d.ny), block(256);
    cfl_kernel<<<grid, block, 0, s>>>(d, slot);
    return hipGetLastError();
}

hipError_t launch_frame_static(const Dom &d, hipStream_t s)
{
    const int n = frame_cells(d) + frame_corners(d);
    hipLaunchKernelGGL(frame_static_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_frame_state(const Dom &d, int parity, hipStream_t s)
{
    const int n = frame_cells(d);
    hipLaunchKernelGGL(frame_state_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, parity);
    return hipGetLastError();
}

hipError_t launch_ctrl_reset(Ctrl *c, double t, int slot, hipStream_t s)
{
    ctrl_reset_kernel<<<1, 64, 0, s>>>(c, t, slot);
    return hipGetLastError();
}

hipError_t launch_policy_reset(Ctrl *c, int parity, hipStream_t s)
{
    ctrl_policy_reset_kernel<<<1, 64, 0, s>>>(c, parity);
    return hipGetLastError();
}

hipError_t launch_set_t_end(Ctrl *c, double te, hipStream_t s)
{
    ctrl_set_t_end_kernel<<<1, 64, 0, s>>>(c, te);
    return hipGetLastError();
}

hipError_t launch_diagnostics(const Dom &d, hipStream_t s)
{
    diag_partial_kernel<<<d.ny, kDiagThreads, 0, s>>>(d);
    diag_final_kernel<<<1, kDiagThreads, 0, s>>>(d);
    return hipGetLastError();
}

}  // namespace swe
