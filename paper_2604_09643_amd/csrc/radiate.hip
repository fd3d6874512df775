// radiate.hip -- gfx950 kernels and C ABI of the differentiable acoustic radiation model.
//
// Model (main text Eq. (1); kernel from Appendix A, Eq. (A13) with K_G):
//   s[e,k] = sum_v p0[v] * phi(d - c t_k) / (2 d),  phi(u) = u exp(-u^2/(2 sigma^2)),
//   t_k = k/fs, terms kept iff |d - c t_k| <= trunc*sigma, e = f*M + m,
//   x_e = R_f e_m + t_f (rigid array of Stage 4).
//
// GPU formulation (FP32 VALU, no matrix cores: the model is a windowed sum,
// not a contraction).
//   * Voxels are processed in regions: boxes of voxels around a common centre.
//     One workgroup owns one region.  Its four wavefronts take 64-element
//     chunks in turn, one element per lane, and walk the region's voxels in
//     lock-step.  Voxel offsets and p0 values are wave-uniform (loads of a
//     wave-uniform address).
//   * Distances.  Each (region, element) pair gets a reference distance d_c
//     to the region centre, computed in double-float (pairs of FP32 values).
//     Each (voxel, element) pair then forms d_v - d_c from
//     N = |D+o|^2 - |D|^2 = 2 D.o + o.o and one Newton step on
//     y = sqrt(dh^2 + N).  So u = d - c t keeps ~1e-10 m absolute accuracy
//     although d ~ 1e-2 m.
//   * Samples.  Around the centre sample k0 = round(d/delta) with offset
//     u0 = d - k0 delta, the Gaussian of sample k0 +- j factorises as
//     e0 * H^{+-j} * Gamma_j, with e0 = exp(-u0^2/2s^2), H = exp(u0 delta/s^2)
//     and Gamma_j = exp(-j^2 delta^2/2s^2) a per-call table.  So each sample
//     costs one multiply of a running power of H plus one or two FMAs, with
//     no transcendental; two or three exponentials are evaluated per pair.
//   * Forward: every lane owns a private row of signal samples in LDS (layout
//     [sample][lane], bank = lane, no conflicts) and updates it by
//     read-modify-write; two z-neighbouring voxels share one pass over the rows
//     (the Gaussian's rows about each voxel's centre sample are taken whole).
//     At the end of each region the rows are added into the signals with
//     global atomics (transposed, so each atomic instruction covers consecutive
//     samples of one element): FP32 up to 4096 regions, FP64 sums beyond.
//   * Adjoints with the Gaussian (single calls and the batched step): Taylor
//     moments of dL/ds per sample (a table built once per call), two LDS
//     reads and a Horner sum per pair, with its derivative for the element
//     gradients (mom_region).
//   * Adjoints otherwise (other profiles, or where the expansion's bound
//     fails): each lane stages its element's dL/ds window in the same
//     private-row layout and gathers.  dL/dp0 of a voxel is summed across the
//     64 lanes with DPP and across the four wavefronts in LDS.  It is written
//     once, with no atomics.  The element gradient is accumulated per lane in
//     FP64 over the region's voxels.  It goes to a per-region partial buffer,
//     then to a deterministic FP64 reduction over regions and the per-frame
//     chain rule to (dL/dR, dL/dt).
//   * The other source profiles of Appendix A (exponential, power law, uniform
//     sphere) swap the pair functions; the exponential factorises per leg.
//   * Around the model: the Stage 2/4 negative-correlation loss (FP64 row
//     statistics), the TGV regulariser (one LDS-tiled pass), the axis-angle and
//     Euler-angle pose maps, and the batched serving step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>

#include "radiate.h"

// Scratch of radiate_forward_static, for callers that cannot allocate: one copy per device
// (each device that loads the library holds it until the process ends), shared by every call
// on that device.  Host code never passes this name to a kernel: it resolves the device's
// address once (static_scratch_of, at ra_create) and uses that.
constexpr size_t STATIC_SCRATCH_BYTES = RA_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int WAVE = 64;
constexpr int WAVES = 4;              // wavefronts per region workgroup
constexpr int BLOCK = WAVE * WAVES;
constexpr int JMAX = 40;              // largest supported window half-width in samples
constexpr int GEN_STEP = 8;           // spacing of the generic window bounds (8, 16, ..., 40)
#ifdef RA_FAST_BUILD
constexpr int EXP_STEP = 8;           // spacing of the exponential profile's window bounds
#else
constexpr int EXP_STEP = 4;
#endif
constexpr int RS_MAX = 47;            // largest |row - kc| of the row-referenced dL/dp0 adjoint
constexpr int PAIR_D = 3;             // largest centre-sample spread of two voxels the paired forward takes
constexpr int NC_THREADS = 256;       // workgroup of the negative-correlation row kernel
constexpr int NXCD = 8;               // MI355X compute dies; workgroups are dealt round-robin
constexpr int RESID_BLOCKS = 1024;    // partial sums of the loss
constexpr int FWD_F32_MAX_REGIONS = 4096;   // forward regions up to which partial rows are summed in FP32
constexpr size_t LDS_FWD_BUDGET = 80 * 1024;   // forward: two region workgroups per CU
constexpr size_t LDS_ADJ_BUDGET = 80 * 1024;   // adjoint with element gradients: two per CU
constexpr size_t LDS_ADJ0_BUDGET = 53 * 1024;  // adjoint for dL/dp0 only: three per CU
constexpr int NMOM = 8;               // Taylor moments per sample of the moment-form dL/dp0 adjoint
constexpr double MOM_TOL = 1e-6;      // its largest admitted truncation error, relative to the peak
constexpr size_t LDS_MOM_BUDGET = 78 * 1024;   // moment-form adjoint: two region workgroups per CU
constexpr int MOM_WAVES = 8;          // wavefronts of its region workgroup
constexpr int MOM_PER = 5;            // its table rows staged per wavefront and chunk, at most

// ------------------------------------------------------------------------------------------
// double-float arithmetic (value = h + l, |l| <= ulp(h)/2)
// ------------------------------------------------------------------------------------------
// Double-float (hi + lo) arithmetic.  Each helper turns off FMA contraction: fusing a
// product of one step into the sum of the next (e.g. the rounded product of two_prod into the
// quick_two_sum that follows) silently breaks the error-free transformations, leaving FP32
// precision (about one ulp of a 60 mm distance, 4e-9 m).
struct DF {
    float h, l;
};
__device__ __forceinline__ DF two_sum(float a, float b) {
#pragma clang fp contract(off)
    float s = a + b;
    float v = s - a;
    float e = (a - (s - v)) + (b - v);
    return {s, e};
}
__device__ __forceinline__ DF quick_two_sum(float a, float b) {
#pragma clang fp contract(off)
    float s = a + b;
    float e = b - (s - a);
    return {s, e};
}
__device__ __forceinline__ DF two_prod(float a, float b) {
#pragma clang fp contract(off)
    float p = a * b;
    float e = fmaf(a, b, -p);
    return {p, e};
}
__device__ __forceinline__ DF df_add(DF a, DF b) {
#pragma clang fp contract(off)
    DF s = two_sum(a.h, b.h);
    return quick_two_sum(s.h, s.l + (a.l + b.l));
}
__device__ __forceinline__ DF df_neg(DF a) { return {-a.h, -a.l}; }
__device__ __forceinline__ DF df_mul(DF a, DF b) {
#pragma clang fp contract(off)
    DF p = two_prod(a.h, b.h);
    return quick_two_sum(p.h, p.l + (a.h * b.l + a.l * b.h));
}
__device__ __forceinline__ DF df_sqrt(DF a) {
#pragma clang fp contract(off)
    float s = sqrtf(a.h);
    DF p = two_prod(s, s);
    float r = ((a.h - p.h) - p.l) + a.l;
    return quick_two_sum(s, r / (2.0f * s));
}
__device__ __forceinline__ DF df_from_double(double x) {
#pragma clang fp contract(off)
    float h = (float)x;
    return {h, (float)(x - (double)h)};
}

// ------------------------------------------------------------------------------------------
// per-call constants
// ------------------------------------------------------------------------------------------
struct Geo {
    int nx, ny, nz;
    long long vsx, vsy;    // element strides of p0 along x and y (z is contiguous)
    long long gsx, gsy;    // element strides of dL/dp0 along x and y
    int rx, ry, rz;        // region size in voxels
    int nrx, nry, nrz;     // regions per axis
    int nreg;
    int K, E, M, F;
    int jin;               // steps |j| <= jin always lie inside the window
    int jclamp;            // |k0 - kc| bound within a region
    float jclampf;
    int kmargin;           // row index of the region's reference sample kc
    int L;                 // LDS row length in samples
    int nvpad;             // voxels per region, padded to a multiple of 4
    int zero;              // always 0 (keeps table loads per-lane, see forward_region)
    float org_h[3], org_l[3];
    float sp_h, sp_l;
    float dlt_h, dlt_l, inv_dlt;   // sample length delta = c/fs
    float tsig;                    // trunc*sigma
    float kappa;                   // e0 = exp2(kappa * u0^2)
    float alpha;                   // H = exp2(alpha * u0)
    float inv_s2;                  // 1/sigma^2
    float gmin;                    // geometry check: minimum element-to-grid distance
    float edge;                    // JT delta - trunc sigma: sample k0 +- JT is in the window iff +-u0 >= edge
    float gam[JMAX + 1];           // Gamma_j
    float jdg[JMAX + 1];           // j delta Gamma_j
    float jjdg[JMAX + 1];          // (j delta)^2 Gamma_j
    float gamr[RS_MAX + 1];        // Gamma_m = exp(-m^2 delta^2 / 2 sigma^2) by LDS row offset m from kc
    int ktype;                     // source profile, RA_KERNEL_*
    int jwin;                      // other profiles: window half-width in steps (JT = 0 kernels)
    float kexp;                    // exponential: K(x) = exp2(kexp x)
    float kinv_w, kinv_w2;         // 1/w, 1/w^2
    float knu, k2nu;               // power law: K(x) = exp2(knu log2(1 + x^2/w^2)), knu = -nu; 2 nu
    double mom_dd, mom_sigma;      // moment forms: delta / sigma and sigma
};

// Workgroup -> region, so that each compute die (XCD) gets a contiguous run of
// regions: neighbouring regions read overlapping signal windows, which then
// hit in that die's L2.
__device__ __forceinline__ int region_of_block(int b, int nreg) {
    int q = nreg / NXCD, rm = nreg % NXCD;
    int x = b % NXCD, i = b / NXCD;
    return x * q + min(x, rm) + i;
}

struct Region {
    int i0, j0, k0;        // first voxel
    int ni, nj, nk;        // voxels inside the grid
    DF cx, cy, cz;         // centre
};

__device__ __forceinline__ Region region_info(const Geo& g, int reg) {
    Region R;
    int a = reg / (g.nry * g.nrz), b = (reg / g.nrz) % g.nry, c = reg % g.nrz;
    R.i0 = a * g.rx; R.j0 = b * g.ry; R.k0 = c * g.rz;
    R.ni = min(g.rx, g.nx - R.i0); R.nj = min(g.ry, g.ny - R.j0); R.nk = min(g.rz, g.nz - R.k0);
    DF sp{g.sp_h, g.sp_l};
    R.cx = df_add(DF{g.org_h[0], g.org_l[0]}, df_mul(DF{(float)R.i0 + 0.5f * (float)(g.rx - 1), 0.f}, sp));
    R.cy = df_add(DF{g.org_h[1], g.org_l[1]}, df_mul(DF{(float)R.j0 + 0.5f * (float)(g.ry - 1), 0.f}, sp));
    R.cz = df_add(DF{g.org_h[2], g.org_l[2]}, df_mul(DF{(float)R.k0 + 0.5f * (float)(g.rz - 1), 0.f}, sp));
    return R;
}

// Per (region, element) reference: D = centre - x_e, d_c = |D| = dh + dl,
// kc = round(dh/delta), uc0 = d_c - kc*delta.
struct Ref {
    float Dx, Dy, Dz;
    float dh, dh2, uc0;
    float hdh;             // dh / 2
    int kbase;             // sample index of LDS row 0
};

__device__ __forceinline__ Ref make_ref(const Geo& g, const float* __restrict__ xe, int e, const Region& R) {
#pragma clang fp contract(off)
    const float* x = xe + 6 * e;
    DF Dx = df_add(R.cx, df_neg(DF{x[0], x[3]}));
    DF Dy = df_add(R.cy, df_neg(DF{x[1], x[4]}));
    DF Dz = df_add(R.cz, df_neg(DF{x[2], x[5]}));
    DF d2 = df_add(df_add(df_mul(Dx, Dx), df_mul(Dy, Dy)), df_mul(Dz, Dz));
    DF d = df_sqrt(d2);
    float kc = rintf(d.h * g.inv_dlt);
    DF kd = df_add(two_prod(kc, g.dlt_h), DF{kc * g.dlt_l, 0.f});
    DF u = df_add(d, df_neg(kd));
    Ref r;
    r.Dx = Dx.h; r.Dy = Dy.h; r.Dz = Dz.h;
    r.dh = d.h;
    r.dh2 = d.h * d.h;
    r.uc0 = u.h;
    r.hdh = 0.5f * d.h;
    r.kbase = (int)kc - g.kmargin;
    return r;
}

// Per (voxel, element) pair: centre-sample offset j0 (relative to kc), residual u0,
// 1/(2d), and the Gaussian factors e0, H, 1/H.
struct Pair {
    int j0;
    float u0, hr, e0, H, Hi;
};

// Copy a wave-uniform value into a VGPR.
__device__ __forceinline__ float to_vgpr(float x) {
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
    return v;
}

// Per-call constants of the pair loops.  With VG they are copied into vector registers
// once (VALU instructions then read no scalar register), otherwise they stay in scalar
// registers; which is faster depends on the kernel's register pressure and schedule, and
// was measured per kernel.
template <int JT, bool M2>
struct VConst {
    float gam[JT + 1], jdg[JT + 1], jjdg[M2 ? JT + 1 : 1];
    float inv_dlt, dlt_h, dlt_l, kappa, alpha, jclampf, njclampf, edge, nedge, tsig, inv_s2;
};

template <bool VG>
__device__ __forceinline__ float cst_copy(float x) {
    if constexpr (VG) return to_vgpr(x);
    return x;
}

template <bool VG, int JT, bool M2>
__device__ __forceinline__ void load_vconst(VConst<JT, M2>& v, const Geo& g) {
#pragma unroll
    for (int j = 0; j <= JT; ++j) {
        v.gam[j] = cst_copy<VG>(g.gam[j]);
        v.jdg[j] = cst_copy<VG>(g.jdg[j]);
        if (M2) v.jjdg[j] = cst_copy<VG>(g.jjdg[j]);
    }
    v.inv_dlt = cst_copy<VG>(g.inv_dlt);
    v.dlt_h = cst_copy<VG>(g.dlt_h);
    v.dlt_l = cst_copy<VG>(g.dlt_l);
    v.kappa = cst_copy<VG>(g.kappa);
    v.alpha = cst_copy<VG>(g.alpha);
    v.jclampf = cst_copy<VG>(g.jclampf);
    v.njclampf = cst_copy<VG>(-g.jclampf);
    v.edge = cst_copy<VG>(g.edge);
    v.nedge = cst_copy<VG>(-g.edge);
    v.tsig = cst_copy<VG>(g.tsig);
    v.inv_s2 = cst_copy<VG>(g.inv_s2);
}

// Distance part of a pair: uc = d_v - kc delta (compensated), 1/d_v and 1/(2 d_v).  The voxel
// table holds o and |o|^2 / 2, so Nh = D.o + |o|^2/2 = (|D+o|^2 - |D|^2) / 2 is three FMAs; with
// y = sqrt(dh^2 + 2 Nh) ~ d_v, a = y - dh (exact), one Newton step gives d_v - dh = a + (N - a (y
// + dh)) / (2 y), carried here in halves.
struct Dist {
    float uc, rs, hr;
};

__device__ __forceinline__ Dist pair_dist(const Ref& r, float4 o) {
#pragma clang fp contract(off)    // a = y - dh must be exact (Sterbenz) for the Newton step
    const float Nh = fmaf(r.Dx, o.x, fmaf(r.Dy, o.y, fmaf(r.Dz, o.z, o.w)));
    const float S = fmaf(2.0f, Nh, r.dh2);
    Dist q;
    q.rs = __builtin_amdgcn_rsqf(S);          // 1/d_v
    const float y = S * q.rs;                 // ~ d_v
    const float a = y - r.dh;                 // exact (Sterbenz)
    const float bh = fmaf(0.5f, y, r.hdh);    // (y + dh) / 2
    const float th = fmaf(-a, bh, Nh);        // (N - a (y + dh)) / 2
    q.hr = 0.5f * q.rs;                       // 1/(2 d_v)
    q.uc = r.uc0 + fmaf(th, q.rs, a);         // d_v - kc delta
    return q;
}

// Nearest sample offset from kc, as a float.  |j| <= jclamp holds by the triangle
// inequality; the clamp keeps LDS indices in range whatever the inputs (NaN converts to 0).
template <int NJ, bool M2>
__device__ __forceinline__ float centre_step(const VConst<NJ, M2>& c, float uc) {
    return __builtin_amdgcn_fmed3f(rintf(uc * c.inv_dlt), c.njclampf, c.jclampf);
}

// uc - j delta with delta in double-float.
template <int NJ, bool M2>
__device__ __forceinline__ float residual(const VConst<NJ, M2>& c, float uc, float jf) {
    return fmaf(-jf, c.dlt_l, fmaf(-jf, c.dlt_h, uc));
}

template <int JT, bool M2>
__device__ __forceinline__ Pair make_pair(const VConst<JT, M2>& c, const Ref& r, float4 o) {
    const Dist q = pair_dist(r, o);
    const float jf = centre_step(c, q.uc);
    const float u0 = residual(c, q.uc, jf);
    Pair p;
    p.j0 = (int)jf;
    p.u0 = u0;
    p.hr = q.hr;
    p.e0 = __builtin_amdgcn_exp2f(c.kappa * (u0 * u0));
    float au = c.alpha * u0;
    p.H = __builtin_amdgcn_exp2f(au);
    p.Hi = __builtin_amdgcn_exp2f(-au);
    return p;
}

// 64-lane sum; the total lands in lane 63 (other lanes hold partial sums).  Every step writes all
// rows with zeros for lanes without a source, so each folds into one v_add_f32_dpp: after the four
// row shifts lane 15 of a row holds the row's total, and lane 63 then adds lane 47 (row 2) and
// lane 31 (rows 0 and 1).
__device__ __forceinline__ float wave_sum_to_63(float v) {
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x142, 0xf, 0xf, true);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0.0f, v, 0x143, 0xf, 0xf, true);  // row_bcast:31
    return v;
}

// Sums of four values over the 64 lanes, left as one partial per row of 16 lanes: on return lanes
// 12..15 of row r hold row r's sums of v0, v2, v1, v3 (in that order).  Two exchange steps within
// quads leave each lane with one quad sum (lane & 3 = 0, 1, 2, 3: v0, v2, v1, v3), then two row
// shifts add the four quads of a row: 11 VALU for four values where four full sums take 24.
__device__ __forceinline__ float wave_sum4_rows(float v0, float v1, float v2, float v3, int lane) {
    const bool odd = lane & 1, hi2 = lane & 2;
    // quad_perm [1,0,3,2]: even lanes add their odd neighbour's v0 / v1, odd lanes the even one's v2 / v3
    const float s02 = (odd ? v2 : v0) + __builtin_amdgcn_update_dpp(0.0f, odd ? v0 : v2, 0xB1, 0xf, 0xf, true);
    const float s13 = (odd ? v3 : v1) + __builtin_amdgcn_update_dpp(0.0f, odd ? v1 : v3, 0xB1, 0xf, 0xf, true);
    // quad_perm [2,3,0,1]: lanes 0, 1 of a quad keep s02 and add lanes 2, 3's; lanes 2, 3 keep s13
    float s = (hi2 ? s13 : s02) + __builtin_amdgcn_update_dpp(0.0f, hi2 ? s02 : s13, 0x4E, 0xf, 0xf, true);
    s += __builtin_amdgcn_update_dpp(0.0f, s, 0x114, 0xf, 0xf, true);   // row_shr:4
    s += __builtin_amdgcn_update_dpp(0.0f, s, 0x118, 0xf, 0xf, true);   // row_shr:8
    return s;
}

// ------------------------------------------------------------------------------------------
// element positions (prologue) and geometry check
// ------------------------------------------------------------------------------------------
__global__ void k_elements(Geo g, const double* __restrict__ elem, const double* __restrict__ poses,
                           float* __restrict__ xe, int* __restrict__ status, float3 box_lo, float3 box_hi) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.E) return;
    int f = e / g.M, m = e % g.M;
    const double* P = poses + 12 * f;
    const double* em = elem + 3 * m;
    DF ev[3] = {df_from_double(em[0]), df_from_double(em[1]), df_from_double(em[2])};
    float out[6];
    for (int i = 0; i < 3; ++i) {
        DF acc = df_from_double(P[9 + i]);
        for (int j = 0; j < 3; ++j) acc = df_add(acc, df_mul(df_from_double(P[3 * i + j]), ev[j]));
        out[i] = acc.h;
        out[3 + i] = acc.l;
    }
    for (int q = 0; q < 6; ++q) xe[6 * e + q] = out[q];
    float dx = fmaxf(fmaxf(box_lo.x - out[0], out[0] - box_hi.x), 0.f);
    float dy = fmaxf(fmaxf(box_lo.y - out[1], out[1] - box_hi.y), 0.f);
    float dz = fmaxf(fmaxf(box_lo.z - out[2], out[2] - box_hi.z), 0.f);
    if (dx * dx + dy * dy + dz * dz < g.gmin * g.gmin) atomicOr(status, 1);
}

// Voxels of a region, in the order they are visited: offset from the region centre and
// |o|^2 (vtab), and region-relative indices plus the p0 offset from the region's first
// voxel (itab).  Entries past rx*ry*rz (padding to a multiple of 4) sit at the centre
// with index -1, i.e. outside every region.
__global__ void k_voxel_table(Geo g, float4* __restrict__ vtab, int4* __restrict__ itab) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int n = g.rx * g.ry * g.rz;
    if (t >= g.nvpad) return;
    if (t >= n) {
        vtab[t] = make_float4(0.f, 0.f, 0.f, 0.f);
        itab[t] = make_int4(1 << 30, 1 << 30, 1 << 30, 0);
        return;
    }
    int i = t / (g.ry * g.rz), j = (t / g.rz) % g.ry, k = t % g.rz;
    itab[t] = make_int4(i, j, k, (int)(i * g.vsx + j * g.vsy + k));
    DF sp{g.sp_h, g.sp_l};
    float ox = (float)i - 0.5f * (float)(g.rx - 1);
    float oy = (float)j - 0.5f * (float)(g.ry - 1);
    float oz = (float)k - 0.5f * (float)(g.rz - 1);
    DF x = df_mul(DF{ox, 0.f}, sp), y = df_mul(DF{oy, 0.f}, sp), z = df_mul(DF{oz, 0.f}, sp);
    DF oo = df_add(df_add(df_mul(x, x), df_mul(y, y)), df_mul(z, z));
    vtab[t] = make_float4(x.h, y.h, z.h, 0.5f * oo.h);       // |o|^2 / 2
}

__global__ void k_fill(float* __restrict__ p, size_t n, float v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f64(double* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_to_f32(const double* __restrict__ a, size_t n, float* __restrict__ out) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (float)a[i];
}

__global__ void k_copy(const float* __restrict__ a, size_t n, float* __restrict__ out) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = a[i];
}

// Fixed-order FP64 sum of the loss partials (one workgroup of 256 threads, n <= 1024 floats).
__global__ __launch_bounds__(256) void k_loss_total(const float* __restrict__ part, int n,
                                                    double* __restrict__ out) {
    __shared__ double red[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += (double)part[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------------------------------------------
// forward
// ------------------------------------------------------------------------------------------
// With EXACT, JT = floor(T sigma / delta + 1/2) is the largest |j| any pair's window can reach,
// and the Gaussian forward takes the 2 JT + 1 rows about the centre sample whole: every term of
// the window is among them, and the ones they add beyond |u| = T sigma are each below psi(T) of
// the kernel's peak (1.5e-7 at T = 6), below the FP32 rounding of a signal sample, so no row
// carries a window test.  Otherwise JT comes from a list spaced GEN_STEP apart, so every step up
// to JT - GEN_STEP lies inside (the host checks it) and only the last GEN_STEP steps are tested,
// each with a compile-time decision.

// One (voxel, element) pair of the forward model: add p0 * phi(u_k)/(2d) to the lane's
// private LDS row for the 2*JT+1 samples around the centre sample.
template <int JT, bool EXACT>
__device__ __forceinline__ void fwd_pair(const Geo& g, const VConst<JT, false>& c, const Ref& ref, float4 o,
                                         float pv, float* lane_rows) {
    const Pair p = make_pair(c, ref, o);
    const float A = pv * p.hr;
    float Rf = A * p.e0, Rb = Rf;
    float* lo = lane_rows + p.j0 * WAVE;
    float rw[2 * JT + 1];                  // rows j0-JT .. j0+JT: all reads issued first
#pragma unroll
    for (int i = 0; i <= 2 * JT; ++i) rw[i] = lo[i * WAVE];
    rw[JT] = fmaf(p.u0, Rf, rw[JT]);
#pragma unroll
    for (int jj = 1; jj <= JT; ++jj) {
        Rf *= p.H;
        Rb *= p.Hi;
        // (u0 -+ j delta) Gamma_j, one FMA each
        float wf = fmaf(p.u0, c.gam[jj], -c.jdg[jj]), wb = fmaf(p.u0, c.gam[jj], c.jdg[jj]);
        if (!EXACT && jj > JT - GEN_STEP) {
            const float uf = fmaf(-(float)jj, c.dlt_h, p.u0), ub = fmaf((float)jj, c.dlt_h, p.u0);
            wf = fabsf(uf) <= c.tsig ? wf : 0.0f;
            wb = fabsf(ub) <= c.tsig ? wb : 0.0f;
        }
        rw[JT + jj] = fmaf(wf, Rf, rw[JT + jj]);
        rw[JT - jj] = fmaf(wb, Rb, rw[JT - jj]);
    }
#pragma unroll
    for (int i = 0; i <= 2 * JT; ++i) lo[i * WAVE] = rw[i];
}

// Source profiles other than the Gaussian (Appendix A, normalised to K(0) = 1, width w):
// K(x) at x = |u|, and phi'(u) = K(x) + x K'(x) given k = K(x).  KT_POWER2 is the power law
// with nu = 2, K = 1/(1 + x^2/w^2)^2 by one reciprocal instead of a logarithm and an exponential
// (the host picks it when nu is exactly 2).
constexpr int KT_POWER2 = 4;

template <int KT>
__device__ __forceinline__ float prof(const Geo& g, float x) {
    if constexpr (KT == RA_KERNEL_EXPONENTIAL) return __builtin_amdgcn_exp2f(g.kexp * x);
    if constexpr (KT == RA_KERNEL_POWER)
        return __builtin_amdgcn_exp2f(g.knu * __builtin_amdgcn_logf(fmaf(x * x, g.kinv_w2, 1.0f)));
    if constexpr (KT == KT_POWER2) {
        const float r = __builtin_amdgcn_rcpf(fmaf(x * x, g.kinv_w2, 1.0f));
        return r * r;
    }
    return 1.0f;
}

template <int KT>
__device__ __forceinline__ float dprof(const Geo& g, float x, float k) {
    if constexpr (KT == RA_KERNEL_EXPONENTIAL) return k * fmaf(-x, g.kinv_w, 1.0f);
    if constexpr (KT == RA_KERNEL_POWER || KT == KT_POWER2) {
        const float q = x * x * g.kinv_w2;
        return k * fmaf(-g.k2nu * q, __builtin_amdgcn_rcpf(1.0f + q), 1.0f);
    }
    return 1.0f;
}

// One (voxel, element) pair of the forward model for a profile other than the Gaussian.
// These do not factor into a per-pair constant times fixed weights, so every sample of the
// window, |j| <= g.jwin steps from the centre sample, evaluates K(|u|) and its own window
// test |u| <= trunc sigma.  `centre` points at the lane's row of the reference sample kc.
template <int KT>
__device__ __forceinline__ void fwd_pair_var(const Geo& g, const VConst<0, false>& c, const Ref& ref, float4 o,
                                             float pv, float* centre) {
    const Dist q = pair_dist(ref, o);
    const float jf = centre_step(c, q.uc);
    const float u0 = residual(c, q.uc, jf);
    const float A = pv * q.hr;
    float* lo = centre + (int)jf * WAVE;
    const int jw = g.jwin;
#pragma unroll 4
    for (int jj = -jw; jj <= jw; ++jj) {
        const float u = residual(c, u0, (float)jj);      // u0 - jj delta
        const float x = fabsf(u);
        const float t = x <= c.tsig ? u * prof<KT>(g, x) : 0.0f;
        lo[jj * WAVE] = fmaf(A, t, lo[jj * WAVE]);
    }
}

// One pair of the forward model for the exponential profile.  Its exponent is linear in
// |u|, so each leg factors exactly: at step j >= 1 after the centre sample u = u0 - j delta
// < 0 and K = exp(u0/w) G_j, before it u = u0 + j delta > 0 and K = exp(-u0/w) G_j, with
// G_j = exp(-j delta/w) in the per-call table gam[] (jdg[] = j delta G_j).  Each sample then
// costs one FMA for its weight (u0 -+ j delta) G_j and one to accumulate, with no
// recurrence.  JT comes from a list spaced EXP_STEP apart; the last EXP_STEP steps carry their
// own window test.
template <int JT>
__device__ __forceinline__ void fwd_pair_exp(const Geo& g, const VConst<JT, false>& c, const Ref& ref, float4 o,
                                             float pv, float* lane_rows) {
    const Dist q = pair_dist(ref, o);
    const float jf = centre_step(c, q.uc);
    const float u0 = residual(c, q.uc, jf);
    const float A = pv * q.hr;
    const float x0 = u0 * g.kexp;                         // u0/w in log2 units
    const float Rf = A * __builtin_amdgcn_exp2f(-x0);     // A exp(u0/w)
    const float Rb = A * __builtin_amdgcn_exp2f(x0);      // A exp(-u0/w)
    float* lo = lane_rows + (int)jf * WAVE;
    float rw[2 * JT + 1];
#pragma unroll
    for (int i = 0; i <= 2 * JT; ++i) rw[i] = lo[i * WAVE];
    rw[JT] = fmaf(u0 * A, __builtin_amdgcn_exp2f(fabsf(u0) * g.kexp), rw[JT]);
#pragma unroll
    for (int jj = 1; jj <= JT; ++jj) {
        float wf = fmaf(u0, c.gam[jj], -c.jdg[jj]), wb = fmaf(u0, c.gam[jj], c.jdg[jj]);
        if (jj > JT - EXP_STEP) {
            const float uf = fmaf(-(float)jj, c.dlt_h, u0), ub = fmaf((float)jj, c.dlt_h, u0);
            wf = fabsf(uf) <= c.tsig ? wf : 0.0f;
            wb = fabsf(ub) <= c.tsig ? wb : 0.0f;
        }
        rw[JT + jj] = fmaf(wf, Rf, rw[JT + jj]);
        rw[JT - jj] = fmaf(wb, Rb, rw[JT - jj]);
    }
#pragma unroll
    for (int i = 0; i <= 2 * JT; ++i) lo[i * WAVE] = rw[i];
}

// Forward contributions of two neighbouring voxels a, b, added to the rows in one pass.  Both are
// expanded about the smaller of their centre samples, base: with u' = d - (kc + base) delta, the
// kernel value at row base + j is R_j (u' - j delta) Gamma_j with R_j = e0' H'^j (e0' =
// exp(-u'^2/2s^2), H' = exp(u' delta/s^2)), so each row is read and written once for both voxels.
// The voxel whose centre sample is the base ("lo", |u'| <= delta/2) takes its own rows -JT .. JT;
// the other ("hi", u' in [-delta/2, (D + 1/2) delta]) takes rows -JT .. JT + D, which hold its
// own 2 JT + 1 rows; its rows beyond those lie further out than any window row (|u| > (JT + 1/2)
// delta), each below the bound of the whole-row reading above.  Each voxel's R_j is one chain of
// multiplies by H' from row -JT, started at p exp2(u'(kappa u' - JT alpha) - 1) / d (the -1
// halves 1/d to 1/(2d)): two exponentials per voxel.  Requires |j0(a) - j0(b)| <= D, which
// holds when a and b are grid neighbours and spacing < D delta.
template <int JT, int D>
__device__ __forceinline__ void fwd_two(const VConst<JT + D, false>& c, const Ref& ref, float4 oa, float pa,
                                        float4 ob, float pb, float* lane_rows) {
    const Dist A = pair_dist(ref, oa), B = pair_dist(ref, ob);
    const float ja = rintf(A.uc * c.inv_dlt), jb = rintf(B.uc * c.inv_dlt);
    // |j| <= jclamp by the triangle inequality; the clamp keeps LDS indices in range whatever the
    // inputs (NaN converts to 0)
    const float bf = __builtin_amdgcn_fmed3f(fminf(ja, jb), c.njclampf, c.jclampf);
    const float ua = residual(c, A.uc, bf), ub = residual(c, B.uc, bf);
    const bool alo = ja <= jb;
    const float ul = alo ? ua : ub, uh = alo ? ub : ua;
    const float al = alo ? pa * A.rs : pb * B.rs, ah = alo ? pb * B.rs : pa * A.rs;
    const float ctop = -(float)JT * c.alpha;
    const float Hl = __builtin_amdgcn_exp2f(c.alpha * ul), Hh = __builtin_amdgcn_exp2f(c.alpha * uh);
    float Rl = al * __builtin_amdgcn_exp2f(fmaf(ul, fmaf(c.kappa, ul, ctop), -1.0f));
    float Rh = ah * __builtin_amdgcn_exp2f(fmaf(uh, fmaf(c.kappa, uh, ctop), -1.0f));
    float* lo = lane_rows + (int)bf * WAVE;
    constexpr int NR = 2 * JT + 1 + D;
    float rw[NR];                          // rows base-JT .. base+JT+D: all reads issued first
#pragma unroll
    for (int i = 0; i < NR; ++i) rw[i] = lo[i * WAVE];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int j = i - JT;
        // (u' - j delta) Gamma_j, one FMA
        const float wh = j == 0 ? uh : (j > 0 ? fmaf(uh, c.gam[j], -c.jdg[j]) : fmaf(uh, c.gam[-j], c.jdg[-j]));
        if (i > 0) Rh *= Hh;
        if (j <= JT) {
            const float wl = j == 0 ? ul : (j > 0 ? fmaf(ul, c.gam[j], -c.jdg[j]) : fmaf(ul, c.gam[-j], c.jdg[-j]));
            if (i > 0) Rl *= Hl;
            rw[i] = fmaf(wl, Rl, fmaf(wh, Rh, rw[i]));
        } else {
            rw[i] = fmaf(wh, Rh, rw[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) lo[i * WAVE] = rw[i];
}

// The forward work of one region: every element chunk of the region, shared among the
// workgroup's wavefronts (chunks wave, wave + WAVES, ...).  `rows` is the calling
// wavefront's private LDS block of g.L sample rows, zero on entry and on exit.
template <int JT, bool EXACT, int D, typename SumT, int KT = RA_KERNEL_GAUSSIAN>
__device__ __forceinline__ void forward_region(const Geo& g, int reg, const float* __restrict__ p0,
                                               const float* __restrict__ xe, const float4* __restrict__ vtab,
                                               const int4* __restrict__ itab, SumT* __restrict__ s,
                                               float* rows, int lane, int wave) {
    const Region R = region_info(g, reg);
    const float* pbase = p0 + (size_t)R.i0 * g.vsx + (size_t)R.j0 * g.vsy + R.k0;
    const int nchunk = (g.E + WAVE - 1) / WAVE;
    VConst<JT + D, false> cst;
    // per-call constants in VGPRs where the register file allows it (measured faster for the
    // Gaussian up to 24 steps; beyond that they would cost occupancy)
    load_vconst<KT == RA_KERNEL_GAUSSIAN && JT + D <= 27>(cst, g);
    // g.zero is 0: the per-lane index makes the voxel loads vector loads (VGPR results)
    const int zl = lane * g.zero;
    // regions wholly inside the grid whose z-rows hold a multiple of 4 voxels skip the per-voxel
    // bounds tests
    const bool interior = R.ni == g.rx && R.nj == g.ry && R.nk == g.rz && (g.rz & 3) == 0;

    for (int c = wave; c < nchunk; c += WAVES) {
        const int e = c * WAVE + lane;
        const bool valid = e < g.E;
        // lanes past the last element model element 0; their rows are cleared, not flushed
        const Ref ref = make_ref(g, xe, valid ? e : 0, R);
        float* lane_rows = rows + lane + (g.kmargin - JT) * WAVE;
        // voxels four at a time, the next four loading while the current are processed
        float4 oa[4], ob[4];
        float pa[4], pb[4];
        auto fetch = [&](float4* o, float* pv, int t) {
            if (interior) {            // four consecutive voxels along z, all inside the grid
                const int off = itab[t].w;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    o[q] = vtab[t + q + zl];
                    pv[q] = pbase[off + q + zl];
                }
                return;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                o[q] = vtab[t + q + zl];
                const int4 ix = itab[t + q];
                const bool inside = ix.x < R.ni && ix.y < R.nj && ix.z < R.nk;
                const float v = pbase[(inside ? ix.w : 0) + zl];
                pv[q] = inside ? v : 0.0f;
            }
        };
        auto work = [&](const float4* o, const float* pv) {
            if constexpr (KT == RA_KERNEL_EXPONENTIAL) {
#pragma unroll
                for (int q = 0; q < 4; ++q) fwd_pair_exp<JT>(g, cst, ref, o[q], pv[q], lane_rows);
            } else if constexpr (KT != RA_KERNEL_GAUSSIAN) {
#pragma unroll
                for (int q = 0; q < 4; ++q) fwd_pair_var<KT>(g, cst, ref, o[q], pv[q], lane_rows);
            } else if constexpr (D == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) fwd_pair<JT, EXACT>(g, cst, ref, o[q], pv[q], lane_rows);
            } else {
                fwd_two<JT, D>(cst, ref, o[0], pv[0], o[1], pv[1], lane_rows);
                fwd_two<JT, D>(cst, ref, o[2], pv[2], o[3], pv[3], lane_rows);
            }
        };
        fetch(oa, pa, 0);
        for (int t = 0; t < g.nvpad; t += 8) {
            const bool more = t + 4 < g.nvpad;
            if (more) fetch(ob, pb, t + 4);
            work(oa, pa);
            if (!more) break;
            if (t + 8 < g.nvpad) fetch(oa, pa, t + 8);
            work(ob, pb);
        }
        // Add the rows to HBM and clear them.  The single-call forward adds into FP64 sums, so
        // that its rounding does not grow with the number of regions whose partial rows meet in
        // one sample (thousands at 256^3 seen from 60 mm).  Lane ix takes
        // row ix of four elements at a time (one 16-byte LDS access: all lanes read the same four
        // banks, so four elements cost what one did); each atomic instruction covers consecutive
        // samples of one element.
        for (int qb = 0; qb < WAVE; qb += 4) {
            int kb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) kb[i] = __builtin_amdgcn_readlane(ref.kbase, qb + i);
            for (int ix = lane; ix < g.L; ix += WAVE) {
                float4* slot = reinterpret_cast<float4*>(rows + ix * WAVE + qb);
                const float4 v4 = *slot;
                *slot = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                const float v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int eq = c * WAVE + qb + i;
                    const int k = kb[i] + ix;
                    if (eq < g.E && v[i] != 0.0f && k >= 0 && k < g.K)
                        atomicAdd(&s[(size_t)eq * g.K + k], (SumT)v[i]);
                }
            }
        }
    }
}

// SumT: the type the region's partial rows are added into in memory (float: straight into the
// caller's signals; double: FP64 sums converted afterwards).
template <int JT, bool EXACT, int D, int KT = RA_KERNEL_GAUSSIAN, typename SumT = double>
__global__ __launch_bounds__(BLOCK) void k_forward(Geo g, const float* __restrict__ p0,
                                                   const float* __restrict__ xe,
                                                   const float4* __restrict__ vtab,
                                                   const int4* __restrict__ itab,
                                                   SumT* __restrict__ s) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    float* rows = lds + (size_t)wave * g.L * WAVE;
    for (int ix = 0; ix < g.L; ++ix) rows[ix * WAVE + lane] = 0.0f;
    forward_region<JT, EXACT, D, SumT, KT>(g, region_of_block(blockIdx.x, g.nreg), p0, xe, vtab, itab, s, rows,
                                           lane, wave);
}

// ------------------------------------------------------------------------------------------
// adjoint: dL/dp0 and/or per-region element-gradient partials
// ------------------------------------------------------------------------------------------
// Moments of one (voxel, element) pair over its sample window, with r = dL/ds:
//   M0 = sum r e0 H^j G_j,  M1 = sum (j delta) r e0 H^j G_j (sign by side),  M2 = sum (j delta)^2 ...
// so that sum r u e = u0 M0 - M1 and sum r u^2 e = u0^2 M0 - 2 u0 M1 + M2.
struct Moments {
    float M0, M1, M2;
};

template <int JT, bool EXACT, bool WANT_M2>
__device__ __forceinline__ Moments adj_moments(const Geo& g, const VConst<JT, WANT_M2>& c, const Pair& p,
                                               const float* lane_rows) {
    const float* lo = lane_rows + p.j0 * WAVE;
    float rw[2 * JT + 1];                  // the window's residuals, all reads issued first
#pragma unroll
    for (int i = 0; i <= 2 * JT; ++i) rw[i] = lo[i * WAVE];
    // residual at row j0 + jj, zero outside the window
    auto inwin = [&](int jj) -> float {
        const int a = jj < 0 ? -jj : jj;
        float rv = rw[JT + jj];
        if (EXACT && a == JT) {
            rv = (jj > 0 ? p.u0 >= c.edge : p.u0 <= c.nedge) ? rv : 0.0f;
        } else if (!EXACT && a > JT - GEN_STEP) {
            const float uj = fmaf(-(float)jj, c.dlt_h, p.u0);
            rv = fabsf(uj) <= c.tsig ? rv : 0.0f;
        }
        return rv;
    };
    Moments m;
    if constexpr (!WANT_M2) {
        // Both sums by Horner's rule in H (rows j0 + j, j >= 0) and in 1/H (rows j0 - j, j >= 1):
        // P(H) = sum Gamma_j r_j H^j, Q(1/H) = sum Gamma_j r_-j H^-(j-1), with their derivatives,
        // give sum Gamma r H^jj = P + Q/H and sum jj Gamma r H^jj = H P' - (Q + Q'/H)/H.
        float pf = c.gam[JT] * inwin(JT), df = 0.0f;
#pragma unroll
        for (int j = JT - 1; j >= 0; --j) {
            df = fmaf(df, p.H, pf);
            pf = fmaf(pf, p.H, j == 0 ? inwin(0) : c.gam[j] * inwin(j));
        }
        float qb = c.gam[JT] * inwin(-JT), db = 0.0f;
#pragma unroll
        for (int j = JT - 1; j >= 1; --j) {
            db = fmaf(db, p.Hi, qb);
            qb = fmaf(qb, p.Hi, c.gam[j] * inwin(-j));
        }
        m.M0 = p.e0 * fmaf(p.Hi, qb, pf);
        const float gb = p.Hi * fmaf(p.Hi, db, qb);
        m.M1 = (c.dlt_h * p.e0) * fmaf(p.H, df, -gb);
        m.M2 = 0.0f;
        return m;
    }
    float Rf = p.e0, Rb = p.e0;
    m.M0 = rw[JT] * Rf;
    m.M1 = 0.0f;
    m.M2 = 0.0f;
#pragma unroll
    for (int jj = 1; jj <= JT; ++jj) {
        Rf *= p.H;
        Rb *= p.Hi;
        const float rf = inwin(jj), rb = inwin(-jj);
        const float tb = rb * Rb;
        const float sp = fmaf(rf, Rf, tb), sm = fmaf(rf, Rf, -tb);
        m.M0 = fmaf(c.gam[jj], sp, m.M0);
        m.M1 = fmaf(c.jdg[jj], sm, m.M1);
        if (WANT_M2) m.M2 = fmaf(c.jjdg[jj], sp, m.M2);
    }
    return m;
}

// dL/dp0 part of one pair with the Gaussian referenced to the region's sample kc instead of
// the pair's centre.  Row m (from kc) of the window has weight exp(-(uc - m delta)^2 / 2 s^2)
// = E_c Hc^m Gamma_m, with uc = d - kc delta, Hc = exp(uc delta / s^2), E_c = exp(-uc^2 / 2 s^2);
// Gamma_m depends on the row alone and was multiplied into the staged residuals (with the
// lane's power-of-two scale), so that over the window's rows i = 0..2 JT (m = mlow + i)
//   A = sum r phi / K = E_c Hc^mlow [ (uc - mlow delta) S0 - delta S1 ],
//   S0 = sum c_i Hc^i, S1 = sum i c_i Hc^i,
// by Horner's rule in Hc: two FMAs per sample and two exponentials per pair.  The host admits
// this form only where every factor stays inside the FP32 range.  Returns A / (lane scale).
template <int JT>
__device__ __forceinline__ float adj_rowref(const VConst<JT, false>& c, const Ref& ref, float4 o,
                                            const float* lane_rows, float& hr) {
    const Dist q = pair_dist(ref, o);
    const float jf = centre_step(c, q.uc);
    const float u0 = residual(c, q.uc, jf);
    const float* lo = lane_rows + (int)jf * WAVE;
    float rw[2 * JT + 1];
#pragma unroll
    for (int i = 0; i <= 2 * JT; ++i) rw[i] = lo[i * WAVE];
    // the outermost rows j0 -+ JT are inside the window iff u0 <= -edge / u0 >= edge
    rw[0] = u0 <= c.nedge ? rw[0] : 0.0f;
    rw[2 * JT] = u0 >= c.edge ? rw[2 * JT] : 0.0f;
    const float mlow = jf - (float)JT;
    const float xa = c.alpha * q.uc;
    const float Hc = __builtin_amdgcn_exp2f(xa);
    const float pref = __builtin_amdgcn_exp2f(fmaf(c.kappa * q.uc, q.uc, xa * mlow));
    float p = rw[2 * JT], dv = 0.0f;
#pragma unroll
    for (int i = 2 * JT - 1; i >= 0; --i) {
        dv = fmaf(dv, Hc, p);
        p = fmaf(p, Hc, rw[i]);
    }
    const float ulow = residual(c, q.uc, mlow);               // uc - mlow delta
    hr = q.hr;
    return pref * fmaf(ulow, p, -c.dlt_h * (Hc * dv));
}

// Window sums of one pair for a profile other than the Gaussian: A = sum r phi(u) and,
// with WANT_B, B = sum r phi'(u), each sample with its own window test.
struct VarSums {
    float A, B, hr;
};

template <int KT, bool WANT_B>
__device__ __forceinline__ VarSums adj_var(const Geo& g, const VConst<0, WANT_B>& c, const Ref& ref, float4 o,
                                           const float* centre) {
    const Dist q = pair_dist(ref, o);
    const float jf = centre_step(c, q.uc);
    const float u0 = residual(c, q.uc, jf);
    const float* lo = centre + (int)jf * WAVE;
    const int jw = g.jwin;
    VarSums v{0.0f, 0.0f, q.hr};
#pragma unroll 4
    for (int jj = -jw; jj <= jw; ++jj) {
        const float u = residual(c, u0, (float)jj);
        const float x = fabsf(u);
        const float rv = x <= c.tsig ? lo[jj * WAVE] : 0.0f;
        const float k = prof<KT>(g, x);
        v.A = fmaf(rv * u, k, v.A);
        if (WANT_B) v.B = fmaf(rv, dprof<KT>(g, x, k), v.B);
    }
    return v;
}

// Window sums of one pair for the exponential profile, by the leg factorisation of
// fwd_pair_exp: per leg S0 = sum r G_j and S1 = sum r j delta G_j (two FMAs per sample), then
//   A = exp(u0/w) (u0 S0f - S1f) + exp(-u0/w) (u0 S0b + S1b) + r_0 u0 K(|u0|),
//   B = exp(u0/w) ((1 + u0/w) S0f - S1f/w) + exp(-u0/w) ((1 - u0/w) S0b - S1b/w)
//       + r_0 K(|u0|) (1 - |u0|/w),
// from phi'(u) = K(|u|) (1 - |u|/w).
template <int JT, bool WANT_B>
__device__ __forceinline__ VarSums adj_exp(const Geo& g, const VConst<JT, WANT_B>& c, const Ref& ref, float4 o,
                                           const float* lane_rows) {
    const Dist q = pair_dist(ref, o);
    const float jf = centre_step(c, q.uc);
    const float u0 = residual(c, q.uc, jf);
    const float* lo = lane_rows + (int)jf * WAVE;
    float rw[2 * JT + 1];
#pragma unroll
    for (int i = 0; i <= 2 * JT; ++i) rw[i] = lo[i * WAVE];
    float s0f = 0.0f, s1f = 0.0f, s0b = 0.0f, s1b = 0.0f;
#pragma unroll
    for (int jj = 1; jj <= JT; ++jj) {
        float rf = rw[JT + jj], rb = rw[JT - jj];
        if (jj > JT - EXP_STEP) {
            const float uf = fmaf(-(float)jj, c.dlt_h, u0), ub = fmaf((float)jj, c.dlt_h, u0);
            rf = fabsf(uf) <= c.tsig ? rf : 0.0f;
            rb = fabsf(ub) <= c.tsig ? rb : 0.0f;
        }
        s0f = fmaf(rf, c.gam[jj], s0f);
        s1f = fmaf(rf, c.jdg[jj], s1f);
        s0b = fmaf(rb, c.gam[jj], s0b);
        s1b = fmaf(rb, c.jdg[jj], s1b);
    }
    const float x0 = u0 * g.kexp;                         // -u0/w in log2 units
    const float Ef = __builtin_amdgcn_exp2f(-x0), Eb = __builtin_amdgcn_exp2f(x0);
    const float a0 = fabsf(u0);
    const float K0 = __builtin_amdgcn_exp2f(a0 * g.kexp);
    VarSums v;
    v.hr = q.hr;
    v.A = fmaf(Ef, fmaf(u0, s0f, -s1f), fmaf(Eb, fmaf(u0, s0b, s1b), rw[JT] * u0 * K0));
    if (WANT_B) {
        const float iw = g.kinv_w, t = u0 * iw;
        const float bf = fmaf(1.0f + t, s0f, -s1f * iw), bb = fmaf(1.0f - t, s0b, -s1b * iw);
        v.B = fmaf(Ef, bf, fmaf(Eb, bb, rw[JT] * K0 * fmaf(-a0, iw, 1.0f)));
    } else {
        v.B = 0.0f;
    }
    return v;
}

// The adjoint work of one region.  dL/dp0 of each voxel is summed over the element
// chunks of the region in LDS (`gsum`, one array of g.nvpad values per wavefront, then
// across wavefronts) and written once; element gradients go to pose_part[reg][e].
// Contains workgroup barriers: every thread of the workgroup must call it.
template <int JT, bool EXACT, bool WANT_P0, bool WANT_POSE, int KT = RA_KERNEL_GAUSSIAN, bool RS = false>
__device__ __forceinline__ void adjoint_region(const Geo& g, int reg, const float* __restrict__ p0,
                                               const float* __restrict__ xe, const float4* __restrict__ vtab,
                                               const int4* __restrict__ itab, const float* __restrict__ r,
                                               float* __restrict__ grad_p0, int accumulate,
                                               double* __restrict__ pose_part, float* rows, float* gsum_all,
                                               int lane, int wave) {
    float* gsum = gsum_all + (size_t)wave * g.nvpad;
    if (WANT_P0)
        for (int t = lane; t < g.nvpad; t += WAVE) gsum[t] = 0.0f;

    const Region R = region_info(g, reg);
    const float* pbase = p0 ? p0 + (size_t)R.i0 * g.vsx + (size_t)R.j0 * g.vsy + R.k0 : nullptr;
    const int nchunk = (g.E + WAVE - 1) / WAVE;
    VConst<JT, WANT_POSE> cst;
    load_vconst<false>(cst, g);
    const bool interior = R.ni == g.rx && R.nj == g.ry && R.nk == g.rz && (g.rz & 3) == 0;

    for (int c = wave; c < nchunk; c += WAVES) {
        const int e = c * WAVE + lane;
        const bool valid = e < g.E;
        const Ref ref = make_ref(g, xe, valid ? e : 0, R);
        int rs_exp = 0;                    // row-referenced form: the lane's window scale 2^-rs_exp
        {   // stage this lane's window of dL/ds in its private row (zeros past the last element
            // and outside [0, K)); loads go out 16 at a time, clamped into the row, before any
            // is waited for
            const float* rrow = r + (size_t)(valid ? e : 0) * g.K;
            float vmax = 0.0f;
            for (int ix0 = 0; ix0 < g.L; ix0 += 16) {
                float v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int k = min(max(ref.kbase + ix0 + q, 0), g.K - 1);
                    v[q] = rrow[k];
                }
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int ix = ix0 + q, k = ref.kbase + ix;
                    const float x = (valid && k >= 0 && k < g.K) ? v[q] : 0.0f;
                    if (ix < g.L) rows[ix * WAVE + lane] = x;
                    if (RS) vmax = fmaxf(vmax, fabsf(x));
                }
            }
            if constexpr (RS) {
                // row-referenced form: scale the lane's window by a power of two (largest value in
                // [1/2, 1)) and by Gamma of each row's offset from kc
                rs_exp = vmax > 0.0f ? __builtin_amdgcn_frexp_expf(vmax) : 0;
                for (int ix0 = 0; ix0 < g.L; ix0 += 16) {      // 16 rows in flight
                    float v[16];
#pragma unroll
                    for (int q = 0; q < 16; ++q)
                        if (ix0 + q < g.L) v[q] = rows[(ix0 + q) * WAVE + lane];
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        const int ix = ix0 + q, m = ix - g.kmargin;
                        if (ix < g.L)
                            rows[ix * WAVE + lane] = __builtin_amdgcn_ldexpf(v[q], -rs_exp) * g.gamr[m < 0 ? -m : m];
                    }
                }
            }
        }
        const float* lane_rows = rows + lane + (g.kmargin - JT) * WAVE;
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int t = 0; t < g.nvpad; t += 4) {
            float G[4];
            float fx = 0.0f, fy = 0.0f, fz = 0.0f;     // four pairs in FP32, then into FP64
            float pv4[4];
            if (WANT_POSE) {
                if (interior) {                          // four consecutive voxels along z
                    const int off = itab[t].w;
#pragma unroll
                    for (int q = 0; q < 4; ++q) pv4[q] = pbase[off + q];
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int4 ix = itab[t + q];
                        const bool inside = ix.x < R.ni && ix.y < R.nj && ix.z < R.nk;
                        const float v = pbase[inside ? ix.w : 0];
                        pv4[q] = inside ? v : 0.0f;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 o = vtab[t + q];
                float A, B = 0.0f, hr;             // sum_k r phi(u), sum_k r phi'(u), 1/(2d)
                if constexpr (RS) {
                    A = __builtin_amdgcn_ldexpf(adj_rowref<JT>(cst, ref, o, lane_rows, hr), rs_exp);
                } else if constexpr (KT == RA_KERNEL_GAUSSIAN) {
                    const Pair p = make_pair(cst, ref, o);
                    const Moments m = adj_moments<JT, EXACT, WANT_POSE>(g, cst, p, lane_rows);
                    A = fmaf(p.u0, m.M0, -m.M1);                                       // sum r u e
                    if (WANT_POSE) {
                        const float Su2 = fmaf(p.u0, fmaf(p.u0, m.M0, -2.0f * m.M1), m.M2);  // sum r u^2 e
                        B = fmaf(-Su2, cst.inv_s2, m.M0);
                    }
                    hr = p.hr;
                } else {
                    VarSums v;
                    if constexpr (KT == RA_KERNEL_EXPONENTIAL)
                        v = adj_exp<JT, WANT_POSE>(g, cst, ref, o, lane_rows);
                    else
                        v = adj_var<KT, WANT_POSE>(g, cst, ref, o, lane_rows);
                    A = v.A;
                    B = v.B;
                    hr = v.hr;
                }
                G[q] = A * hr;                     // sum_k r phi / (2d); 0 for lanes past the last element
                if (WANT_POSE) {
                    const float pv = pv4[q];
                    const float twohr = 2.0f * hr;                                          // 1/d
                    // p0 (B/(2d) - A/(2d^2)) / d times (x_e - x_v) = -(D + o)
                    const float coef = -pv * hr * twohr * fmaf(-twohr, A, B);
                    fx = fmaf(coef, ref.Dx + o.x, fx);
                    fy = fmaf(coef, ref.Dy + o.y, fy);
                    fz = fmaf(coef, ref.Dz + o.z, fz);
                }
            }
            if (WANT_POSE) {
                gx += (double)fx;
                gy += (double)fy;
                gz += (double)fz;
            }
            if (WANT_P0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) G[q] = wave_sum_to_63(G[q]);
                if (lane == WAVE - 1) {
                    float4* dst = reinterpret_cast<float4*>(gsum + t);
                    float4 a = *dst;
                    a.x += G[0]; a.y += G[1]; a.z += G[2]; a.w += G[3];
                    *dst = a;
                }
            }
        }
        if (WANT_POSE && valid) {
            double* out = pose_part + ((size_t)reg * g.E + e) * 3;
            out[0] = gx; out[1] = gy; out[2] = gz;
        }
    }
    if (WANT_P0) {
        __syncthreads();
        float* gbase = grad_p0 + (size_t)R.i0 * g.gsx + (size_t)R.j0 * g.gsy + R.k0;
        for (int t = threadIdx.x; t < g.nvpad; t += BLOCK) {
            const int4 ix = itab[t];
            if (!(ix.x < R.ni && ix.y < R.nj && ix.z < R.nk)) continue;
            const float v = gsum_all[t] + gsum_all[g.nvpad + t] + gsum_all[2 * g.nvpad + t] +
                            gsum_all[3 * g.nvpad + t];
            float* dst = gbase + ix.x * g.gsx + ix.y * g.gsy + ix.z;
            *dst = accumulate ? *dst + v : v;
        }
        __syncthreads();
    }
}

template <int JT, bool EXACT, bool WANT_P0, bool WANT_POSE, int KT = RA_KERNEL_GAUSSIAN, bool RS = false>
__global__ __launch_bounds__(BLOCK) void k_adjoint(Geo g, const float* __restrict__ p0,
                                                   const float* __restrict__ xe,
                                                   const float4* __restrict__ vtab,
                                                   const int4* __restrict__ itab,
                                                   const float* __restrict__ r,
                                                   float* __restrict__ grad_p0, int accumulate,
                                                   double* __restrict__ pose_part) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    float* rows = lds + (size_t)wave * g.L * WAVE;
    float* gsum = lds + (size_t)WAVES * g.L * WAVE;
    adjoint_region<JT, EXACT, WANT_P0, WANT_POSE, KT, RS>(g, region_of_block(blockIdx.x, g.nreg), p0, xe, vtab,
                                                           itab, r, grad_p0, accumulate, pose_part, rows, gsum,
                                                           lane, wave);
}

// ------------------------------------------------------------------------------------------
// dL/dp0 adjoint in moment form (Gaussian profile)
// ------------------------------------------------------------------------------------------
// Write a pair's distance as d = (kc + x) delta with kc its nearest sample and |x| <= 1/2.  The
// window row kc + j carries phi((x - j) delta) = sigma psi((x - j) Delta), psi(y) = y exp(-y^2/2),
// Delta = delta / sigma.  A Taylor expansion in x about the sample (the local expansion of the fast
// Gauss transform of Greengard and Strain), with psi^(n)(-y) = -He_{n+1}(y) exp(-y^2/2) in the
// probabilists' Hermite polynomials, gives
//   sum_j r[kc + j] phi((x - j) delta) = sum_{n < NMOM} x^n Q_n[kc],
//   Q_n[k] = sum_{|j| <= JT} r[k + j] D_n(j),  D_n(j) = -sigma Delta^n He_{n+1}(j Delta) e^{-(j Delta)^2/2} / n!.
// The tables Q are built once per call from dL/ds; a pair then costs its distance, two LDS reads
// and NMOM - 1 FMAs of Horner's rule instead of a pass over its 2 JT + 1 window rows.  Cramer's
// bound on Hermite functions, |He_m(y)| e^{-y^2/2} <= 1.0865 sqrt(m!), bounds the truncation error
// by 1.791 (Delta/2)^NMOM sqrt((NMOM + 1) / NMOM!) of the kernel's peak; the host takes this form
// only where that is at most MOM_TOL.  Rows are taken whole about kc, so a term with
// T sigma < |u| <= (JT + 1/2) delta (at most psi(T) ~ 1e-7 of the peak at T = 6) is added where the
// exact window leaves it out.

// D_n(j) for n < NMOM and |j| <= jt into c[n (2 jt + 1) + j + jt]; one workgroup of 2 jt + 1 threads.
__global__ void k_moment_coefs(int jt, double dd, double sigma, float* __restrict__ c) {
    const int j = (int)threadIdx.x - jt;
    if (j > jt) return;
    const double y = j * dd;
    const double gy = exp(-0.5 * y * y);
    double hprev = 1.0, h = y;             // He_n(y), He_{n+1}(y)
    double dn = 1.0, fact = 1.0;           // Delta^n, n!
    for (int n = 0; n < NMOM; ++n) {
        c[n * (2 * jt + 1) + j + jt] = (float)(-sigma * dn * h * gy / fact);
        const double hnext = y * h - (double)(n + 1) * hprev;   // He_{n+2} = y He_{n+1} - (n+1) He_n
        hprev = h;
        h = hnext;
        dn *= dd;
        fact *= (double)(n + 1);
    }
}

// Q[e][kk][n] = sum_{|j| <= jt} r[e][kk - jt + j] D_n(j) for table rows kk in [0, K + 2 jt) (sample
// kk - jt), with dL/ds zero outside [0, K); each row is two float4 (n = 0..3, 4..7).  One zero row
// follows the last element's rows.
__global__ __launch_bounds__(256) void k_moment_table(int E, int K, int jt, const float* __restrict__ r,
                                                      const float* __restrict__ coef, float4* __restrict__ q) {
    __shared__ float cs[NMOM * (2 * JMAX + 1)];
    const int nj = 2 * jt + 1;
    for (int i = threadIdx.x; i < NMOM * nj; i += blockDim.x) cs[i] = coef[i];
    __syncthreads();
    const int kq = K + 2 * jt;
    const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (idx == (long long)E * kq) {        // the zero row after the last element's rows
        q[2 * idx] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        q[2 * idx + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    if (idx >= (long long)E * kq) return;
    const int e = (int)(idx / kq), kk = (int)(idx % kq);
    const float* row = r + (size_t)e * K;
    float acc[NMOM];
#pragma unroll
    for (int n = 0; n < NMOM; ++n) acc[n] = 0.0f;
    for (int i = 0; i < nj; ++i) {
        const int k = kk - 2 * jt + i;
        const float v = (k >= 0 && k < K) ? row[k] : 0.0f;
#pragma unroll
        for (int n = 0; n < NMOM; ++n) acc[n] = fmaf(v, cs[n * nj + i], acc[n]);
    }
    q[2 * idx] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    q[2 * idx + 1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
}

// Reference of a (region, element) pair from the element's position x (hi: x[0..2], lo: x[3..5]),
// as make_ref.
__device__ __forceinline__ Ref make_ref_x(const Geo& g, const float* x, const Region& R) {
#pragma clang fp contract(off)
    DF Dx = df_add(R.cx, df_neg(DF{x[0], x[3]}));
    DF Dy = df_add(R.cy, df_neg(DF{x[1], x[4]}));
    DF Dz = df_add(R.cz, df_neg(DF{x[2], x[5]}));
    DF d2 = df_add(df_add(df_mul(Dx, Dx), df_mul(Dy, Dy)), df_mul(Dz, Dz));
    DF d = df_sqrt(d2);
    float kc = rintf(d.h * g.inv_dlt);
    DF kd = df_add(two_prod(kc, g.dlt_h), DF{kc * g.dlt_l, 0.f});
    DF u = df_add(d, df_neg(kd));
    Ref r;
    r.Dx = Dx.h; r.Dy = Dy.h; r.Dz = Dz.h;
    r.dh = d.h;
    r.dh2 = d.h * d.h;
    r.uc0 = u.h;
    r.hdh = 0.5f * d.h;
    r.kbase = (int)kc - g.kmargin;
    return r;
}

// Position of this lane's element in chunk c (the last element past the end).
__device__ __forceinline__ void mom_load_x(const Geo& g, const float* __restrict__ xe, int c, int lane, float* xn) {
    const int e = min(c * WAVE + lane, g.E - 1);
#pragma unroll
    for (int i = 0; i < 6; ++i) xn[i] = xe[6 * e + i];
}

// Four floats as a native vector: copies of it are plain vector moves (no byte copies through
// memory), so arrays of it stay in registers.
typedef float vf4 __attribute__((ext_vector_type(4)));

// Issue the loads of a wavefront's PER table rows (bins b0 .. b0 + nb - 1) of chunk c; rows that do
// not exist or lie outside the table read the zero row after the table.
template <int PER>
__device__ __forceinline__ void mom_fetch(const Geo& g, const vf4* __restrict__ q, int c, int lane,
                                          const Ref& ref, int jt, int b0, int nb, vf4 (&plo)[PER],
                                          vf4 (&phi)[PER]) {
    const int e = c * WAVE + lane;
    const bool valid = e < g.E;
    const int kq = g.K + 2 * jt;
    // table row of bin 0: sample kc - jclamp, with kc = kbase + kmargin
    const int kk0 = ref.kbase + g.kmargin - g.jclamp + jt + b0;
    const vf4* qe = q + (size_t)(valid ? e : 0) * kq * 2;
    const vf4* zrow = q + (size_t)g.E * kq * 2;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int kk = kk0 + i;
        const bool in = valid && i < nb && kk >= 0 && kk < kq;
        const vf4* src = in ? qe + (size_t)kk * 2 : zrow;
        plo[i] = src[0];
        phi[i] = src[1];
    }
}

// dL/dp0 (with WANT_P0) and/or the per-region element gradients (with WANT_POSE) of one region
// from the moment tables; `qw` is the workgroup's LDS.  The workgroup's NW wavefronts take the
// element chunks together: they stage the chunk's table rows for the region's 2 jclamp + 1 centre
// samples in LDS ([bin][half][lane] float4, so a wavefront's reads of one half are 1 KiB
// contiguous), then each sums its own share of the region's voxels (groups of four, dealt
// round-robin) over the 64 elements of the chunk (eight wavefronts measured 27% faster than four:
// more waves to hide the LDS reads and the staging, which each wavefront then does less of).
// Per-voxel sums (one partial per row of 16 lanes) stay in LDS across chunks; no atomics.  Loads
// run ahead of use: a wavefront's PER table rows of the next chunk are fetched into registers while
// the current chunk's voxels run (the voxel loop issues no other vector memory loads; voxel offsets
// come in through scalar loads) and the element positions two chunks ahead.  With WANT_POSE the
// Horner sum runs together with its derivative, A = sum_n x^n Q_n = sum_k r phi(u) and
// A' = dA/dx, so B = sum_k r phi'(u) = A' / delta; the pair adds p0 (B/(2d) - A/(2d^2)) (x_e - x_v)/d
// to its element's gradient (FP32 over four voxels, then FP64 per lane).  At the end of a chunk the
// wavefronts' FP64 partials meet in LDS and are added in wavefront order into the region's partial
// of each element, so the result does not depend on timing.  The derivative of the 8-term
// expansion is a 7-term expansion of phi', within about 1.8 (Delta/2)^7 sqrt(8/7!) of its peak
// (3e-6 on the sweep).
template <int PER, int NW, bool WANT_P0, bool WANT_POSE>
__device__ __forceinline__ void mom_region(const Geo& g, int reg, const float* __restrict__ p0,
                                           const float* __restrict__ xe, const float4* __restrict__ vtab,
                                           const int4* __restrict__ itab, const float4* __restrict__ q, int jt,
                                           float* __restrict__ grad_p0, int accumulate,
                                           double* __restrict__ pose_part, float4* qw) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int nbin = 2 * g.jclamp + 1;
    float* gsum = reinterpret_cast<float*>(qw + (size_t)nbin * 2 * WAVE);   // [row of 16 lanes][voxel]
    double* pbuf = reinterpret_cast<double*>(gsum + (WANT_P0 ? 4 * g.nvpad : 0));  // [wave][3][lane]
    const Region R = region_info(g, reg);
    const float* pbase = p0 ? p0 + (size_t)R.i0 * g.vsx + (size_t)R.j0 * g.vsy + R.k0 : nullptr;
    const bool interior = R.ni == g.rx && R.nj == g.ry && R.nk == g.rz && (g.rz & 3) == 0;
    if (WANT_P0)
        for (int t = threadIdx.x; t < 4 * g.nvpad; t += NW * WAVE) gsum[t] = 0.0f;
    const bool adder = (lane & 15) >= 12;
    const int vsel = (lane & 3) == 1 ? 2 : ((lane & 3) == 2 ? 1 : (lane & 3));
    float* gsum_row = gsum + (size_t)(lane >> 4) * g.nvpad + vsel;
    const int nchunk = (g.E + WAVE - 1) / WAVE;
    const float jcl = g.jclampf, njcl = -g.jclampf;
    const int b0 = wv * PER, nb = max(0, min(nbin - b0, PER));

    const vf4* qv = reinterpret_cast<const vf4*>(q);
    vf4* qwv = reinterpret_cast<vf4*>(qw);
    vf4 plo[PER], phi[PER];
    float xn[6];
    mom_load_x(g, xe, 0, lane, xn);
    Ref ref = make_ref_x(g, xn, R);
    mom_fetch<PER>(g, qv, 0, lane, ref, jt, b0, nb, plo, phi);
    mom_load_x(g, xe, 1, lane, xn);

    for (int c = 0; c < nchunk; ++c) {
        __syncthreads();                 // the previous chunk's rows and partials have been read
        if (WANT_POSE && c > 0 && wv == 0) {   // the previous chunk's element partials, in wavefront order
            const int e = (c - 1) * WAVE + lane;
            double a[3] = {0.0, 0.0, 0.0};
            for (int w = 0; w < NW; ++w)
#pragma unroll
                for (int i = 0; i < 3; ++i) a[i] += pbuf[((size_t)w * 3 + i) * WAVE + lane];
            if (e < g.E) {
                double* out = pose_part + ((size_t)reg * g.E + e) * 3;
                out[0] = a[0]; out[1] = a[1]; out[2] = a[2];
            }
        }
        if (nb > 0) {
            // every row slot is written, in descending order: slots past this wavefront's last bin
            // write zeros to that bin first, which its own row then overwrites
#pragma unroll
            for (int i = PER - 1; i >= 0; --i) {
                const int row = b0 + min(i, nb - 1);
                qwv[(row * 2) * WAVE + lane] = plo[i];
                qwv[(row * 2 + 1) * WAVE + lane] = phi[i];
            }
        }
        __syncthreads();
        const Ref cur = ref;
        if (c + 1 < nchunk) {
            ref = make_ref_x(g, xn, R);
            mom_fetch<PER>(g, qv, c + 1, lane, ref, jt, b0, nb, plo, phi);
            mom_load_x(g, xe, c + 2, lane, xn);
        }
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int t = 4 * wv; t < g.nvpad; t += 4 * NW) {
            float pv4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (WANT_POSE) {
                if (interior) {                      // four consecutive voxels along z
                    const int off = itab[t].w;
#pragma unroll
                    for (int v = 0; v < 4; ++v) pv4[v] = pbase[off + v];
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int4 ix = itab[t + v];
                        const bool inside = ix.x < R.ni && ix.y < R.nj && ix.z < R.nk;
                        const float val = pbase[inside ? ix.w : 0];
                        pv4[v] = inside ? val : 0.0f;
                    }
                }
            }
            float G[4];
            float fx = 0.0f, fy = 0.0f, fz = 0.0f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float4 o = vtab[t + v];
                const Dist d = pair_dist(cur, o);
                const float tt = d.uc * g.inv_dlt;                           // d / delta - kc
                const float jf = __builtin_amdgcn_fmed3f(rintf(tt), njcl, jcl);
                const float x = tt - jf;
                const int b = (int)jf + g.jclamp;
                const float4 m0 = qw[(b * 2) * WAVE + lane], m1 = qw[(b * 2 + 1) * WAVE + lane];
                float h = m1.w, dh = 0.0f;
                if (WANT_POSE) {                     // A and dA/dx together by Horner's rule
                    dh = fmaf(dh, x, h); h = fmaf(h, x, m1.z);
                    dh = fmaf(dh, x, h); h = fmaf(h, x, m1.y);
                    dh = fmaf(dh, x, h); h = fmaf(h, x, m1.x);
                    dh = fmaf(dh, x, h); h = fmaf(h, x, m0.w);
                    dh = fmaf(dh, x, h); h = fmaf(h, x, m0.z);
                    dh = fmaf(dh, x, h); h = fmaf(h, x, m0.y);
                    dh = fmaf(dh, x, h); h = fmaf(h, x, m0.x);
                } else {
                    h = fmaf(h, x, m1.z);
                    h = fmaf(h, x, m1.y);
                    h = fmaf(h, x, m1.x);
                    h = fmaf(h, x, m0.w);
                    h = fmaf(h, x, m0.z);
                    h = fmaf(h, x, m0.y);
                    h = fmaf(h, x, m0.x);
                }
                const float A = h;                                           // sum r phi
                G[v] = A * d.hr;
                if (WANT_POSE) {
                    const float B = dh * g.inv_dlt;                          // sum r phi'
                    const float twohr = 2.0f * d.hr;                         // 1/d
                    // p0 (B/(2d) - A/(2d^2)) / d times (x_e - x_v) = -(D + o)
                    const float coef = -pv4[v] * d.hr * twohr * fmaf(-twohr, A, B);
                    fx = fmaf(coef, cur.Dx + o.x, fx);
                    fy = fmaf(coef, cur.Dy + o.y, fy);
                    fz = fmaf(coef, cur.Dz + o.z, fz);
                }
            }
            if (WANT_POSE) {
                gx += (double)fx;
                gy += (double)fy;
                gz += (double)fz;
            }
            if (WANT_P0) {
                const float part = wave_sum4_rows(G[0], G[1], G[2], G[3], lane);
                if (adder) gsum_row[t] += part;
            }
        }
        if (WANT_POSE) {
            pbuf[((size_t)wv * 3 + 0) * WAVE + lane] = gx;
            pbuf[((size_t)wv * 3 + 1) * WAVE + lane] = gy;
            pbuf[((size_t)wv * 3 + 2) * WAVE + lane] = gz;
        }
    }
    __syncthreads();
    if (WANT_POSE && wv == 0) {          // the last chunk's element partials
        const int e = (nchunk - 1) * WAVE + lane;
        double a[3] = {0.0, 0.0, 0.0};
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int i = 0; i < 3; ++i) a[i] += pbuf[((size_t)w * 3 + i) * WAVE + lane];
        if (e < g.E) {
            double* out = pose_part + ((size_t)reg * g.E + e) * 3;
            out[0] = a[0]; out[1] = a[1]; out[2] = a[2];
        }
    }
    if (WANT_P0) {
        float* gbase = grad_p0 + (size_t)R.i0 * g.gsx + (size_t)R.j0 * g.gsy + R.k0;
        for (int t = threadIdx.x; t < g.nvpad; t += NW * WAVE) {
            const int4 ix = itab[t];
            if (!(ix.x < R.ni && ix.y < R.nj && ix.z < R.nk)) continue;
            const float v = (gsum[t] + gsum[g.nvpad + t]) + (gsum[2 * g.nvpad + t] + gsum[3 * g.nvpad + t]);
            float* dst = gbase + ix.x * g.gsx + ix.y * g.gsy + ix.z;
            *dst = accumulate ? *dst + v : v;
        }
    }
    __syncthreads();                     // the workgroup's LDS is free for the next region
}

// dL/dp0 alone in moment form: one workgroup per region.
template <int PER, int NW>
__global__ __launch_bounds__(NW * WAVE) __attribute__((amdgpu_waves_per_eu(NW / 2))) void k_adjoint_mom(
    Geo g, const float* __restrict__ xe, const float4* __restrict__ vtab, const int4* __restrict__ itab,
    const float4* __restrict__ q, int jt, float* __restrict__ grad_p0, int accumulate) {
    extern __shared__ float4 qw[];
    mom_region<PER, NW, true, false>(g, region_of_block(blockIdx.x, g.nreg), nullptr, xe, vtab, itab, q, jt, grad_p0,
                                     accumulate, nullptr, qw);
}

template <int PER, int NW, bool WANT_P0>
__global__ __launch_bounds__(NW * WAVE) __attribute__((amdgpu_waves_per_eu(NW / 2))) void k_adjoint_mom_pose(
    Geo g, const float* __restrict__ p0, const float* __restrict__ xe, const float4* __restrict__ vtab,
    const int4* __restrict__ itab, const float4* __restrict__ q, int jt, float* __restrict__ grad_p0,
    int accumulate, double* __restrict__ pose_part) {
    extern __shared__ float4 qw[];
    mom_region<PER, NW, WANT_P0, true>(g, region_of_block(blockIdx.x, g.nreg), p0, xe, vtab, itab, q, jt, grad_p0,
                                       accumulate, pose_part, qw);
}

// Sum the per-region element gradients in FP64 and a fixed order: a workgroup takes 16
// consecutive gradient components; its 16 phases each sum every 16th region (loads of 16
// consecutive doubles), then the phases are added in order.
constexpr int PR_T = 16, PR_P = 16;
__global__ __launch_bounds__(PR_T * PR_P) void k_pose_reduce(Geo g, const double* __restrict__ part,
                                                            double* __restrict__ ge, double* __restrict__ grad_elem,
                                                            int accumulate) {
    __shared__ double red[PR_P][PR_T];
    const int tl = threadIdx.x % PR_T, ph = threadIdx.x / PR_T;
    const int n3 = 3 * g.E;
    const int t = blockIdx.x * PR_T + tl;
    double acc = 0.0;
    if (t < n3)
        for (int rg = ph; rg < g.nreg; rg += PR_P) acc += part[(size_t)rg * n3 + t];
    red[ph][tl] = acc;
    __syncthreads();
    if (ph == 0 && t < n3) {
        double sum = 0.0;
        for (int p = 0; p < PR_P; ++p) sum += red[p][tl];
        ge[t] = sum;
        if (grad_elem) grad_elem[t] = accumulate ? grad_elem[t] + sum : sum;
    }
}

// Per frame: dL/dR = sum_m g_e e_m^T, dL/dt = sum_m g_e (FP64 block reduction).
__global__ __launch_bounds__(256) void k_pose_frame(Geo g, const double* __restrict__ ge,
                                                    const double* __restrict__ elem,
                                                    double* __restrict__ grad_pose, int accumulate) {
    __shared__ double red[12][256];
    const int f = blockIdx.x;
    double acc[12];
    for (int q = 0; q < 12; ++q) acc[q] = 0.0;
    for (int m = threadIdx.x; m < g.M; m += blockDim.x) {
        const double* gv = ge + 3 * ((size_t)f * g.M + m);
        const double* em = elem + 3 * m;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) acc[3 * i + j] += gv[i] * em[j];
            acc[9 + i] += gv[i];
        }
    }
    for (int q = 0; q < 12; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 12; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 12) {
        double v = red[threadIdx.x][0];
        double* out = grad_pose + 12 * f + threadIdx.x;
        *out = accumulate ? *out + v : v;
    }
}

// r = 2 (s - y) in place; per-block FP32 partial sums of (s - y)^2.
__global__ __launch_bounds__(256) void k_residual(float* __restrict__ s, const float* __restrict__ y, size_t n,
                                                  float* __restrict__ partial) {
    __shared__ float red[256];
    float acc = 0.0f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        float d = s[i] - y[i];
        acc = fmaf(d, d, acc);
        s[i] = 2.0f * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Stage 2 negative correlation, one workgroup per signal row (one element): the row's
// means, then its spreads and covariance (two passes, FP64 sums), L_e = -Cov/(sigma_s sigma_y),
// and in place dL/ds = w_e (-(y - ybar) / (K sigma_s sigma_y) + Cov (s - sbar) / (K sigma_s^3
// sigma_y)).  A row with zero spread in either signal gets L_e = 0 and a zero gradient.
__device__ __forceinline__ double block_sum_f64(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = NC_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(NC_THREADS) void k_nc_residual(float* __restrict__ s, const float* __restrict__ y,
                                                            const float* __restrict__ weight, int E, int K,
                                                            double* __restrict__ loss_e,
                                                            double* __restrict__ wloss_e) {
    __shared__ double red[NC_THREADS];
    for (int e = blockIdx.x; e < E; e += gridDim.x) {
        float* se = s + (size_t)e * K;
        const float* ye = y + (size_t)e * K;
        double as = 0.0, ay = 0.0;
        for (int k = threadIdx.x; k < K; k += NC_THREADS) {
            as += (double)se[k];
            ay += (double)ye[k];
        }
        const double ms = block_sum_f64(as, red) / K, my = block_sum_f64(ay, red) / K;
        double c = 0.0, vs = 0.0, vy = 0.0;
        for (int k = threadIdx.x; k < K; k += NC_THREADS) {
            const double ds = (double)se[k] - ms, dy = (double)ye[k] - my;
            c = fma(ds, dy, c);
            vs = fma(ds, ds, vs);
            vy = fma(dy, dy, vy);
        }
        const double C = block_sum_f64(c, red) / K;
        const double Vs = block_sum_f64(vs, red) / K, Vy = block_sum_f64(vy, red) / K;
        const double w = weight ? (double)weight[e] : 1.0;
        double a = 0.0, b = 0.0, L = 0.0;
        if (Vs > 0.0 && Vy > 0.0) {
            const double ss = sqrt(Vs), sy = sqrt(Vy);
            L = -C / (ss * sy);
            a = w / (K * ss * sy);
            b = w * C / (K * ss * Vs * sy);
        }
        if (threadIdx.x == 0) {
            if (loss_e) loss_e[e] = L;
            wloss_e[e] = w * L;
        }
        for (int k = threadIdx.x; k < K; k += NC_THREADS) {
            const double ds = (double)se[k] - ms, dy = (double)ye[k] - my;
            se[k] = (float)(fma(b, ds, -a * dy));
        }
    }
}

// Fixed-order FP64 sum of n values into *out (one workgroup).
__global__ __launch_bounds__(NC_THREADS) void k_sum_f64(const double* __restrict__ v, int n,
                                                        double* __restrict__ out) {
    __shared__ double red[NC_THREADS];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += NC_THREADS) a += v[i];
    const double t = block_sum_f64(a, red);
    if (threadIdx.x == 0) *out = t;
}

// Second-order TGV regulariser of the Stage 1 / Stage 5 objectives, for a volume u and its
// auxiliary vector field w, the discretisation written out: alpha1 sum |D+ u - w|_eps + alpha0 sum |E(w)|_eps, D+ forward
// differences (zero at the last index), E(w) = (D-_a w_b + D-_b w_a) / 2 with backward
// differences (zero at the first index), |x|_eps = sqrt(|x|^2 + eps^2) - eps.  With the
// normalised fields q = alpha1 g/|g|_eps (g = D+u - w) and Q = alpha0 E/|E|_eps the gradients are
//   dR/du   = sum_a [q_a(v - e_a) (v_a >= 1) - q_a(v) (v_a <= n_a - 2)],
//   dR/dw_b = -q_b(v) + sum_a [Q_ab(v) (v_a >= 1) - Q_ab(v + e_a) (v_a <= n_a - 2)],
// so a voxel needs q at itself and its three lower neighbours and Q at itself and its three
// upper neighbours: everything within one voxel of it.  One pass computes them from u and w.
struct TgvDims {
    int nx, ny, nz;
    int n, sx, sy;           // voxels (< 2^31); strides of x and y (z contiguous)
    int bz, by, bx;          // tiles along z (64), y (4) and x (TGV_XC planes)
    float a0, a1, eps;
};

// A workgroup owns 64 (z) x 4 (y) columns and marches along TGV_XC x planes, holding three
// planes of u and w with a one-voxel halo in LDS (a ring: plane x + 1 is loaded while x - 1
// and x are still resident), so each input value is read from memory about once per tile.
constexpr int TGV_TZ = 64, TGV_TY = 4, TGV_XC = 8;
constexpr int TGV_LZ = TGV_TZ + 2, TGV_LY = TGV_TY + 2, TGV_PLANE = TGV_LZ * TGV_LY;

struct TgvTile {
    float u[3][TGV_PLANE];
    float w[3][3][TGV_PLANE];     // [component][ring slot][...]
};

__device__ __forceinline__ void tgv_load_plane(const TgvDims& d, const float* __restrict__ u,
                                               const float* __restrict__ w, TgvTile& T, int x, int j0, int k0,
                                               int t) {
    const int slot = (x + 3) % 3;
    for (int q = t; q < TGV_PLANE; q += TGV_TZ * TGV_TY) {
        const int ly = q / TGV_LZ, lz = q % TGV_LZ;
        const int j = j0 + ly - 1, k = k0 + lz - 1;
        float a = 0.0f, b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;
        if (x >= 0 && x < d.nx && j >= 0 && j < d.ny && k >= 0 && k < d.nz) {
            const int v = x * d.sx + j * d.sy + k;
            a = u[v];
            b0 = w[v];
            b1 = w[d.n + v];
            b2 = w[2 * d.n + v];
        }
        T.u[slot][q] = a;
        T.w[0][slot][q] = b0;
        T.w[1][slot][q] = b1;
        T.w[2][slot][q] = b2;
    }
}

// Accessors relative to the voxel (i, j, k) at tile position (ly, lz) of plane slot s0 = i % 3.
struct TgvView {
    const TgvTile* T;
    int s[3];                // ring slots of planes i - 1, i, i + 1
    int q0;                  // LDS index of the voxel within a plane
    __device__ __forceinline__ float U(int dx, int dy, int dz) const {
        return T->u[s[dx + 1]][q0 + dy * TGV_LZ + dz];
    }
    __device__ __forceinline__ float W(int c, int dx, int dy, int dz) const {
        return T->w[c][s[dx + 1]][q0 + dy * TGV_LZ + dz];
    }
};

// g = D+u - w at the voxel offset by (dx, dy, dz) from the view's voxel, whose grid indices are p.
__device__ __forceinline__ void tgv_g(const TgvDims& d, const TgvView& V, int dx, int dy, int dz, const int p[3],
                                      float g[3]) {
    const float u0 = V.U(dx, dy, dz);
    g[0] = (p[0] < d.nx - 1 ? V.U(dx + 1, dy, dz) - u0 : 0.0f) - V.W(0, dx, dy, dz);
    g[1] = (p[1] < d.ny - 1 ? V.U(dx, dy + 1, dz) - u0 : 0.0f) - V.W(1, dx, dy, dz);
    g[2] = (p[2] < d.nz - 1 ? V.U(dx, dy, dz + 1) - u0 : 0.0f) - V.W(2, dx, dy, dz);
}

// E = symmetrised D-w at the offset voxel; components xx yy zz xy xz yz.
__device__ __forceinline__ void tgv_e(const TgvView& V, int dx, int dy, int dz, const int p[3], float E[6]) {
    float D[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            D[a][b] = p[a] > 0 ? V.W(b, dx, dy, dz) - V.W(b, dx - (a == 0), dy - (a == 1), dz - (a == 2)) : 0.0f;
    E[0] = D[0][0];
    E[1] = D[1][1];
    E[2] = D[2][2];
    E[3] = 0.5f * (D[0][1] + D[1][0]);
    E[4] = 0.5f * (D[0][2] + D[2][0]);
    E[5] = 0.5f * (D[1][2] + D[2][1]);
}

// Norms and their reciprocals by the hardware square root and reciprocal (about 1 ulp each;
// the arguments are at least eps^2, far from the denormal range).
__device__ __forceinline__ float tgv_n1(const TgvDims& d, const float g[3]) {
    return __builtin_amdgcn_sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + d.eps * d.eps);
}

__device__ __forceinline__ float tgv_n0(const TgvDims& d, const float E[6]) {
    return __builtin_amdgcn_sqrtf(E[0] * E[0] + E[1] * E[1] + E[2] * E[2] +
                                  2.0f * (E[3] * E[3] + E[4] * E[4] + E[5] * E[5]) + d.eps * d.eps);
}

__device__ __forceinline__ float tgv_ratio(float a, float n) {
    return a * __builtin_amdgcn_rcpf(n);
}

// Value partials (one per workgroup) and, when asked, both gradients, in one pass.
__global__ __launch_bounds__(TGV_TZ * TGV_TY) void k_tgv(TgvDims d, const float* __restrict__ u,
                                                          const float* __restrict__ w, float scale, int accumulate,
                                                          float* __restrict__ gu, float* __restrict__ gw,
                                                          double* __restrict__ partial) {
    __shared__ TgvTile T;
    __shared__ double red[TGV_TZ * TGV_TY];
    // tiles in x order, each compute die (XCD) taking a contiguous run of them so that the
    // halo planes shared with the neighbouring tiles stay in that die's L2
    const int b = region_of_block(blockIdx.x, gridDim.x);
    const int bk = b % d.bz, bj = (b / d.bz) % d.by, bi = b / (d.bz * d.by);
    const int k0 = bk * TGV_TZ, j0 = bj * TGV_TY, x0 = bi * TGV_XC;
    const int x1 = min(x0 + TGV_XC, d.nx);
    const int t = threadIdx.y * TGV_TZ + threadIdx.x;
    const int k = k0 + threadIdx.x, j = j0 + threadIdx.y;
    const bool mine = k < d.nz && j < d.ny;
    double acc = 0.0;
    tgv_load_plane(d, u, w, T, x0 - 1, j0, k0, t);
    tgv_load_plane(d, u, w, T, x0, j0, k0, t);
    for (int i = x0; i < x1; ++i) {
        tgv_load_plane(d, u, w, T, i + 1, j0, k0, t);
        __syncthreads();
        if (mine) {
            TgvView V;
            V.T = &T;
            V.s[0] = (i + 2) % 3;
            V.s[1] = i % 3;
            V.s[2] = (i + 1) % 3;
            V.q0 = (threadIdx.y + 1) * TGV_LZ + threadIdx.x + 1;
            const int v = i * d.sx + j * d.sy + k;
            const int ix[3] = {i, j, k};
            const int nn[3] = {d.nx, d.ny, d.nz};
            float g[3], E[6];
            tgv_g(d, V, 0, 0, 0, ix, g);
            tgv_e(V, 0, 0, 0, ix, E);
            const float n1 = tgv_n1(d, g), n0 = tgv_n0(d, E);
            const float s1 = tgv_ratio(d.a1, n1), s0 = tgv_ratio(d.a0, n0);
            acc += (double)d.a1 * (double)(n1 - d.eps) + (double)d.a0 * (double)(n0 - d.eps);
            if (gu) {
                float gs = 0.0f;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (ix[a] >= 1) {
                        const int pn[3] = {i - (a == 0), j - (a == 1), k - (a == 2)};
                        float gn[3];
                        tgv_g(d, V, -(a == 0), -(a == 1), -(a == 2), pn, gn);
                        gs += tgv_ratio(d.a1, tgv_n1(d, gn)) * gn[a];
                    }
                    if (ix[a] <= nn[a] - 2) gs -= s1 * g[a];
                }
                gu[v] = accumulate ? fmaf(scale, gs, gu[v]) : scale * gs;
            }
            if (gw) {
                // Q_ab as an index into E by (a, b)
                const int qi[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
                float gb[3] = {-(s1 * g[0]), -(s1 * g[1]), -(s1 * g[2])};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    float En[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, sn = 0.0f;
                    const bool up = ix[a] <= nn[a] - 2;
                    if (up) {
                        const int pn[3] = {i + (a == 0), j + (a == 1), k + (a == 2)};
                        tgv_e(V, (a == 0), (a == 1), (a == 2), pn, En);
                        sn = tgv_ratio(d.a0, tgv_n0(d, En));
                    }
#pragma unroll
                    for (int bb = 0; bb < 3; ++bb) {
                        if (ix[a] >= 1) gb[bb] += s0 * E[qi[a][bb]];
                        if (up) gb[bb] -= sn * En[qi[a][bb]];
                    }
                }
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) {
                    float* dst = gw + (size_t)bb * d.n + v;
                    *dst = accumulate ? fmaf(scale, gb[bb], *dst) : scale * gb[bb];
                }
            }
        }
        __syncthreads();          // plane i - 1's slot is overwritten next
    }
    red[t] = acc;
    __syncthreads();
    for (int s2 = TGV_TZ * TGV_TY / 2; s2 > 0; s2 >>= 1) {
        if (t < s2) red[t] += red[t + s2];
        __syncthreads();
    }
    if (t == 0) partial[b] = red[0];
}

static inline unsigned tgv_blocks(int nx, int ny, int nz) {
    return (unsigned)((nz + TGV_TZ - 1) / TGV_TZ) * (unsigned)((ny + TGV_TY - 1) / TGV_TY) *
           (unsigned)((nx + TGV_XC - 1) / TGV_XC);
}

// ------------------------------------------------------------------------------------------
// axis-angle poses.  R = exp([w]x) = I + a [w]x + b [w]x^2, and
// dL/dw = J_r(w)^T vee(R^T G - G^T R) / 1 with J_r the right Jacobian of SO(3):
//   J_r = I - b [w]x + c [w]x^2,  a = sin th/th, b = (1-cos th)/th^2, c = (th - sin th)/th^3.
// ------------------------------------------------------------------------------------------
__device__ void so3_coefs(double th, double& a, double& b, double& c) {
    double t2 = th * th;
    if (th < 0.05) {
        a = 1.0 - t2 / 6.0 * (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0 * (1.0 - t2 / 72.0)));
        b = 0.5 * (1.0 - t2 / 12.0 * (1.0 - t2 / 30.0 * (1.0 - t2 / 56.0 * (1.0 - t2 / 90.0))));
        c = (1.0 / 6.0) * (1.0 - t2 / 20.0 * (1.0 - t2 / 42.0 * (1.0 - t2 / 72.0 * (1.0 - t2 / 110.0))));
    } else {
        double sn = sin(th), cs = cos(th);
        a = sn / th;
        b = (1.0 - cs) / t2;
        c = (th - sn) / (t2 * th);
    }
}

__device__ void so3_exp(const double* w, double* R) {
    const double w0 = w[0], w1 = w[1], w2 = w[2];
    const double th = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    double a, b, c;
    so3_coefs(th, a, b, c);
    const double K[9] = {0, -w2, w1, w2, 0, -w0, -w1, w0, 0};
    const double W[3] = {w0, w1, w2};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double k2 = W[i] * W[j] - (i == j ? th * th : 0.0);  // [w]x^2 = w w^T - th^2 I
            R[3 * i + j] = (i == j ? 1.0 : 0.0) + a * K[3 * i + j] + b * k2;
        }
}

// gw = J_r(w)^T vee(R^T G - G^T R)... with M = R^T G and m = vee(M - M^T).
__device__ void so3_vjp(const double* w, const double* G, double* gw) {
    double R[9];
    so3_exp(w, R);
    const double w0 = w[0], w1 = w[1], w2 = w[2];
    const double th = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
    double a, b, c;
    so3_coefs(th, a, b, c);
    double Mx[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Mx[3 * i + j] = R[i] * G[j] + R[3 + i] * G[3 + j] + R[6 + i] * G[6 + j];
    const double m[3] = {Mx[7] - Mx[5], Mx[2] - Mx[6], Mx[3] - Mx[1]};
    // J_r^T m = m + b [w]x m + c [w]x^2 m
    const double Km[3] = {w1 * m[2] - w2 * m[1], w2 * m[0] - w0 * m[2], w0 * m[1] - w1 * m[0]};
    const double KKm[3] = {w1 * Km[2] - w2 * Km[1], w2 * Km[0] - w0 * Km[2], w0 * Km[1] - w1 * Km[0]};
    for (int i = 0; i < 3; ++i) gw[i] = m[i] + b * Km[i] + c * KKm[i];
}

// Euler angles of Stage 4 (extrinsic x, then y, then z): R = Rz(a2) Ry(a1) Rx(a0).
__device__ void mat3_mul(const double* A, const double* B, double* C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// Elementary rotations about x, y, z and their derivatives with respect to the angle.
__device__ void euler_factors(const double* a, double* Rx, double* Ry, double* Rz, double* Dx, double* Dy,
                              double* Dz) {
    const double cx = cos(a[0]), sx = sin(a[0]), cy = cos(a[1]), sy = sin(a[1]), cz = cos(a[2]), sz = sin(a[2]);
    const double rx[9] = {1, 0, 0, 0, cx, -sx, 0, sx, cx}, dx[9] = {0, 0, 0, 0, -sx, -cx, 0, cx, -sx};
    const double ry[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy}, dy[9] = {-sy, 0, cy, 0, 0, 0, -cy, 0, -sy};
    const double rz[9] = {cz, -sz, 0, sz, cz, 0, 0, 0, 1}, dz[9] = {-sz, -cz, 0, cz, -sz, 0, 0, 0, 0};
    for (int i = 0; i < 9; ++i) {
        Rx[i] = rx[i]; Ry[i] = ry[i]; Rz[i] = rz[i];
        Dx[i] = dx[i]; Dy[i] = dy[i]; Dz[i] = dz[i];
    }
}

__global__ void k_pose_from_euler(const double* __restrict__ pose6, int F, double* __restrict__ poses) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double* p = pose6 + 6 * f;
    double Rx[9], Ry[9], Rz[9], Dx[9], Dy[9], Dz[9], T[9];
    euler_factors(p, Rx, Ry, Rz, Dx, Dy, Dz);
    double* R = poses + 12 * f;
    mat3_mul(Ry, Rx, T);
    mat3_mul(Rz, T, R);
    R[9] = p[3]; R[10] = p[4]; R[11] = p[5];
}

__global__ void k_pose_grad_euler(const double* __restrict__ pose6, const double* __restrict__ gpose, int F,
                                  double* __restrict__ g6) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double* G = gpose + 12 * f;
    double Rx[9], Ry[9], Rz[9], Dx[9], Dy[9], Dz[9], T[9], U[9];
    euler_factors(pose6 + 6 * f, Rx, Ry, Rz, Dx, Dy, Dz);
    double* out = g6 + 6 * f;
    double acc[3];
    mat3_mul(Ry, Dx, T);                   // dR/da0 = Rz Ry Dx
    mat3_mul(Rz, T, U);
    acc[0] = 0.0;
    for (int i = 0; i < 9; ++i) acc[0] += G[i] * U[i];
    mat3_mul(Dy, Rx, T);                   // dR/da1 = Rz Dy Rx
    mat3_mul(Rz, T, U);
    acc[1] = 0.0;
    for (int i = 0; i < 9; ++i) acc[1] += G[i] * U[i];
    mat3_mul(Ry, Rx, T);                   // dR/da2 = Dz Ry Rx
    mat3_mul(Dz, T, U);
    acc[2] = 0.0;
    for (int i = 0; i < 9; ++i) acc[2] += G[i] * U[i];
    out[0] = acc[0]; out[1] = acc[1]; out[2] = acc[2];
    out[3] = G[9]; out[4] = G[10]; out[5] = G[11];
}

__global__ void k_pose_from_aa(const double* __restrict__ pose6, int F, double* __restrict__ poses) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double* p = pose6 + 6 * f;
    double* R = poses + 12 * f;
    so3_exp(p, R);
    R[9] = p[3]; R[10] = p[4]; R[11] = p[5];
}

__global__ void k_pose_grad_aa(const double* __restrict__ pose6, const double* __restrict__ gpose, int F,
                               double* __restrict__ g6) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const double* G = gpose + 12 * f;
    double* out = g6 + 6 * f;
    so3_vjp(pose6 + 6 * f, G, out);
    out[3] = G[9]; out[4] = G[10]; out[5] = G[11];
}

// ------------------------------------------------------------------------------------------
// exact update count (FP64, decided as |d - c*(k/fs)| <= trunc*sigma)
// ------------------------------------------------------------------------------------------
__global__ void k_elements_f64(int M, int E, const double* __restrict__ elem, const double* __restrict__ poses,
                               double* __restrict__ xe) {
#pragma clang fp contract(off)
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    int f = e / M, m = e % M;
    const double* R = poses + 12 * f;
    const double* em = elem + 3 * m;
    for (int i = 0; i < 3; ++i)
        xe[3 * e + i] = R[3 * i + 0] * em[0] + R[3 * i + 1] * em[1] + R[3 * i + 2] * em[2] + R[9 + i];
}

__global__ __launch_bounds__(256) void k_count(int nx, int ny, int nz, double ox, double oy, double oz, double h,
                                               int E, const double* __restrict__ xe, double c, double fs, int K,
                                               double tsig, unsigned long long* __restrict__ total) {
#pragma clang fp contract(off)
    __shared__ unsigned long long red[256];
    long long nvox = (long long)nx * ny * nz;
    long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    unsigned long long cnt = 0;
    if (v < nvox) {
        long long i = v / ((long long)ny * nz), j = (v / nz) % ny, k = v % nz;
        double px = ox + (double)i * h, py = oy + (double)j * h, pz = oz + (double)k * h;
        for (int e = 0; e < E; ++e) {
            double dx = px - xe[3 * e], dy = py - xe[3 * e + 1], dz = pz - xe[3 * e + 2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            long a = (long)ceil((d - tsig) * fs / c) - 1;
            long b = (long)floor((d + tsig) * fs / c) + 1;
            if (a < 0) a = 0;
            if (b > K - 1) b = K - 1;
            while (a <= b && !(fabs(d - c * ((double)a / fs)) <= tsig)) ++a;
            while (b >= a && !(fabs(d - c * ((double)b / fs)) <= tsig)) --b;
            if (b >= a) cnt += (unsigned long long)(b - a + 1);
        }
    }
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(total, red[0]);
}


// ------------------------------------------------------------------------------------------
// issue-rate probes (calibration of the roofline figures): every thread runs PROBE_CHAINS
// independent chains of FP32 FMAs, or of v_exp_f32, so the issue rate, not latency, bounds them
// ------------------------------------------------------------------------------------------
constexpr int PROBE_CHAINS = 8;
constexpr int PROBE_BLOCKS = 4096;

__global__ __launch_bounds__(256) void k_probe_fma(float* __restrict__ out, int iters, float a, float b) {
    float x[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = 1e-3f * (float)(threadIdx.x + c);
#pragma unroll 4
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = fmaf(x[c], a, b);
    float t = 0.0f;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) t += x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_probe_exp(float* __restrict__ out, int iters) {
    float x[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = 1e-3f * (float)(threadIdx.x + c);
#pragma unroll 4
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);    // stays in (1/2, 1]
    float t = 0.0f;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) t += x[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

// ==========================================================================================
// batched steps (serving): one gradient step for every request of a batch, each request
// with its own array size, sample count and box of the resident volume.  Work lists and
// their lengths live in device memory and every launch uses a fixed grid that walks its
// list, so a captured HIP graph replays the step for whatever batch the lists describe.
// ==========================================================================================
constexpr int BATCH_THREADS = 256;

__global__ void k_batch_elements(const Geo* __restrict__ geos, const ra_batch_request* __restrict__ reqs,
                                 const int2* __restrict__ items, const int* __restrict__ counts) {
    const int n = counts[3];
    for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < n; it += gridDim.x * blockDim.x) {
        const int2 w = items[it];
        const ra_batch_request& q = reqs[w.x];
        double R[9];
        so3_exp(q.pose6, R);
        const double* em = q.elem + 3 * w.y;
        const DF ev[3] = {df_from_double(em[0]), df_from_double(em[1]), df_from_double(em[2])};
        float* out = q.xe + 6 * w.y;
        for (int i = 0; i < 3; ++i) {
            DF acc = df_from_double(q.pose6[3 + i]);
            for (int j = 0; j < 3; ++j) acc = df_add(acc, df_mul(df_from_double(R[3 * i + j]), ev[j]));
            out[i] = acc.h;
            out[3 + i] = acc.l;
        }
    }
}

// zero the signal buffer of every request (slot-major, one workgroup per slot at a time)
__global__ void k_batch_zero(const Geo* __restrict__ geos, const ra_batch_request* __restrict__ reqs,
                             const int* __restrict__ counts) {
    const int ns = counts[4];
    for (int slot = blockIdx.x; slot < ns; slot += gridDim.x) {
        if (reqs[slot].kind < 0) continue;      // slot not in this batch
        const Geo& g = geos[slot];
        float* s = reqs[slot].s;
        const int n = g.E * g.K;
        for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] = 0.0f;
    }
}

// r = 2 (s - y) in place and the loss sum (s - y)^2 of every request
__global__ __launch_bounds__(BATCH_THREADS) void k_batch_residual(const Geo* __restrict__ geos,
                                                                  const ra_batch_request* __restrict__ reqs,
                                                                  const int* __restrict__ counts) {
    __shared__ float red[BATCH_THREADS];
    const int ns = counts[4];
    for (int slot = blockIdx.x; slot < ns; slot += gridDim.x) {
        const ra_batch_request& q = reqs[slot];
        if (q.kind < 0) continue;               // slot not in this batch (uniform per block)
        const Geo& g = geos[slot];
        const int n = g.E * g.K;
        float acc = 0.0f;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const float d = q.s[i] - q.y[i];
            acc = fmaf(d, d, acc);
            q.s[i] = 2.0f * d;
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = BATCH_THREADS / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) q.loss[0] = red[0];
        __syncthreads();
    }
}

template <int JT, bool EXACT, int D>
__global__ __launch_bounds__(BLOCK) void k_forward_batch(const Geo* __restrict__ geos,
                                                         const ra_batch_request* __restrict__ reqs,
                                                         const float4* __restrict__ vtab,
                                                         const int4* __restrict__ itab,
                                                         const int2* __restrict__ items,
                                                         const int* __restrict__ counts, int lmax) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    float* rows = lds + (size_t)wave * lmax * WAVE;
    for (int ix = 0; ix < lmax; ++ix) rows[ix * WAVE + lane] = 0.0f;
    const int n = counts[0];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = items[it];
        const ra_batch_request& q = reqs[w.x];
        forward_region<JT, EXACT, D, float>(geos[w.x], w.y, q.p0, q.xe, vtab, itab, q.s, rows, lane, wave);
    }
}

template <int JT, bool EXACT, bool WANT_P0, bool WANT_POSE>
__global__ __launch_bounds__(BLOCK) void k_adjoint_batch(const Geo* __restrict__ geos,
                                                         const ra_batch_request* __restrict__ reqs,
                                                         const float4* __restrict__ vtab,
                                                         const int4* __restrict__ itab,
                                                         const int2* __restrict__ items,
                                                         const int* __restrict__ counts, int which, int lmax) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    float* rows = lds + (size_t)wave * lmax * WAVE;
    float* gsum = lds + (size_t)WAVES * lmax * WAVE;
    const int n = counts[which];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = items[it];
        const ra_batch_request& q = reqs[w.x];
        adjoint_region<JT, EXACT, WANT_P0, WANT_POSE>(geos[w.x], w.y, q.p0, q.xe, vtab, itab, q.s, q.grad_p0, 0,
                                                       q.pose_part, rows, gsum, lane, wave);
    }
}

// Moment form of the batched adjoints (requests sharing the window code, region size and
// moment coefficients).  The coefficients come from the first active slot's descriptor; each
// request's table is built from its own dL/ds into its `q` buffer.
__global__ void k_batch_moment_coefs(const Geo* __restrict__ geos, const ra_batch_request* __restrict__ reqs,
                                     const int* __restrict__ counts, int jt, float* __restrict__ c) {
    const int ns = counts[4];
    int first = -1;
    for (int slot = 0; slot < ns && first < 0; ++slot)
        if (reqs[slot].kind >= 0) first = slot;
    if (first < 0) return;
    const Geo& g = geos[first];
    const int j = (int)threadIdx.x - jt;
    if (j > jt) return;
    const double y = j * g.mom_dd;
    const double gy = exp(-0.5 * y * y);
    double hprev = 1.0, h = y, dn = 1.0, fact = 1.0;
    for (int n = 0; n < NMOM; ++n) {
        c[n * (2 * jt + 1) + j + jt] = (float)(-g.mom_sigma * dn * h * gy / fact);
        const double hnext = y * h - (double)(n + 1) * hprev;
        hprev = h;
        h = hnext;
        dn *= g.mom_dd;
        fact *= (double)(n + 1);
    }
}

__global__ __launch_bounds__(256) void k_batch_moment_table(const Geo* __restrict__ geos,
                                                            const ra_batch_request* __restrict__ reqs,
                                                            const int* __restrict__ counts, int jt,
                                                            const float* __restrict__ coef) {
    __shared__ float cs[NMOM * (2 * JMAX + 1)];
    const int nj = 2 * jt + 1;
    for (int i = threadIdx.x; i < NMOM * nj; i += blockDim.x) cs[i] = coef[i];
    __syncthreads();
    const int ns = counts[4];
    for (int slot = 0; slot < ns; ++slot) {
        const ra_batch_request& rq = reqs[slot];
        if (rq.kind < 0) continue;                         // uniform per block
        const Geo& g = geos[slot];
        const int kq = g.K + 2 * jt;
        const long long nrow = (long long)g.E * kq;
        float4* q = reinterpret_cast<float4*>(rq.q);
        for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx <= nrow;
             idx += (long long)gridDim.x * blockDim.x) {
            if (idx == nrow) {                             // the zero row after the table
                q[2 * idx] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                q[2 * idx + 1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                continue;
            }
            const int e = (int)(idx / kq), kk = (int)(idx % kq);
            const float* row = rq.s + (size_t)e * g.K;     // dL/ds after k_batch_residual
            float acc[NMOM];
#pragma unroll
            for (int n = 0; n < NMOM; ++n) acc[n] = 0.0f;
            for (int i = 0; i < nj; ++i) {
                const int k = kk - 2 * jt + i;
                const float v = (k >= 0 && k < g.K) ? row[k] : 0.0f;
#pragma unroll
                for (int n = 0; n < NMOM; ++n) acc[n] = fmaf(v, cs[n * nj + i], acc[n]);
            }
            q[2 * idx] = make_float4(acc[0], acc[1], acc[2], acc[3]);
            q[2 * idx + 1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
        }
    }
}

// which: 1 = pose requests (element gradients), 2 = volume requests (dL/dp0).  The LDS window was
// sized for nbin bins; a request whose window needs more (a descriptor from another batch layout)
// is skipped rather than overrun it.
template <bool WANT_P0, bool WANT_POSE>
__global__ __launch_bounds__(MOM_WAVES * WAVE) __attribute__((amdgpu_waves_per_eu(MOM_WAVES / 2)))
void k_adjoint_mom_batch(const Geo* __restrict__ geos, const ra_batch_request* __restrict__ reqs,
                         const float4* __restrict__ vtab, const int4* __restrict__ itab,
                         const int2* __restrict__ items, const int* __restrict__ counts, int which, int jt,
                         int nbin) {
    extern __shared__ float4 qw[];
    const int n = counts[which];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = items[it];
        if (2 * geos[w.x].jclamp + 1 > nbin) continue;     // uniform per workgroup
        const ra_batch_request& rq = reqs[w.x];
        mom_region<MOM_PER, MOM_WAVES, WANT_P0, WANT_POSE>(geos[w.x], w.y, rq.p0, rq.xe, vtab, itab,
                                                           reinterpret_cast<const float4*>(rq.q), jt, rq.grad_p0, 0,
                                                           rq.pose_part, qw);
    }
}

// Pose requests: element gradients summed over regions (FP64, fixed order), chained to
// (dL/dR, dL/dt), then to (dL/dw, dL/dt), followed by one Adam step on the pose.
// First stage of the pose update: the per-region element gradients of a pose request are
// summed in POSE_CHUNKS fixed chunks of regions, each over the chunk's first row (FP64, in
// region order), so that the per-request stage below adds POSE_CHUNKS rows instead of
// nreg.  Work items run over (chunk, element) with the element fastest (coalesced rows).
constexpr int POSE_CHUNKS = 32;
__global__ void k_batch_pose_chunks(const Geo* __restrict__ geos, const ra_batch_request* __restrict__ reqs,
                                    const int2* __restrict__ items, const int* __restrict__ counts) {
    const int ne = counts[3];
    const long long n = (long long)ne * POSE_CHUNKS;
    for (long long it = blockIdx.x * (long long)blockDim.x + threadIdx.x; it < n;
         it += (long long)gridDim.x * blockDim.x) {
        const int2 w = items[it % ne];
        const int c = (int)(it / ne);
        const ra_batch_request& q = reqs[w.x];
        if (q.kind != RA_REQ_POSE) continue;
        const Geo& g = geos[w.x];
        const int cs = (q.nreg + POSE_CHUNKS - 1) / POSE_CHUNKS;
        const int r0 = c * cs, r1 = min(r0 + cs, q.nreg);
        if (r0 >= r1) continue;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int rg = r0; rg < r1; ++rg) {
            const double* pp = q.pose_part + ((size_t)rg * g.E + w.y) * 3;
            a0 += pp[0]; a1 += pp[1]; a2 += pp[2];
        }
        double* out = q.pose_part + ((size_t)r0 * g.E + w.y) * 3;
        out[0] = a0; out[1] = a1; out[2] = a2;
    }
}

__global__ __launch_bounds__(BATCH_THREADS) void k_batch_pose_update(const Geo* __restrict__ geos,
                                                                     const ra_batch_request* __restrict__ reqs,
                                                                     const int* __restrict__ counts) {
    __shared__ double red[12][BATCH_THREADS];
    const int ns = counts[4];
    for (int slot = blockIdx.x; slot < ns; slot += gridDim.x) {
        const ra_batch_request& q = reqs[slot];
        if (q.kind != RA_REQ_POSE) continue;
        const Geo& g = geos[slot];
        double acc[12];
        for (int i = 0; i < 12; ++i) acc[i] = 0.0;
        const int cs = (q.nreg + POSE_CHUNKS - 1) / POSE_CHUNKS;      // chunk sums from k_batch_pose_chunks
        for (int m = threadIdx.x; m < g.M; m += blockDim.x) {
            double ge[3] = {0.0, 0.0, 0.0};
            for (int rg = 0; rg < q.nreg; rg += cs) {
                const double* pp = q.pose_part + ((size_t)rg * g.E + m) * 3;
                ge[0] += pp[0]; ge[1] += pp[1]; ge[2] += pp[2];
            }
            const double* em = q.elem + 3 * m;
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) acc[3 * i + j] += ge[i] * em[j];
                acc[9 + i] += ge[i];
            }
        }
        for (int i = 0; i < 12; ++i) red[i][threadIdx.x] = acc[i];
        __syncthreads();
        for (int w = BATCH_THREADS / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                for (int i = 0; i < 12; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double G[9], g6[6];
            for (int i = 0; i < 9; ++i) G[i] = red[i][0];
            so3_vjp(q.pose6, G, g6);
            g6[3] = red[9][0]; g6[4] = red[10][0]; g6[5] = red[11][0];
            double* st = q.adam;                 // m[6], v[6], step
            const double b1 = 0.9, b2 = 0.999, eps = 1e-8;     // torch.optim.Adam's defaults
            const double t = st[12] + 1.0;
            st[12] = t;
            const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
            for (int i = 0; i < 6; ++i) {
                st[i] = b1 * st[i] + (1.0 - b1) * g6[i];
                st[6 + i] = b2 * st[6 + i] + (1.0 - b2) * g6[i] * g6[i];
                const double lr = i < 3 ? q.lr_w : q.lr_t;
                q.pose6[i] -= lr * (st[i] / c1) / (sqrt(st[6 + i] / c2) + eps);
            }
        }
        __syncthreads();
    }
}

// Volume requests: p0 -= lr * dL/dp0 over the request's box (atomic: boxes may overlap).
__global__ __launch_bounds__(BLOCK) void k_batch_volume_apply(const Geo* __restrict__ geos,
                                                              const ra_batch_request* __restrict__ reqs,
                                                              const int4* __restrict__ itab,
                                                              const int2* __restrict__ items,
                                                              const int* __restrict__ counts) {
    const int n = counts[2];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int2 w = items[it];
        const Geo& g = geos[w.x];
        const ra_batch_request& q = reqs[w.x];
        const Region R = region_info(g, w.y);
        float* pbase = q.p0 + (size_t)R.i0 * g.vsx + (size_t)R.j0 * g.vsy + R.k0;
        const float* gbase = q.grad_p0 + (size_t)R.i0 * g.gsx + (size_t)R.j0 * g.gsy + R.k0;
        const float lr = (float)q.lr_w;
        for (int t = threadIdx.x; t < g.nvpad; t += blockDim.x) {
            const int4 ix = itab[t];
            if (!(ix.x < R.ni && ix.y < R.nj && ix.z < R.nk)) continue;
            atomicAdd(pbase + ix.w, -lr * gbase[ix.x * g.gsx + ix.y * g.gsy + ix.z]);
        }
    }
}

}  // namespace

// ==============================================================================================
// host side
// ==============================================================================================
struct ra_ctx {
    int device = 0;
    int* d_status = nullptr;
    char* arena = nullptr;                  // the context's scratch (grown by ensure_scratch)
    size_t arena_bytes = 0;
    char* static_scratch = nullptr;         // this device's static array (radiate_forward_static)
    unsigned long long* h_count = nullptr;  // pinned
    double* h_f64 = nullptr;                // pinned, one value
    double* d_f64 = nullptr;                // device, one value
    int sums_mode = RA_SUMS_AUTO;           // how the forward adds its partial rows (ra_set_forward_sums)
    std::string err;
};

namespace {

int fail(ra_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return code;
}

#define RA_HIP(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, RA_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Window half-widths with a kernel compiled for exactly that many steps.  Others run
// the next larger generic kernel, which tests its last GEN_STEP steps.
#ifdef RA_FAST_BUILD
#define RA_EXACT_LIST(X) X(12) X(16)
#else
#define RA_EXACT_LIST(X) \
    X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24)
#endif
#define RA_GENERIC_LIST(X) X(8) X(16) X(24) X(32) X(40)
#ifdef RA_FAST_BUILD
#define RA_EXP_LIST(X) X(8) X(16) X(24) X(32) X(40)
#else
#define RA_EXP_LIST(X) X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(36) X(40)
#endif
// Window bounds of the per-sample kernels of the other source profiles.

void choose_jt(int jout, int& jt, bool& exact) {
#define RA_TRY_EXACT(n) \
    if (jout == n) {    \
        jt = n;         \
        exact = true;   \
        return;         \
    }
    RA_EXACT_LIST(RA_TRY_EXACT)
#undef RA_TRY_EXACT
    exact = false;
    jt = -1;
#define RA_TRY_GENERIC(n) \
    if (jt < 0 && jout <= n) jt = n;
    RA_GENERIC_LIST(RA_TRY_GENERIC)
#undef RA_TRY_GENERIC
}

// Per-call plan.  The forward and the adjoint use different region sizes: the forward
// keeps only sample rows in LDS and can afford larger regions (fewer partial rows to
// add into HBM); the adjoint also keeps per-voxel dL/dp0 sums.
struct Plan {
    Geo g;              // adjoint regions (element gradients: per-region partials are kept, so larger)
    Geo ga;             // adjoint regions for dL/dp0 alone
    Geo gf;             // forward regions
    int jt;
    bool exact;
    int pair_d;         // forward takes voxels two at a time with this spread (0: one at a time)
    bool pair_ok;       // sampling and spacing allow pairs (regions with an even depth still needed)
    bool rowref;        // the dL/dp0-only adjoint may use the row-referenced form (adj_rowref)
    bool moment;        // the dL/dp0-only adjoint takes the moment form (k_adjoint_mom) on regions ga
    bool pose_moment;   // the adjoint with element gradients takes it too (k_adjoint_mom_pose) on regions g
    double mom_dd, mom_sigma;   // its delta / sigma and sigma
    bool f64_sums;      // the forward adds its partial rows into FP64 sums (else FP32, straight into s)
    size_t lds_adj, lds_adj0, lds_fwd;
    // scratch layout (byte offsets)
    size_t off_xe, off_vtab, off_itab, off_vtab_a, off_itab_a, off_vtab_f, off_itab_f, off_part, off_ge, off_s,
        off_partial, off_count, off_nc, off_ncw, off_nct, off_s64,
        off_xe64, off_qc, off_q, total;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int validate(ra_ctx* ctx, const ra_grid* grid, int32_t M, int32_t F, const ra_sampling* samp) {
    if (!ctx) return RA_EINVAL;
    if (!grid || !samp) return fail(ctx, RA_EINVAL, "grid and sampling descriptors are required");
    if (grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0)
        return fail(ctx, RA_EINVAL, "grid dimensions must be positive");
    if ((long long)grid->nx * grid->ny * grid->nz >= (1LL << 31))
        return fail(ctx, RA_EINVAL, "grid has 2^31 or more voxels");
    if (!finite_pos(grid->spacing)) return fail(ctx, RA_EINVAL, "grid spacing must be finite and positive");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(grid->origin[a])) return fail(ctx, RA_EINVAL, "grid origin must be finite");
    if (M <= 0 || F <= 0) return fail(ctx, RA_EINVAL, "M and F must be positive");
    if ((long long)M * F >= (1LL << 31)) return fail(ctx, RA_EINVAL, "M*F too large");
    if (samp->K <= 0) return fail(ctx, RA_EINVAL, "K must be positive");
    if (!finite_pos(samp->c) || !finite_pos(samp->fs) || !finite_pos(samp->sigma) || !finite_pos(samp->trunc))
        return fail(ctx, RA_EINVAL, "c, fs, sigma and trunc must be finite and positive");
    double delta = samp->c / samp->fs;
    double tsig = samp->trunc * samp->sigma;
    if (tsig < 0.5 * delta) return fail(ctx, RA_EINVAL, "trunc*sigma must be at least half a sample length");
    int jout = (int)std::floor(tsig / delta + 0.5);
    if (jout > JMAX) return fail(ctx, RA_EINVAL, "trunc*sigma exceeds 40 sample lengths");
    if (samp->kernel < RA_KERNEL_GAUSSIAN || samp->kernel > RA_KERNEL_UNIFORM)
        return fail(ctx, RA_EINVAL, "unknown source profile (kernel)");
    if (samp->kernel == RA_KERNEL_POWER && !(std::isfinite(samp->nu) && samp->nu > 0.5))
        return fail(ctx, RA_EINVAL, "power-law exponent nu must be finite and above 1/2");
    return RA_OK;
}

// Region size: the largest candidate box whose LDS footprint (sample rows of every
// wavefront, plus per-voxel sums for the adjoint) fits the byte budget per workgroup.
size_t set_regions(Geo& g, const ra_grid* grid, double delta, int jt, bool with_gsum, int extra_rows,
                   size_t budget, int moments = 0) {
    static const int cand[][3] = {{8, 8, 16}, {8, 8, 8}, {4, 8, 8}, {4, 4, 8}, {4, 4, 4},
                                  {2, 4, 4},  {2, 2, 4}, {2, 2, 2}, {1, 1, 2}, {1, 1, 1}};
    size_t lds = 0;
    for (const auto& c : cand) {
        int rx = std::min(c[0], g.nx), ry = std::min(c[1], g.ny), rz = std::min(c[2], g.nz);
        double rad = 0.5 * grid->spacing *
                     std::sqrt((double)(rx - 1) * (rx - 1) + (double)(ry - 1) * (ry - 1) + (double)(rz - 1) * (rz - 1));
        int jclamp = (int)std::ceil(rad / delta * (1.0 + 1e-6)) + 1;
        int L = 2 * (jclamp + jt) + 1 + extra_rows;
        int nvpad = (rx * ry * rz + 3) & ~3;
        lds = (size_t)WAVES * L * WAVE * sizeof(float) + (with_gsum ? (size_t)WAVES * nvpad * sizeof(float) : 0);
        if (moments)     // moment-form adjoint: one shared window of 2 jclamp + 1 table rows, four sums per voxel
            lds = (size_t)(2 * jclamp + 1) * 2 * WAVE * sizeof(float4) + (size_t)4 * nvpad * sizeof(float);
        if (moments == 2)   // and with element gradients: the wavefronts' FP64 partials of a chunk
            lds += (size_t)MOM_WAVES * 3 * WAVE * sizeof(double);
        g.rx = rx; g.ry = ry; g.rz = rz;
        g.nvpad = nvpad;
        g.jclamp = jclamp;
        g.jclampf = (float)jclamp;
        g.kmargin = jclamp + jt;
        g.L = L;
        if (lds <= budget) break;
    }
    g.nrx = (g.nx + g.rx - 1) / g.rx;
    g.nry = (g.ny + g.ry - 1) / g.ry;
    g.nrz = (g.nz + g.rz - 1) / g.rz;
    g.nreg = g.nrx * g.nry * g.nrz;
    return lds;
}

// allow_moment false: the row forms only (the batched serving step, whose kernels and region sizes
// are those of the row forms).
void make_plan(const ra_grid* grid, int32_t M, int32_t F, const ra_sampling* samp, Plan& P, int sums_mode = RA_SUMS_AUTO,
               bool allow_moment = true) {
    Geo& g = P.g;
    std::memset(&g, 0, sizeof(g));
    g.nx = grid->nx; g.ny = grid->ny; g.nz = grid->nz;
    g.vsx = (long long)grid->ny * grid->nz;
    g.vsy = grid->nz;
    g.gsx = g.vsx;
    g.gsy = g.vsy;
    g.K = samp->K; g.M = M; g.F = F; g.E = M * F;
    const double delta = samp->c / samp->fs;
    const double sigma = samp->sigma;
    const double tsig = samp->trunc * sigma;
    const int jout = (int)std::floor(tsig / delta + 0.5);
    choose_jt(jout, P.jt, P.exact);
    g.ktype = samp->kernel;
    if (g.ktype != RA_KERNEL_GAUSSIAN) {
        P.exact = false;
        if (g.ktype == RA_KERNEL_EXPONENTIAL) {
            // factorised legs (fwd_pair_exp): the smallest listed window bound, tables of
            // G_j = exp(-j delta/w)
            P.jt = -1;
#define RA_TRY_EXP(n) \
    if (P.jt < 0 && jout <= n) P.jt = n;
            RA_EXP_LIST(RA_TRY_EXP)
#undef RA_TRY_EXP
        } else {
            // per-sample kernels with a run-time window of jout steps either side
            P.jt = jout;
        }
        g.jwin = jout;
        const double log2e = 1.4426950408889634;
        g.kexp = (float)(-log2e / sigma);
        g.kinv_w = (float)(1.0 / sigma);
        g.kinv_w2 = (float)(1.0 / (sigma * sigma));
        g.knu = (float)(-samp->nu);
        g.k2nu = (float)(2.0 * samp->nu);
    }
    g.edge = (float)(P.jt * delta - tsig);
    g.jin = (int)std::floor(tsig / delta - 0.5);
    for (int a = 0; a < 3; ++a) {
        g.org_h[a] = (float)grid->origin[a];
        g.org_l[a] = (float)(grid->origin[a] - (double)g.org_h[a]);
    }
    g.sp_h = (float)grid->spacing;
    g.sp_l = (float)(grid->spacing - (double)g.sp_h);
    g.dlt_h = (float)delta;
    g.dlt_l = (float)(delta - (double)g.dlt_h);
    g.inv_dlt = (float)(1.0 / delta);
    g.tsig = (float)tsig;
    const double log2e = 1.4426950408889634;
    g.kappa = (float)(-log2e / (2.0 * sigma * sigma));
    g.alpha = (float)(log2e * delta / (sigma * sigma));
    g.inv_s2 = (float)(1.0 / (sigma * sigma));
    g.gmin = (float)(10.0 * sigma);
    for (int j = 0; j <= JMAX; ++j) {
        double gj = g.ktype == RA_KERNEL_EXPONENTIAL ? std::exp(-(double)j * delta / sigma)
                                                     : std::exp(-(double)j * j * delta * delta / (2.0 * sigma * sigma));
        g.gam[j] = (float)gj;
        g.jdg[j] = (float)(j * delta * gj);
        g.jjdg[j] = (float)((j * delta) * (j * delta) * gj);
    }
    for (int m = 0; m <= RS_MAX; ++m) {
        g.gamr[m] = (float)std::exp(-(double)m * m * delta * delta / (2.0 * sigma * sigma));
    }
    // Paired forward: z-neighbours (distance h) have centre samples at most D apart when
    // h < D delta.
    P.pair_d = 0;
    P.pair_ok = P.exact && g.ktype == RA_KERNEL_GAUSSIAN && grid->spacing <= (PAIR_D - 0.01) * delta;
    if (P.pair_ok) P.pair_d = PAIR_D;
    P.gf = g;
    P.ga = g;
    P.lds_adj = set_regions(g, grid, delta, P.jt, true, 0, LDS_ADJ_BUDGET);
    P.lds_adj0 = set_regions(P.ga, grid, delta, P.jt, true, 0, LDS_ADJ0_BUDGET);
    // Row-referenced dL/dp0 adjoint: its factors reach exp(+-(kmargin + 1)^2 (delta/sigma)^2 / 2)
    // (Hc^(2 JT), E_c Hc^mlow and Gamma_m at the window's ends), which must stay well inside the
    // FP32 range (e^88); the staged window is normalised to [1/2, 1).
    {
        const double km = P.ga.kmargin + 1.0, ds = delta / sigma;
        P.rowref = P.exact && g.ktype == RA_KERNEL_GAUSSIAN && P.ga.kmargin <= RS_MAX && km * km * ds * ds / 2.0 <= 75.0;
    }
    // Moment-form dL/dp0 adjoint (k_adjoint_mom) where its truncation bound holds; it replaces the
    // row-referenced form and takes regions sized for its shared table window.
    {
        double fact = 1.0;
        for (int n = 2; n <= NMOM; ++n) fact *= n;
        const double bound = 1.791 * std::pow(0.5 * delta / sigma, NMOM) * std::sqrt((NMOM + 1) / fact);
        P.moment = allow_moment && P.exact && g.ktype == RA_KERNEL_GAUSSIAN && bound <= MOM_TOL;
        P.mom_dd = delta / sigma;
        P.mom_sigma = sigma;
        g.mom_dd = delta / sigma;
        g.mom_sigma = sigma;
        if (P.moment) {
            Geo gm = P.ga;
            const size_t lds = set_regions(gm, grid, delta, P.jt, true, 0, LDS_MOM_BUDGET, 1);
            P.moment = lds <= LDS_MOM_BUDGET && 2 * gm.jclamp + 1 <= MOM_WAVES * MOM_PER;
            if (P.moment) {
                P.ga = gm;
                P.lds_adj0 = lds;
                P.rowref = false;
            }
        }
        // the adjoint with element gradients in moment form, on regions sized for its LDS (the
        // per-region partials then follow these regions)
        P.pose_moment = false;
        if (P.moment) {
            Geo gp = g;
            const size_t lds = set_regions(gp, grid, delta, P.jt, true, 0, LDS_ADJ_BUDGET, 2);
            if (lds <= LDS_ADJ_BUDGET && 2 * gp.jclamp + 1 <= MOM_WAVES * MOM_PER) {
                g = gp;
                P.lds_adj = lds;
                P.pose_moment = true;
            }
        }
    }
    P.lds_fwd = set_regions(P.gf, grid, delta, P.jt, false, P.pair_d, LDS_FWD_BUDGET);
    // pairs are (k, k+1) of the visiting order, so the forward region needs an even rz
    if (P.pair_d && (P.gf.rz & 1)) {
        P.pair_d = 0;
        P.lds_fwd = set_regions(P.gf, grid, delta, P.jt, false, 0, LDS_FWD_BUDGET);
    }
    // Profiles that do not vanish at the window edge (RA_KERNEL_* other than the Gaussian): the
    // dL/dp0 adjoint takes the forward's regions where they fit its LDS budget, so that both compute
    // every pair's u from the same reference, bit for bit, and decide its window edge alike (then
    // <A p0, r> = <p0, A^T r> holds to summation rounding; with other regions an edge term within
    // rounding of the edge can fall in on one side and out on the other).
    if (g.ktype != RA_KERNEL_GAUSSIAN) {
        Geo ga2 = P.ga;
        const size_t lds2 = set_regions(ga2, grid, delta, P.jt, true, 0, LDS_FWD_BUDGET);
        if (lds2 <= LDS_FWD_BUDGET && ga2.rx == P.gf.rx && ga2.ry == P.gf.ry && ga2.rz == P.gf.rz) {
            P.ga = ga2;
            P.lds_adj0 = lds2;
        }
    }
    // FP32 rounding of the forward's sums grows with the number of regions whose partial rows
    // meet in one sample; past FWD_F32_MAX_REGIONS forward regions the rows go into FP64 sums.
    P.f64_sums = sums_mode == RA_SUMS_F64 || (sums_mode == RA_SUMS_AUTO && P.gf.nreg > FWD_F32_MAX_REGIONS);

    size_t o = 0;
    P.off_xe = o; o = align_up(o + (size_t)g.E * 6 * sizeof(float));
    P.off_vtab = o; o = align_up(o + (size_t)g.nvpad * sizeof(float4));
    P.off_itab = o; o = align_up(o + (size_t)g.nvpad * sizeof(int4));
    P.off_vtab_a = o; o = align_up(o + (size_t)P.ga.nvpad * sizeof(float4));
    P.off_itab_a = o; o = align_up(o + (size_t)P.ga.nvpad * sizeof(int4));
    P.off_vtab_f = o; o = align_up(o + (size_t)P.gf.nvpad * sizeof(float4));
    P.off_itab_f = o; o = align_up(o + (size_t)P.gf.nvpad * sizeof(int4));
    P.off_part = o; o = align_up(o + (size_t)g.nreg * g.E * 3 * sizeof(double));
    P.off_ge = o; o = align_up(o + (size_t)g.E * 3 * sizeof(double));
    P.off_s = o; o = align_up(o + (size_t)g.E * g.K * sizeof(float));
    P.off_partial = o; o = align_up(o + RESID_BLOCKS * sizeof(float));
    P.off_count = o; o = align_up(o + sizeof(unsigned long long));
    P.off_nc = o; o = align_up(o + (size_t)g.E * sizeof(double));
    P.off_ncw = o; o = align_up(o + (size_t)g.E * sizeof(double));
    P.off_nct = o; o = align_up(o + sizeof(double));
    P.off_s64 = o; o = align_up(o + (P.f64_sums ? (size_t)g.E * g.K * sizeof(double) : 0));
    P.off_xe64 = o; o = align_up(o + (size_t)g.E * 3 * sizeof(double));
    P.off_qc = o; o = align_up(o + (P.moment ? (size_t)NMOM * (2 * P.jt + 1) * sizeof(float) : 0));
    P.off_q = o; o = align_up(o + (P.moment ? ((size_t)g.E * (g.K + 2 * P.jt) + 1) * NMOM * sizeof(float) : 0));
    P.total = o;
}

int ensure_scratch(ra_ctx* ctx, size_t bytes, hipStream_t stream) {
    if (bytes <= ctx->arena_bytes) return RA_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(ctx, RA_ENOMEM, "scratch must be reserved (ra_reserve) before stream capture");
    RA_HIP(ctx, hipStreamSynchronize(stream));
    if (ctx->arena) RA_HIP(ctx, hipFree(ctx->arena));
    ctx->arena = nullptr;
    ctx->arena_bytes = 0;
    if (hipMalloc(&ctx->arena, bytes) != hipSuccess) {
        ctx->arena = nullptr;
        (void)hipGetLastError();
        return fail(ctx, RA_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes of scratch failed");
    }
    ctx->arena_bytes = bytes;
    return RA_OK;
}

// Allow a kernel the full LDS of a CU, once per kernel (so not again under stream capture).
template <typename K>
hipError_t allow_full_lds(K kern) {
    static std::mutex mu;
    static std::set<const void*> done;
    const void* f = (const void*)kern;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count(f)) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess) done.insert(f);
    return e;
}

template <typename T>
T* at(ra_ctx* ctx, size_t off) {
    return reinterpret_cast<T*>(ctx->arena + off);
}

template <typename T>
T* at(char* base, size_t off) {
    return reinterpret_cast<T*>(base + off);
}

int prologue(ra_ctx* ctx, char* base, const ra_grid* grid, const Plan& P, const double* elem, const double* poses,
             hipStream_t stream, bool forward_only = false) {
    const Geo& g = P.g;
    float3 lo = make_float3((float)grid->origin[0], (float)grid->origin[1], (float)grid->origin[2]);
    float3 hi = make_float3((float)(grid->origin[0] + (g.nx - 1) * grid->spacing),
                            (float)(grid->origin[1] + (g.ny - 1) * grid->spacing),
                            (float)(grid->origin[2] + (g.nz - 1) * grid->spacing));
    hipLaunchKernelGGL(k_elements, dim3((g.E + 255) / 256), dim3(256), 0, stream, g, elem, poses,
                       at<float>(base, P.off_xe), ctx->d_status, lo, hi);
    if (!forward_only) {
        hipLaunchKernelGGL(k_voxel_table, dim3((g.nvpad + 255) / 256), dim3(256), 0, stream, g,
                           at<float4>(base, P.off_vtab), at<int4>(base, P.off_itab));
        hipLaunchKernelGGL(k_voxel_table, dim3((P.ga.nvpad + 255) / 256), dim3(256), 0, stream, P.ga,
                           at<float4>(base, P.off_vtab_a), at<int4>(base, P.off_itab_a));
    }
    hipLaunchKernelGGL(k_voxel_table, dim3((P.gf.nvpad + 255) / 256), dim3(256), 0, stream, P.gf,
                       at<float4>(base, P.off_vtab_f), at<int4>(base, P.off_itab_f));
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

// Scratch layout of a forward-only call (element positions, the forward's voxel tables and, with
// FP64 sums, the sums): the offsets of P the forward reads, rewritten from 0; returns the bytes.
size_t forward_layout(Plan& P) {
    size_t o = 0;
    P.off_xe = o; o = align_up(o + (size_t)P.g.E * 6 * sizeof(float));
    P.off_vtab_f = o; o = align_up(o + (size_t)P.gf.nvpad * sizeof(float4));
    P.off_itab_f = o; o = align_up(o + (size_t)P.gf.nvpad * sizeof(int4));
    P.off_s64 = o; o = align_up(o + (P.f64_sums ? (size_t)P.g.E * P.g.K * sizeof(double) : 0));
    return o;
}

// Device address of this device's static scratch array, resolved once per device (the
// current device must be `device`).
hipError_t static_scratch_of(int device, char** out) {
    static std::mutex mu;
    static std::map<int, char*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        it = addr.emplace(device, static_cast<char*>(p)).first;
    }
    *out = it->second;
    return hipSuccess;
}

template <int JT, bool EXACT, int D, int KT = RA_KERNEL_GAUSSIAN>
int launch_forward_t(ra_ctx* ctx, char* base, const Plan& P, const float* p0, float* s, hipStream_t stream) {
    const size_t n = (size_t)P.g.E * P.g.K;
    if (!P.f64_sums) {
        auto kern = k_forward<JT, EXACT, D, KT, float>;
        RA_HIP(ctx, allow_full_lds(kern));
        hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, stream, s, n, 0.0f);
        hipLaunchKernelGGL(kern, dim3(P.gf.nreg), dim3(BLOCK), P.lds_fwd, stream, P.gf, p0,
                           at<float>(base, P.off_xe), at<float4>(base, P.off_vtab_f), at<int4>(base, P.off_itab_f), s);
        RA_HIP(ctx, hipGetLastError());
        return RA_OK;
    }
    auto kern = k_forward<JT, EXACT, D, KT, double>;
    RA_HIP(ctx, allow_full_lds(kern));
    double* s64 = at<double>(base, P.off_s64);
    hipLaunchKernelGGL(k_fill_f64, dim3(1024), dim3(256), 0, stream, s64, n);
    hipLaunchKernelGGL(kern, dim3(P.gf.nreg), dim3(BLOCK), P.lds_fwd, stream, P.gf, p0, at<float>(base, P.off_xe),
                       at<float4>(base, P.off_vtab_f), at<int4>(base, P.off_itab_f), s64);
    hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, stream, s64, n, s);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

// Kernels with a listed window bound JT test only their last GEN_STEP (Gaussian) or
// EXP_STEP (exponential) steps, which needs every earlier step inside the window.
bool generic_bound_ok(const Plan& P) {
    if (P.g.ktype == RA_KERNEL_EXPONENTIAL) return P.g.jin >= P.jt - EXP_STEP;
    return P.exact || P.g.ktype != RA_KERNEL_GAUSSIAN || P.g.jin >= P.jt - GEN_STEP;
}

int launch_forward(ra_ctx* ctx, char* base, const Plan& P, const float* p0, float* s, hipStream_t stream) {
    if (!generic_bound_ok(P)) return fail(ctx, RA_ENOTSUP, "window half-width not supported");
    // other profiles; the per-sample kernels index from the centre row kmargin (JT = 0)
    switch (P.g.ktype) {
        case RA_KERNEL_EXPONENTIAL:
#define RA_CASE(n) \
    if (P.jt == n) return launch_forward_t<n, false, 0, RA_KERNEL_EXPONENTIAL>(ctx, base, P, p0, s, stream);
            RA_EXP_LIST(RA_CASE)
#undef RA_CASE
            break;
        case RA_KERNEL_POWER:
            if (P.g.knu == -2.0f) return launch_forward_t<0, false, 0, KT_POWER2>(ctx, base, P, p0, s, stream);
            return launch_forward_t<0, false, 0, RA_KERNEL_POWER>(ctx, base, P, p0, s, stream);
        case RA_KERNEL_UNIFORM: return launch_forward_t<0, false, 0, RA_KERNEL_UNIFORM>(ctx, base, P, p0, s, stream);
        default: break;
    }
#define RA_CASE(n)                                                                       \
    if (P.exact && P.jt == n)                                                            \
        return P.pair_d ? launch_forward_t<n, true, PAIR_D>(ctx, base, P, p0, s, stream)       \
                        : launch_forward_t<n, true, 0>(ctx, base, P, p0, s, stream);
    RA_EXACT_LIST(RA_CASE)
#undef RA_CASE
#define RA_CASE(n) \
    if (!P.exact && P.jt == n) return launch_forward_t<n, false, 0>(ctx, base, P, p0, s, stream);
    RA_GENERIC_LIST(RA_CASE)
#undef RA_CASE
    return fail(ctx, RA_ENOTSUP, "window half-width not supported");
}

template <int JT, bool EXACT, bool P0, bool POSE, int KT = RA_KERNEL_GAUSSIAN>
int launch_adjoint_t(ra_ctx* ctx, const Plan& P, const float* p0, const float* r, float* gp0, int acc,
                     hipStream_t stream) {
    auto kern = k_adjoint<JT, EXACT, P0, POSE, KT>;
    if constexpr (P0 && !POSE && EXACT && KT == RA_KERNEL_GAUSSIAN)
        if (P.rowref) kern = k_adjoint<JT, EXACT, P0, POSE, KT, true>;
    RA_HIP(ctx, allow_full_lds(kern));
    const bool alone = P0 && !POSE;        // dL/dp0 alone: the smaller regions
    const Geo& g = alone ? P.ga : P.g;
    hipLaunchKernelGGL(kern, dim3(g.nreg), dim3(BLOCK), alone ? P.lds_adj0 : P.lds_adj, stream, g, p0,
                       at<float>(ctx, P.off_xe), at<float4>(ctx, alone ? P.off_vtab_a : P.off_vtab),
                       at<int4>(ctx, alone ? P.off_itab_a : P.off_itab), r, gp0, acc, at<double>(ctx, P.off_part));
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

template <int JT, bool EXACT, int KT = RA_KERNEL_GAUSSIAN>
int launch_adjoint_j(ra_ctx* ctx, const Plan& P, const float* p0, const float* r, float* gp0, bool pose, int acc,
                     hipStream_t stream) {
    if (gp0 && pose) return launch_adjoint_t<JT, EXACT, true, true, KT>(ctx, P, p0, r, gp0, acc, stream);
    if (gp0) return launch_adjoint_t<JT, EXACT, true, false, KT>(ctx, P, p0, r, gp0, acc, stream);
    return launch_adjoint_t<JT, EXACT, false, true, KT>(ctx, P, p0, r, gp0, acc, stream);
}

// dL/dp0 alone in moment form: coefficient and moment tables, then one workgroup per region.
int launch_adjoint_mom(ra_ctx* ctx, const Plan& P, const float* r, float* gp0, int acc, hipStream_t stream) {
    const Geo& g = P.ga;
    const int jt = P.jt;
    hipLaunchKernelGGL(k_moment_coefs, dim3(1), dim3(2 * jt + 1), 0, stream, jt, P.mom_dd, P.mom_sigma,
                       at<float>(ctx, P.off_qc));
    const long long rows = (long long)g.E * (g.K + 2 * jt) + 1;      // and the zero row
    hipLaunchKernelGGL(k_moment_table, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, stream, g.E, g.K, jt, r,
                       at<float>(ctx, P.off_qc), at<float4>(ctx, P.off_q));
    auto kern = k_adjoint_mom<MOM_PER, MOM_WAVES>;     // the host checked 2 jclamp + 1 <= MOM_WAVES * MOM_PER
    RA_HIP(ctx, allow_full_lds(kern));
    hipLaunchKernelGGL(kern, dim3(g.nreg), dim3(MOM_WAVES * WAVE), P.lds_adj0, stream, g, at<float>(ctx, P.off_xe),
                       at<float4>(ctx, P.off_vtab_a), at<int4>(ctx, P.off_itab_a), at<float4>(ctx, P.off_q), jt, gp0,
                       acc);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

// The adjoint with element gradients (and dL/dp0 if gp0) in moment form, on the regions of P.g.
int launch_adjoint_mom_pose(ra_ctx* ctx, const Plan& P, const float* p0, const float* r, float* gp0, int acc,
                            hipStream_t stream) {
    const Geo& g = P.g;
    const int jt = P.jt;
    hipLaunchKernelGGL(k_moment_coefs, dim3(1), dim3(2 * jt + 1), 0, stream, jt, P.mom_dd, P.mom_sigma,
                       at<float>(ctx, P.off_qc));
    const long long rows = (long long)g.E * (g.K + 2 * jt) + 1;      // and the zero row
    hipLaunchKernelGGL(k_moment_table, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, stream, g.E, g.K, jt, r,
                       at<float>(ctx, P.off_qc), at<float4>(ctx, P.off_q));
    auto kern = gp0 ? k_adjoint_mom_pose<MOM_PER, MOM_WAVES, true> : k_adjoint_mom_pose<MOM_PER, MOM_WAVES, false>;
    RA_HIP(ctx, allow_full_lds(kern));
    hipLaunchKernelGGL(kern, dim3(g.nreg), dim3(MOM_WAVES * WAVE), P.lds_adj, stream, g, p0, at<float>(ctx, P.off_xe),
                       at<float4>(ctx, P.off_vtab), at<int4>(ctx, P.off_itab), at<float4>(ctx, P.off_q), jt, gp0, acc,
                       at<double>(ctx, P.off_part));
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

int launch_adjoint(ra_ctx* ctx, const Plan& P, const float* p0, const float* r, float* gp0, bool pose, int acc,
                   hipStream_t stream) {
    if (!generic_bound_ok(P)) return fail(ctx, RA_ENOTSUP, "window half-width not supported");
    if (P.moment && gp0 && !pose) return launch_adjoint_mom(ctx, P, r, gp0, acc, stream);
    if (P.pose_moment && pose) return launch_adjoint_mom_pose(ctx, P, p0, r, gp0, acc, stream);
    switch (P.g.ktype) {
        case RA_KERNEL_EXPONENTIAL:
#define RA_CASE(n) \
    if (P.jt == n) return launch_adjoint_j<n, false, RA_KERNEL_EXPONENTIAL>(ctx, P, p0, r, gp0, pose, acc, stream);
            RA_EXP_LIST(RA_CASE)
#undef RA_CASE
            break;
        case RA_KERNEL_POWER:
            if (P.g.knu == -2.0f) return launch_adjoint_j<0, false, KT_POWER2>(ctx, P, p0, r, gp0, pose, acc, stream);
            return launch_adjoint_j<0, false, RA_KERNEL_POWER>(ctx, P, p0, r, gp0, pose, acc, stream);
        case RA_KERNEL_UNIFORM:
            return launch_adjoint_j<0, false, RA_KERNEL_UNIFORM>(ctx, P, p0, r, gp0, pose, acc, stream);
        default: break;
    }
#define RA_CASE(n) \
    if (P.exact && P.jt == n) return launch_adjoint_j<n, true>(ctx, P, p0, r, gp0, pose, acc, stream);
    RA_EXACT_LIST(RA_CASE)
#undef RA_CASE
#define RA_CASE(n) \
    if (!P.exact && P.jt == n) return launch_adjoint_j<n, false>(ctx, P, p0, r, gp0, pose, acc, stream);
    RA_GENERIC_LIST(RA_CASE)
#undef RA_CASE
    return fail(ctx, RA_ENOTSUP, "window half-width not supported");
}

int adjoint_body(ra_ctx* ctx, const Plan& P, const float* p0, const double* elem, const float* r,
                 float* grad_p0, double* grad_pose, double* grad_elem, uint32_t flags, hipStream_t stream) {
    const int acc = (flags & RA_ACCUMULATE) ? 1 : 0;
    const bool pose = grad_pose || grad_elem;
    if (!grad_p0 && !pose) return RA_OK;
    int rc = launch_adjoint(ctx, P, p0, r, grad_p0, pose, acc, stream);
    if (rc != RA_OK) return rc;
    if (pose) {
        const Geo& g = P.g;
        hipLaunchKernelGGL(k_pose_reduce, dim3((3 * g.E + PR_T - 1) / PR_T), dim3(PR_T * PR_P), 0, stream, g,
                           at<double>(ctx, P.off_part), at<double>(ctx, P.off_ge), grad_elem, acc);
        if (grad_pose)
            hipLaunchKernelGGL(k_pose_frame, dim3(g.F), dim3(256), 0, stream, g, at<double>(ctx, P.off_ge), elem,
                               grad_pose, acc);
        RA_HIP(ctx, hipGetLastError());
    }
    return RA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// exported API
// ---------------------------------------------------------------------------------------------
extern "C" {

int ra_create(ra_ctx** out, int device) {
    if (!out) return RA_EINVAL;
    *out = nullptr;
    ra_ctx* ctx = new (std::nothrow) ra_ctx();
    if (!ctx) return RA_ENOMEM;
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess || hipMalloc(&ctx->d_status, sizeof(int)) != hipSuccess ||
        hipMemset(ctx->d_status, 0, sizeof(int)) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_count, sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ctx->h_f64, sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&ctx->d_f64, sizeof(double)) != hipSuccess ||
        static_scratch_of(device, &ctx->static_scratch) != hipSuccess) {
        (void)hipGetLastError();
        ra_destroy(ctx);
        return RA_EHIP;
    }
    *out = ctx;
    return RA_OK;
}

void ra_destroy(ra_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->arena) (void)hipFree(ctx->arena);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
    if (ctx->h_count) (void)hipHostFree(ctx->h_count);
    if (ctx->h_f64) (void)hipHostFree(ctx->h_f64);
    if (ctx->d_f64) (void)hipFree(ctx->d_f64);
    delete ctx;
}

const char* ra_last_error(const ra_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ra_status(ra_ctx* ctx, void* stream) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    hipStream_t st = (hipStream_t)stream;
    int h = 0;
    RA_HIP(ctx, hipMemcpyAsync(&h, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost, st));
    RA_HIP(ctx, hipStreamSynchronize(st));
    RA_HIP(ctx, hipMemsetAsync(ctx->d_status, 0, sizeof(int), st));
    RA_HIP(ctx, hipStreamSynchronize(st));
    if (h) return fail(ctx, RA_EGEOM, "an element came closer than 10 sigma to the voxel grid");
    return RA_OK;
}

int ra_reserve(ra_ctx* ctx, size_t bytes) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    RA_HIP(ctx, hipSetDevice(ctx->device));
    return ensure_scratch(ctx, bytes, nullptr);
}

size_t ra_scratch_bytes(const ra_grid* grid, int32_t M, int32_t F, const ra_sampling* samp) {
    ra_ctx tmp;
    if (validate(&tmp, grid, M, F, samp) != RA_OK) return 0;
    Plan P;
    make_plan(grid, M, F, samp, P, RA_SUMS_F64);      // the largest of the forward's sum modes
    return P.total;
}

int ra_set_forward_sums(ra_ctx* ctx, int32_t mode) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    if (mode != RA_SUMS_AUTO && mode != RA_SUMS_F32 && mode != RA_SUMS_F64)
        return fail(ctx, RA_EINVAL, "mode must be RA_SUMS_AUTO, RA_SUMS_F32 or RA_SUMS_F64");
    ctx->sums_mode = mode;
    return RA_OK;
}

int radiate_forward(ra_ctx* ctx, const ra_grid* grid, const float* p0, int32_t M, const double* elem,
                    const double* poses, int32_t F, const ra_sampling* samp, float* s, void* stream) {
    int rc = validate(ctx, grid, M, F, samp);
    if (rc != RA_OK) return rc;
    ctx->err.clear();
    if (!p0 || !elem || !poses || !s) return fail(ctx, RA_EINVAL, "p0, elem, poses and s are required");
    hipStream_t st = (hipStream_t)stream;
    RA_HIP(ctx, hipSetDevice(ctx->device));
    Plan P;
    make_plan(grid, M, F, samp, P, ctx->sums_mode);
    if ((rc = ensure_scratch(ctx, P.total, st)) != RA_OK) return rc;
    if ((rc = prologue(ctx, ctx->arena, grid, P, elem, poses, st)) != RA_OK) return rc;
    return launch_forward(ctx, ctx->arena, P, p0, s, st);
}

int radiate_forward_static(ra_ctx* ctx, const ra_grid* grid, const float* p0, int32_t M, const double* elem,
                           const double* poses, int32_t F, const ra_sampling* samp, float* s, void* stream) {
    int rc = validate(ctx, grid, M, F, samp);
    if (rc != RA_OK) return rc;
    ctx->err.clear();
    if (!p0 || !elem || !poses || !s) return fail(ctx, RA_EINVAL, "p0, elem, poses and s are required");
    if (!ctx->static_scratch) return fail(ctx, RA_EHIP, "the static scratch of this device was not resolved");
    hipStream_t st = (hipStream_t)stream;
    RA_HIP(ctx, hipSetDevice(ctx->device));
    Plan P;
    make_plan(grid, M, F, samp, P, ctx->sums_mode);
    const size_t need = forward_layout(P);
    if (need > STATIC_SCRATCH_BYTES)
        return fail(ctx, RA_ENOMEM, "radiate_forward_static needs " + std::to_string(need) +
                                        " bytes of scratch; its static array holds " +
                                        std::to_string(STATIC_SCRATCH_BYTES));
    if ((rc = prologue(ctx, ctx->static_scratch, grid, P, elem, poses, st, true)) != RA_OK) return rc;
    return launch_forward(ctx, ctx->static_scratch, P, p0, s, st);
}

int radiate_adjoint(ra_ctx* ctx, const ra_grid* grid, const float* p0, int32_t M, const double* elem,
                    const double* poses, int32_t F, const ra_sampling* samp, const float* r, float* grad_p0,
                    double* grad_pose, double* grad_elem, uint32_t flags, void* stream) {
    int rc = validate(ctx, grid, M, F, samp);
    if (rc != RA_OK) return rc;
    ctx->err.clear();
    if (!elem || !poses || !r) return fail(ctx, RA_EINVAL, "elem, poses and r are required");
    if ((grad_pose || grad_elem) && !p0) return fail(ctx, RA_EINVAL, "p0 is required for pose gradients");
    if (flags & ~RA_ACCUMULATE) return fail(ctx, RA_EINVAL, "unknown flag bits");
    hipStream_t st = (hipStream_t)stream;
    RA_HIP(ctx, hipSetDevice(ctx->device));
    Plan P;
    make_plan(grid, M, F, samp, P, ctx->sums_mode);
    if ((rc = ensure_scratch(ctx, P.total, st)) != RA_OK) return rc;
    if ((rc = prologue(ctx, ctx->arena, grid, P, elem, poses, st)) != RA_OK) return rc;
    return adjoint_body(ctx, P, p0, elem, r, grad_p0, grad_pose, grad_elem, flags, st);
}

int loss_and_grad(ra_ctx* ctx, const ra_grid* grid, const float* p0, int32_t M, const double* elem,
                  const double* poses, int32_t F, const ra_sampling* samp, const float* y, double* loss,
                  float* s_out, float* grad_p0, double* grad_pose, double* grad_elem, uint32_t flags,
                  void* stream) {
    int rc = validate(ctx, grid, M, F, samp);
    if (rc != RA_OK) return rc;
    ctx->err.clear();
    if (!p0 || !elem || !poses || !y) return fail(ctx, RA_EINVAL, "p0, elem, poses and y are required");
    if (flags & ~(RA_ACCUMULATE | RA_LOSS_ON_DEVICE | RA_SIGNALS_GIVEN))
        return fail(ctx, RA_EINVAL, "unknown flag bits");
    const bool given = (flags & RA_SIGNALS_GIVEN) != 0;
    if (given && !s_out) return fail(ctx, RA_EINVAL, "RA_SIGNALS_GIVEN needs the signals in s_out");
    hipStream_t st = (hipStream_t)stream;
    RA_HIP(ctx, hipSetDevice(ctx->device));
    Plan P;
    make_plan(grid, M, F, samp, P, ctx->sums_mode);
    if ((rc = ensure_scratch(ctx, P.total, st)) != RA_OK) return rc;
    if ((rc = prologue(ctx, ctx->arena, grid, P, elem, poses, st)) != RA_OK) return rc;
    float* s = at<float>(ctx, P.off_s);
    const size_t n = (size_t)P.g.E * P.g.K;
    if (given) {
        // the caller's signals; the residual below overwrites the scratch copy, not them
        hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, st, s_out, n, s);
    } else {
        if ((rc = launch_forward(ctx, ctx->arena, P, p0, s, st)) != RA_OK) return rc;
        if (s_out) hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, st, s, n, s_out);
    }
    float* partial = at<float>(ctx, P.off_partial);
    hipLaunchKernelGGL(k_residual, dim3(RESID_BLOCKS), dim3(256), 0, st, s, y, n, partial);
    RA_HIP(ctx, hipGetLastError());
    if ((rc = adjoint_body(ctx, P, p0, elem, s, grad_p0, grad_pose, grad_elem, flags & RA_ACCUMULATE, st)) != RA_OK)
        return rc;
    if (loss) {
        // FP64 sum of the per-block FP32 partials, in a fixed order, on the device
        double* dst = (flags & RA_LOSS_ON_DEVICE) ? loss : ctx->d_f64;
        hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, st, partial, RESID_BLOCKS, dst);
        RA_HIP(ctx, hipGetLastError());
        if (!(flags & RA_LOSS_ON_DEVICE)) {
            RA_HIP(ctx, hipMemcpyAsync(ctx->h_f64, ctx->d_f64, sizeof(double), hipMemcpyDeviceToHost, st));
            RA_HIP(ctx, hipStreamSynchronize(st));
            *loss = *ctx->h_f64;
        }
    }
    return RA_OK;
}

int nc_loss_and_grad(ra_ctx* ctx, const ra_grid* grid, const float* p0, int32_t M, const double* elem,
                     const double* poses, int32_t F, const ra_sampling* samp, const float* y,
                     const float* weight, double* loss, double* loss_elem, float* s_out, float* grad_p0,
                     double* grad_pose, double* grad_elem, uint32_t flags, void* stream) {
    int rc = validate(ctx, grid, M, F, samp);
    if (rc != RA_OK) return rc;
    ctx->err.clear();
    if (!p0 || !elem || !poses || !y) return fail(ctx, RA_EINVAL, "p0, elem, poses and y are required");
    if (flags & ~RA_ACCUMULATE) return fail(ctx, RA_EINVAL, "unknown flag bits");
    hipStream_t st = (hipStream_t)stream;
    RA_HIP(ctx, hipSetDevice(ctx->device));
    Plan P;
    make_plan(grid, M, F, samp, P, ctx->sums_mode);
    if ((rc = ensure_scratch(ctx, P.total, st)) != RA_OK) return rc;
    if ((rc = prologue(ctx, ctx->arena, grid, P, elem, poses, st)) != RA_OK) return rc;
    float* s = at<float>(ctx, P.off_s);
    if ((rc = launch_forward(ctx, ctx->arena, P, p0, s, st)) != RA_OK) return rc;
    const int E = P.g.E;
    if (s_out) hipLaunchKernelGGL(k_copy, dim3(1024), dim3(256), 0, st, s, (size_t)E * P.g.K, s_out);
    double* wl = at<double>(ctx, P.off_ncw);
    hipLaunchKernelGGL(k_nc_residual, dim3(std::min(E, 65536)), dim3(NC_THREADS), 0, st, s, y, weight, E, P.g.K,
                       loss_elem, wl);
    RA_HIP(ctx, hipGetLastError());
    if ((rc = adjoint_body(ctx, P, p0, elem, s, grad_p0, grad_pose, grad_elem, flags, st)) != RA_OK) return rc;
    if (loss) {
        double* d_total = at<double>(ctx, P.off_nct);
        hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(NC_THREADS), 0, st, wl, E, d_total);
        RA_HIP(ctx, hipMemcpyAsync(ctx->h_f64, d_total, sizeof(double), hipMemcpyDeviceToHost, st));
        RA_HIP(ctx, hipStreamSynchronize(st));
        *loss = *ctx->h_f64;
    }
    return RA_OK;
}

int ra_pose_from_axis_angle(ra_ctx* ctx, const double* pose6, int32_t F, double* poses, void* stream) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    if (!pose6 || !poses || F <= 0) return fail(ctx, RA_EINVAL, "pose6, poses and F > 0 are required");
    RA_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_pose_from_aa, dim3((F + 127) / 128), dim3(128), 0, (hipStream_t)stream, pose6, F, poses);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

int ra_pose_grad_axis_angle(ra_ctx* ctx, const double* pose6, const double* grad_pose, int32_t F, double* grad6,
                            void* stream) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    if (!pose6 || !grad_pose || !grad6 || F <= 0)
        return fail(ctx, RA_EINVAL, "pose6, grad_pose, grad6 and F > 0 are required");
    RA_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_pose_grad_aa, dim3((F + 127) / 128), dim3(128), 0, (hipStream_t)stream, pose6, grad_pose, F,
                       grad6);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

size_t ra_tgv_scratch_bytes(int32_t nx, int32_t ny, int32_t nz) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return 0;
    return align_up((size_t)tgv_blocks(nx, ny, nz) * sizeof(double));
}

int tgv_loss_and_grad(ra_ctx* ctx, int32_t nx, int32_t ny, int32_t nz, const float* u, const float* w,
                      double alpha0, double alpha1, double eps, double scale, double* loss, float* grad_u,
                      float* grad_w, uint32_t flags, void* stream) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    if (nx <= 0 || ny <= 0 || nz <= 0) return fail(ctx, RA_EINVAL, "grid dimensions must be positive");
    if ((long long)nx * ny * nz >= (1LL << 31)) return fail(ctx, RA_EINVAL, "grid has 2^31 or more voxels");
    if (!u || !w) return fail(ctx, RA_EINVAL, "u and w are required");
    if (!(alpha0 >= 0.0) || !(alpha1 >= 0.0) || !(eps >= 1e-18) || !std::isfinite(scale) || !std::isfinite(alpha0) ||
        !std::isfinite(alpha1) || !std::isfinite(eps))
        return fail(ctx, RA_EINVAL, "alpha0, alpha1 >= 0, eps >= 1e-18 and a finite scale are required");
    if (flags & ~RA_ACCUMULATE) return fail(ctx, RA_EINVAL, "unknown flag bits");
    hipStream_t st = (hipStream_t)stream;
    RA_HIP(ctx, hipSetDevice(ctx->device));
    int rc = ensure_scratch(ctx, ra_tgv_scratch_bytes(nx, ny, nz), st);
    if (rc != RA_OK) return rc;
    TgvDims d;
    d.nx = nx; d.ny = ny; d.nz = nz;
    d.n = nx * ny * nz;
    d.sy = nz;
    d.sx = ny * nz;
    d.bz = (nz + TGV_TZ - 1) / TGV_TZ;
    d.by = (ny + TGV_TY - 1) / TGV_TY;
    d.bx = (nx + TGV_XC - 1) / TGV_XC;
    d.a0 = (float)alpha0; d.a1 = (float)alpha1; d.eps = (float)eps;
    const unsigned nblocks = tgv_blocks(nx, ny, nz);      // at most one per voxel: below 2^31
    const dim3 gr(nblocks), blk(TGV_TZ, TGV_TY);
    double* partial = at<double>(ctx, 0);
    hipLaunchKernelGGL(k_tgv, gr, blk, 0, st, d, u, w, (float)scale, (flags & RA_ACCUMULATE) ? 1 : 0, grad_u, grad_w,
                       partial);
    RA_HIP(ctx, hipGetLastError());
    if (loss) {
        hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(NC_THREADS), 0, st, partial, (int)nblocks, ctx->d_f64);
        RA_HIP(ctx, hipMemcpyAsync(ctx->h_f64, ctx->d_f64, sizeof(double), hipMemcpyDeviceToHost, st));
        RA_HIP(ctx, hipStreamSynchronize(st));
        *loss = scale * *ctx->h_f64;
    }
    return RA_OK;
}

int ra_pose_from_euler(ra_ctx* ctx, const double* pose6, int32_t F, double* poses, void* stream) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    if (!pose6 || !poses || F <= 0) return fail(ctx, RA_EINVAL, "pose6, poses and F > 0 are required");
    RA_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_pose_from_euler, dim3((F + 127) / 128), dim3(128), 0, (hipStream_t)stream, pose6, F, poses);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

int ra_pose_grad_euler(ra_ctx* ctx, const double* pose6, const double* grad_pose, int32_t F, double* grad6,
                       void* stream) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    if (!pose6 || !grad_pose || !grad6 || F <= 0)
        return fail(ctx, RA_EINVAL, "pose6, grad_pose, grad6 and F > 0 are required");
    RA_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_pose_grad_euler, dim3((F + 127) / 128), dim3(128), 0, (hipStream_t)stream, pose6, grad_pose,
                       F, grad6);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

int ra_count_updates(ra_ctx* ctx, const ra_grid* grid, int32_t M, const double* elem, const double* poses,
                     int32_t F, const ra_sampling* samp, long long* count, void* stream) {
    int rc = validate(ctx, grid, M, F, samp);
    if (rc != RA_OK) return rc;
    ctx->err.clear();
    if (!elem || !poses || !count) return fail(ctx, RA_EINVAL, "elem, poses and count are required");
    hipStream_t st = (hipStream_t)stream;
    RA_HIP(ctx, hipSetDevice(ctx->device));
    Plan P;
    make_plan(grid, M, F, samp, P, ctx->sums_mode);
    if ((rc = ensure_scratch(ctx, P.total, st)) != RA_OK) return rc;
    const Geo& g = P.g;
    double* xe64 = at<double>(ctx, P.off_xe64);
    unsigned long long* d_count = at<unsigned long long>(ctx, P.off_count);
    hipLaunchKernelGGL(k_elements_f64, dim3((g.E + 255) / 256), dim3(256), 0, st, g.M, g.E, elem, poses, xe64);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, st, reinterpret_cast<float*>(d_count), (size_t)2, 0.0f);
    long long nvox = (long long)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_count, dim3((unsigned)((nvox + 255) / 256)), dim3(256), 0, st, g.nx, g.ny, g.nz,
                       grid->origin[0], grid->origin[1], grid->origin[2], grid->spacing, g.E, xe64, samp->c,
                       samp->fs, samp->K, samp->trunc * samp->sigma, d_count);
    RA_HIP(ctx, hipGetLastError());
    RA_HIP(ctx, hipMemcpyAsync(ctx->h_count, d_count, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    RA_HIP(ctx, hipStreamSynchronize(st));
    *count = (long long)*ctx->h_count;
    return RA_OK;
}

int ra_probe_rates(ra_ctx* ctx, double* fma_per_s, double* exp_per_s, void* stream) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    if (!fma_per_s || !exp_per_s) return fail(ctx, RA_EINVAL, "fma_per_s and exp_per_s are required");
    hipStream_t st = (hipStream_t)stream;
    RA_HIP(ctx, hipSetDevice(ctx->device));
    int rc = ensure_scratch(ctx, align_up((size_t)PROBE_BLOCKS * 256 * sizeof(float)), st);
    if (rc != RA_OK) return rc;
    float* out = at<float>(ctx, 0);
    const int it_fma = 16384, it_exp = 4096;
    hipEvent_t e0, e1;
    RA_HIP(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, RA_EHIP, "hipEventCreate failed");
    }
    auto timed = [&](bool exp_probe, int iters, double& rate) -> hipError_t {
        for (int rep = 0; rep < 2; ++rep) {          // the first launch warms up; the second is timed
            hipError_t e = hipEventRecord(e0, st);
            if (e != hipSuccess) return e;
            if (exp_probe)
                hipLaunchKernelGGL(k_probe_exp, dim3(PROBE_BLOCKS), dim3(256), 0, st, out, iters);
            else
                hipLaunchKernelGGL(k_probe_fma, dim3(PROBE_BLOCKS), dim3(256), 0, st, out, iters, 0.999f, 1e-3f);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
        }
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, e0, e1);
        rate = (double)PROBE_BLOCKS * 256.0 * PROBE_CHAINS * iters / (ms * 1e-3);
        return e;
    };
    hipError_t e = timed(false, it_fma, *fma_per_s);
    if (e == hipSuccess) e = timed(true, it_exp, *exp_per_s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(ctx, RA_EHIP, std::string("rate probe: ") + hipGetErrorString(e));
    return RA_OK;
}

}  // extern "C"

extern "C" {

size_t ra_batch_geo_bytes(void) { return sizeof(Geo); }

int ra_batch_describe(ra_ctx* ctx, const ra_grid* box, int64_t stride_x, int64_t stride_y, int32_t M,
                      const ra_sampling* samp, void* geo, ra_batch_info* info) {
    int rc = validate(ctx, box, M, 1, samp);
    if (rc != RA_OK) return rc;
    ctx->err.clear();
    if (!geo || !info) return fail(ctx, RA_EINVAL, "geo and info are required");
    if (samp->kernel != RA_KERNEL_GAUSSIAN)
        return fail(ctx, RA_ENOTSUP, "the batched step supports the Gaussian profile only");
    if (stride_y < box->nz || stride_x < (int64_t)stride_y * box->ny)
        return fail(ctx, RA_EINVAL, "volume strides smaller than the box");
    Plan P;
    make_plan(box, M, 1, samp, P, RA_SUMS_AUTO, false);
    Geo g = P.g;
    g.vsx = stride_x;
    g.vsy = stride_y;
    g.gsx = (long long)box->ny * box->nz;
    g.gsy = box->nz;
    // the batched forward pairs z-neighbours when it can: D more rows (the adjoint stages
    // them too, and never reads them)
    const int pd = (P.pair_ok && !(g.rz & 1)) ? PAIR_D : 0;
    g.L += pd;
    std::memcpy(geo, &g, sizeof(Geo));
    info->nreg = g.nreg;
    info->jt = P.jt;
    info->exact = P.exact ? 1 : 0;
    info->pair_d = pd;
    info->lmax = g.L;
    info->nvpad = g.nvpad;
    info->rx = g.rx; info->ry = g.ry; info->rz = g.rz;
    // the moment form of the adjoints where the single-call plan takes it and its LDS fits one
    // workgroup on these regions
    Plan Pm;
    make_plan(box, M, 1, samp, Pm);
    const int nbin = 2 * g.jclamp + 1;
    const size_t lds_p = (size_t)nbin * 2 * WAVE * sizeof(float4) + (size_t)MOM_WAVES * 3 * WAVE * sizeof(double);
    const size_t lds_v = (size_t)nbin * 2 * WAVE * sizeof(float4) + (size_t)4 * g.nvpad * sizeof(float);
    info->moment = (Pm.moment && nbin <= MOM_WAVES * MOM_PER && std::max(lds_p, lds_v) <= 160 * 1024) ? 1 : 0;
    info->nbin = nbin;
    info->q_bytes = info->moment ? ((int64_t)M * (samp->K + 2 * P.jt) + 1) * NMOM * (int64_t)sizeof(float) : 0;
    return RA_OK;
}

int ra_batch_tables(ra_ctx* ctx, const void* geo, void* vtab, void* itab, void* stream) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    if (!geo || !vtab || !itab) return fail(ctx, RA_EINVAL, "geo, vtab and itab are required");
    Geo g;
    std::memcpy(&g, geo, sizeof(Geo));
    RA_HIP(ctx, hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_voxel_table, dim3((g.nvpad + 255) / 256), dim3(256), 0, (hipStream_t)stream, g,
                       (float4*)vtab, (int4*)itab);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

}  // extern "C"

namespace {

template <int JT, bool EXACT, int D>
int batch_step_t(ra_ctx* ctx, const ra_batch* b, uint32_t flags, hipStream_t st) {
    const Geo* geos = (const Geo*)b->geos;
    const float4* vtab = (const float4*)b->vtab;
    const int4* itab = (const int4*)b->itab;
    const int2* ifwd = (const int2*)b->items_fwd;
    const int2* ipose = (const int2*)b->items_pose;
    const int2* ivol = (const int2*)b->items_vol;
    const int2* ielem = (const int2*)b->items_elem;
    const int grid = b->grid_blocks > 0 ? b->grid_blocks : 1024;
    const size_t lds_f = (size_t)WAVES * b->lmax * WAVE * sizeof(float);
    const size_t lds_a = lds_f + (size_t)WAVES * b->nvpad * sizeof(float);
    auto kf = k_forward_batch<JT, EXACT, D>;
    auto kp = k_adjoint_batch<JT, EXACT, false, true>;
    auto kv = k_adjoint_batch<JT, EXACT, true, false>;
    RA_HIP(ctx, allow_full_lds(kf));
    RA_HIP(ctx, allow_full_lds(kp));
    RA_HIP(ctx, allow_full_lds(kv));
    hipLaunchKernelGGL(k_batch_elements, dim3(64), dim3(256), 0, st, geos, b->reqs, ielem, b->counts);
    hipLaunchKernelGGL(k_batch_zero, dim3(grid), dim3(256), 0, st, geos, b->reqs, b->counts);
    hipLaunchKernelGGL(kf, dim3(grid), dim3(BLOCK), lds_f, st, geos, b->reqs, vtab, itab, ifwd, b->counts, b->lmax);
    hipLaunchKernelGGL(k_batch_residual, dim3(grid), dim3(BATCH_THREADS), 0, st, geos, b->reqs, b->counts);
    if (b->moment) {
        // moment form: coefficients, each request's table from its dL/ds, then the adjoints
        const size_t lds_v = (size_t)b->nbin * 2 * WAVE * sizeof(float4) + (size_t)4 * b->nvpad * sizeof(float);
        const size_t lds_p = (size_t)b->nbin * 2 * WAVE * sizeof(float4) + (size_t)MOM_WAVES * 3 * WAVE * sizeof(double);
        auto mp = k_adjoint_mom_batch<false, true>;
        auto mv = k_adjoint_mom_batch<true, false>;
        RA_HIP(ctx, allow_full_lds(mp));
        RA_HIP(ctx, allow_full_lds(mv));
        hipLaunchKernelGGL(k_batch_moment_coefs, dim3(1), dim3(2 * b->jt + 1), 0, st, geos, b->reqs, b->counts, b->jt,
                           b->coef);
        hipLaunchKernelGGL(k_batch_moment_table, dim3(grid), dim3(256), 0, st, geos, b->reqs, b->counts, b->jt,
                           b->coef);
        hipLaunchKernelGGL(mp, dim3(grid), dim3(MOM_WAVES * WAVE), lds_p, st, geos, b->reqs, vtab, itab, ipose,
                           b->counts, 1, b->jt, b->nbin);
        hipLaunchKernelGGL(mv, dim3(grid), dim3(MOM_WAVES * WAVE), lds_v, st, geos, b->reqs, vtab, itab, ivol,
                           b->counts, 2, b->jt, b->nbin);
    } else {
        hipLaunchKernelGGL(kp, dim3(grid), dim3(BLOCK), lds_a, st, geos, b->reqs, vtab, itab, ipose, b->counts, 1,
                           b->lmax);
        hipLaunchKernelGGL(kv, dim3(grid), dim3(BLOCK), lds_a, st, geos, b->reqs, vtab, itab, ivol, b->counts, 2,
                           b->lmax);
    }
    hipLaunchKernelGGL(k_batch_pose_chunks, dim3(grid), dim3(256), 0, st, geos, b->reqs, ielem, b->counts);
    hipLaunchKernelGGL(k_batch_pose_update, dim3(grid), dim3(BATCH_THREADS), 0, st, geos, b->reqs, b->counts);
    if (flags & RA_BATCH_APPLY_UPDATES)
        hipLaunchKernelGGL(k_batch_volume_apply, dim3(grid), dim3(BLOCK), 0, st, geos, b->reqs, itab, ivol,
                           b->counts);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

}  // namespace

extern "C" int ra_batch_step(ra_ctx* ctx, const ra_batch* b, uint32_t flags, void* stream) {
    if (!ctx) return RA_EINVAL;
    ctx->err.clear();
    if (!b || !b->geos || !b->reqs || !b->vtab || !b->itab || !b->items_fwd || !b->items_pose || !b->items_vol ||
        !b->items_elem || !b->counts)
        return fail(ctx, RA_EINVAL, "every table of the batch is required");
    if (flags & ~RA_BATCH_APPLY_UPDATES) return fail(ctx, RA_EINVAL, "unknown flag bits");
    if (b->lmax <= 0 || b->nvpad <= 0 || b->nvpad % 4) return fail(ctx, RA_EINVAL, "bad lmax or nvpad");
    if ((size_t)WAVES * b->lmax * WAVE * sizeof(float) + (size_t)WAVES * b->nvpad * sizeof(float) > 160 * 1024)
        return fail(ctx, RA_EINVAL, "lmax / nvpad exceed the LDS of a workgroup");
    const bool ex = b->exact != 0;
    if (b->moment) {
        // the moment form exists for the exact Gaussian window only; its LDS window holds nbin bins
        // of 2 x 64 float4 plus the dL/dp0 sums or the wavefronts' FP64 pose partials
        if (!b->coef) return fail(ctx, RA_EINVAL, "the moment form needs the coefficient scratch (coef)");
        if (!ex || b->jt < 1 || b->jt > JMAX) return fail(ctx, RA_EINVAL, "moment form with a window it does not cover");
        if (b->nbin < 1 || b->nbin > MOM_WAVES * MOM_PER)
            return fail(ctx, RA_EINVAL, "nbin must be the value ra_batch_describe reported");
        const size_t win = (size_t)b->nbin * 2 * WAVE * sizeof(float4);
        if (win + std::max((size_t)4 * b->nvpad * sizeof(float), (size_t)MOM_WAVES * 3 * WAVE * sizeof(double)) >
            160 * 1024)
            return fail(ctx, RA_EINVAL, "nbin / nvpad exceed the LDS of a workgroup");
    }
    RA_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    if (b->pair_d != 0 && (b->pair_d != PAIR_D || !ex))
        return fail(ctx, RA_EINVAL, "pair_d must be the value ra_batch_describe reported");
#define RA_CASE(n)                                                                                      \
    if (ex && b->jt == n)                                                                               \
        return b->pair_d ? batch_step_t<n, true, PAIR_D>(ctx, b, flags, st)                             \
                         : batch_step_t<n, true, 0>(ctx, b, flags, st);
    RA_EXACT_LIST(RA_CASE)
#undef RA_CASE
#define RA_CASE(n) \
    if (!ex && b->jt == n) return batch_step_t<n, false, 0>(ctx, b, flags, st);
    RA_GENERIC_LIST(RA_CASE)
#undef RA_CASE
    return fail(ctx, RA_ENOTSUP, "window half-width not supported");
}
