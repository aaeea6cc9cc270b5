// lbm_internal.h -- shared definitions of the library: lattice tables, kernel argument
// blocks and the kernel launchers. Not part of the public ABI (see include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

namespace lbm {

// ---------------------------------------------------------------------------------
// Lattice vectors e_a (Sec. 8, Table 1) in the library's order, with opposites.
// D2V9: rest, 4 axis, 4 diagonals. D3V19: rest, 6 axis, 12 face diagonals; every
// non-rest vector at an odd index is followed by its opposite.
// ---------------------------------------------------------------------------------
template <int LAT>
struct Lat;

template <>
struct Lat<LBM_D2V9> {
    static constexpr int Q = 9, D = 2;
    static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
};

template <>
struct Lat<LBM_D3V19> {
    static constexpr int Q = 19, D = 3;
    static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
};

// ---------------------------------------------------------------------------------
// Kernel argument block (passed by value). Float constants are the FP64 host constants
// rounded once to FP32.
// ---------------------------------------------------------------------------------
// n / d for 0 <= n < 2^31 as (n m) >> sh, with l = ceil(log2 d), m = ceil(2^(31+l) / d)
// and sh = 31 + l: m < 2^32, and the excess n (m d - 2^(31+l)) / (d 2^(31+l)) < 1/d never
// carries n / d past the next integer.
struct FastDiv {
    uint32_t m;
    uint32_t sh;
};

inline FastDiv make_fastdiv(int d)
{
    uint32_t l = 0;
    while ((1ll << l) < (long long)d) ++l;
    return FastDiv{(uint32_t)(((1ull << (31 + l)) + (uint64_t)d - 1) / (uint64_t)d), 31 + l};
}

struct Geometry {
    int nx, ny, nz;
    int stride;       // elements between population arrays
    int ntx;          // 256-node tiles per x row
    int nblocks;      // tiles in the grid = ntx * ny * nz
    FastDiv div_ntx;  // division by ntx
    FastDiv div_ny;   // division by ny
    int slip;         // free-slip wall planes (LBM_SLIP_Y | LBM_SLIP_Z)
    const uint8_t *mask;  // nullable
    const float *s;       // nullable
};

constexpr int kQMax = 19;

struct Physics {
    float rho0;
    float omega;      // 1 / tau
    float what[4];    // w_k / I_0 by shell k = |e|^2
    float lam[4];     // what_k A / c_s^2: weight of e.j in the equilibrium, rounded so that
                      // sum_a lam_a e_a e_a = identity holds exactly in FP32 constants
    float A, Bc;      // reduced EDF coefficients
    float C[4];       // C_k (source term)
    float C2[4];      // 2 C_k
    float Cp[4];      // C_k c_s^2 (equilibrium, U = u / c_s)
    float cs, inv_cs2;
    float E[3];       // xi-units per step
    float B[3];
    float c1q[kQMax]; // A (e_q.E) / c_s, library velocity order
    float c2q[kQMax]; // 2 Bc (e_q.E) / c_s
    float scale, inv_scale;  // storage scale (F16: 2^k), 1 otherwise
    // Forward step in stored units (deviations x scale), omega folded per shell:
    // o_q = c0 D_q + ol_k e_q.j + owhat_k drho + whatS_k rho [omega (Bc (e_q.U)^2 + Cp_k U^2)
    //       + source_q], and o_0 from mass closure.
    float c0;         // 1 - omega
    float ol[4];      // ~omega lam_k, with c0 + n1 ol_1 + n2 ol_2 = 1 exactly
    float owhat[4];   // omega what_k
    float whatS[4];   // what_k scale
    float omBc;       // omega Bc
    float oCp[4];     // omega Cp_k
    float c1v[3];     // A E / c_s, so that c1q = e_q . c1v
    float inv_cs2S;   // inv_cs2 / scale
    float shE[3];     // velocity shift: scale tau c_s E
    float shB;        //   and scale tau c_s^2 (multiplies U x B)
};

struct StepArgs {
    Geometry g;
    Physics ph;
    int remap;          // XCD-contiguous block order
    int sr;             // stochastic rounding of the stored 16-bit values
    uint32_t sr_key;    // the step's key for the random bits of stochastic rounding
    const void *links;  // per-node link masks (nullable: no solids)
    const void *src;
    void *dst;
};

struct InitArgs {
    Geometry g;
    Physics ph;
    const double *rho;
    const double *u;     // nullable
    const void *links;   // per-node link masks (nullable: no solids)
    void *dst;
};

struct GatherArgs {
    Geometry g;
    Physics ph;
    const void *links;
    const void *src;
    float *rho;       // nullable
    float *u;         // nullable
    double *f64;      // nullable (export)
    double *partials; // nullable (reduction)
    double what_rho0[4];  // what_k rho0 in FP64 (export of full populations)
    int N;
    int odd;          // src is in the odd layout of the in-place step
};

struct AdjointArgs {
    Geometry g;
    Physics ph;
    int remap;
    const void *links;
    const void *state;
    const float *lam_in;
    float *lam_out;
    float *grad_s;    // nullable
    double *partials; // per-wave (dE_x, dE_y, dE_z, dtau)
    int accumulate;   // add this step's wave sums to partials instead of overwriting
};

// Fourth-order thermal model on D1V7 (lbm_thermal.hip), deviations d_a = f_a - rho0 what_a.
// The equilibrium is what_a p(xi_a) with sum_a what_a p(xi_a) xi_a^k = M_k, k = 0..4; the
// deviation of p from rho0 has coefficients dc = H^-1 dM, split into the even block
// (k = 0, 2, 4) and the odd block (k = 1, 3) of the Hankel matrix of the what moments.
// Constants of the D1V7 thermal step. Inside the step, velocities are the integer e_a
// (lattice units: u_e = c_s u, thetabar_e = c_s^2 thetabar), so that every power of e_a
// is exact in FP32; the fields convert to xi = e / c_s only on input and output.
struct ThermalPhysics {
    float omega;       // 1 / tau
    float rho0;
    float scale, inv_scale;  // stored value = deviation * scale (2^k for FP16, else 1)
    float tb_hi, tb_lo;  // T = sum what e^2 = c_s^2 I_2 / I_0 (thetabar_e of the weight), two FP32 parts
    float g0;          // g held at the weight's value, I_4 I_0 / I_2^2
    float what[7];     // w / I_0 in the order e = 0, +1, -1, +2, -2, +3, -3
    // Polynomial coefficients c = H^-1 M of the moment targets, with the linear parts of
    // M_3, M_4 folded in (H the Hankel matrices of the e-moments of what, in long double):
    //   (c0, c2, c4) = (drho, 0, 0) + pe * D + he * r4,   (c1, c3) = ko * j + ho * r3
    float pe[3], he[3], ko[2], ho[2];
    float k6;          // 6 T (1 - g0)
    double T;          // T in FP64 (init)
    double cs;         // c_s (conversion of the fields)
    double what_rho0[7];  // rho0 what_a in FP64 (export)
};

struct ThermalArgs {
    int n;             // nodes
    int stride;        // elements between population arrays
    ThermalPhysics ph;
    const void *src;   // states: FP32, FP16 x 2^k or BF16 deviations (lbm_params.storage)
    void *dst;
    const double *rho, *u, *tb;   // init fields (u, tb nullable)
    float *out_rho, *out_u, *out_tb;  // moment fields (nullable)
    double *f64;       // export (nullable)
    double *partials;  // per-block (sum drho, sum j_e, sum dE_e), lattice units (nullable)
    int odd;           // src holds the streamed ("odd") layout of the in-place step
};

// mode 0: step src -> dst; 1: init into dst; 2: fields; 3: export; 4: partial sums;
// 5, 6: the two phases of the in-place step (src == dst); 7: odd layout src -> even dst
hipError_t launch_thermal(int mode, int storage, const ThermalArgs &a, int nblocks_reduce, hipStream_t st);

// Launchers (lbm_kernels.hip). Each returns hipSuccess or the launch error.
// force: 0 no field, 1 E only, 2 E and B.
hipError_t launch_step(int lattice, int storage, int force, const StepArgs &a, hipStream_t st);
// the same with stochastic rounding (16-bit storage; a.sr set)
hipError_t launch_step_sr(int lattice, int storage, int force, const StepArgs &a, hipStream_t st);
// rho <-> mu of the weight (lbm_density.hip); to_mu selects the inverse
hipError_t launch_density(int D, int stats, double theta, const double *in, double *out, size_t n, bool to_mu,
                          hipStream_t st);
// Per-node link masks from g.mask into links (link_mask_bytes(lattice) per node).
hipError_t launch_links(int lattice, const Geometry &g, void *links, hipStream_t st);
size_t link_mask_bytes(int lattice);
hipError_t launch_init(int lattice, int storage, const InitArgs &a, hipStream_t st);
hipError_t launch_gather(int lattice, int storage, const GatherArgs &a, int nblocks_reduce,
                         hipStream_t st);
// Sum per-block partials [nparts][ncomp] (ncomp <= 8) into out (+= if accumulate).
// `stage` (kReduceStage * ncomp doubles, nullable) enables a two-stage reduction.
// Convergence measure of Sec. 9.4 (lbm_speed_change): per-block partials [block][2]
// Threads per block of the node kernels (k_step, the in-place phases, the adjoint) for rows
// of nx nodes at V nodes per thread: kBlock, or, where one block covers a whole row, the row
// rounded up to whole waves, so that short rows (e.g. 128 nodes) launch no idle waves.
int row_block_threads(int nx, int V);

// Device address (per device, looked up once) and size of the library's static scratch
// array, and the FP64 totals of lbm_current reduced through it into device out[4].
hipError_t static_scratch(int device, double **ptr, size_t *bytes);
size_t totals_scratch_bytes();
hipError_t launch_totals_noalloc(int lattice, int storage, const GatherArgs &a, double rho0, double cs, double *out,
                                 hipStream_t st, double *scratch_dev);
hipError_t launch_speed_change(const float *u, int D, int N, float *speed, int have_prev, double *partials,
                               int nblocks, hipStream_t st);
hipError_t launch_reduce_final(const double *partials, int nparts, int ncomp, double *out,
                               int accumulate, hipStream_t st, double *stage);
int step_vector_width(int lattice, int storage, int nx, bool local_phase_solids = false);
int use_xcd_remap(int lattice, bool mask, bool soft);
int remap_code(int remap, int ntx);
// shift: the adjoint of the velocity-shift forcing (k_adjoint_shift), else of the source
hipError_t launch_adjoint(int lattice, int storage, bool mag, bool shift, const AdjointArgs &a, hipStream_t st);
// In-place step (lbm_aa.hip), a.src == a.dst: phase 0 takes the state from the two-buffer
// layout to the odd layout, phase 1 back. launch_canon writes the two-buffer layout of an
// odd-layout state a.src into a.dst (a distinct buffer).
hipError_t launch_step_aa(int lattice, int storage, int force, int phase, const StepArgs &a, hipStream_t st);
hipError_t launch_step_aa_sr(int lattice, int storage, int force, int phase, const StepArgs &a, hipStream_t st);
hipError_t launch_canon(int lattice, int storage, const StepArgs &a, hipStream_t st);
hipError_t launch_seed(int lattice, const Geometry &g, float value_per_unit_e, int axis, float *lam,
                       hipStream_t st);

// Host constants (lbm_consts.cpp).
int weight_integrals(int stats, int D, double theta, double mu, double out[4]);
int weight_integrals_n(int stats, int D, double theta, double mu, int n, double *out);
int d1v7_constants(const double I[5], double *cs, double w[4]);
int compute_constants(const lbm_params *p, lbm_constants *k);

constexpr int kBlock = 256;        // threads per block of the node kernels
constexpr int kReduceBlocks = 1024;  // blocks of the gather/reduce kernel
constexpr int kReduceStage = 256;    // blocks of the first stage of a partials reduction

}  // namespace lbm
