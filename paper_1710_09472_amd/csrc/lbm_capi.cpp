// lbm_capi.cpp -- the extern "C" boundary of the library (declared in include/lbm.h):
// argument validation, constants, buffer binding and kernel launches on the caller's
// stream. No device memory is allocated here.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "lbm_internal.h"

using namespace lbm;

// Extra elements between population arrays (a multiple of 256), so that the Q arrays do
// not all start at the same offset modulo large powers of two (measured: +1-4 % on
// MI355X). LBM_STRIDE_PAD overrides it (rounded to a multiple of 256).
static int stride_pad()
{
    static const int pad = [] {
        const char *e = std::getenv("LBM_STRIDE_PAD");
        const int v = e ? std::atoi(e) : 1024;
        return v < 0 ? 0 : (v + 255) / 256 * 256;
    }();
    return pad;
}

struct lbm_s {
    lbm_params p;
    lbm_constants k;
    int D = 0, Q = 0;
    int N = 0, stride = 0;
    size_t elem = 4;
    const uint8_t *mask = nullptr;
    const float *s = nullptr;
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;
    bool aa = false;  // one state buffer: in-place steps (AA pattern)
    int parity = 0;   // in-place steps since the last even layout, mod 2
    unsigned long long t = 0;  // index of the next step (selects the stochastic-rounding bits)
    unsigned char *work = nullptr;
    hipStream_t stream = nullptr;
    Geometry g{};
    Physics ph{};
    void *links = nullptr;  // per-node link masks inside the work buffer
    bool initialized = false;
    bool adj_held = false;  // work_adj holds adjoint contributions not yet reduced
    bool thermal = false;   // D1V7: the fourth-order thermal model
    ThermalPhysics tph{};
    std::string err;
};

namespace {

thread_local std::string g_create_error;

int fail(lbm_t h, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(lbm_t h, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (h)
        h->err = buf;
    else
        g_create_error = buf;
    return code;
}

int hip_fail(lbm_t h, hipError_t e, const char *what)
{
    return fail(h, LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

int lattice_dims(int lattice, int *Q, int *D)
{
    if (lattice == LBM_D2V9) {
        *Q = 9;
        *D = 2;
        return LBM_OK;
    }
    if (lattice == LBM_D3V19) {
        *Q = 19;
        *D = 3;
        return LBM_OK;
    }
    if (lattice == LBM_D3V15) {
        *Q = 15;
        *D = 3;
        return LBM_OK;
    }
    if (lattice == LBM_D1V7) {
        *Q = 7;
        *D = 1;
        return LBM_OK;
    }
    return LBM_EINVAL;
}

constexpr int kD1V7E[7] = {0, 1, -1, 2, -2, 3, -3};

size_t elem_size(int storage) { return storage == LBM_F32 ? 4 : 2; }

struct Sizes {
    int N, stride, nblocks, ntx;
    size_t state, work, adjoint;
};

// Workspace layout (bytes from its start): FP64 totals; per-block partials of the
// reductions; second-stage scratch; link masks (256-byte aligned); FP64 per-block
// partials of dJ/dE, dJ/dtau, one per wave, held across adjoint steps (256-byte aligned).
struct WorkLayout {
    size_t parts, stage, links, adj, total;
};

WorkLayout work_layout(int nblocks, int stride)
{
    WorkLayout w;
    const size_t parts = std::max((size_t)kReduceBlocks * 5, (size_t)nblocks * 4);
    w.parts = 64;
    w.stage = w.parts + parts * sizeof(double);
    w.links = (w.stage + (size_t)kReduceStage * 8 * sizeof(double) + 255) / 256 * 256;
    w.adj = (w.links + (size_t)stride * 4 + 255) / 256 * 256;
    w.total = w.adj + (size_t)nblocks * (kBlock / 64) * 4 * sizeof(double);
    return w;
}

// Validation shared by create and the size query. Writes the message through fail().
// The key of step t for the random bits of stochastic rounding: the SplitMix64 output
// function (Steele, Lea and Flood, OOPSLA 2014) of t, upper half. The kernels hash it
// with the node index (sr_node).
uint32_t sr_step_key(unsigned long long t)
{
    uint64_t z = (uint64_t)t + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (uint32_t)(z >> 32);
}

int validate(const lbm_params *p, lbm_t h, Sizes *sz)
{
    if (!p) return fail(h, LBM_EINVAL, "null params");
    int Q, D;
    if (lattice_dims(p->lattice, &Q, &D) != LBM_OK) return fail(h, LBM_EINVAL, "unknown lattice %d", p->lattice);
    if (p->stats != LBM_FERMI_DIRAC && p->stats != LBM_BOSE_EINSTEIN && p->stats != LBM_HERMITE)
        return fail(h, LBM_EINVAL, "unknown weight function %d", p->stats);
    if (p->storage != LBM_F32 && p->storage != LBM_F16 && p->storage != LBM_BF16)
        return fail(h, LBM_EINVAL, "unknown storage %d", p->storage);
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(h, LBM_EINVAL, "grid sizes must be >= 1");
    if (D == 2 && p->nz != 1) return fail(h, LBM_EINVAL, "D2V9 needs nz = 1");
    if (D == 1) {
        if (p->ny != 1 || p->nz != 1) return fail(h, LBM_EINVAL, "D1V7 needs ny = nz = 1");
        for (int i = 0; i < 3; ++i)
            if (p->E[i] != 0.0 || p->B[i] != 0.0) return fail(h, LBM_EINVAL, "D1V7 (thermal model): no E or B");
        if (p->slip) return fail(h, LBM_EINVAL, "D1V7 (thermal model): no free-slip walls");
        if (p->order != 0 && p->order != 3 && p->order != 4)
            return fail(h, LBM_EINVAL, "D1V7 (thermal model): order must be 3 or 4 (0 = 4)");
    } else if (p->order != 0) {
        return fail(h, LBM_EINVAL, "order: the D2V9/D3V19 model is of second order (order must be 0)");
    }
    const double N = (double)p->nx * p->ny * p->nz;
    const double stride = std::ceil(N / 256.0) * 256.0 + stride_pad();
    if (stride * Q >= 2147483647.0) return fail(h, LBM_EINVAL, "grid too large (Q * N must stay below 2^31)");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(h, LBM_EINVAL, "tau must be finite and > 1/2");
    if (!(p->rho0 > 0) || !std::isfinite(p->rho0)) return fail(h, LBM_EINVAL, "rho0 must be finite and > 0");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->E[i]) || !std::isfinite(p->B[i])) return fail(h, LBM_EINVAL, "E and B must be finite");
    if (D == 2 && (p->E[2] != 0.0 || p->B[0] != 0.0 || p->B[1] != 0.0))
        return fail(h, LBM_EINVAL, "2D lattice: only E_x, E_y and B_z may be non-zero");
    if (p->storage == LBM_F16 && (p->dev_scale_log2 < 0 || p->dev_scale_log2 > 40))
        return fail(h, LBM_EINVAL, "F16 storage: dev_scale_log2 must be in 0..40");
    if (p->stats == LBM_FERMI_DIRAC && (!(p->theta > 0) || !std::isfinite(p->theta) || !std::isfinite(p->mu)))
        return fail(h, LBM_EINVAL, "Fermi-Dirac weight needs finite theta > 0 and finite mu");
    if (p->stats == LBM_BOSE_EINSTEIN && (!(p->theta > 0) || !std::isfinite(p->theta) || !(p->mu < 0) ||
                                          !std::isfinite(p->mu)))
        return fail(h, LBM_EINVAL, "Bose-Einstein weight needs finite theta > 0 and finite mu < 0");
    if (p->forcing != LBM_FORCE_SOURCE && p->forcing != LBM_FORCE_SHIFT)
        return fail(h, LBM_EINVAL, "unknown forcing scheme %d", p->forcing);
    if (p->slip & ~(LBM_SLIP_Y | LBM_SLIP_Z)) return fail(h, LBM_EINVAL, "slip: only LBM_SLIP_Y and LBM_SLIP_Z bits");
    if (D == 2 && (p->slip & LBM_SLIP_Z)) return fail(h, LBM_EINVAL, "2D lattice: no z walls");
    if (((p->slip & LBM_SLIP_Y) && p->ny < 3) || ((p->slip & LBM_SLIP_Z) && p->nz < 3))
        return fail(h, LBM_EINVAL, "a free-slip axis needs at least 3 planes (2 walls and fluid)");
    if (p->rounding != LBM_ROUND_NEAREST && p->rounding != LBM_ROUND_STOCHASTIC)
        return fail(h, LBM_EINVAL, "unknown rounding %d", p->rounding);
    if (p->rounding == LBM_ROUND_STOCHASTIC && (p->storage == LBM_F32 || p->lattice == LBM_D1V7))
        return fail(h, LBM_EINVAL, "stochastic rounding: FP16 or BF16 storage of D2V9/D3V19 only");
    if (sz) {
        sz->N = (int)N;
        sz->stride = (int)stride;
        sz->ntx = (p->nx + kBlock - 1) / kBlock;
        sz->nblocks = sz->ntx * p->ny * p->nz;
        sz->state = (size_t)Q * (size_t)sz->stride * elem_size(p->storage);
        sz->adjoint = (size_t)Q * (size_t)sz->stride * sizeof(float);
        sz->work = work_layout(sz->nblocks, sz->stride).total;
    }
    return LBM_OK;
}

void fill_physics(lbm_t h)
{
    const lbm_constants &k = h->k;
    Physics &ph = h->ph;
    ph = Physics{};
    ph.rho0 = (float)h->p.rho0;
    ph.omega = (float)(1.0 / h->p.tau);
    for (int s = 0; s < 4; ++s) {
        ph.what[s] = (float)k.what[s];
        ph.C[s] = (float)k.C[s];
        ph.Cp[s] = (float)(k.C[s] * k.cs * k.cs);
    }
    // lam_k = what_k A / c_s^2. Round the diagonal-shell value to a multiple of 2^-26 and
    // solve the axis-shell value from n1 lam_1 + n2 lam_2 = 1 (n1, n2: vectors of each
    // shell with e_x != 0), so the identity holds exactly for the FP32 constants.
    {
        const double l2 = k.what[2] * k.A / (k.cs * k.cs);
        const float l2f = (float)(std::nearbyint(l2 * 67108864.0) / 67108864.0);
        const double n1 = 2.0, n2 = (h->D == 2) ? 4.0 : 8.0;
        const float l1f = (float)((1.0 - n2 * (double)l2f) / n1);
        ph.lam[0] = 0.0f;
        ph.lam[1] = l1f;
        ph.lam[2] = l2f;
        ph.lam[3] = 0.0f;
    }
    ph.A = (float)k.A;
    ph.Bc = (float)k.Bc;
    for (int s = 0; s < 4; ++s) ph.C2[s] = (float)(2.0 * k.C[s]);
    {
        int Q = 0, D = 0, e[3 * kQMax];
        lbm_lattice_info(h->p.lattice, &Q, &D, e);
        for (int q = 0; q < Q; ++q) {
            const double eE = (e[3 * q] * h->p.E[0] + e[3 * q + 1] * h->p.E[1] + e[3 * q + 2] * h->p.E[2]) / k.cs;
            ph.c1q[q] = (float)(k.A * eE);
            ph.c2q[q] = (float)(2.0 * k.Bc * eE);
        }
    }
    ph.cs = (float)k.cs;
    ph.inv_cs2 = (float)(1.0 / (k.cs * k.cs));
    for (int i = 0; i < 3; ++i) {
        ph.E[i] = (float)h->p.E[i];
        ph.B[i] = (float)h->p.B[i];
    }
    if (h->p.storage == LBM_F16) {
        ph.scale = std::ldexp(1.0f, h->p.dev_scale_log2);
        ph.inv_scale = std::ldexp(1.0f, -h->p.dev_scale_log2);
    } else {
        ph.scale = 1.0f;
        ph.inv_scale = 1.0f;
    }
    // Forward-step constants. c0 = 1 - omega in FP32 (exact for omega >= 1/2); the linear
    // equilibrium weights times omega are split as for lam above, with the diagonal-shell
    // value a multiple of 2^-m for the largest m that keeps both values exact FP32 numbers
    // and c0 + n1 ol_1 + n2 ol_2 = 1 exact, so that momentum relaxes without a bias from
    // the rounding of the constants.
    ph.c0 = 1.0f - ph.omega;
    {
        const double R = 1.0 - (double)ph.c0;
        const double l2 = k.what[2] * k.A / (k.cs * k.cs);
        const double n1 = 2.0, n2 = (h->D == 2) ? 4.0 : 8.0;
        for (int m = 30; m >= 12; --m) {
            const double sc = std::ldexp(1.0, m);
            const double o2 = std::nearbyint(R * l2 * sc) / sc;
            const double o1 = (R - n2 * o2) / n1;
            if ((double)(float)o2 == o2 && (double)(float)o1 == o1 && n1 * o1 + n2 * o2 == R) {
                ph.ol[1] = (float)o1;
                ph.ol[2] = (float)o2;
                break;
            }
        }
    }
    const double om = (double)ph.omega;
    ph.omBc = (float)(om * k.Bc);
    for (int s = 0; s < 4; ++s) {
        ph.owhat[s] = (float)(om * k.what[s]);
        ph.whatS[s] = (float)(k.what[s] * (double)ph.scale);
        ph.oCp[s] = (float)(om * k.C[s] * k.cs * k.cs);
    }
    for (int i = 0; i < 3; ++i) ph.c1v[i] = (float)(k.A * h->p.E[i] / k.cs);
    // velocity shift: j_eq - j = rho (shE + shB (U x B)) in stored lattice units
    for (int i = 0; i < 3; ++i) ph.shE[i] = (float)((double)ph.scale * h->p.tau * k.cs * h->p.E[i]);
    ph.shB = (float)((double)ph.scale * h->p.tau * k.cs * k.cs);
    ph.inv_cs2S = (float)(1.0 / (k.cs * k.cs) / (double)ph.scale);
}

bool has_B(const lbm_t h) { return h->p.B[0] != 0.0 || h->p.B[1] != 0.0 || h->p.B[2] != 0.0; }
bool has_E(const lbm_t h) { return h->p.E[0] != 0.0 || h->p.E[1] != 0.0 || h->p.E[2] != 0.0; }
// kernel forcing variant: 0 none, 1 source with E, 2 source with E and B, 3 velocity shift
int force_level(const lbm_t h)
{
    if (h->p.forcing == LBM_FORCE_SHIFT) return (has_E(h) || has_B(h)) ? 3 : 0;
    return has_B(h) ? 2 : (has_E(h) ? 1 : 0);
}
// link masks exist where there are solids: obstacles of the mask, or slip wall planes
bool has_solids(const lbm_t h) { return h->mask != nullptr || h->p.slip != 0; }
const void *links_of(const lbm_t h) { return has_solids(h) ? h->links : nullptr; }
bool adjoint_supported(const lbm_t h) { return !h->thermal; }

// Constants of the thermal kernel (D1V7) from the weights: what, xi, the weight's
// thetabar and g, and the inverses of the even and odd blocks of the Hankel matrix of the
// what moments, m_k = sum_a what_a xi_a^k (equal to the weight's moments up to order 9).
void fill_thermal(lbm_t h)
{
    ThermalPhysics &t = h->tph;
    t = ThermalPhysics{};
    const lbm_constants &k = h->k;
    t.omega = (float)(1.0 / h->p.tau);
    t.rho0 = (float)h->p.rho0;
    t.scale = h->p.storage == LBM_F16 ? (float)std::ldexp(1.0, h->p.dev_scale_log2) : 1.f;
    t.inv_scale = 1.f / t.scale;  // a power of two: exact
    long double what[7], m[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // e-moments sum what e^j
    for (int a = 0; a < 7; ++a) {
        what[a] = (long double)k.w[std::abs(kD1V7E[a])] / (long double)k.I0;
        t.what[a] = (float)what[a];
        t.what_rho0[a] = (double)(what[a] * (long double)h->p.rho0);
        long double pw = 1.0L;
        for (int j = 0; j < 9; ++j) {
            m[j] += what[a] * pw;
            pw *= kD1V7E[a];
        }
    }
    t.T = (double)m[2];
    t.tb_hi = (float)m[2];
    t.tb_lo = (float)(m[2] - (long double)t.tb_hi);
    t.cs = k.cs;
    t.g0 = (float)(m[4] / (3.0L * m[2] * m[2]));  // I_4 I_0 / I_2^2 (the same in any unit of velocity)
    // even block over (0, 2, 4): E[i][j] = m[2i + 2j]; odd block over (1, 3): m[2i + 2j + 2]
    const long double E[3][3] = {{m[0], m[2], m[4]}, {m[2], m[4], m[6]}, {m[4], m[6], m[8]}};
    const long double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                            E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                            E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    long double Ei[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            // inverse = adjugate / det; adj[i][j] = cofactor of E[j][i]
            const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
            Ei[i][j] = (E[r0][c0] * E[r1][c1] - E[r0][c1] * E[r1][c0]) / det;
        }
    const long double O[2][2] = {{m[2], m[4]}, {m[4], m[6]}};
    const long double dO = O[0][0] * O[1][1] - O[0][1] * O[1][0];
    const long double Oi[2][2] = {{O[1][1] / dO, -O[0][1] / dO}, {-O[1][0] / dO, O[0][0] / dO}};
    // With D = dE - T drho and dtb = D / rho - u^2, the targets split into linear parts and
    // remainders of second order:
    //   dM_3 = 3 T j + r3,   r3 = j (u^2 + 3 dtb)
    //   dM_4 = 3 g0 (2 T D + T^2 drho) + r4,   r4 = rho [u^2 (u^2 + 6 dtb + 6 T (1 - g0)) + 3 g0 dtb^2]
    // and H^-1 applied to the weight's own moments (m0, m2, m4) = (1, T, 3 g0 T^2) is (1, 0, 0),
    // so the drho column of the even solve is exactly (1, 0, 0).
    const long double T = m[2], g0 = m[4] / (3.0L * m[2] * m[2]);
    if (h->p.order == 3) {
        // third-order truncation: degree 3, even block over (0, 2) only; M_4 is not matched
        // (c4 = 0, no r4 term), and (1, 0) is again the drho column
        const long double d2 = m[0] * m[4] - m[2] * m[2];
        t.pe[0] = (float)(-m[2] / d2);
        t.pe[1] = (float)(m[0] / d2);
        t.pe[2] = 0.f;
        t.he[0] = t.he[1] = t.he[2] = 0.f;
    } else {
        for (int i = 0; i < 3; ++i) {
            t.pe[i] = (float)(Ei[i][1] + 6.0L * g0 * T * Ei[i][2]);
            t.he[i] = (float)Ei[i][2];
        }
    }
    for (int i = 0; i < 2; ++i) {
        t.ko[i] = (float)(Oi[i][0] + 3.0L * T * Oi[i][1]);
        t.ho[i] = (float)Oi[i][1];
    }
    t.k6 = (float)(6.0L * T * (1.0L - g0));
}

ThermalArgs thermal_args(const lbm_t h)
{
    ThermalArgs a{};
    a.n = h->N;
    a.stride = h->stride;
    a.ph = h->tph;
    return a;
}

double *work_out(lbm_t h) { return reinterpret_cast<double *>(h->work); }
double *work_parts(lbm_t h) { return reinterpret_cast<double *>(h->work + work_layout(h->g.nblocks, h->stride).parts); }
double *work_stage(lbm_t h) { return reinterpret_cast<double *>(h->work + work_layout(h->g.nblocks, h->stride).stage); }
void *work_links(lbm_t h) { return h->work + work_layout(h->g.nblocks, h->stride).links; }
double *work_adj(lbm_t h) { return reinterpret_cast<double *>(h->work + work_layout(h->g.nblocks, h->stride).adj); }

}  // namespace

extern "C" {

const char *lbm_status_string(int status)
{
    switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_EUNSUPPORTED: return "unsupported configuration";
    case LBM_EDEVICE: return "HIP device error";
    case LBM_ENONFINITE: return "non-finite value in reduction";
    case LBM_ESTATE: return "call out of order";
    default: return "unknown status";
    }
}

const char *lbm_last_error(lbm_t h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int lbm_compute_constants(const lbm_params *p, lbm_constants *out)
{
    if (!p || !out) return fail(nullptr, LBM_EINVAL, "null argument");
    const int rc = compute_constants(p, out);
    if (rc == LBM_EUNSUPPORTED) return fail(nullptr, rc, "a quadrature weight is not positive for this lattice and weight");
    if (rc != LBM_OK) return fail(nullptr, rc, "invalid lattice, weight function or weight parameters");
    return LBM_OK;
}

int lbm_lattice_info(int lattice, int *Q, int *D, int *e)
{
    int q, d;
    if (lattice_dims(lattice, &q, &d) != LBM_OK || lattice == LBM_D3V15)
        return fail(nullptr, LBM_EINVAL, "lattice %d has no kernels", lattice);
    if (Q) *Q = q;
    if (D) *D = d;
    if (e) {
        for (int a = 0; a < q; ++a) {
            if (lattice == LBM_D1V7) {
                e[3 * a] = kD1V7E[a];
                e[3 * a + 1] = 0;
                e[3 * a + 2] = 0;
            } else if (lattice == LBM_D2V9) {
                e[3 * a] = Lat<LBM_D2V9>::ex[a];
                e[3 * a + 1] = Lat<LBM_D2V9>::ey[a];
                e[3 * a + 2] = 0;
            } else {
                e[3 * a] = Lat<LBM_D3V19>::ex[a];
                e[3 * a + 1] = Lat<LBM_D3V19>::ey[a];
                e[3 * a + 2] = Lat<LBM_D3V19>::ez[a];
            }
        }
    }
    return LBM_OK;
}

int lbm_buffer_sizes(const lbm_params *p, size_t *state_bytes, size_t *work_bytes, size_t *adjoint_bytes,
                     size_t *stride)
{
    Sizes sz;
    const int rc = validate(p, nullptr, &sz);
    if (rc != LBM_OK) return rc;
    if (state_bytes) *state_bytes = sz.state;
    if (work_bytes) *work_bytes = sz.work;
    if (adjoint_bytes) *adjoint_bytes = sz.adjoint;
    if (stride) *stride = (size_t)sz.stride;
    return LBM_OK;
}

int lbm_workspace_bytes(const lbm_params *p, size_t *state_bytes, size_t *work_bytes)
{
    return lbm_buffer_sizes(p, state_bytes, work_bytes, nullptr, nullptr);
}

int lbm_create(const lbm_params *p, const uint8_t *mask, const float *s, void *state_a, void *state_b, void *work,
               void *stream, lbm_t *out)
{
    if (!out) return fail(nullptr, LBM_EINVAL, "null output handle pointer");
    *out = nullptr;
    Sizes sz;
    int rc = validate(p, nullptr, &sz);
    if (rc != LBM_OK) return rc;
    if (p->lattice == LBM_D3V15) {
        lbm_constants k;
        rc = compute_constants(p, &k);
        return fail(nullptr, rc == LBM_OK ? LBM_EUNSUPPORTED : rc,
                    "D3V15 is not supported (its rest weight is negative under the electron weight)");
    }
    if (!state_a || !work) return fail(nullptr, LBM_EINVAL, "state_a and work are required");
    if (state_a == state_b) return fail(nullptr, LBM_EINVAL, "state_a and state_b must be distinct buffers");
    if (p->lattice == LBM_D1V7) {
        if (mask || s) return fail(nullptr, LBM_EUNSUPPORTED, "D1V7 (thermal model): no solids or porosity");
    }
    lbm_s *h = new (std::nothrow) lbm_s;
    if (!h) return fail(nullptr, LBM_EDEVICE, "out of host memory");
    h->p = *p;
    rc = compute_constants(p, &h->k);
    if (rc != LBM_OK) {
        delete h;
        return fail(nullptr, rc, rc == LBM_EUNSUPPORTED ? "a quadrature weight is not positive"
                                                          : "invalid weight parameters");
    }
    lattice_dims(p->lattice, &h->Q, &h->D);
    h->N = sz.N;
    h->stride = sz.stride;
    h->elem = elem_size(p->storage);
    h->mask = mask;
    h->s = s;
    h->buf[0] = state_a;
    h->buf[1] = state_b;
    h->aa = state_b == nullptr;
    h->work = static_cast<unsigned char *>(work);
    h->stream = static_cast<hipStream_t>(stream);
    h->g.nx = p->nx;
    h->g.ny = p->ny;
    h->g.nz = p->nz;
    h->g.stride = sz.stride;
    h->g.ntx = sz.ntx;
    h->g.nblocks = sz.nblocks;
    h->g.div_ntx = make_fastdiv(sz.ntx);
    h->g.div_ny = make_fastdiv(p->ny);
    h->g.mask = mask;
    h->g.s = s;
    h->g.slip = p->slip;
    h->thermal = p->lattice == LBM_D1V7;
    if (h->thermal)
        fill_thermal(h);
    else
        fill_physics(h);
    h->links = work_links(h);
    if (has_solids(h)) {
        const hipError_t e = launch_links(p->lattice, h->g, h->links, h->stream);
        if (e != hipSuccess) {
            delete h;
            return fail(nullptr, LBM_EDEVICE, "link mask kernel launch: %s", hipGetErrorString(e));
        }
    }
    *out = h;
    return LBM_OK;
}

void lbm_destroy(lbm_t h) { delete h; }

namespace {
int density_common(const lbm_params *p, const double *in, double *out, size_t n, void *stream, bool to_mu)
{
    if (!p) return fail(nullptr, LBM_EINVAL, "null params");
    int Q, D;
    if (lattice_dims(p->lattice, &Q, &D) != LBM_OK) return fail(nullptr, LBM_EINVAL, "unknown lattice %d", p->lattice);
    if (D == 1) return fail(nullptr, LBM_EUNSUPPORTED, "rho(mu) is provided in 2D and 3D");
    if (p->stats != LBM_FERMI_DIRAC && p->stats != LBM_BOSE_EINSTEIN)
        return fail(nullptr, LBM_EINVAL, "rho(mu) needs the Fermi-Dirac or Bose-Einstein weight");
    if (!(p->theta > 0) || !std::isfinite(p->theta)) return fail(nullptr, LBM_EINVAL, "theta must be finite and > 0");
    if (n > 0 && (!in || !out)) return fail(nullptr, LBM_EINVAL, "null array");
    const hipError_t e = launch_density(D, p->stats, p->theta, in, out, n, to_mu, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(nullptr, LBM_EDEVICE, "density kernel launch: %s", hipGetErrorString(e));
    return LBM_OK;
}
}  // namespace

int lbm_density_from_mu(const lbm_params *p, const double *mu, double *rho, size_t n, void *stream)
{
    return density_common(p, mu, rho, n, stream, false);
}

int lbm_mu_from_density(const lbm_params *p, const double *rho, double *mu, size_t n, void *stream)
{
    return density_common(p, rho, mu, n, stream, true);
}

int lbm_init_thermal(lbm_t h, const double *rho, const double *u, const double *thetabar)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!h->thermal) return fail(h, LBM_EUNSUPPORTED, "lbm_init_thermal needs the D1V7 thermal model");
    if (!rho) return fail(h, LBM_EINVAL, "rho is required");
    ThermalArgs a = thermal_args(h);
    a.rho = rho;
    a.u = u;
    a.tb = thetabar;
    a.dst = h->buf[h->cur];
    const hipError_t e = launch_thermal(1, h->p.storage, a, 0, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "thermal init kernel launch");
    h->initialized = true;
    h->parity = 0;
    h->t = 0;
    return LBM_OK;
}

int lbm_init(lbm_t h, const double *rho, const double *u)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!rho) return fail(h, LBM_EINVAL, "rho is required");
    if (h->thermal) return lbm_init_thermal(h, rho, u, nullptr);
    InitArgs a{};
    a.g = h->g;
    a.ph = h->ph;
    a.rho = rho;
    a.u = u;
    a.links = links_of(h);
    a.dst = h->buf[h->cur];
    const hipError_t e = launch_init(h->p.lattice, h->p.storage, a, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "init kernel launch");
    h->initialized = true;
    h->parity = 0;
    h->t = 0;
    return LBM_OK;
}

int lbm_step(lbm_t h, int nsteps)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (nsteps < 0) return fail(h, LBM_EINVAL, "nsteps must be >= 0");
    if (!h->initialized) return fail(h, LBM_ESTATE, "lbm_step before lbm_init or lbm_set_state");
    StepArgs a{};
    a.g = h->g;
    a.ph = h->ph;
    a.links = links_of(h);
    a.remap = use_xcd_remap(h->p.lattice, has_solids(h), h->s != nullptr);
    a.sr = h->p.rounding == LBM_ROUND_STOCHASTIC ? 1 : 0;
    if (h->thermal && h->aa) {
        ThermalArgs ta = thermal_args(h);
        ta.src = ta.dst = h->buf[0];
        for (int t = 0; t < nsteps; ++t) {
            const hipError_t e = launch_thermal(5 + h->parity, h->p.storage, ta, 0, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "in-place thermal step kernel launch");
            h->parity ^= 1;
            ++h->t;
        }
        return LBM_OK;
    }
    if (h->thermal) {
        ThermalArgs ta = thermal_args(h);
        for (int t = 0; t < nsteps; ++t) {
            ta.src = h->buf[h->cur];
            ta.dst = h->buf[h->cur ^ 1];
            const hipError_t e = launch_thermal(0, h->p.storage, ta, 0, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "thermal step kernel launch");
            h->cur ^= 1;
            ++h->t;
        }
        return LBM_OK;
    }
    const int force = force_level(h);
    if (h->aa) {
        a.src = a.dst = h->buf[0];
        for (int t = 0; t < nsteps; ++t) {
            a.sr_key = sr_step_key(h->t);
            const hipError_t e = launch_step_aa(h->p.lattice, h->p.storage, force, h->parity, a, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "in-place step kernel launch");
            h->parity ^= 1;
            ++h->t;
        }
        return LBM_OK;
    }
    for (int t = 0; t < nsteps; ++t) {
        a.src = h->buf[h->cur];
        a.dst = h->buf[h->cur ^ 1];
        a.sr_key = sr_step_key(h->t);
        const hipError_t e = launch_step(h->p.lattice, h->p.storage, force, a, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "step kernel launch");
        h->cur ^= 1;
        ++h->t;
    }
    return LBM_OK;
}

int lbm_step_from(lbm_t h, const void *src, void *dst)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!src || !dst || src == dst) return fail(h, LBM_EINVAL, "src and dst must be distinct non-null buffers");
    if (h->thermal) {
        ThermalArgs ta = thermal_args(h);
        ta.src = src;
        ta.dst = dst;
        const hipError_t e = launch_thermal(0, h->p.storage, ta, 0, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "thermal step kernel launch");
        ++h->t;
        return LBM_OK;
    }
    StepArgs a{};
    a.g = h->g;
    a.ph = h->ph;
    a.links = links_of(h);
    a.remap = use_xcd_remap(h->p.lattice, has_solids(h), h->s != nullptr);
    a.sr = h->p.rounding == LBM_ROUND_STOCHASTIC ? 1 : 0;
    a.sr_key = sr_step_key(h->t);
    a.src = src;
    a.dst = dst;
    const hipError_t e = launch_step(h->p.lattice, h->p.storage, force_level(h), a, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "step kernel launch");
    ++h->t;
    return LBM_OK;
}

static int thermal_gather(lbm_t h, const void *state, float *rho, float *u, float *tb, double *f64, double *parts)
{
    ThermalArgs a = thermal_args(h);
    a.src = state ? state : h->buf[h->cur];
    a.odd = (!state && h->aa && h->parity) ? 1 : 0;
    a.out_rho = rho;
    a.out_u = u;
    a.out_tb = tb;
    a.f64 = f64;
    a.partials = parts;
    const hipError_t e = launch_thermal(parts ? 4 : (f64 ? 3 : 2), h->p.storage, a, kReduceBlocks, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "thermal gather kernel launch");
    return LBM_OK;
}

// Reduce the thermal per-block partials (already in work_parts) to (sum drho, sum j, sum dE).
static int thermal_totals(lbm_t h, double tot[3])
{
    hipError_t e = launch_reduce_final(work_parts(h), kReduceBlocks, 3, work_out(h), 0, h->stream, work_stage(h));
    if (e != hipSuccess) return hip_fail(h, e, "reduce kernel launch");
    e = hipMemcpyAsync(tot, work_out(h), 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "copy of totals");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
    return LBM_OK;
}

static int gather_common(lbm_t h, const void *state, float *rho, float *u, double *f64, double *parts)
{
    if (h->thermal) return thermal_gather(h, state, rho, u, nullptr, f64, parts);
    GatherArgs a{};
    a.g = h->g;
    a.ph = h->ph;
    a.links = links_of(h);
    a.src = state ? state : h->buf[h->cur];
    a.rho = rho;
    a.u = u;
    a.f64 = f64;
    a.partials = parts;
    a.N = h->N;
    a.odd = (!state && h->aa && h->parity) ? 1 : 0;
    for (int k = 0; k < 4; ++k) a.what_rho0[k] = h->k.what[k] * h->p.rho0;
    const hipError_t e = launch_gather(h->p.lattice, h->p.storage, a, kReduceBlocks, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "gather kernel launch");
    return LBM_OK;
}

int lbm_moments(lbm_t h, float *rho, float *u)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!h->initialized) return fail(h, LBM_ESTATE, "lbm_moments before lbm_init or lbm_set_state");
    if (!rho && !u) return LBM_OK;
    return gather_common(h, nullptr, rho, u, nullptr, nullptr);
}

int lbm_thetabar(lbm_t h, float *thetabar)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!h->thermal) return fail(h, LBM_EUNSUPPORTED, "thetabar is a field of the D1V7 thermal model");
    if (!thetabar) return fail(h, LBM_EINVAL, "thetabar is required");
    if (!h->initialized) return fail(h, LBM_ESTATE, "lbm_thetabar before lbm_init or lbm_set_state");
    return thermal_gather(h, nullptr, nullptr, nullptr, thetabar, nullptr, nullptr);
}

int lbm_energy(lbm_t h, double *out)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!h->thermal) return fail(h, LBM_EUNSUPPORTED, "lbm_energy is a total of the D1V7 thermal model");
    if (!out) return fail(h, LBM_EINVAL, "out is required");
    if (!h->initialized) return fail(h, LBM_ESTATE, "lbm_energy before lbm_init or lbm_set_state");
    int rc = thermal_gather(h, nullptr, nullptr, nullptr, nullptr, nullptr, work_parts(h));
    if (rc != LBM_OK) return rc;
    double tot[3];
    rc = thermal_totals(h, tot);
    if (rc != LBM_OK) return rc;
    // sum over nodes of sum_a f xi^2; the weight's state contributes rho0 I_2 / I_0 per node
    *out = (double)h->N * h->p.rho0 * (h->k.I2 / h->k.I0) + tot[2] / (h->tph.cs * h->tph.cs);
    if (!std::isfinite(*out)) return fail(h, LBM_ENONFINITE, "non-finite energy total");
    return LBM_OK;
}

int lbm_speed_change(lbm_t h, const float *u, float *speed, int have_previous, double *out)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!u || !speed || !out) return fail(h, LBM_EINVAL, "u, speed and out are required");
    hipError_t e = launch_speed_change(u, h->D, (int)h->N, speed, have_previous ? 1 : 0, work_parts(h), kReduceBlocks,
                                       h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "speed change kernel launch");
    e = launch_reduce_final(work_parts(h), kReduceBlocks, 2, work_out(h), 0, h->stream, work_stage(h));
    if (e != hipSuccess) return hip_fail(h, e, "reduce kernel launch");
    double tot[2];
    e = hipMemcpyAsync(tot, work_out(h), sizeof(tot), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "copy of totals");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
    *out = (have_previous && tot[1] > 0) ? tot[0] / tot[1] : 0.0;
    if (!std::isfinite(*out)) return fail(h, LBM_ENONFINITE, "non-finite speed change");
    return LBM_OK;
}

int lbm_export_f64(lbm_t h, const void *state, double *dst)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!dst) return fail(h, LBM_EINVAL, "dst is required");
    if (!state && !h->initialized) return fail(h, LBM_ESTATE, "export of the current state before init");
    return gather_common(h, state, nullptr, nullptr, dst, nullptr);
}

int lbm_current(lbm_t h, double out[4])
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!out) return fail(h, LBM_EINVAL, "out is required");
    if (!h->initialized) return fail(h, LBM_ESTATE, "lbm_current before lbm_init or lbm_set_state");
    int rc = gather_common(h, nullptr, nullptr, nullptr, nullptr, work_parts(h));
    if (rc != LBM_OK) return rc;
    if (h->thermal) {
        double tot[3];
        rc = thermal_totals(h, tot);
        if (rc != LBM_OK) return rc;
        out[0] = (double)h->N * h->p.rho0 + tot[0];
        out[1] = tot[1] / h->tph.cs;  // lattice units to xi
        out[2] = out[3] = 0.0;
        for (int i = 0; i < 2; ++i)
            if (!std::isfinite(out[i])) return fail(h, LBM_ENONFINITE, "non-finite total (component %d)", i);
        return LBM_OK;
    }
    hipError_t e = launch_reduce_final(work_parts(h), kReduceBlocks, 5, work_out(h), 0, h->stream, work_stage(h));
    if (e != hipSuccess) return hip_fail(h, e, "reduce kernel launch");
    double tot[5];
    e = hipMemcpyAsync(tot, work_out(h), sizeof(tot), hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "copy of totals");
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "stream synchronize");
    // tot = (sum drho, sum d e_x, sum d e_y, sum d e_z, fluid nodes); momentum to xi-units
    out[0] = tot[4] * h->p.rho0 + tot[0];
    for (int i = 0; i < 3; ++i) out[1 + i] = tot[1 + i] / h->k.cs;
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(out[i])) return fail(h, LBM_ENONFINITE, "non-finite total (component %d)", i);
    return LBM_OK;
}

int lbm_current_noalloc(lbm_t h, double *out)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!out) return fail(h, LBM_EINVAL, "out is required");
    if (!h->initialized) return fail(h, LBM_ESTATE, "lbm_current_noalloc before lbm_init or lbm_set_state");
    if (h->thermal) return fail(h, LBM_EUNSUPPORTED, "lbm_current_noalloc covers the D2V9 and D3V19 lattices");
    int device = 0;
    hipError_t e = h->stream ? hipStreamGetDevice(h->stream, &device) : hipGetDevice(&device);
    if (e != hipSuccess) return hip_fail(h, e, "device of the handle's stream");
    double *scratch = nullptr;
    size_t bytes = 0;
    e = static_scratch(device, &scratch, &bytes);
    if (e != hipSuccess) return hip_fail(h, e, "address of the static scratch array");
    if (totals_scratch_bytes() > bytes)
        return fail(h, LBM_EINVAL, "the totals reduction needs %zu bytes of scratch, above the %zu of the static array",
                    totals_scratch_bytes(), bytes);
    GatherArgs a{};
    a.g = h->g;
    a.ph = h->ph;
    a.links = links_of(h);
    a.src = h->buf[h->cur];
    a.N = h->N;
    a.odd = (h->aa && h->parity) ? 1 : 0;
    for (int k = 0; k < 4; ++k) a.what_rho0[k] = h->k.what[k] * h->p.rho0;
    e = launch_totals_noalloc(h->p.lattice, h->p.storage, a, h->p.rho0, h->k.cs, out, h->stream, scratch);
    if (e != hipSuccess) return hip_fail(h, e, "totals kernel launch");
    return LBM_OK;
}

int lbm_get_state(lbm_t h, void *dst)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!dst) return fail(h, LBM_EINVAL, "dst is required");
    if (h->aa && h->parity) {
        if (dst == h->buf[0]) return fail(h, LBM_EINVAL, "dst must not be the handle's own state buffer");
        if (h->thermal) {
            ThermalArgs ta = thermal_args(h);
            ta.src = h->buf[0];
            ta.dst = dst;
            const hipError_t e = launch_thermal(7, h->p.storage, ta, 0, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "state layout kernel launch");
            return LBM_OK;
        }
        StepArgs a{};
        a.g = h->g;
        a.ph = h->ph;
        a.links = links_of(h);
        a.src = h->buf[0];
        a.dst = dst;
        const hipError_t e = launch_canon(h->p.lattice, h->p.storage, a, h->stream);
        if (e != hipSuccess) return hip_fail(h, e, "state layout kernel launch");
        return LBM_OK;
    }
    const hipError_t e = hipMemcpyAsync(dst, h->buf[h->cur], (size_t)h->Q * h->stride * h->elem,
                                        hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "state copy");
    return LBM_OK;
}

int lbm_set_state(lbm_t h, const void *src)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!src) return fail(h, LBM_EINVAL, "src is required");
    const hipError_t e = hipMemcpyAsync(h->buf[h->cur], src, (size_t)h->Q * h->stride * h->elem,
                                        hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "state copy");
    h->initialized = true;
    h->parity = 0;
    h->t = 0;
    return LBM_OK;
}

int lbm_set_step_index(lbm_t h, unsigned long long t)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    h->t = t;
    return LBM_OK;
}

int lbm_set_fields(lbm_t h, const double E[3], const double B[3])
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!E || !B) return fail(h, LBM_EINVAL, "E and B are required");
    lbm_params q = h->p;
    for (int i = 0; i < 3; ++i) {
        q.E[i] = E[i];
        q.B[i] = B[i];
    }
    const int rc = validate(&q, h, nullptr);
    if (rc != LBM_OK) return rc;
    h->p = q;
    if (h->thermal)
        fill_thermal(h);
    else
        fill_physics(h);
    return LBM_OK;
}

int lbm_set_tau(lbm_t h, double tau)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    lbm_params q = h->p;
    q.tau = tau;
    const int rc = validate(&q, h, nullptr);
    if (rc != LBM_OK) return rc;
    h->p = q;
    if (h->thermal)
        fill_thermal(h);
    else
        fill_physics(h);
    return LBM_OK;
}

int lbm_adjoint_seed(lbm_t h, int axis, double norm, float *lam)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!lam) return fail(h, LBM_EINVAL, "lam is required");
    if (!adjoint_supported(h))
        return fail(h, LBM_EUNSUPPORTED, "the adjoint covers the isothermal model only");
    if (axis < 0 || axis >= h->D) return fail(h, LBM_EINVAL, "axis must be in 0..D-1");
    if (!(norm != 0.0) || !std::isfinite(norm)) return fail(h, LBM_EINVAL, "norm must be finite and non-zero");
    const hipError_t e = launch_seed(h->p.lattice, h->g, (float)(1.0 / (h->k.cs * norm)), axis, lam, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "seed kernel launch");
    h->adj_held = false;  // a new reverse pass
    return LBM_OK;
}

int lbm_adjoint_step(lbm_t h, const void *state, const float *lam_in, float *lam_out, float *grad_s,
                     double *grad_scalars)
{
    if (!h) return fail(nullptr, LBM_EINVAL, "null handle");
    if (!state || !lam_in || !lam_out) return fail(h, LBM_EINVAL, "state, lam_in and lam_out are required");
    if (lam_in == lam_out) return fail(h, LBM_EINVAL, "lam_in and lam_out must be distinct buffers");
    if (!adjoint_supported(h))
        return fail(h, LBM_EUNSUPPORTED, "the adjoint covers the isothermal model only");
    AdjointArgs a{};
    a.g = h->g;
    a.ph = h->ph;
    a.links = links_of(h);
    a.remap = use_xcd_remap(h->p.lattice, has_solids(h), h->s != nullptr);
    a.state = state;
    a.lam_in = lam_in;
    a.lam_out = lam_out;
    a.grad_s = grad_s;
    a.partials = work_adj(h);
    a.accumulate = h->adj_held ? 1 : 0;
    hipError_t e = launch_adjoint(h->p.lattice, h->p.storage, has_B(h), h->p.forcing == LBM_FORCE_SHIFT, a, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "adjoint kernel launch");
    h->adj_held = true;
    if (grad_scalars) {
        e = launch_reduce_final(work_adj(h), h->g.nblocks * (row_block_threads(h->g.nx, 1) / 64), 4, grad_scalars, 1,
                                h->stream,
                                work_stage(h));
        if (e != hipSuccess) return hip_fail(h, e, "reduce kernel launch");
        h->adj_held = false;
    }
    return LBM_OK;
}

}  // extern "C"
