// Green's-function block assembly, plane-wave right-hand sides and DoF permutations.
//
// Entries of the discretised VIE (§2 eq. 2.4, §3 eq. 3.5, pulse-basis reading):
//   Z[(m,a),(n,b)] = -k^2 V_m V_n G_ab(r_m - r_n)          distinct cells m != n
//   Z[(m,a),(m,b)] = V_m delta_ab [1/chi_m - s(a_m)]       cell diagonal
//   G(d) = g(R) [(1 - j/kR - 1/(kR)^2) I + (-1 + 3j/kR + 3/(kR)^2) d^d^],  g = e^{-jkR}/(4 pi R)
//   s(a) = (2/3) [(1 + j k a) e^{-jka} - 1] - 1/3
// One thread evaluates one (row cell, column cell) pair: one sqrt, one reciprocal and one
// sincos give the 6 distinct entries of the symmetric 3x3 tile, written as 9 entries.
#include "internal.h"

namespace qrvie {

namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ c128 cmul(c128 a, c128 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

struct GeomView {
    const double* center; const int32_t* ptype; const double* tvol; const double* taeq;
    const c128* tchi; const double* toff; double k;
};

__device__ __forceinline__ void cell_pos(const GeomView& g, int p, int cell, double& x, double& y, double& z) {
    const int t = g.ptype[p];
    const double* o = g.toff + ((size_t)t * kCells + cell) * 3;
    x = g.center[3 * p + 0] + o[0];
    y = g.center[3 * p + 1] + o[1];
    z = g.center[3 * p + 2] + o[2];
}

// scale * G(d) as the 6 distinct entries xx, yy, zz, xy, xz, yz.
__device__ __forceinline__ void dyadic6(double dx, double dy, double dz, double k, double scale, c128 e[6]) {
    const double R = sqrt(dx * dx + dy * dy + dz * dz);
    const double iR = 1.0 / R;
    const double kr = k * R;
    const double ikr = 1.0 / kr;
    const double ikr2 = ikr * ikr;
    double sn, cs;
    sincos(kr, &sn, &cs);
    const double g0 = scale * iR * (1.0 / (4.0 * kPi));
    const c128 g = make_double2(g0 * cs, -g0 * sn);          // scale * e^{-jkR} / (4 pi R)
    const c128 gA = cmul(g, make_double2(1.0 - ikr2, -ikr));
    const c128 gB = cmul(g, make_double2(-1.0 + 3.0 * ikr2, 3.0 * ikr));
    const double ux = dx * iR, uy = dy * iR, uz = dz * iR;
    e[0] = make_double2(gA.x + gB.x * ux * ux, gA.y + gB.y * ux * ux);
    e[1] = make_double2(gA.x + gB.x * uy * uy, gA.y + gB.y * uy * uy);
    e[2] = make_double2(gA.x + gB.x * uz * uz, gA.y + gB.y * uz * uz);
    e[3] = make_double2(gB.x * ux * uy, gB.y * ux * uy);
    e[4] = make_double2(gB.x * ux * uz, gB.y * ux * uz);
    e[5] = make_double2(gB.x * uy * uz, gB.y * uy * uz);
}

// V [1/chi - s(a)]: the cell-diagonal entry.
__device__ __forceinline__ c128 diag_entry(double vol, double a, c128 chi, double k) {
    const double ka = k * a;
    double sn, cs;
    sincos(ka, &sn, &cs);
    // (1 + j ka)(cos ka - j sin ka) = cos + ka sin + j (ka cos - sin)
    const double s_re = (2.0 / 3.0) * (cs + ka * sn - 1.0) - 1.0 / 3.0;
    const double s_im = (2.0 / 3.0) * (ka * cs - sn);
    const double den = chi.x * chi.x + chi.y * chi.y;
    const double ic_re = chi.x / den, ic_im = -chi.y / den;
    return make_double2(vol * (ic_re - s_re), vol * (ic_im - s_im));
}

// The 3x3 tile of Z for particle p cell cm (rows) and particle q cell cn (columns).
__device__ __forceinline__ void tile(const GeomView& g, int p, int cm, int q, int cn, c128 e[6], bool& diag) {
    diag = false;
    const int tp = g.ptype[p];
    if (p == q) {
        if (cm == cn) {
            diag = true;
            e[0] = diag_entry(g.tvol[tp], g.taeq[tp], g.tchi[tp], g.k);
            return;
        }
        const double* o = g.toff + (size_t)tp * kCells * 3;
        const double v = g.tvol[tp];
        dyadic6(o[3 * cm] - o[3 * cn], o[3 * cm + 1] - o[3 * cn + 1], o[3 * cm + 2] - o[3 * cn + 2],
                g.k, -g.k * g.k * v * v, e);
        return;
    }
    double xm, ym, zm, xn, yn, zn;
    cell_pos(g, p, cm, xm, ym, zm);
    cell_pos(g, q, cn, xn, yn, zn);
    const double sc = -g.k * g.k * g.tvol[tp] * g.tvol[g.ptype[q]];
    dyadic6(xm - xn, ym - yn, zm - zn, g.k, sc, e);
}

__device__ __forceinline__ void store_tile(c128* B, int64_t ldb, int64_t row, int64_t col, const c128 e[6], bool diag) {
    const c128 z = make_double2(0.0, 0.0);
    // column-major: B[row + a + (col + b) * ldb]
    c128* c0 = B + row + col * ldb;
    c128* c1 = c0 + ldb;
    c128* c2 = c1 + ldb;
    if (diag) {
        c0[0] = e[0]; c0[1] = z; c0[2] = z;
        c1[0] = z; c1[1] = e[0]; c1[2] = z;
        c2[0] = z; c2[1] = z; c2[2] = e[0];
        return;
    }
    c0[0] = e[0]; c0[1] = e[3]; c0[2] = e[4];
    c1[0] = e[3]; c1[1] = e[1]; c1[2] = e[5];
    c2[0] = e[4]; c2[1] = e[5]; c2[2] = e[2];
}

GeomView view(const qrvie_geom* g) {
    return GeomView{g->d_center, g->d_ptype, g->d_tvol, g->d_taeq, g->d_tchi, g->d_toff, g->k};
}

// Self block of each particle type, from cell offsets only (identical atoms give
// bitwise-identical blocks).  One workgroup per type.
__global__ void __launch_bounds__(256) k_assemble_self(GeomView g, const int32_t* type_rep, c128* out) {
    const int t = blockIdx.x;
    const int p = type_rep[t];
    c128* B = out + (size_t)t * kNp * kNp;
    for (int e = threadIdx.x; e < kCells * kCells; e += blockDim.x) {
        const int cm = e % kCells, cn = e / kCells;
        c128 v[6];
        bool d;
        tile(g, p, cm, p, cn, v, d);
        store_tile(B, kNp, 3 * cm, 3 * cn, v, d);
    }
}

// Far blocks: work item = (block descriptor, column particle).
__global__ void __launch_bounds__(256) k_assemble_far(GeomView g, const AsmDesc* descs, const int32_t* wblock,
                                                      const int32_t* wcol) {
    const AsmDesc d = descs[wblock[blockIdx.x]];
    const int qi = wcol[blockIdx.x];
    const int q = d.c0 + qi;
    const int nrc = d.rn * kCells;
    for (int e = threadIdx.x; e < nrc * kCells; e += blockDim.x) {
        const int rc = e % nrc, cn = e / nrc;
        const int p = d.r0 + rc / kCells, cm = rc % kCells;
        c128 v[6];
        bool dg;
        tile(g, p, cm, q, cn, v, dg);
        store_tile(d.B, d.ldb, 3 * (int64_t)rc, 3 * ((int64_t)qi * kCells + cn), v, dg);
    }
}

// Arbitrary particle lists (internal indices): B (3*48*nr x 3*48*nc).
__global__ void __launch_bounds__(256) k_assemble_lists(GeomView g, const int32_t* rows, int nr, const int32_t* cols,
                                                        c128* B, int64_t ldb) {
    const int qi = blockIdx.x;
    const int q = cols[qi];
    const int nrc = nr * kCells;
    for (int e = threadIdx.x; e < nrc * kCells; e += blockDim.x) {
        const int rc = e % nrc, cn = e / nrc;
        const int p = rows[rc / kCells], cm = rc % kCells;
        c128 v[6];
        bool dg;
        tile(g, p, cm, q, cn, v, dg);
        store_tile(B, ldb, 3 * (int64_t)rc, 3 * ((int64_t)qi * kCells + cn), v, dg);
    }
}

// Plane waves: par[r] = (khat.xyz, e.xyz) per RHS; output in caller order.
__global__ void k_rhs(GeomView g, int32_t N, const int32_t* i2c, int nrhs, const double* par, c128* v, int64_t ldv) {
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (cell >= (int64_t)N * kCells || r >= nrhs) return;
    const int p = (int)(cell / kCells), c = (int)(cell % kCells);
    double x, y, z;
    cell_pos(g, p, c, x, y, z);
    const double* pr = par + 6 * r;
    const double ph = g.k * (x * pr[0] + y * pr[1] + z * pr[2]);
    double sn, cs;
    sincos(ph, &sn, &cs);
    const double vol = g.tvol[g.ptype[p]];
    const int64_t dof = ((int64_t)i2c[p] * kCells + c) * 3;
    c128* out = v + r * ldv + dof;
    for (int a = 0; a < 3; ++a) out[a] = make_double2(vol * pr[3 + a] * cs, -vol * pr[3 + a] * sn);
}

// to_internal: out[p*144 + i] = in[i2c[p]*144 + i]; else the inverse.
__global__ void k_permute(int32_t N, const int32_t* i2c, const c128* in, c128* out, int to_internal) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)N * kNp) return;
    const int p = (int)(e / kNp), i = (int)(e % kNp);
    const int64_t ext = (int64_t)i2c[p] * kNp + i;
    if (to_internal) out[e] = in[ext];
    else out[ext] = in[e];
}

}  // namespace

void launch_assemble_self(hipStream_t s, const qrvie_geom* g, c128* out, int ntypes) {
    hipLaunchKernelGGL(k_assemble_self, dim3(ntypes), dim3(256), 0, s, view(g), g->d_trep, out);
}

void launch_assemble_far(hipStream_t s, const qrvie_geom* g, const AsmDesc* d_descs, const int32_t* d_wb,
                         const int32_t* d_wc, int64_t nwork) {
    if (nwork <= 0) return;
    hipLaunchKernelGGL(k_assemble_far, dim3((unsigned)nwork), dim3(256), 0, s, view(g), d_descs, d_wb, d_wc);
}

void launch_assemble_lists(hipStream_t s, const qrvie_geom* g, const int32_t* d_rows, int32_t nr,
                           const int32_t* d_cols, int32_t nc, c128* B, int64_t ldb) {
    if (nr <= 0 || nc <= 0) return;
    hipLaunchKernelGGL(k_assemble_lists, dim3(nc), dim3(256), 0, s, view(g), d_rows, nr, d_cols, B, ldb);
}

void launch_rhs(hipStream_t s, const qrvie_geom* g, int nrhs, const double* d_par, c128* v, int64_t ldv) {
    const int64_t ncell = (int64_t)g->N * kCells;
    dim3 grid((unsigned)((ncell + 255) / 256), nrhs);
    hipLaunchKernelGGL(k_rhs, grid, dim3(256), 0, s, view(g), g->N, g->d_i2c, nrhs, d_par, v, ldv);
}

void launch_permute(hipStream_t s, int32_t N, const int32_t* d_i2c, const c128* in, c128* out, int to_internal) {
    const int64_t n = (int64_t)N * kNp;
    hipLaunchKernelGGL(k_permute, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, d_i2c, in, out, to_internal);
}

}  // namespace qrvie
