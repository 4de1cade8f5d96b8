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

// ----------------------------------------------------------------- cross approximation
// Far blocks couple distinct particles, so every 3 x 3 tile is a full dyadic tile: entry
// (a, b) is e[a] on the diagonal and e[a + b + 2] off it (xy = e3, xz = e4, yz = e5).
__device__ __forceinline__ c128 tile_comp(const c128 e[6], int a, int b) { return a == b ? e[a] : e[a + b + 2]; }

// Row a of scale * G(d) (a known only at run time): gA delta_ab + gB u_a u_b, formed from the
// direction cosine u_a so that no register array is indexed at run time.
__device__ __forceinline__ void dyadic_row(double dx, double dy, double dz, double k, double scale, int a, c128 r[3]) {
    const double R = sqrt(dx * dx + dy * dy + dz * dz);
    const double iR = 1.0 / R;
    const double kr = k * R;
    const double ikr = 1.0 / kr;
    const double ikr2 = ikr * ikr;
    double sn, cs;
    sincos(kr, &sn, &cs);
    const double g0 = scale * iR * (1.0 / (4.0 * kPi));
    const c128 g = make_double2(g0 * cs, -g0 * sn);
    const c128 gA = cmul(g, make_double2(1.0 - ikr2, -ikr));
    const c128 gB = cmul(g, make_double2(-1.0 + 3.0 * ikr2, 3.0 * ikr));
    const double u[3] = {dx * iR, dy * iR, dz * iR};
    const double ua = a == 0 ? u[0] : (a == 1 ? u[1] : u[2]);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const double w = ua * u[b];
        const double dg = a == b ? 1.0 : 0.0;
        r[b] = make_double2(gA.x * dg + gB.x * w, gA.y * dg + gB.y * w);
    }
}

// Row a of the 3 x 3 tile of a far pair (cell cm of particle p, cell cn of particle q); by
// symmetry also column a.
__device__ __forceinline__ void far_row(const GeomView& g, int p, int cm, int q, int cn, int a, c128 r[3]) {
    double xm, ym, zm, xn, yn, zn;
    cell_pos(g, p, cm, xm, ym, zm);
    cell_pos(g, q, cn, xn, yn, zn);
    dyadic_row(xm - xn, ym - yn, zm - zn, g.k, -g.k * g.k * g.tvol[g.ptype[p]] * g.tvol[g.ptype[q]], a, r);
}

__device__ __forceinline__ void far_tile(const GeomView& g, int p, int cm, int q, int cn, c128 e[6]) {
    double xm, ym, zm, xn, yn, zn;
    cell_pos(g, p, cm, xm, ym, zm);
    cell_pos(g, q, cn, xn, yn, zn);
    dyadic6(xm - xn, ym - yn, zm - zn, g.k, -g.k * g.k * g.tvol[g.ptype[p]] * g.tvol[g.ptype[q]], e);
}

template <int NW>
__device__ __forceinline__ double wg_argmax(double v, int& idx, double* rv, int* ri) {
    // maximum of v over the NW waves of the workgroup (ties to the smallest index), its index in idx
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const int oi = __shfl_xor(idx, o, 64);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { rv[threadIdx.x >> 6] = v; ri[threadIdx.x >> 6] = idx; }
    __syncthreads();
    v = rv[0];
    idx = ri[0];
    for (int k = 1; k < NW; ++k)
        if (rv[k] > v || (rv[k] == v && ri[k] < idx)) { v = rv[k]; idx = ri[k]; }
    return v;
}

template <int NW>
__device__ __forceinline__ double wg_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < NW; ++k) s += red[k];
    return s;
}

__device__ __forceinline__ void csub_mul(c128& r, c128 u, c128 w) {
    r.x -= u.x * w.x - u.y * w.y;
    r.y -= u.x * w.y + u.y * w.x;
}

// Cross approximation with partial pivoting of one far block per workgroup (§6.5, Table of
// assembly times: the reported compression step is a cross approximation after Kurz et al.
// 2002, which needs only the pivot rows and columns of a block):
// B ~ U V with U (m x k, ld m) the residual columns and V (k x n, stored by rows: V(l, j) at
// V[j + l n], so a step's reads of the earlier rows are coalesced) the residual rows divided by
// their pivots.  Step k generates pivot row i from the Green's function, subtracts
// the earlier crosses, takes its largest entry j as the pivot, then does the same for column j;
// the next pivot row is the largest entry of that column among rows not used yet.  It stops
// once the newest cross is at most eps times the running Frobenius estimate
// (sum_l ||u_l||^2 ||v_l||^2, cross terms left out), when a residual row or the unused part of
// a column vanishes, or at kmax crosses.  One thread evaluates one cell pair (3 entries of the
// pivot row or column) per visit.  A resumed approximation (k0 > 0: the crosses of an earlier
// launch copied into wider buffers) continues from the saved pivot rows and state.
template <int NT>
__global__ void __launch_bounds__(NT) k_aca(GeomView g, const AcaDesc* descs) {
    constexpr int NW = NT / 64;
    const AcaDesc d = descs[blockIdx.x];
    const int m = d.rn * kNp, n = d.cn * kNp;
    __shared__ unsigned used[kAcaMaxRows / 32];
    __shared__ c128 urow[kAcaMaxRank], vcol[kAcaMaxRank];
    __shared__ double rv[NW], red[NW];
    __shared__ int ri[NW];
    const int t = threadIdx.x;
    for (int e = t; e < (m + 31) / 32; e += NT) used[e] = 0u;
    int i = 0, k = d.k0;
    double normS2 = 0.0;
    if (k > 0) {
        normS2 = d.state[0];
        i = (int)d.state[1];
        __syncthreads();
        if (t == 0)
            for (int l = 0; l < k; ++l) used[d.piv[l] >> 5] |= 1u << (d.piv[l] & 31);
    }
    for (; k < d.kmax; ++k) {
        __syncthreads();
        for (int l = t; l < k; l += NT) urow[l] = d.U[i + (int64_t)l * m];
        __syncthreads();
        // residual of pivot row i: each thread one cell (3 consecutive columns) at a time
        const int p = d.r0 + i / kNp, cm = (i % kNp) / 3, a = i % 3;
        double best = -1.0;
        int bj = n;
        for (int c = t; c < n / 3; c += NT) {
            c128 r[3];
            far_row(g, p, cm, d.c0 + c / kCells, c % kCells, a, r);
            const c128* v = d.V + 3 * c;
            for (int l = 0; l < k; ++l, v += n) {
                const c128 u = urow[l];
                csub_mul(r[0], u, v[0]);
                csub_mul(r[1], u, v[1]);
                csub_mul(r[2], u, v[2]);
            }
            c128* out = d.V + 3 * c + (int64_t)k * n;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                out[b] = r[b];
                const double a2 = r[b].x * r[b].x + r[b].y * r[b].y;
                if (a2 > best) { best = a2; bj = 3 * c + b; }
            }
        }
        best = wg_argmax<NW>(best, bj, rv, ri);
        if (!(best > 0.0)) break;                          // the residual row vanishes
        const c128 piv = d.V[bj + (int64_t)k * n];
        __syncthreads();                                   // every wave holds the pivot before the
                                                           // wave owning it normalises it in place
        const c128 inv = make_double2(piv.x / best, -piv.y / best);
        double vn2 = 0.0;
        for (int c = t; c < n / 3; c += NT) {
            c128* w = d.V + 3 * c + (int64_t)k * n;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const c128 r = w[b];
                const c128 q = make_double2(r.x * inv.x - r.y * inv.y, r.x * inv.y + r.y * inv.x);
                w[b] = q;
                vn2 += q.x * q.x + q.y * q.y;
            }
        }
        vn2 = wg_sum<NW>(vn2, red);
        for (int l = t; l <= k; l += NT) vcol[l] = d.V[bj + (int64_t)l * n];
        if (t == 0) {
            used[i >> 5] |= 1u << (i & 31);
            d.piv[k] = i;
        }
        __syncthreads();
        // residual of pivot column bj, the same way over the rows
        const int q = d.c0 + bj / kNp, cn = (bj % kNp) / 3, b = bj % 3;
        double un2 = 0.0, bc = -1.0;
        int bi = m;
        for (int c = t; c < m / 3; c += NT) {
            c128 v[3];
            far_row(g, d.r0 + c / kCells, c % kCells, q, cn, b, v);   // the tile is symmetric
            const c128* u = d.U + 3 * c;
            for (int l = 0; l < k; ++l, u += m) {
                const c128 w = vcol[l];
                csub_mul(v[0], u[0], w);
                csub_mul(v[1], u[1], w);
                csub_mul(v[2], u[2], w);
            }
            c128* out = d.U + 3 * c + (int64_t)k * m;
#pragma unroll
            for (int aa = 0; aa < 3; ++aa) {
                const int r = 3 * c + aa;
                out[aa] = v[aa];
                const double a2 = v[aa].x * v[aa].x + v[aa].y * v[aa].y;
                un2 += a2;
                if (!((used[r >> 5] >> (r & 31)) & 1u) && a2 > bc) { bc = a2; bi = r; }
            }
        }
        un2 = wg_sum<NW>(un2, red);
        bc = wg_argmax<NW>(bc, bi, rv, ri);
        normS2 += un2 * vn2;
        if (un2 * vn2 <= d.eps * d.eps * normS2 || !(bc > 0.0)) { ++k; break; }
        i = bi;
    }
    if (t == 0) {
        *d.rank_out = k;
        d.state[0] = normS2;
        d.state[1] = (double)i;
    }
}

// Certification without the assembled block: each workgroup covers 48 rows and up to
// kCertGroup column tiles of 48 of one block (16 x 16 cell pairs per tile, one per thread),
// generates the entries of B from the Green's function and accumulates Q R from LDS-staged
// 32-term chunks.  partial[w] = ||B - Q R||^2 and partial[nwg + w] = ||B||^2 over its region.
// descs are found from the prefix sums wg_first (nd + 1 entries) of their workgroup counts.
constexpr int kCertGroup = 4;

__global__ void __launch_bounds__(256) k_cert_fused(GeomView g, const CertDesc* descs, const int64_t* wg_first,
                                                    int nd, double* partial) {
    const int64_t w = blockIdx.x;
    int lo = 0, hi = nd - 1;
    while (lo < hi) {                                      // last descriptor with wg_first <= w
        const int mid = (lo + hi + 1) >> 1;
        if (wg_first[mid] <= w) lo = mid;
        else hi = mid - 1;
    }
    const CertDesc d = descs[lo];
    const int64_t local = w - wg_first[lo];
    const int ntn = d.cn * kNp / 48, ngrp = (ntn + kCertGroup - 1) / kCertGroup;
    const int i0 = 48 * (int)(local / ngrp), tj0 = kCertGroup * (int)(local % ngrp);
    const int tj1 = min(ntn, tj0 + kCertGroup);
    const int t = threadIdx.x, cr = t >> 4, cc = t & 15;
    __shared__ c128 Qs[48][33];
    __shared__ c128 Rs[32][49];
    __shared__ double red[4];
    double e2 = 0.0, b2 = 0.0;
    for (int tj = tj0; tj < tj1; ++tj) {
        const int j0 = 48 * tj;
        c128 acc[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) acc[a][b] = make_double2(0.0, 0.0);
        for (int k0 = 0; k0 < d.r; k0 += 32) {
            const int kc = min(32, d.r - k0);
            __syncthreads();
            for (int e = t; e < 48 * 32; e += 256) {
                const int rr = e % 48, kk = e / 48;
                Qs[rr][kk] = kk < kc ? d.Q[(i0 + rr) + (int64_t)(k0 + kk) * d.ldq] : make_double2(0.0, 0.0);
                const int kr = e % 32, jc = e / 32;
                Rs[kr][jc] = kr < kc ? d.R[(k0 + kr) + (int64_t)(j0 + jc) * d.ldr] : make_double2(0.0, 0.0);
            }
            __syncthreads();
            for (int l = 0; l < kc; ++l) {
                c128 qv[3], rw[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) qv[a] = Qs[3 * cr + a][l];
#pragma unroll
                for (int b = 0; b < 3; ++b) rw[b] = Rs[l][3 * cc + b];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        acc[a][b].x = fma(qv[a].x, rw[b].x, fma(-qv[a].y, rw[b].y, acc[a][b].x));
                        acc[a][b].y = fma(qv[a].x, rw[b].y, fma(qv[a].y, rw[b].x, acc[a][b].y));
                    }
            }
        }
        const int rc = i0 / 3 + cr, ccell = j0 / 3 + cc;     // cell rows / columns of the block
        c128 e[6];
        far_tile(g, d.r0 + rc / kCells, rc % kCells, d.c0 + ccell / kCells, ccell % kCells, e);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const c128 v = tile_comp(e, a, b);
                const double dx = v.x - acc[a][b].x, dy = v.y - acc[a][b].y;
                e2 += dx * dx + dy * dy;
                b2 += v.x * v.x + v.y * v.y;
            }
    }
    e2 = wg_sum<4>(e2, red);
    b2 = wg_sum<4>(b2, red);
    if (t == 0) {
        partial[w] = e2;
        partial[gridDim.x + w] = b2;
    }
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

void launch_aca(hipStream_t s, const qrvie_geom* g, const AcaDesc* d, int n, bool wide) {
    if (n <= 0) return;
    if (wide) hipLaunchKernelGGL(k_aca<1024>, dim3((unsigned)n), dim3(1024), 0, s, view(g), d);
    else hipLaunchKernelGGL(k_aca<256>, dim3((unsigned)n), dim3(256), 0, s, view(g), d);
}
void launch_cert_fused(hipStream_t s, const qrvie_geom* g, const CertDesc* d, const int64_t* wg_first, int nd,
                       int64_t nwg, double* partial) {
    if (nwg > 0) hipLaunchKernelGGL(k_cert_fused, dim3((unsigned)nwg), dim3(256), 0, s, view(g), d, wg_first, nd, partial);
}
int64_t cert_workgroups(int32_t rn, int32_t cn) {
    const int64_t ntn = (int64_t)cn * kNp / 48;
    return (int64_t)rn * kNp / 48 * ((ntn + kCertGroup - 1) / kCertGroup);
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
