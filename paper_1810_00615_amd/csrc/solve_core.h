// Partition solve of a constant-coefficient (Toeplitz) tridiagonal system by one
// workgroup: Thomas elimination of per-thread chunks, cyclic reduction of the
// separator system in LDS down to one wave, parallel cyclic reduction of the last
// (at most 64) equations with cross-lane moves, back substitution.  Shared by the
// shifted solves (single problem and batched) and the trajectory recomputation.
#pragma once
#include "aao_internal.h"

namespace aao {

// LDS needed by partition_solve: the table (3 CW + 8 entries) followed by the
// reduced-system area (6 NT entries).
__host__ __device__ constexpr int psolve_tab_entries(int CW) { return 3 * CW + 8; }
__host__ __device__ constexpr int psolve_lds_entries(int CW, int NT)
{
    return psolve_tab_entries(CW) + 6 * NT;
}

// Normalised tridiagonal equation a X_{k-1} + X_k + c X_{k+1} = d.
template <typename A> struct TriEq {
    cx<A> a, c, d;
};

// Eliminate the neighbours k -+ s from equation k (both normalised); missing
// neighbours pass zeros.  Returns the new equation, normalised.
template <typename A>
__device__ __forceinline__ TriEq<A> reduce_eq(TriEq<A> m, TriEq<A> l, TriEq<A> r)
{
    const cx<A> one = {A(1), A(0)};
    TriEq<A> o;
    const cx<A> dg = cfms(cfms(one, m.a, l.c), m.c, r.a);   // 1 - a cl - c ar
    const cx<A> nd = cfms(cfms(m.d, m.a, l.d), m.c, r.d);   // d - a dl - c dr
    const cx<A> q = recip(dg);
    o.a = -((m.a * l.a) * q);
    o.c = -((m.c * r.c) * q);
    o.d = nd * q;
    return o;
}

template <typename A>
__device__ __forceinline__ cx<A> csel(bool b, cx<A> x, cx<A> y)
{
    return {b ? x.x : y.x, b ? x.y : y.y};
}

template <typename A>
__device__ __forceinline__ cx<A> shfl_cx(cx<A> v, int src)
{
    return {__shfl(v.x, src, 64), __shfl(v.y, src, 64)};
}

// Solve tridiag(e, d, e) x = r with n unknowns.  Thread t owns unknowns
// [t*CW, t*CW + len); y[] holds its part of r on entry and of x on exit.
//
// Chunk t is split into an interior (its first len-1 unknowns) and a separator
// (its last unknown).  With the interior eliminated, x_i = y_i + u_i X_{t-1} +
// v_i X_t, where y is the interior solution with zero neighbours and u, v its
// responses to the left / right separator.  The matrix being Toeplitz, the
// elimination factors (1/pivot, e/pivot), the forward part of u and the end values
// of u and v are the same for every full chunk: one thread tabulates them (and the
// end values for the shorter last chunk) in LDS, every thread regenerates u and v
// backwards from the table, so a thread keeps only y in registers.
//
// The separators satisfy a tridiagonal system with one equation per chunk.  Its
// equations are normalised to a unit diagonal and reduced by cyclic reduction
// (even-numbered unknowns survive each level, compacted) until at most 64 remain;
// one wave solves those by parallel cyclic reduction with lane shuffles, and the
// eliminated unknowns are recovered level by level.  No pivoting, as in the
// Thomas algorithm the method prescribes per block.
//
// tab: psolve_tab_entries(CW) entries of LDS; red: 6*NT entries (may alias a
// staging area the caller has finished reading: the first barrier below precedes
// every write to it, and the last barrier follows every read).  Every thread of
// the block must call it.  Returns true if a value is not finite.
// Table of the interior elimination of a chunk of CW unknowns (one thread):
// tab[0..CW-2] 1/pivot, tab[CW..2CW-2] e/pivot, tab[2CW..3CW-2] the forward part of
// the response to the left separator, tab[3CW..3CW+7] the first / last values of
// both responses for full chunks (slots 0-3) and for the last chunk, whose interior
// has mlast unknowns (slots 4-7).
template <typename A, int CW, typename P>
__device__ __forceinline__ void build_tab(cx<A> d, cx<A> e, int mlast, P tab)
{
    const cx<A> zero = {A(0), A(0)};
    // pivots of the interior elimination and the forward part of u (the response to
    // -e in the first interior equation)
    cx<A> cprev = zero, g = zero;
    for (int i = 0; i < CW - 1; ++i) {
        const cx<A> ip = recip(cfms(d, e, cprev));
        tab[i] = ip;
        cprev = e * ip;
        tab[CW + i] = cprev;
        g = (i == 0) ? -(e * ip) : -((e * g) * ip);
        tab[2 * CW + i] = g;
    }
    for (int k = 0; k < 2; ++k) {
        const int mi = k == 0 ? CW - 1 : mlast;
        cx<A> uf = zero, ul = zero, vf = zero, vl = zero;
        if (mi > 0) {
            ul = tab[2 * CW + mi - 1];
            vl = -(e * tab[mi - 1]);
            uf = ul;
            vf = vl;
            for (int i = mi - 2; i >= 0; --i) {
                uf = cfms(tab[2 * CW + i], tab[CW + i], uf);
                vf = -(tab[CW + i] * vf);
            }
        }
        tab[3 * CW + 4 * k + 0] = uf;
        tab[3 * CW + 4 * k + 1] = ul;
        tab[3 * CW + 4 * k + 2] = vf;
        tab[3 * CW + 4 * k + 3] = vl;
    }
}

// Solve tridiag(e, d, e) x = r with n unknowns.  Thread t owns unknowns
// [t*CW, t*CW + len); y[] holds its part of r on entry and of x on exit.
//
// Chunk t is split into an interior (its first len-1 unknowns) and a separator
// (its last unknown).  With the interior eliminated, x_i = y_i + u_i X_{t-1} +
// v_i X_t, where y is the interior solution with zero neighbours and u, v its
// responses to the left / right separator.  The matrix being Toeplitz, the
// elimination factors (1/pivot, e/pivot), the forward part of u and the end values
// of u and v are the same for every full chunk: they form one table per row
// (build_tab) in LDS, built by one thread or copied from a table precomputed per
// row, and every thread regenerates u and v backwards from it, so a thread
// keeps only y in registers.
//
// The separators satisfy a tridiagonal system with one equation per chunk.  Its
// equations are normalised to a unit diagonal and reduced by cyclic reduction
// (even-numbered unknowns survive each level, compacted) until at most 64 remain;
// one wave solves those by parallel cyclic reduction with lane shuffles, and the
// eliminated unknowns are recovered level by level.  No pivoting, as in the
// Thomas algorithm the method prescribes per block.
//
// Where partition_solve finds the table: built by thread 0, or already written to LDS
// by the caller (the shifted solves copy a table precomputed per row).
enum TabSource { kTabBuild = 0, kTabReady = 2 };

// tab: psolve_tab_entries(CW) entries of LDS; red:
// 6*NT entries (may alias a staging area the caller has finished reading: the first
// barrier below precedes every write to it, and the last barrier follows every read).
// With kTabReady the caller's writes to tab must precede the call's first barrier.
// Every thread of the block must call it.  Returns true if a value is not finite.
template <typename A, int CW, int TABSRC = kTabBuild>
__device__ bool partition_solve(cx<A> (&y)[CW], int n, cx<A> d, cx<A> e, cx<A> *tab, cx<A> *red)
{
    const int NT = blockDim.x;
    const int t = threadIdx.x;
    const cx<A> zero = {A(0), A(0)};
    const int P = (n + CW - 1) / CW;                     // number of chunks / separators
    const int mlast = n - (P - 1) * CW - 1;              // interior length of the last chunk
    if (TABSRC == kTabBuild && t == 0) build_tab<A, CW>(d, e, mlast, tab);
    const cx<A> *s_ip = tab, *s_cp = tab + CW, *s_gu = tab + 2 * CW, *s_end = tab + 3 * CW;
    // level-0 reduced system (a | c | d, NT each), then the neighbour terms and the
    // compacted deeper levels in the second half
    cx<A> *a0 = red, *c0 = red + NT, *d0 = red + 2 * NT, *ny = red + 3 * NT;
    __syncthreads();

    const int a0i = t * CW;
    const int len = (t < P) ? min(CW, n - a0i) : 0;
    const int mi = len - 1;                              // interior length (may be 0)
    const bool last = (t == P - 1);

    cx<A> rsep = zero;
#pragma unroll
    for (int i = 0; i < CW; ++i)
        if (i == mi) rsep = y[i];
    // interior: forward elimination in place (y becomes the forward sweep g); the
    // back substitution is deferred until the separators are known, only its
    // first value y_0 = g_0 - cp_0 (g_1 - cp_1 (...)) is formed now
    cx<A> gy = zero;
#pragma unroll
    for (int i = 0; i < CW - 1; ++i) {
        if (i < mi) {
            gy = cfms(y[i], e, gy) * s_ip[i];
            y[i] = gy;
        }
    }
    cx<A> ylast = zero;
#pragma unroll
    for (int i = 0; i < CW - 1; ++i)
        if (i == mi - 1) ylast = y[i];
    cx<A> yfirst = ylast;
#pragma unroll
    for (int i = CW - 3; i >= 0; --i)
        if (i < mi - 1) yfirst = cfms(y[i], s_cp[i], yfirst);

    const int eo = last ? 4 : 0;
    const cx<A> ulast = mi > 0 ? s_end[eo + 1] : zero;
    const cx<A> vlast = mi > 0 ? s_end[eo + 3] : zero;

    // equation t:  lo X_{t-1} + di X_t + up X_{t+1} = rh, where the next chunk's
    // first unknown (interior or separator) has been eliminated
    if (t < P) ny[t] = (mi > 0) ? e * yfirst : zero;
    __syncthreads();
    if (t < P) {
        cx<A> lo = (mi > 0) ? e * ulast : e;
        cx<A> di = (mi > 0) ? cfma(d, e, vlast) : d;
        cx<A> rh = (mi > 0) ? cfms(rsep, e, ylast) : rsep;
        if (t == 0) lo = zero;
        cx<A> up = zero;
        if (t + 1 < P) {
            const int mn = (t + 1 == P - 1) ? mlast : CW - 1;
            const int no = (t + 1 == P - 1) ? 4 : 0;
            if (mn > 0) {
                di = cfma(di, e, s_end[no + 0]);
                up = e * s_end[no + 2];
                rh = rh - ny[t + 1];
            } else {
                up = e;
            }
        }
        const cx<A> q = recip(di);
        a0[t] = lo * q;
        c0[t] = up * q;
        d0[t] = rh * q;
    }
    __syncthreads();

    // cyclic reduction down to at most 64 equations; level s arrays (a, c, d) of
    // length Ps; level s+1 keeps the even unknowns of level s
    int Ps = P;
    cx<A> *as = a0, *cs = c0, *ds = d0;
    cx<A> *next = red + 3 * NT;
    int levels = 0;
    while (Ps > 64) {
        const int Pn = (Ps + 1) / 2;
        cx<A> *an = next, *cn = next + Pn, *dn = next + 2 * Pn;
        for (int u = t; u < Pn; u += NT) {
            const int k = 2 * u;
            TriEq<A> m{as[k], cs[k], ds[k]}, l{zero, zero, zero}, r{zero, zero, zero};
            if (k >= 1) l = {as[k - 1], cs[k - 1], ds[k - 1]};
            if (k + 1 < Ps) r = {as[k + 1], cs[k + 1], ds[k + 1]};
            const TriEq<A> o = reduce_eq(m, l, r);
            an[u] = o.a;
            cn[u] = o.c;
            dn[u] = o.d;
        }
        __syncthreads();
        as = an;
        cs = cn;
        ds = dn;
        next = dn + Pn;
        Ps = Pn;
        ++levels;
    }
    // one wave: parallel cyclic reduction of the remaining Ps <= 64 equations.  Lanes
    // t >= Ps hold zero equations and are never a neighbour of a live lane (a right
    // neighbour t + sd >= Ps is replaced by zeros), so every lane updates
    // unconditionally; the selects are per component, which keeps them in registers.
    if (t < 64) {
        const bool live = t < Ps;
        TriEq<A> m{csel(live, as[min(t, Ps - 1)], zero), csel(live, cs[min(t, Ps - 1)], zero),
                   csel(live, ds[min(t, Ps - 1)], zero)};
        for (int sd = 1; sd < Ps; sd <<= 1) {
            const bool hl = t - sd >= 0, hr = t + sd < Ps;
            const TriEq<A> l{csel(hl, shfl_cx(m.a, t - sd), zero), csel(hl, shfl_cx(m.c, t - sd), zero),
                             csel(hl, shfl_cx(m.d, t - sd), zero)};
            const TriEq<A> r{csel(hr, shfl_cx(m.a, t + sd), zero), csel(hr, shfl_cx(m.c, t + sd), zero),
                             csel(hr, shfl_cx(m.d, t + sd), zero)};
            m = reduce_eq(m, l, r);
        }
        if (live) ds[t] = m.d;                           // X at the deepest level
    }
    __syncthreads();
    // back substitution, level by level: level s recovers its odd unknowns from
    // the even ones (level s+1); the d arrays are overwritten with X
    for (int lv = levels; lv > 0; --lv) {
        // arrays of level lv-1: recompute their position
        int P0 = P;
        cx<A> *ap = a0, *cp = c0, *dp = d0;
        cx<A> *nx = red + 3 * NT;
        for (int q = 0; q < lv - 1; ++q) {
            const int Pn = (P0 + 1) / 2;
            ap = nx;
            cp = nx + Pn;
            dp = nx + 2 * Pn;
            nx = dp + Pn;
            P0 = Pn;
        }
        const int Pn = (P0 + 1) / 2;
        const cx<A> *dn = nx + 2 * Pn;                  // X of level lv
        for (int u = t; u < Pn; u += NT) {
            const int k = 2 * u;
            const cx<A> xk = dn[u];
            if (k + 1 < P0) {
                const cx<A> xr = (k + 2 < P0) ? dn[u + 1] : zero;
                dp[k + 1] = cfms(cfms(dp[k + 1], ap[k + 1], xk), cp[k + 1], xr);
            }
            dp[k] = xk;
        }
        __syncthreads();
    }
    // d0[t] now holds the separator value X_t
    cx<A> XL = zero, XR = zero;
    if (t < P) {
        XL = (t > 0) ? d0[t - 1] : zero;
        XR = d0[t];
    }
    __syncthreads();   // the caller may reuse `red` from here on
    // interior: the forward sweep of the full right-hand side r - e XL e_0 - e XR
    // e_last is g + XL gu (+ vlast XR in the last entry); back substitution
    bool bad = false;
    if (t < P) {
        cx<A> xn = XR;   // x_{i+1}; the separator for i = mi - 1
#pragma unroll
        for (int i = CW - 2; i >= 0; --i) {
            if (i < mi) {
                cx<A> g = cfma(y[i], s_gu[i], XL);
                if (i == mi - 1) {
                    g = cfma(g, vlast, XR);
                    xn = g;
                } else {
                    xn = cfms(g, s_cp[i], xn);
                }
                y[i] = xn;
                bad |= !(isfinite((double)xn.x) && isfinite((double)xn.y));
            }
        }
#pragma unroll
        for (int i = 0; i < CW; ++i)
            if (i == mi) y[i] = XR;
        bad |= !(isfinite((double)XR.x) && isfinite((double)XR.y));
    }
    return bad;
}

}  // namespace aao
