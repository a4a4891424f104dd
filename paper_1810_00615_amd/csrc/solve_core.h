// Partition solve of a constant-coefficient (Toeplitz) tridiagonal system by one
// workgroup: Thomas elimination of per-thread chunks, parallel cyclic reduction
// of the separator system in LDS, back substitution.  Shared by the shifted
// solves (single problem and batched) and the trajectory recomputation.
#pragma once
#include "aao_internal.h"

namespace aao {

// LDS needed by partition_solve: tables (3 CW) + reduced system (6 NT) entries.
__host__ __device__ constexpr int psolve_lds_entries(int CW, int NT) { return 3 * CW + 6 * NT; }

// Solve tridiag(e, d, e) x = r with n unknowns.  Thread t owns unknowns
// [t*CW, t*CW + len); y[] holds its part of r on entry and of x on exit.
//
// Chunk t is split into an interior (its first len-1 unknowns) and a separator
// (its last unknown).  With the interior eliminated, x_i = y_i + u_i X_{t-1} +
// v_i X_t, where y is the interior solution with zero neighbours and u, v its
// responses to the left / right separator.  Because the matrix is Toeplitz, the
// elimination factors (1/pivot, e/pivot) and the forward part of u are the same
// for every chunk: one thread tabulates them per row in LDS and every thread
// regenerates u and v backwards from the table, so a thread keeps only y in
// registers.  The separators satisfy a tridiagonal system (one equation per
// chunk), solved by parallel cyclic reduction with every equation normalised to
// a unit diagonal (one complex reciprocal per equation and step).
//
// tab: 3*CW entries of LDS; red: 6*NT entries (may alias a staging area the caller
// has finished reading: the first barrier below precedes every write to it, and
// the last barrier follows every read).  Every thread of the block must call it.
// Returns true if a value is not finite.
template <typename A, int CW>
__device__ bool partition_solve(cx<A> (&y)[CW], int n, cx<A> d, cx<A> e, cx<A> *tab, cx<A> *red)
{
    const int NT = blockDim.x;
    const int t = threadIdx.x;
    cx<A> *s_ip = tab, *s_cp = tab + CW, *s_gu = tab + 2 * CW;
    cx<A> *pa = red, *pc = red + NT, *pd = red + 2 * NT, *nb = red + 3 * NT;
    const cx<A> zero = {A(0), A(0)};
    const cx<A> me = {-e.x, -e.y};
    if (t == 0) {
        // pivots of the interior elimination and the forward part of u (the
        // response to -e in the first interior equation)
        cx<A> cprev = zero, g = zero;
        for (int i = 0; i < CW - 1; ++i) {
            const cx<A> ip = recip(d - e * cprev);
            s_ip[i] = ip;
            cprev = e * ip;
            s_cp[i] = cprev;
            g = (i == 0) ? me * ip : (me * g) * ip;
            s_gu[i] = g;
        }
    }
    __syncthreads();

    const int P = (n + CW - 1) / CW;                     // number of chunks / separators
    const int a0 = t * CW;
    const int len = (t < P) ? min(CW, n - a0) : 0;
    const int mi = len - 1;                              // interior length (may be 0)

    cx<A> rsep = zero;
#pragma unroll
    for (int i = 0; i < CW; ++i)
        if (i == mi) rsep = y[i];
    // interior: forward elimination and back substitution in place
    cx<A> gy = zero;
#pragma unroll
    for (int i = 0; i < CW - 1; ++i) {
        if (i < mi) {
            gy = (y[i] - e * gy) * s_ip[i];
            y[i] = gy;
        }
    }
#pragma unroll
    for (int i = CW - 3; i >= 0; --i)
        if (i < mi - 1) y[i] = y[i] - s_cp[i] * y[i + 1];

    // ends of u and v for this chunk's interior length
    cx<A> ulast = zero, ufirst = zero, vlast = zero, vfirst = zero;
    if (mi > 0) {
        ulast = s_gu[mi - 1];
        vlast = me * s_ip[mi - 1];
        ufirst = ulast;
        vfirst = vlast;
        for (int i = mi - 2; i >= 0; --i) {
            const cx<A> cp = s_cp[i];
            ufirst = s_gu[i] - cp * ufirst;
            vfirst = zero - cp * vfirst;
        }
    }
    cx<A> ylast = zero, yfirst = y[0];
#pragma unroll
    for (int i = 0; i < CW - 1; ++i)
        if (i == mi - 1) ylast = y[i];

    // reduced (separator) system, equation t:  lo X_{t-1} + di X_t + up X_{t+1} = rh
    if (t < P) {
        cx<A> lo, di, rh;
        if (mi > 0) {
            lo = e * ulast;
            di = d + e * vlast;
            rh = rsep - e * ylast;
        } else {
            lo = e;
            di = d;
            rh = rsep;
        }
        if (t == 0) lo = zero;
        pa[t] = lo;
        pc[t] = di;        // diagonal kept in pc until the neighbour terms are added
        pd[t] = rh;
        // what this chunk adds to equation t-1 (its left neighbour separator)
        if (mi > 0) {
            nb[3 * t + 0] = e * ufirst;        // to the diagonal
            nb[3 * t + 1] = e * vfirst;        // upper coefficient (to X_t)
            nb[3 * t + 2] = e * yfirst;        // subtracted from the rhs
        } else {
            nb[3 * t + 0] = zero;
            nb[3 * t + 1] = e;
            nb[3 * t + 2] = zero;
        }
    }
    __syncthreads();
    cx<A> a = zero, c = zero, dd = zero;
    if (t < P) {
        cx<A> di = pc[t];
        dd = pd[t];
        a = pa[t];
        if (t + 1 < P) {
            di = di + nb[3 * (t + 1) + 0];
            c = nb[3 * (t + 1) + 1];
            dd = dd - nb[3 * (t + 1) + 2];
        }
        const cx<A> r = recip(di);                       // unit diagonal
        a = a * r;
        c = c * r;
        dd = dd * r;
    }
    __syncthreads();
    if (t < P) {
        pa[t] = a;
        pc[t] = c;
        pd[t] = dd;
    }
    __syncthreads();

    // parallel cyclic reduction on unit-diagonal equations
    for (int sd = 1; sd < P; sd <<= 1) {
        cx<A> na = zero, nc = zero, nd = dd, nbd = {A(1), A(0)};
        if (t < P) {
            if (t - sd >= 0) {
                const cx<A> al = pa[t - sd], cl = pc[t - sd], dl = pd[t - sd];
                na = zero - a * al;
                nbd = nbd - a * cl;
                nd = nd - a * dl;
            }
            if (t + sd < P) {
                const cx<A> ar = pa[t + sd], cr = pc[t + sd], dr = pd[t + sd];
                nc = zero - c * cr;
                nbd = nbd - c * ar;
                nd = nd - c * dr;
            }
            const cx<A> r = recip(nbd);
            a = na * r;
            c = nc * r;
            dd = nd * r;
        }
        __syncthreads();
        if (t < P) {
            pa[t] = a;
            pc[t] = c;
            pd[t] = dd;
        }
        __syncthreads();
    }
    // pd[t] now holds the separator value X_t
    cx<A> XL = zero, XR = zero;
    if (t < P) {
        XL = (t > 0) ? pd[t - 1] : zero;
        XR = dd;
    }
    __syncthreads();   // the caller may reuse `red` from here on
    // interior: x_i = y_i + u_i XL + v_i XR, u and v regenerated from the back
    bool bad = false;
    if (t < P) {
        cx<A> ui = ulast, vi = vlast;
#pragma unroll
        for (int i = CW - 2; i >= 0; --i) {
            if (i < mi) {
                if (i < mi - 1) {
                    const cx<A> cp = s_cp[i];
                    ui = s_gu[i] - cp * ui;
                    vi = zero - cp * vi;
                }
                y[i] = y[i] + ui * XL + vi * XR;
                bad |= !(isfinite((double)y[i].x) && isfinite((double)y[i].y));
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
