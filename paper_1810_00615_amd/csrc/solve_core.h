// Partition solve of a constant-coefficient (Toeplitz) tridiagonal system by one
// workgroup: Thomas elimination of per-thread chunks, parallel cyclic reduction
// of the separator system in LDS, back substitution.  Shared by the shifted
// solves (single problem and batched) and the trajectory recomputation.
#pragma once
#include "aao_internal.h"

namespace aao {

// Partition solve of tridiag(e, d, e) x = r with n unknowns by one workgroup.
// Thread t owns unknowns [t*CW, t*CW + len); y[] holds its part of r on entry and
// of x on exit.  s_ip / s_cp: CW entries of LDS each; red: 7*NT entries of LDS
// (may alias a staging area the caller has finished reading: the first barrier
// below precedes every write to it, and the last barrier follows every read).
// Every thread of the block must call it.  Returns true if a value is not finite.
template <typename A, int CW>
__device__ bool partition_solve(cx<A> (&y)[CW], int n, cx<A> d, cx<A> e, cx<A> *s_ip,
                                cx<A> *s_cp, cx<A> *red)
{
    const int NT = blockDim.x;
    const int t = threadIdx.x;
    cx<A> *pa = red, *pb = red + NT, *pc = red + 2 * NT, *pd = red + 3 * NT, *nb = red + 4 * NT;
    const cx<A> zero = {A(0), A(0)};
    const cx<A> me = {-e.x, -e.y};
    if (t == 0) {
        cx<A> cprev = zero;
        for (int i = 0; i < CW - 1; ++i) {
            const cx<A> ip = recip(d - e * cprev);
            s_ip[i] = ip;
            cprev = e * ip;
            s_cp[i] = cprev;
        }
    }
    __syncthreads();

    const int P = (n + CW - 1) / CW;                     // number of chunks / separators
    const int a0 = t * CW;
    const int len = (t < P) ? min(CW, n - a0) : 0;
    const int mi = len - 1;                              // interior length (may be 0)

    cx<A> u[CW];
    cx<A> rsep = zero;
#pragma unroll
    for (int i = 0; i < CW; ++i) {
        u[i] = zero;
        if (i == mi) rsep = y[i];
    }
    // forward elimination of the interior: particular solution y and the
    // response u to the left separator (right-hand side -e at interior 0)
    cx<A> gy = zero, gu = zero;
#pragma unroll
    for (int i = 0; i < CW - 1; ++i) {
        if (i < mi) {
            const cx<A> ip = s_ip[i];
            gy = (y[i] - e * gy) * ip;
            gu = (i == 0) ? me * ip : (me * gu) * ip;
            y[i] = gy;
            u[i] = gu;
        }
    }
    // back substitution; v (response to the right separator) only at its ends
    cx<A> vlast = zero, vfirst = zero;
    if (mi > 0) {
        vlast = me * s_ip[mi - 1];
        vfirst = vlast;
    }
#pragma unroll
    for (int i = CW - 3; i >= 0; --i) {
        if (i < mi - 1) {
            const cx<A> cp = s_cp[i];
            y[i] = y[i] - cp * y[i + 1];
            u[i] = u[i] - cp * u[i + 1];
            vfirst = zero - cp * vfirst;
        }
    }

    // reduced (separator) system, equation c = t
    if (t < P) {
        cx<A> lo, di, rh;
        if (mi > 0) {
            cx<A> ul = zero, yl = zero;
#pragma unroll
            for (int i = 0; i < CW - 1; ++i)
                if (i == mi - 1) {
                    ul = u[i];
                    yl = y[i];
                }
            lo = e * ul;
            di = d + e * vlast;
            rh = rsep - e * yl;
        } else {
            lo = e;
            di = d;
            rh = rsep;
        }
        if (t == 0) lo = zero;
        pa[t] = lo;
        pb[t] = di;
        pd[t] = rh;
        // what this chunk adds to equation t-1 (its left neighbour separator)
        if (mi > 0) {
            nb[3 * t + 0] = e * u[0];          // to the diagonal
            nb[3 * t + 1] = e * vfirst;        // upper coefficient (to X_t)
            nb[3 * t + 2] = e * y[0];          // subtracted from the rhs
        } else {
            nb[3 * t + 0] = zero;
            nb[3 * t + 1] = e;
            nb[3 * t + 2] = zero;
        }
    }
    __syncthreads();
    if (t < P) {
        if (t + 1 < P) {
            pb[t] = pb[t] + nb[3 * (t + 1) + 0];
            pc[t] = nb[3 * (t + 1) + 1];
            pd[t] = pd[t] - nb[3 * (t + 1) + 2];
        } else {
            pc[t] = zero;
        }
    }
    __syncthreads();

    // parallel cyclic reduction
    for (int sd = 1; sd < P; sd <<= 1) {
        cx<A> na = zero, nbv = zero, nc = zero, nd = zero;
        if (t < P) {
            const cx<A> a = pa[t], b = pb[t], c = pc[t], dd = pd[t];
            nbv = b;
            nd = dd;
            if (t - sd >= 0) {
                const cx<A> k1 = a * recip(pb[t - sd]);
                na = zero - pa[t - sd] * k1;
                nbv = nbv - pc[t - sd] * k1;
                nd = nd - pd[t - sd] * k1;
            }
            if (t + sd < P) {
                const cx<A> k2 = c * recip(pb[t + sd]);
                nc = zero - pc[t + sd] * k2;
                nbv = nbv - pa[t + sd] * k2;
                nd = nd - pd[t + sd] * k2;
            }
        }
        __syncthreads();
        if (t < P) {
            pa[t] = na;
            pb[t] = nbv;
            pc[t] = nc;
            pd[t] = nd;
        }
        __syncthreads();
    }
    if (t < P) pd[t] = pd[t] * recip(pb[t]);            // separator values X_t
    __syncthreads();
    cx<A> XL = zero, XR = zero;
    if (t < P) {
        XL = (t > 0) ? pd[t - 1] : zero;
        XR = pd[t];
    }
    __syncthreads();   // the caller may reuse `red` from here on
    // interior: x_i = y_i + u_i XL + v_i XR, v from the back
    bool bad = false;
    if (t < P) {
        cx<A> vi = vlast;
#pragma unroll
        for (int i = CW - 2; i >= 0; --i) {
            if (i < mi) {
                if (i < mi - 1) vi = zero - s_cp[i] * vi;
                y[i] = y[i] + u[i] * XL + vi * XR;
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
