// Device functions of the EM-PIC particle step for gfx950, templated on the
// real type T (float: split-precision mode, double) and the shape order O.
//
// One implementation of each operation is shared by the fused tile kernel
// (fields and current in LDS) and the untiled kernels (global memory): the
// callers pass precomputed index offsets per direction, so the same loops
// address either an LDS tile with halo or the periodic global arrays.
//
// Paper: "Porting WarpX to GPU-accelerated platforms" (arXiv 2101.12149).
// Shapes: Sec. 4.1.1 (third-order shape functions); gather: Sec. 3.1 and 4.2
// (fused gather+push, energy-conserving gather); deposit: Sec. 3.4.1 and
// 4.1.1 (Esirkepov); Yee staggering: Sec. 2.4.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// ---------------------------------------------------------------------------
// Per-node weights of the order-O B-spline in the frame of one cell: a
// particle at offset d in [0,1) of node j0 touches nodes j0+NB .. j0+NB+O.

template <int O, typename T>
struct Shape;

template <typename T>
struct Shape<1, T> {
    static constexpr int NW = 2;   // nodes touched
    static constexpr int NB = 0;   // first node relative to the cell
    __device__ static inline void w(T d, T *s)
    {
        s[0] = T(1) - d;
        s[1] = d;
    }
    __device__ static inline void dw(T, T *s)
    {
        s[0] = T(-1);
        s[1] = T(1);
    }
    // divided difference (w(b) - w(a)) / (b - a), free of cancellation
    __device__ static inline void q(T, T, T *s)
    {
        s[0] = T(-1);
        s[1] = T(1);
    }
};

template <typename T>
struct Shape<3, T> {
    static constexpr int NW = 4;
    static constexpr int NB = -1;
    __device__ static inline void w(T d, T *s)
    {
        const T e = T(1) - d, d2 = d * d, d3 = d2 * d;
        const T sixth = T(1) / T(6);
        s[0] = e * e * e * sixth;
        s[1] = (T(4) - T(6) * d2 + T(3) * d3) * sixth;
        s[2] = (T(1) + T(3) * d + T(3) * d2 - T(3) * d3) * sixth;
        s[3] = d3 * sixth;
    }
    __device__ static inline void dw(T d, T *s)
    {
        const T e = T(1) - d, d2 = d * d;
        s[0] = T(-0.5) * e * e;
        s[1] = T(-2) * d + T(1.5) * d2;
        s[2] = T(0.5) + d - T(1.5) * d2;
        s[3] = T(0.5) * d2;
    }
    __device__ static inline void q(T a, T b, T *s)
    {
        const T p2 = a * a + a * b + b * b, sm = a + b;
        const T sixth = T(1) / T(6);
        s[0] = -(T(3) - T(3) * sm + p2) * sixth;
        s[1] = T(0.5) * (p2 - T(2) * sm);
        s[2] = T(0.5) * (T(1) + sm - p2);
        s[3] = p2 * sixth;
    }
};

// Nodal and half-cell-staggered weights of one coordinate, with the offset of
// the first touched node relative to the particle's cell.
template <int O, typename T>
struct AxisW {
    T wn[Shape<O, T>::NW], ws[Shape<O, T>::NW];
    int bn, bs;
};

template <int O, typename T>
__device__ inline void axis_weights(T f, AxisW<O, T> &a)
{
    using S = Shape<O, T>;
    S::w(f, a.wn);
    a.bn = S::NB;
    // staggered sample points sit at node + 1/2: coordinate f - 1/2
    if (f >= T(0.5)) {
        S::w(f - T(0.5), a.ws);
        a.bs = S::NB;
    } else {
        S::w(f + T(0.5), a.ws);
        a.bs = S::NB - 1;
    }
}

template <int O, typename T>
__device__ inline void axis_dweights(T f, T *dn, T *ds)
{
    using S = Shape<O, T>;
    S::dw(f, dn);
    if (f >= T(0.5))
        S::dw(f - T(0.5), ds);
    else
        S::dw(f + T(0.5), ds);
}

// sum_k wz[k] sum_j wy[j] sum_i wx[i] F[xo[i] + yo[j] + zo[k]]
template <int NW, typename T>
__device__ inline T contract3(const T *__restrict__ F, const int *xo, const int *yo, const int *zo, const T *wx,
                              const T *wy, const T *wz)
{
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        T accy = T(0);
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const T *row = F + yo[j] + zo[k];
            T accx = T(0);
#pragma unroll
            for (int i = 0; i < NW; ++i)
                accx += wx[i] * row[xo[i]];
            accy += wy[j] * accx;
        }
        acc += wz[k] * accy;
    }
    return acc;
}

// Index offsets of the touched nodes along one axis: (pos + base + a) * stride
// in a tile region (no wrap) or wrapped into [0,n) for global arrays.
template <int NW>
__device__ inline void axis_offsets_local(int pos, int base, int stride, int *o)
{
#pragma unroll
    for (int a = 0; a < NW; ++a)
        o[a] = (pos + base + a) * stride;
}

template <int NW>
__device__ inline void axis_offsets_global(int cell, int base, int n, int stride, int *o)
{
#pragma unroll
    for (int a = 0; a < NW; ++a) {
        int v = cell + base + a;
        v = v < 0 ? v + n : (v >= n ? v - n : v);
        // tiny grids (n < stencil) can need more than one wrap
        while (v < 0)
            v += n;
        while (v >= n)
            v -= n;
        o[a] = v * stride;
    }
}

// Field pointers (global arrays or the six LDS blocks), E then B.
template <typename T>
struct FieldSrc {
    const T *c[6];
};

// Gather E and B at one particle (energy-conserving: each component with its
// own staggering, same order in all directions).  nodal/staggered offsets
// per axis: on[d][], os[d][].
template <int O, typename T>
__device__ inline void gather_eb(const FieldSrc<T> &F, const AxisW<O, T> *aw, const int (*on)[Shape<O, T>::NW],
                                 const int (*os)[Shape<O, T>::NW], T *E, T *B)
{
    constexpr int NW = Shape<O, T>::NW;
    // E_x (s,n,n) E_y (n,s,n) E_z (n,n,s)
    E[0] = contract3<NW>(F.c[0], os[0], on[1], on[2], aw[0].ws, aw[1].wn, aw[2].wn);
    E[1] = contract3<NW>(F.c[1], on[0], os[1], on[2], aw[0].wn, aw[1].ws, aw[2].wn);
    E[2] = contract3<NW>(F.c[2], on[0], on[1], os[2], aw[0].wn, aw[1].wn, aw[2].ws);
    // B_x (n,s,s) B_y (s,n,s) B_z (s,s,n)
    B[0] = contract3<NW>(F.c[3], on[0], os[1], os[2], aw[0].wn, aw[1].ws, aw[2].ws);
    B[1] = contract3<NW>(F.c[4], os[0], on[1], os[2], aw[0].ws, aw[1].wn, aw[2].ws);
    B[2] = contract3<NW>(F.c[5], os[0], os[1], on[2], aw[0].ws, aw[1].ws, aw[2].wn);
}

// ---------------------------------------------------------------------------
// Relativistic Boris push (h = q dt / 2m): half electric kick, rotation by
// t = h B / gamma and s = 2 t / (1 + t^2), second half kick.

template <typename T>
struct BorisTape {
    T a[3], gbar, t[3], s[3], up[3], tt;
};

template <typename T>
__device__ inline void cross3(const T *a, const T *b, T *r)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename T>
__device__ inline void boris(T h, T inv_c2, const T *u0, const T *E, const T *B, T *u1, BorisTape<T> &tp)
{
#pragma unroll
    for (int d = 0; d < 3; ++d)
        tp.a[d] = u0[d] + h * E[d];
    tp.gbar = sqrt(T(1) + (tp.a[0] * tp.a[0] + tp.a[1] * tp.a[1] + tp.a[2] * tp.a[2]) * inv_c2);
    const T hg = h / tp.gbar;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        tp.t[d] = hg * B[d];
    tp.tt = tp.t[0] * tp.t[0] + tp.t[1] * tp.t[1] + tp.t[2] * tp.t[2];
    const T sc = T(2) / (T(1) + tp.tt);
#pragma unroll
    for (int d = 0; d < 3; ++d)
        tp.s[d] = sc * tp.t[d];
    T axt[3];
    cross3(tp.a, tp.t, axt);
#pragma unroll
    for (int d = 0; d < 3; ++d)
        tp.up[d] = tp.a[d] + axt[d];
    T upxs[3];
    cross3(tp.up, tp.s, upxs);
#pragma unroll
    for (int d = 0; d < 3; ++d)
        u1[d] = tp.a[d] + upxs[d] + h * E[d];
}

// Transpose of the Boris map: given ub = dL/du1, return dL/du0, dL/dE, dL/dB.
template <typename T>
__device__ inline void boris_adjoint(T h, T inv_c2, const T *B, const BorisTape<T> &tp, const T *ub, T *u0b, T *Eb,
                                     T *Bb)
{
    T ab[3], upb[3], sb[3], tb[3], tmp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Eb[d] = h * ub[d];
        ab[d] = ub[d];
    }
    cross3(tp.s, ub, upb);     // d(u' x s)/du'^T ub = s x ub
    cross3(ub, tp.up, sb);     // d(u' x s)/ds^T ub  = ub x u'
    cross3(tp.t, upb, tmp);    // d(a x t)/da^T upb  = t x upb
#pragma unroll
    for (int d = 0; d < 3; ++d)
        ab[d] += upb[d] + tmp[d];
    cross3(upb, tp.a, tb);     // d(a x t)/dt^T upb  = upb x a
    const T den = T(1) + tp.tt;
    const T tsb = tp.t[0] * sb[0] + tp.t[1] * sb[1] + tp.t[2] * sb[2];
    const T c1 = T(2) / den, c2 = T(4) * tsb / (den * den);
#pragma unroll
    for (int d = 0; d < 3; ++d)
        tb[d] += c1 * sb[d] - c2 * tp.t[d];
    const T hg = h / tp.gbar;
    T Btb = T(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Bb[d] = hg * tb[d];
        Btb += B[d] * tb[d];
    }
    const T gb = -hg * Btb / tp.gbar;           // dL/dgbar
    const T ga = gb * inv_c2 / tp.gbar;         // dgbar/da = a / (c^2 gbar)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ab[d] += ga * tp.a[d];
        u0b[d] = ab[d];
        Eb[d] += h * ab[d];
    }
}

// ---------------------------------------------------------------------------
// Vay's relativistic push (Vay 2008; the paper's pusher for relativistic
// beams, Sec. 4.2).  The magnetic force uses the mean of the old and new
// velocities, an equation implicit in u1.  With the known part
// w = u0 + 2h E + h (u0/g0) x B and tau = h B it is u1 - u1 x (tau/g1) = w:
// for the new gamma, G = g1^2 solves G^2 - sigma G - X = 0 with
// sigma = 1 + |w|^2/c^2 - |tau|^2 and X = |tau|^2 + (w.tau)^2/c^2 (its
// positive root, in the form without cancellation for sigma < 0); then with
// t = tau/g1 the linear system gives u1 = (w + (w.t) t + w x t) / (1 + |t|^2).

template <typename T>
__device__ inline T dot3(const T *a, const T *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// the known part w, tau = h B and the new gamma's square G (with D = sqrt(sigma^2 + 4X))
template <typename T>
__device__ inline void vay_setup(T h, T inv_c2, const T *u0, const T *E, const T *B, T *v0, T *w, T *tau, T &G,
                                 T &D, T &sigma)
{
    const T ig0 = T(1) / sqrt(T(1) + dot3(u0, u0) * inv_c2);
#pragma unroll
    for (int d = 0; d < 3; ++d)
        v0[d] = u0[d] * ig0;
    T vb[3];
    cross3(v0, B, vb);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        w[d] = u0[d] + T(2) * h * E[d] + h * vb[d];
        tau[d] = h * B[d];
    }
    const T tau2 = dot3(tau, tau), wt = dot3(w, tau);
    sigma = T(1) + dot3(w, w) * inv_c2 - tau2;
    const T X = tau2 + wt * wt * inv_c2;
    D = sqrt(sigma * sigma + T(4) * X);
    G = sigma >= T(0) ? T(0.5) * (sigma + D) : T(2) * X / (D - sigma);
}

template <typename T>
__device__ inline void vay(T h, T inv_c2, const T *u0, const T *E, const T *B, T *u1)
{
    T v0[3], w[3], tau[3], G, D, sigma;
    vay_setup(h, inv_c2, u0, E, B, v0, w, tau, G, D, sigma);
    const T ig1 = T(1) / sqrt(G);
    T t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        t[d] = tau[d] * ig1;
    T wxt[3];
    cross3(w, t, wxt);
    const T a = dot3(w, t), s = T(1) / (T(1) + dot3(t, t));
#pragma unroll
    for (int d = 0; d < 3; ++d)
        u1[d] = s * (w[d] + a * t[d] + wxt[d]);
}

// Transpose of vay(): given ub = dL/du1, return dL/du0, dL/dE, dL/dB.  The
// forward quantities are evaluated again; dG/dsigma = G/D, dG/dX = 1/D.
template <typename T>
__device__ inline void vay_adjoint(T h, T inv_c2, const T *u0, const T *E, const T *B, const T *ub, T *u0b, T *Eb,
                                   T *Bb)
{
    T v0[3], w[3], tau[3], G, D, sigma;
    vay_setup(h, inv_c2, u0, E, B, v0, w, tau, G, D, sigma);
    const T g1 = sqrt(G), ig1 = T(1) / g1;
    T t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        t[d] = tau[d] * ig1;
    T wxt[3];
    cross3(w, t, wxt);
    const T a = dot3(w, t), s = T(1) / (T(1) + dot3(t, t));
    // u1 = s q, q = w + a t + w x t
    T q[3], qb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        q[d] = w[d] + a * t[d] + wxt[d];
        qb[d] = s * ub[d];
    }
    const T sb = dot3(ub, q);
    T wb[3], tb[3], tmp[3];
    cross3(t, qb, tmp);            // d((w x t).qb)/dw = t x qb
#pragma unroll
    for (int d = 0; d < 3; ++d)
        wb[d] = qb[d] + tmp[d];
    cross3(qb, w, tmp);            // d((w x t).qb)/dt = qb x w
    const T ab = dot3(qb, t);      // dL/da, a = w.t
    const T c1 = T(-2) * s * s * sb;   // s = 1/(1 + |t|^2)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        tb[d] = a * qb[d] + tmp[d] + ab * w[d] + c1 * t[d];
        wb[d] += ab * t[d];
    }
    // t = tau / g1, g1 = sqrt(G)
    const T g1b = -dot3(tb, t) * ig1;
    const T Gb = T(0.5) * g1b * ig1;
    const T sigb = Gb * G / D, Xb = Gb / D;
    const T wt = dot3(w, tau);
    const T wtb = T(2) * Xb * wt * inv_c2;   // X = |tau|^2 + (w.tau)^2/c^2
    T taub[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        taub[d] = tb[d] * ig1 + T(2) * Xb * tau[d] - T(2) * sigb * tau[d] + wtb * w[d];
        wb[d] += T(2) * sigb * w[d] * inv_c2 + wtb * tau[d];
    }
    // tau = h B; w = u0 + 2h E + h v0 x B; v0 = u0 / g0
    T v0b[3], wxv[3];
    cross3(B, wb, v0b);            // d((v0 x B).wb)/dv0 = B x wb
    cross3(wb, v0, wxv);           // d((v0 x B).wb)/dB = wb x v0
    const T ig0 = T(1) / sqrt(T(1) + dot3(u0, u0) * inv_c2);
    const T g0b = -h * dot3(v0b, v0) * ig0;   // dL/dg0 through v0 = u0/g0
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Bb[d] = h * (taub[d] + wxv[d]);
        Eb[d] = T(2) * h * wb[d];
        u0b[d] = wb[d] + h * v0b[d] * ig0 + g0b * v0[d] * inv_c2;
    }
}

// ---------------------------------------------------------------------------
// Position update in split representation, one axis: f += disp; the integer
// part moves the cell (|disp| < 1 so the shift is -1, 0 or +1); an offset
// that rounds to exactly 1 belongs to the next cell.
template <typename T>
__device__ inline void move_axis(T f0, T disp, T &f1, int &kappa)
{
    const T xi = f0 + disp;
    const T k = floor(xi);
    T f = xi - k;
    int kk = (int)k;
    if (f >= T(1)) {
        f -= T(1);
        kk += 1;
    }
    f1 = f;
    kappa = kk;
}

// ---------------------------------------------------------------------------
// Esirkepov deposition, per axis data in the frame of the union window of
// NW+1 nodes starting at node (cell + NB + min(kappa,0)).  DS = S1 - S0 is
// formed without cancellation: within one cell it is (d1-d0) times the
// divided difference of the weight polynomial; a cell crossing is split at
// the cell boundary into two such pieces.

template <int O, typename T>
struct EskAxis {
    static constexpr int NW = Shape<O, T>::NW;
    T S0[NW + 1], DS[NW + 1];
    int lo;       // first window node relative to the old cell
    bool cross;   // the particle changed cell along this axis
};

template <int O, typename T>
__device__ inline void esk_axis(T d0, T d1, int kappa, EskAxis<O, T> &e)
{
    using S = Shape<O, T>;
    constexpr int NW = S::NW;
    T w0[NW], qa[NW], qb[NW];
    S::w(d0, w0);
#pragma unroll
    for (int a = 0; a <= NW; ++a) {
        e.S0[a] = T(0);
        e.DS[a] = T(0);
    }
    e.cross = kappa != 0;
    if (kappa == 0) {
        S::q(d0, d1, qa);
        const T dd = d1 - d0;
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            e.S0[a] = w0[a];
            e.DS[a] = dd * qa[a];
        }
        e.lo = S::NB;
    } else if (kappa > 0) {
        // old cell from d0 to its upper face, then new cell from 0 to d1
        S::q(d0, T(1), qa);
        S::q(T(0), d1, qb);
        const T da = T(1) - d0;
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            e.S0[a] = w0[a];
            e.DS[a] += da * qa[a];
            e.DS[a + 1] += d1 * qb[a];
        }
        e.lo = S::NB;
    } else {
        // old cell from d0 down to its lower face, then new cell from 1 to d1
        S::q(d0, T(0), qa);
        S::q(T(1), d1, qb);
        const T db = d1 - T(1);
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            e.S0[a + 1] = w0[a];
            e.DS[a + 1] += -d0 * qa[a];
            e.DS[a] += db * qb[a];
        }
        e.lo = S::NB - 1;
    }
}

// Derivatives of the window S0 and DS with respect to d0 and d1 (adjoint).
template <int O, typename T>
__device__ inline void esk_axis_deriv(T d0, T d1, int kappa, T *dS0, T *dDS1)
{
    using S = Shape<O, T>;
    constexpr int NW = S::NW;
    T g0[NW], g1[NW];
    S::dw(d0, g0);
    S::dw(d1, g1);
#pragma unroll
    for (int a = 0; a <= NW; ++a) {
        dS0[a] = T(0);
        dDS1[a] = T(0);
    }
    // dDS/dd0 = -dS0/dd0 everywhere
    if (kappa == 0) {
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            dS0[a] = g0[a];
            dDS1[a] = g1[a];
        }
    } else if (kappa > 0) {
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            dS0[a] = g0[a];
            dDS1[a + 1] = g1[a];
        }
    } else {
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            dS0[a + 1] = g0[a];
            dDS1[a] = g1[a];
        }
    }
}

// Current of one particle: J_m(wm,wp,wq) += K_m P_m[wm] C(wp,wq) with
// P_m the running sum of DS_m along m and
// C = S0p S0q + DSp S0q/2 + S0p DSq/2 + DSp DSq/3
// (the Esirkepov weight (S0p S0q + S1p S1q)/3 + (S1p S0q + S0p S1q)/6
// rewritten in S0 and DS).  The products K P C are formed in the
// accumulator type A (double for the LDS current tile, whose FP64 atomics
// are far faster than FP32 ones on gfx950).  `add(m, index, value)`
// performs the scatter; jo[d][a] are the index offsets of window node a
// along axis d.
// With MSEL in 0..2 only that component is scattered.
template <int O, typename T, typename A, int MSEL = -1, typename AddFn>
__device__ __attribute__((always_inline)) inline void esk_scatter(const EskAxis<O, T> *e, const int (*jo)[Shape<O, T>::NW + 1], const T *K,
                                   AddFn &&add)
{
    constexpr int NW = Shape<O, T>::NW;
    const T half = T(0.5), third = T(1) / T(3);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        if (MSEL >= 0 && m != MSEL)
            continue;
        const int p = (m + 1) % 3, q = (m + 2) % 3;
        A P[NW];
        T run = T(0);
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            run += e[m].DS[a];
            P[a] = (A)(K[m] * run);
        }
        // A particle that stays in its cell along an axis has S0 = DS = 0 at
        // the window's last node, and along m its running sum closes to zero
        // one node earlier: those entries are zero and are not scattered.
        // The rim of the window is touched only by cell-crossing particles.
        const bool xm = e[m].cross, xp = e[p].cross, xq = e[q].cross;
#pragma unroll
        for (int c = 0; c <= NW; ++c) {
#pragma unroll
            for (int b = 0; b <= NW; ++b) {
                if ((c == NW && !xq) || (b == NW && !xp))
                    continue;
                const A C = (A)(e[p].S0[b] * (e[q].S0[c] + half * e[q].DS[c]) +
                                e[p].DS[b] * (half * e[q].S0[c] + third * e[q].DS[c]));
                const int base = jo[p][b] + jo[q][c];
#pragma unroll
                for (int a = 0; a < NW; ++a) {
                    if (a == NW - 1 && !xm)
                        continue;
                    add(m, base + jo[m][a], P[a] * C);
                }
            }
        }
    }
}

// The window of a particle that stays in its cell along every axis: the
// kappa = 0 case of esk_axis without the rim node (same arithmetic).
template <int O, typename T>
__device__ inline void esk_axis_still(T d0, T d1, T *S0, T *DS)
{
    using S = Shape<O, T>;
    constexpr int NW = S::NW;
    T qa[NW];
    S::w(d0, S0);
    S::q(d0, d1, qa);
    const T dd = d1 - d0;
#pragma unroll
    for (int a = 0; a < NW; ++a)
        DS[a] = dd * qa[a];
}

// esk_scatter for a particle that stays in its cell along every axis: the
// NW x NW cross-section and the NW - 1 nodes along m that carry current (the
// same sums as esk_scatter, without its rim branches).  jo[d][a] are the
// index offsets of the window nodes starting at the first gather node.
template <int O, typename T, typename A, typename AddFn>
__device__ __attribute__((always_inline)) inline void esk_scatter_still(const T (*S0)[Shape<O, T>::NW], const T (*DS)[Shape<O, T>::NW],
                                         const int (*jo)[Shape<O, T>::NW], const T *K, AddFn &&add)
{
    constexpr int NW = Shape<O, T>::NW;
    const T half = T(0.5), third = T(1) / T(3);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int p = (m + 1) % 3, q = (m + 2) % 3;
        A P[NW - 1];
        T run = T(0);
#pragma unroll
        for (int a = 0; a < NW - 1; ++a) {
            run += DS[m][a];
            P[a] = (A)(K[m] * run);
        }
#pragma unroll
        for (int c = 0; c < NW; ++c) {
#pragma unroll
            for (int b = 0; b < NW; ++b) {
                const A C = (A)(S0[p][b] * (S0[q][c] + half * DS[q][c]) + DS[p][b] * (half * S0[q][c] + third * DS[q][c]));
                const int base = jo[p][b] + jo[q][c];
#pragma unroll
                for (int a = 0; a < NW - 1; ++a)
                    add(m, base + jo[m][a], P[a] * C);
            }
        }
    }
}

// Transpose of esk_scatter_still (a particle that stays in its cell along
// every axis): the NW x NW cross-section and the NW - 1 nodes along m that
// carry current.  S0, DS and jo as for esk_scatter_still; returns
// d phi / d d0 and d phi / d d1 per axis for phi = <lJ, J_particle>.
template <int O, typename T, typename GetFn>
__device__ __attribute__((always_inline)) inline void esk_gather_adjoint_still(
    const T (*S0)[Shape<O, T>::NW], const T (*DS)[Shape<O, T>::NW], const T *d0, const T *d1,
    const int (*jo)[Shape<O, T>::NW], const T *K, GetFn &&get, T *g0, T *g1)
{
    constexpr int NW = Shape<O, T>::NW;
    const T half = T(0.5), third = T(1) / T(3);
    T gS0[3][NW], gDS[3][NW];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            gS0[d][a] = T(0);
            gDS[d][a] = T(0);
        }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int p = (m + 1) % 3, q = (m + 2) % 3;
        T P[NW - 1];
        T run = T(0);
#pragma unroll
        for (int a = 0; a < NW - 1; ++a) {
            run += DS[m][a];
            P[a] = run;
        }
        T G[NW - 1];
#pragma unroll
        for (int a = 0; a < NW - 1; ++a)
            G[a] = T(0);
#pragma unroll
        for (int c = 0; c < NW; ++c) {
#pragma unroll
            for (int b = 0; b < NW; ++b) {
                const T C = S0[p][b] * (S0[q][c] + half * DS[q][c]) + DS[p][b] * (half * S0[q][c] + third * DS[q][c]);
                const int base = jo[p][b] + jo[q][c];
                T H = T(0);
#pragma unroll
                for (int a = 0; a < NW - 1; ++a) {
                    const T l = get(m, base + jo[m][a]);
                    G[a] += l * C;
                    H += l * P[a];
                }
                H *= K[m];
                gS0[p][b] += H * (S0[q][c] + half * DS[q][c]);
                gDS[p][b] += H * (half * S0[q][c] + third * DS[q][c]);
                gS0[q][c] += H * (S0[p][b] + half * DS[p][b]);
                gDS[q][c] += H * (half * S0[p][b] + third * DS[p][b]);
                // finish this entry here (see esk_gather_adjoint)
#pragma unroll
                for (int a = 0; a < NW - 1; ++a)
                    asm volatile("" : "+v"(G[a]));
                asm volatile("" : "+v"(gS0[p][b]), "+v"(gDS[p][b]), "+v"(gS0[q][c]), "+v"(gDS[q][c]));
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // P[a] = sum_{a' <= a} DS[a'] -> dphi/dDS[a'] = sum_{a' <= a < NW-1} G[a]
        T suf = T(0);
#pragma unroll
        for (int a = NW - 2; a >= 0; --a) {
            suf += G[a];
            gDS[m][a] += K[m] * suf;
        }
    }
    // chain rule: S0 = w(d0) and DS = w(d1) - w(d0) on the same nodes
    using S = Shape<O, T>;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T w0[NW], w1[NW];
        S::dw(d0[d], w0);
        S::dw(d1[d], w1);
        T s0 = T(0), s1 = T(0);
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            s0 += (gS0[d][a] - gDS[d][a]) * w0[a];
            s1 += gDS[d][a] * w1[a];
        }
        g0[d] = s0;
        g1[d] = s1;
    }
}

// Transpose of esk_scatter: given the current adjoint lJ (read through
// `get(m, index)`), return d phi / d d0 and d phi / d d1 per axis for
// phi = <lJ, J_particle>.
template <int O, typename T, typename GetFn>
__device__ __attribute__((always_inline)) inline void esk_gather_adjoint(const EskAxis<O, T> *e, const T *d0, const T *d1, const int *kappa,
                                          const int (*jo)[Shape<O, T>::NW + 1], const T *K, GetFn &&get, T *g0,
                                          T *g1)
{
    constexpr int NW = Shape<O, T>::NW;
    const T half = T(0.5), third = T(1) / T(3);
    T gS0[3][NW + 1], gDS[3][NW + 1];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int a = 0; a <= NW; ++a) {
            gS0[d][a] = T(0);
            gDS[d][a] = T(0);
        }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int p = (m + 1) % 3, q = (m + 2) % 3;
        T P[NW];
        T run = T(0);
#pragma unroll
        for (int a = 0; a < NW; ++a) {
            run += e[m].DS[a];
            P[a] = run;
        }
        T G[NW];
#pragma unroll
        for (int a = 0; a < NW; ++a)
            G[a] = T(0);
#pragma unroll
        for (int c = 0; c <= NW; ++c) {
#pragma unroll
            for (int b = 0; b <= NW; ++b) {
                const T C = e[p].S0[b] * (e[q].S0[c] + half * e[q].DS[c]) +
                            e[p].DS[b] * (half * e[q].S0[c] + third * e[q].DS[c]);
                const int base = jo[p][b] + jo[q][c];
                // the window values enter unscaled: K_m multiplies H here and
                // G after the window
                T H = T(0);
#pragma unroll
                for (int a = 0; a < NW; ++a) {
                    const T l = get(m, base + jo[m][a]);
                    G[a] += l * C;
                    H += l * P[a];
                }
                H *= K[m];
                // dC/dS0p, dC/dDSp, dC/dS0q, dC/dDSq
                gS0[p][b] += H * (e[q].S0[c] + half * e[q].DS[c]);
                gDS[p][b] += H * (half * e[q].S0[c] + third * e[q].DS[c]);
                gS0[q][c] += H * (e[p].S0[b] + half * e[p].DS[b]);
                gDS[q][c] += H * (half * e[p].S0[b] + third * e[p].DS[b]);
                // Finish this window entry's arithmetic here: without the
                // register operands below the compiler issues every window
                // load first and parks the values in scratch memory.
#pragma unroll
                for (int a = 0; a < NW; ++a)
                    asm volatile("" : "+v"(G[a]));
                asm volatile("" : "+v"(gS0[p][b]), "+v"(gDS[p][b]), "+v"(gS0[q][c]), "+v"(gDS[q][c]));
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // P[a] = sum_{a' <= a} DS[a'] -> dphi/dDS[a'] = sum_{a >= a'} G[a]
        T suf = T(0);
#pragma unroll
        for (int a = NW - 1; a >= 0; --a) {
            suf += G[a];
            gDS[m][a] += K[m] * suf;
        }
    }
    // chain rule through the shapes; their derivatives are formed here, not
    // kept live across the loops above
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T dS0[NW + 1], dDS1[NW + 1];
        esk_axis_deriv<O>(d0[d], d1[d], kappa[d], dS0, dDS1);
        T s0 = T(0), s1 = T(0);
#pragma unroll
        for (int a = 0; a <= NW; ++a) {
            // DS = S1 - S0: dDS/dd0 = -dS0/dd0
            s0 += (gS0[d][a] - gDS[d][a]) * dS0[a];
            s1 += gDS[d][a] * dDS1[a];
        }
        g0[d] = s0;
        g1[d] = s1;
    }
}

}  // namespace pic
