/*
 * Scalar robust back-substitution for the right generalized eigenvectors of a real
 * Schur pencil (S, T) -- the CPU oracle.  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path links or calls this code.
 *
 * This file is included twice by tgevc_oracle.c, once with R = double and once with
 * R = long double; FN(x) appends the type suffix to every exported name.
 *
 * What is computed, and where the paper fixes it:
 *   - structure: S is quasi-upper-triangular, T upper triangular, diagonal blocks of
 *     order 1 or 2 (Section 2);
 *   - eigenvalues as pairs (alpha, beta), alpha complex, beta >= 0 (Section 2);
 *   - for eigenvalue (alpha, beta), alpha = a + i b, the eigenvector z solves
 *     (beta S - alpha T) z = 0 (Section 2.1, the lemma and equations DB1/DB2);
 *   - overflow is prevented with the two scalar functions ProtectDivision and
 *     ProtectUpdate of Section 4, whose defining bounds are
 *         xi |b| <= |t| Omega                 (division)
 *         xi (|Y| + |T| |X|) <= Omega         (update),
 *     and the result is an augmented vector <2^-k, w> that represents 2^k w
 *     (definition of an augmented matrix, Section 4; integer power-of-two scale
 *     factors, Section 5).
 * The substitution runs one eigenvector at a time over the 1x1/2x2 blocks from the
 * bottom up, exactly as the scalar solvers that the paper compares against do.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - Omega = 2^(EMAX-4) (2^1020 for double);
 *   - ProtectDivision/ProtectUpdate return the least power-of-two exponent that
 *     meets the bound (the update version keeps a relative margin of 2^-50 to cover
 *     the rounding of its own evaluation);
 *   - ProtectUpdate's argument order is (t, x, y) with bound xi (t x + y) <= Omega;
 *   - complex magnitudes use |Re| + |Im|, the two-column infinity norm;
 *   - the tip of a real eigenvector at p is w_p = 1; the tip of a complex pair at
 *     (p, p+1) has w_{p+1} = 1 and w_p from the second row of the singular 2x2
 *     block, so the phase is fixed;
 *   - pivots of modulus below smin = max(u (beta |S_qq|max + |alpha| |T_qq|max),
 *     tiny), taken over the diagonal block's own entries, are replaced by smin and
 *     flagged (assumption 3 excludes such cases); a threshold from the norm of the
 *     whole pencil would mark every pivot of a badly scaled pencil as singular;
 *   - complex division by Smith's method with the refinements of Baudin and Smith
 *     (2012), the method the paper points to for xLADIV;
 *   - 2x2 diagonal systems are solved by Gaussian elimination with complete
 *     pivoting, every division and update protected as above.
 */

#ifndef R
#error "R must be defined"
#endif

/* ---------------------------------------------------------------- scalars -- */

/* ProtectDivision: q >= 0 least with 2^-q * b <= t * Omega (b = |numerator| <= Omega,
 * t = |divisor| > 0).  The comparison is exact: t * Omega is an exact scaling. */
int FN(oracle_pd)(R b, R t)
{
    if (!(b > 0)) return 0;
    if (t >= 1) return 0;
    R tw = LDEXP(t, OMEGA_EXP);
    if (b <= tw) return 0;
    int eb, et;
    R mb = FREXP(b, &eb);
    R mt = FREXP(tw, &et);
    return eb - et + (mb > mt ? 1 : 0);
}

/* ProtectUpdate: q >= 0 least with 2^-q * (t*x + y) <= Omega * (1 - 2^-50), for
 * t, x, y in [0, Omega].  t*x may exceed the floating-point range, so the sum is
 * formed from mantissas and exponents. */
int FN(oracle_pu)(R t, R x, R y)
{
    int et = 0, ex = 0, ey = 0;
    R mt = (t > 0) ? FREXP(t, &et) : 0;
    R mx = (x > 0) ? FREXP(x, &ex) : 0;
    R my = (y > 0) ? FREXP(y, &ey) : 0;
    R mp = mt * mx;                       /* in [1/4, 1) or 0 */
    int ep = et + ex;
    int E;
    if (mp == 0 && my == 0) return 0;
    if (mp == 0) E = ey;
    else if (my == 0) E = ep;
    else E = ep > ey ? ep : ey;
    R s = (mp == 0 ? 0 : LDEXP(mp, ep - E)) + (my == 0 ? 0 : LDEXP(my, ey - E));
    int es;
    R ms = FREXP(s, &es);
    int q = es + E - OMEGA_EXP + (ms > (R)1 - MARGIN ? 1 : 0);
    return q > 0 ? q : 0;
}

/* Complex division (a + ib) / (c + id) by Smith's method with Baudin and Smith's
 * refinements for underflowing intermediate products. */
static void FN(cdiv_internal)(R a, R b, R c, R d, R *e, R *f)
{
    R r = d / c;
    R t = 1 / (c + d * r);
    if (r != 0) {
        R br = b * r;
        *e = (br != 0) ? (a + br) * t : a * t + (b * t) * r;
        R ar = a * r;
        *f = (ar != 0) ? (b - ar) * t : b * t - (a * t) * r;
    } else {
        *e = (a + d * (b / c)) * t;
        *f = (b - d * (a / c)) * t;
    }
}

void FN(oracle_cdiv)(R a, R b, R c, R d, R *e, R *f)
{
    if (FABS(d) <= FABS(c)) {
        FN(cdiv_internal)(a, b, c, d, e, f);
    } else {
        FN(cdiv_internal)(b, a, d, c, e, f);
        *f = -*f;
    }
}

/* ----------------------------------------------------------- structure (O1) -- */

/* blk[k] = 0 (1x1), 1 (first row of 2x2), 2 (second row).  Returns 0, or the info
 * bit 2 when two consecutive sub-diagonal entries are non-zero. */
int FN(oracle_blocks)(int64_t m, const double *S, int64_t lds, int8_t *blk)
{
    int bad = 0;
    for (int64_t k = 0; k < m; ++k) blk[k] = 0;
    for (int64_t k = 0; k + 1 < m; ++k) {
        if (S[(k + 1) + k * lds] != 0.0) {          /* sub-diagonal entry S[k+1, k] */
            if (blk[k] != 0) { bad = 2; continue; } /* S[k, k-1] is non-zero too */
            blk[k] = 1;
            blk[k + 1] = 2;
        }
    }
    return bad;
}

/* ---------------------------------------------------------- eigenvalues (O2) -- */

/* Scale (alpha, beta) by a power of two so that max(beta, |a| + |b|) is in (1/2, 1]. */
static void FN(normalize_ab)(R *a, R *b, R *be)
{
    R n = FABS(*a) + FABS(*b);
    if (*be > n) n = *be;
    if (n == 0) return;
    int e;
    FREXP(n, &e);
    *a = LDEXP(*a, -e);
    *b = LDEXP(*b, -e);
    *be = LDEXP(*be, -e);
}

/* Eigenvalue of the diagonal block starting at k.  Returns info bits. */
static int FN(block_eig)(int64_t k, int8_t kind, const double *S, int64_t lds,
                         const double *T, int64_t ldt, R *ar, R *ai, R *be)
{
#define SS(i, j) ((R)S[(i) + (j) * lds])
#define TT(i, j) ((R)T[(i) + (j) * ldt])
    int info = 0;
    if (kind == 0) {
        R a = SS(k, k), b = TT(k, k);
        if (b < 0 || (b == 0 && SIGNBIT(b))) { a = -a; b = -b; }
        *ar = a; *ai = 0; *be = b;
        if (a == 0 && b == 0) info |= 8;
    } else {
        R s11 = SS(k, k), s12 = SS(k, k + 1), s21 = SS(k + 1, k), s22 = SS(k + 1, k + 1);
        R t11 = TT(k, k), t12 = TT(k, k + 1), t22 = TT(k + 1, k + 1);
        /* scale the block to unit range; the eigenvalue scales by 2^(es - et) */
        R ms = FABS(s11), mt = FABS(t11);
        if (FABS(s12) > ms) ms = FABS(s12);
        if (FABS(s21) > ms) ms = FABS(s21);
        if (FABS(s22) > ms) ms = FABS(s22);
        if (FABS(t12) > mt) mt = FABS(t12);
        if (FABS(t22) > mt) mt = FABS(t22);
        int es = 0, et = 0;
        if (ms > 0) FREXP(ms, &es);
        if (mt > 0) FREXP(mt, &et);
        s11 = LDEXP(s11, -es); s12 = LDEXP(s12, -es); s21 = LDEXP(s21, -es); s22 = LDEXP(s22, -es);
        t11 = LDEXP(t11, -et); t12 = LDEXP(t12, -et); t22 = LDEXP(t22, -et);
        /* det(S_b - lambda T_b) = A2 lambda^2 - A1 lambda + A0 */
        R A2 = t11 * t22;
        R A1 = s11 * t22 + s22 * t11 - s21 * t12;
        R A0 = s11 * s22 - s12 * s21;
        if (A2 < 0) { A2 = -A2; A1 = -A1; A0 = -A0; }
        R disc = A1 * A1 - 4 * A2 * A0;
        if (disc >= 0) { info |= 4; disc = 0; }
        R a = A1 / 2, b = SQRT(-disc) / 2, bb = A2;
        if (a == 0 && b == 0 && bb == 0) info |= 8;
        /* undo the block scaling: alpha carries 2^es, beta carries 2^et */
        int d = es - et;
        if (d >= 0) bb = LDEXP(bb, -d); else { a = LDEXP(a, d); b = LDEXP(b, d); }
        *ar = a; *ai = b; *be = bb;
    }
    FN(normalize_ab)(ar, ai, be);
    return info;
#undef SS
#undef TT
}

int FN(oracle_eigvals)(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                       double *alpha_re, double *alpha_im, double *beta)
{
    int8_t *blk = (int8_t *)malloc((size_t)(m > 0 ? m : 1));
    int info = FN(oracle_blocks)(m, S, lds, blk);
    for (int64_t k = 0; k < m; ++k) {
        if (blk[k] == 2) continue;
        R ar, ai, be;
        info |= FN(block_eig)(k, blk[k], S, lds, T, ldt, &ar, &ai, &be);
        alpha_re[k] = (double)ar; alpha_im[k] = (double)ai; beta[k] = (double)be;
        if (blk[k] == 1) {
            alpha_re[k + 1] = (double)ar; alpha_im[k + 1] = -(double)ai; beta[k + 1] = (double)be;
        }
    }
    free(blk);
    return info;
}

/* --------------------------------------------------- one eigenvector (O4-O6) -- */

typedef struct {
    int64_t m;
    const double *S, *T;
    int64_t lds, ldt;
    const int8_t *blk;
} FN(pencil_t);

/* The working vector is (wr, wi) (wi unused for a real eigenvalue); k collects the
 * exponent of the scale factor: the represented vector is 2^k * w. */
static void FN(scale_all)(R *wr, R *wi, int64_t n, int q, int cplx)
{
    if (q <= 0) return;
    for (int64_t i = 0; i < n; ++i) {
        wr[i] = LDEXP(wr[i], -q);
        if (cplx) wi[i] = LDEXP(wi[i], -q);
    }
}

static R FN(cabs1)(R x, R y) { return FABS(x) + FABS(y); }

/* Pivot threshold for the diagonal block at r0 (order nb) and eigenvalue
 * (a + ib, be): u times the size of the terms of beta S_qq - alpha T_qq. */
static R FN(block_smin)(const FN(pencil_t) *P, int64_t r0, int nb, R a, R b, R be)
{
    R ms = 0, mt = 0;
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
            R s = FABS((R)P->S[(r0 + i) + (r0 + j) * P->lds]);
            R t = (i > j) ? 0 : FABS((R)P->T[(r0 + i) + (r0 + j) * P->ldt]);
            if (s > ms) ms = s;
            if (t > mt) mt = t;
        }
    R smin = U_ROUND * (be * ms + (FABS(a) + FABS(b)) * mt);
    return smin < TINY ? TINY : smin;
}

/* Solve the 1x1 or 2x2 system C w = y in rows r0..r0+nb-1 of the working vector,
 * where C = beta S_qq - alpha T_qq (trans = 1: C^T w = y, for the left eigenvectors),
 * writing w over y.  Every division and update is protected; the scaling exponents are
 * added to *k and applied to the whole working vector (length n).  Returns info bits. */
static int FN(diag_solve_t)(const FN(pencil_t) *P, int64_t r0, int nb, R a, R b, R be,
                            int cplx, R *wr, R *wi, int64_t n, int64_t *k, int trans)
{
#define SS(i, j) ((R)P->S[(i) + (j) * P->lds])
#define TT(i, j) ((R)P->T[(i) + (j) * P->ldt])
    int info = 0, q;
    R smin = FN(block_smin)(P, r0, nb, a, b, be);
    if (nb == 1) {
        R dr = be * SS(r0, r0) - a * TT(r0, r0);
        R di = -b * TT(r0, r0);
        if (!cplx) {
            if (FABS(dr) < smin) { dr = smin; info |= 16; }
            q = FN(oracle_pd)(FABS(wr[r0]), FABS(dr));
            if (q) { FN(scale_all)(wr, wi, n, q, 0); *k += q; }
            wr[r0] = wr[r0] / dr;
        } else {
            if (FN(cabs1)(dr, di) < smin) { dr = smin; di = 0; info |= 16; }
            /* |y/d|_1 <= 2 |y|_1 / |d|_1 */
            q = FN(oracle_pd)(FN(cabs1)(wr[r0], wi[r0]), FN(cabs1)(dr, di) / 2);
            if (q) { FN(scale_all)(wr, wi, n, q, 1); *k += q; }
            R e, f;
            FN(oracle_cdiv)(wr[r0], wi[r0], dr, di, &e, &f);
            wr[r0] = e; wi[r0] = f;
        }
        return info;
    }
    /* 2x2: C[i][j] = beta S(r0+i, r0+j) - alpha T(r0+i, r0+j), complex */
    R cr[2][2], ci[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            int ii = trans ? j : i, jj = trans ? i : j;   /* entry (i, j) of C or of C^T */
            R s = SS(r0 + ii, r0 + jj);
            R t = (ii > jj) ? 0 : TT(r0 + ii, r0 + jj);
            cr[i][j] = be * s - a * t;
            ci[i][j] = cplx ? -b * t : 0;
        }
    /* complete pivoting on |.|_1 */
    int ip = 0, jp = 0;
    R best = -1;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            R v = FN(cabs1)(cr[i][j], ci[i][j]);
            if (v > best) { best = v; ip = i; jp = j; }
        }
    if (best < smin) {
        cr[0][0] = smin; ci[0][0] = 0; cr[0][1] = 0; ci[0][1] = 0;
        cr[1][0] = 0; ci[1][0] = 0; cr[1][1] = smin; ci[1][1] = 0;
        ip = 0; jp = 0; info |= 16;
    }
    int io = 1 - ip, jo = 1 - jp;
    R u11r = cr[ip][jp], u11i = ci[ip][jp];
    R u12r = cr[ip][jo], u12i = ci[ip][jo];
    R l21r, l21i;
    if (cplx) FN(oracle_cdiv)(cr[io][jp], ci[io][jp], u11r, u11i, &l21r, &l21i);
    else { l21r = cr[io][jp] / u11r; l21i = 0; }
    R u22r = cr[io][jo] - (l21r * u12r - l21i * u12i);
    R u22i = ci[io][jo] - (l21r * u12i + l21i * u12r);
    if (FN(cabs1)(u22r, u22i) < smin) { u22r = smin; u22i = 0; info |= 16; }
    /* forward elimination of the right-hand side: r2 = y_io - l21 y_ip */
    R *y1r = &wr[r0 + ip], *y1i = &wi[r0 + ip];
    R *y2r = &wr[r0 + io], *y2i = &wi[r0 + io];
    R y1i_v = cplx ? *y1i : 0, y2i_v = cplx ? *y2i : 0;
    q = FN(oracle_pu)(FN(cabs1)(l21r, l21i), FN(cabs1)(*y1r, y1i_v), FN(cabs1)(*y2r, y2i_v));
    if (q) { FN(scale_all)(wr, wi, n, q, cplx); *k += q; y1i_v = cplx ? *y1i : 0; y2i_v = cplx ? *y2i : 0; }
    R r2r = *y2r - (l21r * *y1r - l21i * y1i_v);
    R r2i = y2i_v - (l21r * y1i_v + l21i * *y1r);
    R r1r = *y1r, r1i = y1i_v;
    /* w2 = r2 / u22 */
    R x2r, x2i;
    if (cplx) {
        q = FN(oracle_pd)(FN(cabs1)(r2r, r2i), FN(cabs1)(u22r, u22i) / 2);
        if (q) {
            FN(scale_all)(wr, wi, n, q, 1); *k += q;
            r2r = LDEXP(r2r, -q); r2i = LDEXP(r2i, -q); r1r = LDEXP(r1r, -q); r1i = LDEXP(r1i, -q);
        }
        FN(oracle_cdiv)(r2r, r2i, u22r, u22i, &x2r, &x2i);
    } else {
        q = FN(oracle_pd)(FABS(r2r), FABS(u22r));
        if (q) { FN(scale_all)(wr, wi, n, q, 0); *k += q; r2r = LDEXP(r2r, -q); r1r = LDEXP(r1r, -q); }
        x2r = r2r / u22r; x2i = 0;
    }
    /* w1 = (r1 - u12 w2) / u11 */
    q = FN(oracle_pu)(FN(cabs1)(u12r, u12i), FN(cabs1)(x2r, x2i), FN(cabs1)(r1r, r1i));
    if (q) {
        FN(scale_all)(wr, wi, n, q, cplx); *k += q;
        x2r = LDEXP(x2r, -q); x2i = LDEXP(x2i, -q); r1r = LDEXP(r1r, -q); r1i = LDEXP(r1i, -q);
    }
    R n1r = r1r - (u12r * x2r - u12i * x2i);
    R n1i = r1i - (u12r * x2i + u12i * x2r);
    R x1r, x1i;
    if (cplx) {
        q = FN(oracle_pd)(FN(cabs1)(n1r, n1i), FN(cabs1)(u11r, u11i) / 2);
        if (q) {
            FN(scale_all)(wr, wi, n, q, 1); *k += q;
            n1r = LDEXP(n1r, -q); n1i = LDEXP(n1i, -q); x2r = LDEXP(x2r, -q); x2i = LDEXP(x2i, -q);
        }
        FN(oracle_cdiv)(n1r, n1i, u11r, u11i, &x1r, &x1i);
    } else {
        q = FN(oracle_pd)(FABS(n1r), FABS(u11r));
        if (q) { FN(scale_all)(wr, wi, n, q, 0); *k += q; n1r = LDEXP(n1r, -q); x2r = LDEXP(x2r, -q); }
        x1r = n1r / u11r; x1i = 0;
    }
    /* undo the column permutation: unknown jp gets x1, unknown jo gets x2 */
    wr[r0 + jp] = x1r; wr[r0 + jo] = x2r;
    if (cplx) { wi[r0 + jp] = x1i; wi[r0 + jo] = x2i; }
    return info;
#undef SS
#undef TT
}

static int FN(diag_solve)(const FN(pencil_t) *P, int64_t r0, int nb, R a, R b, R be,
                          int cplx, R *wr, R *wi, int64_t n, int64_t *k)
{
    return FN(diag_solve_t)(P, r0, nb, a, b, be, cplx, wr, wi, n, k, 0);
}

/* y[0:r0] -= (beta S[0:r0, cols] - alpha T[0:r0, cols]) w[cols], cols = r0..r0+nb-1,
 * protected by ProtectUpdate with the exact norms of the three operands. */
static void FN(update_above)(const FN(pencil_t) *P, int64_t r0, int nb, R a, R b, R be,
                             int cplx, R *wr, R *wi, int64_t n, int64_t *k)
{
    if (r0 == 0) return;
    const double *S = P->S, *T = P->T;
    int64_t lds = P->lds, ldt = P->ldt;
    R aabs = FABS(a) + FABS(b);
    /* ||C||: max over rows above of sum over the block's columns of |C_il|_1 */
    R cn = 0;
    for (int64_t i = 0; i < r0; ++i) {
        R s = 0;
        for (int l = 0; l < nb; ++l)
            s += be * FABS((R)S[i + (r0 + l) * lds]) + aabs * FABS((R)T[i + (r0 + l) * ldt]);
        if (s > cn) cn = s;
    }
    R wn = 0, yn = 0;
    for (int l = 0; l < nb; ++l) {
        R v = FN(cabs1)(wr[r0 + l], cplx ? wi[r0 + l] : 0);
        if (v > wn) wn = v;
    }
    for (int64_t i = 0; i < r0; ++i) {
        R v = FN(cabs1)(wr[i], cplx ? wi[i] : 0);
        if (v > yn) yn = v;
    }
    int q = FN(oracle_pu)(cn, wn, yn);
    if (q) { FN(scale_all)(wr, wi, n, q, cplx); *k += q; }
    for (int l = 0; l < nb; ++l) {
        int64_t c = r0 + l;
        R xr = wr[c], xi = cplx ? wi[c] : 0;
        const double *Sc = S + c * lds, *Tc = T + c * ldt;
        if (!cplx) {
            R u = be * xr, v = a * xr;      /* beta w and alpha w */
            for (int64_t i = 0; i < r0; ++i)
                wr[i] -= (R)Sc[i] * u - (R)Tc[i] * v;
        } else {
            R ur = be * xr, ui = be * xi;   /* beta w */
            R vr = a * xr - b * xi, vi = b * xr + a * xi;   /* alpha w */
            for (int64_t i = 0; i < r0; ++i) {
                wr[i] -= (R)Sc[i] * ur - (R)Tc[i] * vr;
                wi[i] -= (R)Sc[i] * ui - (R)Tc[i] * vi;
            }
        }
    }
}

/* Eigenvector for the block starting at p.  On return w[0..pe) holds the mantissa
 * (pe = p + block order), *k the exponent.  Returns info bits. */
static int FN(eigvec)(const FN(pencil_t) *P, int64_t p, R *wr, R *wi, int64_t *kout)
{
    const double *S = P->S, *T = P->T;
    int64_t lds = P->lds, ldt = P->ldt;
    const int8_t *blk = P->blk;
    int info = 0;
    R a, b, be;
    info |= FN(block_eig)(p, blk[p], S, lds, T, ldt, &a, &b, &be);
    int cplx = (blk[p] == 1);
    int nbp = cplx ? 2 : 1;
    int64_t n = p + nbp;
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) { wr[i] = 0; wi[i] = 0; }
    if (info & 8) {           /* alpha = beta = 0: return the unit vector */
        wr[p] = 1;
        *kout = 0;
        return info;
    }
    /* tip */
    if (!cplx) {
        wr[p] = 1;
    } else {
        /* second row of M = beta S_b - alpha T_b: M21 w_p + M22 w_{p+1} = 0, w_{p+1} = 1 */
        R m21 = be * (R)S[p + 1 + p * lds];
        R m22r = be * (R)S[p + 1 + (p + 1) * lds] - a * (R)T[p + 1 + (p + 1) * ldt];
        R m22i = -b * (R)T[p + 1 + (p + 1) * ldt];
        R nr = -m22r, ni = -m22i;
        R smin = FN(block_smin)(P, p, 2, a, b, be);
        if (FABS(m21) < smin) { m21 = smin; info |= 16; }
        int q = FN(oracle_pd)(FN(cabs1)(nr, ni), FABS(m21));
        R one = 1;
        if (q) { one = LDEXP(one, -q); nr = LDEXP(nr, -q); ni = LDEXP(ni, -q); k += q; }
        wr[p] = nr / m21; wi[p] = ni / m21;
        wr[p + 1] = one; wi[p + 1] = 0;
    }
    /* right-hand side of the rows above the tip */
    FN(update_above)(P, p, nbp, a, b, be, cplx, wr, wi, n, &k);
    /* back-substitution over the blocks above the tip */
    int64_t r = p - 1;
    while (r >= 0) {
        int64_t r0 = (blk[r] == 2) ? r - 1 : r;
        int nb = (int)(r - r0 + 1);
        info |= FN(diag_solve)(P, r0, nb, a, b, be, cplx, wr, wi, n, &k);
        FN(update_above)(P, r0, nb, a, b, be, cplx, wr, wi, n, &k);
        r = r0 - 1;
    }
    *kout = k;
    return info;
}

/* All selected eigenvectors.  Z is column-major (ldz >= m); column c of a real
 * eigenvalue holds its eigenvector; for a pair in (p, p+1) column p holds the real
 * part and column p+1 the imaginary part of the eigenvector of the eigenvalue with
 * positive imaginary part.  normalize = 1: each eigenvector is divided by
 * max_i (|x_i| + |y_i|) and scales[c] = 0.  normalize = 0: Z holds the mantissa and
 * scales[c] the exponent k of the represented vector 2^k Z_c (only meaningful when
 * the mantissa fits the double range, i.e. for R = double).  Unselected columns are
 * zero.  Returns the OR of the info bits. */
int FN(oracle_tgevc)(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                     const int32_t *select, double *Z, int64_t ldz, int32_t *scales,
                     int normalize, int nthreads)
{
    if (m <= 0) return 0;
    int8_t *blk = (int8_t *)malloc((size_t)m);
    int info = FN(oracle_blocks)(m, S, lds, blk);
    FN(pencil_t) P;
    P.m = m; P.S = S; P.T = T; P.lds = lds; P.ldt = ldt; P.blk = blk;
    int64_t *starts = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t nstart = 0;
    for (int64_t c = 0; c < m; ++c) {
        if (blk[c] == 2) continue;
        int want = 1;
        if (select) {
            want = select[c] != 0;
            if (blk[c] == 1 && select[c + 1] != 0) want = 1;
        }
        if (want) starts[nstart++] = c;
    }
    for (int64_t c = 0; c < m; ++c) {
        for (int64_t i = 0; i < m; ++i) Z[i + c * ldz] = 0;
        scales[c] = 0;
    }
    /* largest first so that the dynamic schedule balances */
    int tinfo = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : tinfo)
    {
        R *wr = (R *)malloc(sizeof(R) * (size_t)(m + 2));
        R *wi = (R *)malloc(sizeof(R) * (size_t)(m + 2));
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = nstart - 1; s >= 0; --s) {
            int64_t p = starts[s];
            int64_t k = 0;
            tinfo |= FN(eigvec)(&P, p, wr, wi, &k);
            int cplx = blk[p] == 1;
            int64_t n = p + (cplx ? 2 : 1);
            if (normalize) {
                R nrm = 0;
                for (int64_t i = 0; i < n; ++i) {
                    R v = FABS(wr[i]) + (cplx ? FABS(wi[i]) : 0);
                    if (v > nrm) nrm = v;
                }
                if (nrm == 0) nrm = 1;
                for (int64_t i = 0; i < n; ++i) {
                    Z[i + p * ldz] = (double)(wr[i] / nrm);
                    if (cplx) Z[i + (p + 1) * ldz] = (double)(wi[i] / nrm);
                }
                scales[p] = 0;
                if (cplx) scales[p + 1] = 0;
            } else {
                for (int64_t i = 0; i < n; ++i) {
                    Z[i + p * ldz] = (double)wr[i];
                    if (cplx) Z[i + (p + 1) * ldz] = (double)wi[i];
                }
                scales[p] = (int32_t)k;
                if (cplx) scales[p + 1] = (int32_t)k;
            }
        }
        free(wr);
        free(wi);
    }
    info |= tinfo;
    if (select)
        for (int64_t c = 0; c + 1 < m; ++c)
            if (blk[c] == 1 && ((select[c] != 0) != (select[c + 1] != 0))) info |= 32;
    free(starts);
    free(blk);
    return info;
}

/* ------------------------------------------- left eigenvectors (Section 7) -- */

/* The left eigenvector u of eigenvalue (alpha, beta): u^H (beta S - alpha T) = 0.  With
 * w = conj(u) this is w^T C = 0, C = beta S - alpha T: a forward substitution over the
 * blocks from the eigenvalue's own block down, row-oriented where the right vectors are
 * column-oriented.  After block q is solved, the columns after it take the update
 *     y[cols after q] -= C[rows of q, cols after q]^T w_q,
 * whose protection needs the 1-norm of that block row (its largest column sum): the
 * conclusion's remark that left eigenvectors are the same computation with the 1-norm in
 * place of the infinity norm.  Diagonal blocks are solved transposed, C_qq^T w_q = y_q. */

/* y[r0+nb : n) -= C[r0 .. r0+nb-1, r0+nb : n)^T w[r0 .. r0+nb-1], protected by
 * ProtectUpdate with the exact 1-norm of the block row. */
static void FN(update_below)(const FN(pencil_t) *P, int64_t r0, int nb, R a, R b, R be,
                             int cplx, R *wr, R *wi, int64_t n, int64_t *k)
{
    int64_t c0 = r0 + nb;
    if (c0 >= n) return;
    const double *S = P->S, *T = P->T;
    int64_t lds = P->lds, ldt = P->ldt;
    R aabs = FABS(a) + FABS(b);
    R cn = 0;                     /* max over the columns after the block of its column sum */
    for (int64_t c = c0; c < n; ++c) {
        R s = 0;
        for (int l = 0; l < nb; ++l)
            s += be * FABS((R)S[(r0 + l) + c * lds]) + aabs * FABS((R)T[(r0 + l) + c * ldt]);
        if (s > cn) cn = s;
    }
    R wn = 0, yn = 0;
    for (int l = 0; l < nb; ++l) {
        R v = FN(cabs1)(wr[r0 + l], cplx ? wi[r0 + l] : 0);
        if (v > wn) wn = v;
    }
    for (int64_t c = c0; c < n; ++c) {
        R v = FN(cabs1)(wr[c], cplx ? wi[c] : 0);
        if (v > yn) yn = v;
    }
    int q = FN(oracle_pu)(cn, wn, yn);
    if (q) { FN(scale_all)(wr, wi, n, q, cplx); *k += q; }
    for (int l = 0; l < nb; ++l) {
        int64_t r = r0 + l;
        R xr = wr[r], xi = cplx ? wi[r] : 0;
        R ur = be * xr, ui = be * xi;                                  /* beta w */
        R vr = a * xr - b * xi, vi = b * xr + a * xi;                  /* alpha w */
        for (int64_t c = c0; c < n; ++c) {
            R s = (R)S[r + c * lds], t = (R)T[r + c * ldt];
            wr[c] -= s * ur - t * vr;
            if (cplx) wi[c] -= s * ui - t * vi;
        }
    }
}

/* w = conj(u) for the block starting at p; w[p .. m) holds the mantissa, *k the exponent.
 * Phase: w_p = 1 (for a pair, w_{p+1} from the first column of the singular block). */
static int FN(left_eigvec)(const FN(pencil_t) *P, int64_t p, R *wr, R *wi, int64_t *kout)
{
    const double *S = P->S, *T = P->T;
    int64_t lds = P->lds, ldt = P->ldt, m = P->m;
    const int8_t *blk = P->blk;
    int info = 0;
    R a, b, be;
    info |= FN(block_eig)(p, blk[p], S, lds, T, ldt, &a, &b, &be);
    int cplx = (blk[p] == 1);
    int nbp = cplx ? 2 : 1;
    int64_t k = 0;
    for (int64_t i = 0; i < m; ++i) { wr[i] = 0; wi[i] = 0; }
    if (info & 8) {
        wr[p] = 1;
        *kout = 0;
        return info;
    }
    if (!cplx) {
        wr[p] = 1;
    } else {
        /* first column of M = beta S_b - alpha T_b: w_p M11 + w_{p+1} M21 = 0, w_p = 1 */
        R m21 = be * (R)S[p + 1 + p * lds];
        R m11r = be * (R)S[p + p * lds] - a * (R)T[p + p * ldt];
        R m11i = -b * (R)T[p + p * ldt];
        R nr = -m11r, ni = -m11i;
        R smin = FN(block_smin)(P, p, 2, a, b, be);
        if (FABS(m21) < smin) { m21 = smin; info |= 16; }
        int q = FN(oracle_pd)(FN(cabs1)(nr, ni), FABS(m21));
        R one = 1;
        if (q) { one = LDEXP(one, -q); nr = LDEXP(nr, -q); ni = LDEXP(ni, -q); k += q; }
        wr[p] = one; wi[p] = 0;
        wr[p + 1] = nr / m21; wi[p + 1] = ni / m21;
    }
    FN(update_below)(P, p, nbp, a, b, be, cplx, wr, wi, m, &k);
    int64_t r = p + nbp;
    while (r < m) {
        int nb = (blk[r] == 1) ? 2 : 1;
        info |= FN(diag_solve_t)(P, r, nb, a, b, be, cplx, wr, wi, m, &k, 1);
        FN(update_below)(P, r, nb, a, b, be, cplx, wr, wi, m, &k);
        r += nb;
    }
    *kout = k;
    return info;
}

/* All selected left eigenvectors, in the layout of oracle_tgevc: column c of a real
 * eigenvalue holds u; for a pair (p, p+1), column p holds Re u and column p+1 Im u of the
 * left eigenvector of the eigenvalue with positive imaginary part (u = conj(w)).
 * normalize = 1: u / max_i (|Re u_i| + |Im u_i|), scales 0; else mantissa and exponent. */
int FN(oracle_tgevc_left)(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                          const int32_t *select, double *Z, int64_t ldz, int32_t *scales,
                          int normalize, int nthreads)
{
    if (m <= 0) return 0;
    int8_t *blk = (int8_t *)malloc((size_t)m);
    int info = FN(oracle_blocks)(m, S, lds, blk);
    FN(pencil_t) P;
    P.m = m; P.S = S; P.T = T; P.lds = lds; P.ldt = ldt; P.blk = blk;
    int64_t *starts = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t nstart = 0;
    for (int64_t c = 0; c < m; ++c) {
        if (blk[c] == 2) continue;
        int want = 1;
        if (select) {
            want = select[c] != 0;
            if (blk[c] == 1 && select[c + 1] != 0) want = 1;
        }
        if (want) starts[nstart++] = c;
    }
    for (int64_t c = 0; c < m; ++c) {
        for (int64_t i = 0; i < m; ++i) Z[i + c * ldz] = 0;
        scales[c] = 0;
    }
    int tinfo = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : tinfo)
    {
        R *wr = (R *)malloc(sizeof(R) * (size_t)(m + 2));
        R *wi = (R *)malloc(sizeof(R) * (size_t)(m + 2));
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nstart; ++s) {
            int64_t p = starts[s];
            int64_t k = 0;
            tinfo |= FN(left_eigvec)(&P, p, wr, wi, &k);
            int cplx = blk[p] == 1;
            R nrm = 1;
            if (normalize) {
                nrm = 0;
                for (int64_t i = p; i < m; ++i) {
                    R v = FABS(wr[i]) + (cplx ? FABS(wi[i]) : 0);
                    if (v > nrm) nrm = v;
                }
                if (nrm == 0) nrm = 1;
            }
            for (int64_t i = p; i < m; ++i) {
                Z[i + p * ldz] = (double)(wr[i] / nrm);
                if (cplx) Z[i + (p + 1) * ldz] = (double)(-wi[i] / nrm);   /* u = conj(w) */
            }
            scales[p] = normalize ? 0 : (int32_t)k;
            if (cplx) scales[p + 1] = scales[p];
        }
        free(wr);
        free(wi);
    }
    info |= tinfo;
    if (select)
        for (int64_t c = 0; c + 1 < m; ++c)
            if (blk[c] == 1 && ((select[c] != 0) != (select[c + 1] != 0))) info |= 32;
    free(starts);
    free(blk);
    return info;
}

/* --------------------------- complex-arithmetic pencils (Section 7, future work) -- */

/* S and T complex upper triangular of order m, stored interleaved (real, imaginary) and
 * column-major with leading dimensions counted in complex entries; there are no 2x2 blocks.
 * Eigenvalue k is lambda = s_kk / t_kk, kept as (alpha, beta) with beta = |t_kk| real >= 0
 * and alpha = s_kk conj(t_kk) / |t_kk| (t_kk = 0: beta = 0 and alpha = |s_kk|; both zero:
 * indefinite, info bit 8), scaled by a power of two so that max(beta, |alpha|_1) lies in
 * (1/2, 1].  Its eigenvector solves (beta S - alpha T) z = 0 with z_k = 1 and z_i = 0 for
 * i > k, by the same scalar robust back-substitution as the real case with 1x1 blocks only:
 * complex divisions protected by ProtectDivision, column updates by ProtectUpdate, pivots
 * below smin = max(u (beta |s_jj| + |alpha| |t_jj|), tiny) perturbed (info bit 16), complex
 * magnitudes |Re| + |Im|. */

#define CRE(A, ld, i, j) ((R)(A)[2 * ((i) + (j) * (int64_t)(ld))])
#define CIM(A, ld, i, j) ((R)(A)[2 * ((i) + (j) * (int64_t)(ld)) + 1])

/* |x + iy| without overflow */
static R FN(cmod)(R x, R y)
{
    R ax = FABS(x), ay = FABS(y);
    R mx = ax > ay ? ax : ay;
    if (mx == 0) return 0;
    R rx = ax / mx, ry = ay / mx;
    return mx * SQRT(rx * rx + ry * ry);
}

static int FN(ceig)(const double *S, int64_t lds, const double *T, int64_t ldt, int64_t k,
                    R *ar, R *ai, R *be)
{
    R sr = CRE(S, lds, k, k), si = CIM(S, lds, k, k);
    R tr = CRE(T, ldt, k, k), ti = CIM(T, ldt, k, k);
    R at = FN(cmod)(tr, ti);
    int info = 0;
    if (at > 0) {
        R ur = tr / at, ui = -ti / at;          /* conj(t) / |t| */
        *ar = sr * ur - si * ui;
        *ai = sr * ui + si * ur;
        *be = at;
    } else {
        *ar = FN(cmod)(sr, si);
        *ai = 0;
        *be = 0;
        if (*ar == 0) info |= 8;
    }
    FN(normalize_ab)(ar, ai, be);
    return info;
}

int FN(oracle_ceigvals)(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                        double *alpha_re, double *alpha_im, double *beta)
{
    int info = 0;
    for (int64_t k = 0; k < m; ++k) {
        R ar, ai, be;
        info |= FN(ceig)(S, lds, T, ldt, k, &ar, &ai, &be);
        alpha_re[k] = (double)ar; alpha_im[k] = (double)ai; beta[k] = (double)be;
    }
    return info;
}

/* y[0:r] -= (beta S[0:r, r] - alpha T[0:r, r]) w_r, protected by ProtectUpdate with the
 * exact bound of the column, the solved entry and the rows above. */
static void FN(cupdate_above)(const double *S, int64_t lds, const double *T, int64_t ldt, int64_t r,
                              R a, R b, R be, R *wr, R *wi, int64_t n, int64_t *k)
{
    if (r == 0) return;
    R aabs = FABS(a) + FABS(b);
    R cn = 0;
    for (int64_t i = 0; i < r; ++i) {
        R v = be * (FABS(CRE(S, lds, i, r)) + FABS(CIM(S, lds, i, r))) +
              aabs * (FABS(CRE(T, ldt, i, r)) + FABS(CIM(T, ldt, i, r)));
        if (v > cn) cn = v;
    }
    R wn = FN(cabs1)(wr[r], wi[r]), yn = 0;
    for (int64_t i = 0; i < r; ++i) {
        R v = FN(cabs1)(wr[i], wi[i]);
        if (v > yn) yn = v;
    }
    int q = FN(oracle_pu)(cn, wn, yn);
    if (q) { FN(scale_all)(wr, wi, n, q, 1); *k += q; }
    R ur = be * wr[r], ui = be * wi[r];                        /* beta w_r */
    R vr = a * wr[r] - b * wi[r], vi = b * wr[r] + a * wi[r];  /* alpha w_r */
    for (int64_t i = 0; i < r; ++i) {
        R sr = CRE(S, lds, i, r), si = CIM(S, lds, i, r);
        R tr = CRE(T, ldt, i, r), ti = CIM(T, ldt, i, r);
        /* S (beta w) - T (alpha w), complex products */
        wr[i] -= (sr * ur - si * ui) - (tr * vr - ti * vi);
        wi[i] -= (sr * ui + si * ur) - (tr * vi + ti * vr);
    }
}

static int FN(ceigvec)(const double *S, int64_t lds, const double *T, int64_t ldt, int64_t p,
                       R *wr, R *wi, int64_t *kout)
{
    int info = 0;
    R a, b, be;
    info |= FN(ceig)(S, lds, T, ldt, p, &a, &b, &be);
    int64_t n = p + 1, k = 0;
    for (int64_t i = 0; i < n; ++i) { wr[i] = 0; wi[i] = 0; }
    wr[p] = 1;
    if (info & 8) { *kout = 0; return info; }
    FN(cupdate_above)(S, lds, T, ldt, p, a, b, be, wr, wi, n, &k);
    for (int64_t j = p - 1; j >= 0; --j) {
        R sr = CRE(S, lds, j, j), si = CIM(S, lds, j, j);
        R tr = CRE(T, ldt, j, j), ti = CIM(T, ldt, j, j);
        /* d = beta s_jj - alpha t_jj */
        R dr = be * sr - (a * tr - b * ti);
        R di = be * si - (a * ti + b * tr);
        R smin = U_ROUND * (be * (FABS(sr) + FABS(si)) + (FABS(a) + FABS(b)) * (FABS(tr) + FABS(ti)));
        if (smin < TINY) smin = TINY;
        if (FN(cabs1)(dr, di) < smin) { dr = smin; di = 0; info |= 16; }
        int q = FN(oracle_pd)(FN(cabs1)(wr[j], wi[j]), FN(cabs1)(dr, di) / 2);
        if (q) { FN(scale_all)(wr, wi, n, q, 1); k += q; }
        R e, f;
        FN(oracle_cdiv)(wr[j], wi[j], dr, di, &e, &f);
        wr[j] = e; wi[j] = f;
        FN(cupdate_above)(S, lds, T, ldt, j, a, b, be, wr, wi, n, &k);
    }
    *kout = k;
    return info;
}

/* All selected eigenvectors of the complex pencil; Z complex (interleaved), column k the
 * eigenvector of eigenvalue k.  normalize = 1: divided by max_i |Re z_i| + |Im z_i|, scales 0;
 * else the mantissa in Z and the exponent in scales (2^scales[k] Z[:, k], with z_k = 1). */
int FN(oracle_ctgevc)(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                      const int32_t *select, double *Z, int64_t ldz, int32_t *scales,
                      int normalize, int nthreads)
{
    if (m <= 0) return 0;
    for (int64_t c = 0; c < m; ++c) {
        for (int64_t i = 0; i < m; ++i) { Z[2 * (i + c * ldz)] = 0; Z[2 * (i + c * ldz) + 1] = 0; }
        scales[c] = 0;
    }
    int tinfo = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : tinfo)
    {
        R *wr = (R *)malloc(sizeof(R) * (size_t)(m + 1));
        R *wi = (R *)malloc(sizeof(R) * (size_t)(m + 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = m - 1; s >= 0; --s) {
            if (select && !select[s]) continue;
            int64_t k = 0;
            tinfo |= FN(ceigvec)(S, lds, T, ldt, s, wr, wi, &k);
            R nrm = 1;
            if (normalize) {
                nrm = 0;
                for (int64_t i = 0; i <= s; ++i) {
                    R v = FN(cabs1)(wr[i], wi[i]);
                    if (v > nrm) nrm = v;
                }
                if (nrm == 0) nrm = 1;
            }
            for (int64_t i = 0; i <= s; ++i) {
                Z[2 * (i + s * ldz)] = (double)(wr[i] / nrm);
                Z[2 * (i + s * ldz) + 1] = (double)(wi[i] / nrm);
            }
            scales[s] = normalize ? 0 : (int32_t)k;
        }
        free(wr);
        free(wi);
    }
    return tinfo;
}
#undef CRE
#undef CIM
