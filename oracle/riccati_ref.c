/*
 * Serial FP64 Riccati recursion for the UFTOC problem P(N).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle of the
 * project: it may be built and called by tests/, by the smoke check and by
 * the CPU-baseline leg of the benchmark, and by nothing else.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Problem (paper, Sec. 2, eq. "org_eqc_problem"): minimise over x_0..x_N and
 * w_0..w_{N-1}
 *     sum_{t<N} ( 1/2 [x_t;w_t]' [[Qx_t, Qxw_t],[Qxw_t', Qw_t]] [x_t;w_t]
 *                 + lx_t' x_t + lw_t' w_t + c_t )
 *     + 1/2 x_N' QxN x_N + lN' x_N + cN
 * subject to x_0 = xbar0 and x_{t+1} = A_t x_t + B_t w_t + a_t.
 *
 * The solution is computed by the serial Riccati recursion of Sec. 3:
 *   Alg. 1 (factorization)   F, G, H, factor G, G K = -H', P = F - K' G K
 *   Alg. 2 (backward)        G k = B'Psi - lw - B'P a, Psi, cbar
 *   Alg. 3 (forward)         w = k + K x, x+ = A x + B w + a, lambda = P x - Psi
 * "A factorization of G" (Alg. 1) is read as the Cholesky factorization
 * G = L L' (G is positive definite, Sec. 3).  P is symmetrised after the
 * update (its exact value is symmetric).  The optimal value is the cost to go
 * at t = 0, 1/2 xbar0' P_0 xbar0 - Psi_0' xbar0 + cbar_0.
 *
 * Storage: every block is row-major; block t of an array of n-by-m blocks
 * starts at element t*n*m.  Qxw, a, lx, lw and c may be NULL (zero).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* y (n) = M (n x m, row-major) * v (m) */
static void mat_vec(int n, int m, const double *M, const double *v, double *y)
{
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += M[i * m + j] * v[j];
        y[i] = s;
    }
}

/* y (m) = M' v, M is n x m.  Every y[j] is summed over i in ascending
 * order; the loops run row by row of M for contiguous reads. */
static void matT_vec(int n, int m, const double *M, const double *v, double *y)
{
    for (int j = 0; j < m; ++j) y[j] = 0.0;
    for (int i = 0; i < n; ++i) {
        const double vi = v[i];
        for (int j = 0; j < m; ++j) y[j] += M[i * m + j] * vi;
    }
}

/* C (p x q) = X' Y with X r-by-p and Y r-by-q.  Every C[i][j] is summed over
 * k in ascending order starting from zero (the plain definition); the loops
 * run k outermost so that rows of X and Y are read contiguously. */
static void matT_mat(int r, int p, int q, const double *X, const double *Y, double *C)
{
    for (int e = 0; e < p * q; ++e) C[e] = 0.0;
    for (int k = 0; k < r; ++k)
        for (int i = 0; i < p; ++i) {
            const double xki = X[k * p + i];
            double *Ci = C + i * q;
            const double *Yk = Y + k * q;
            for (int j = 0; j < q; ++j) Ci[j] += xki * Yk[j];
        }
}

/* C (p x q) = X Y with X p-by-r and Y r-by-q; C[i][j] summed over k in
 * ascending order, rows of Y read contiguously. */
static void mat_mat(int p, int r, int q, const double *X, const double *Y, double *C)
{
    for (int i = 0; i < p; ++i) {
        double *Ci = C + i * q;
        for (int j = 0; j < q; ++j) Ci[j] = 0.0;
        for (int k = 0; k < r; ++k) {
            const double xik = X[i * r + k];
            const double *Yk = Y + k * q;
            for (int j = 0; j < q; ++j) Ci[j] += xik * Yk[j];
        }
    }
}

/* Cholesky G = L L' (lower, row-major, n x n).  Returns 0 on success, -1 if
 * a pivot is not positive (G not positive definite) or not finite. */
static int cholesky(int n, const double *G, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)n * n);
    for (int j = 0; j < n; ++j) {
        double d = G[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0) || !isfinite(d)) return -1;
        double ljj = sqrt(d);
        L[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = G[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / ljj;
        }
    }
    return 0;
}

/* Solve (L L') X = Y in place for an n x q right-hand side Y (row-major). */
static void chol_solve(int n, int q, const double *L, double *Y)
{
    for (int c = 0; c < q; ++c) {
        for (int i = 0; i < n; ++i) {            /* L z = y */
            double s = Y[i * q + c];
            for (int k = 0; k < i; ++k) s -= L[i * n + k] * Y[k * q + c];
            Y[i * q + c] = s / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {       /* L' x = z */
            double s = Y[i * q + c];
            for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * Y[k * q + c];
            Y[i * q + c] = s / L[i * n + i];
        }
    }
}

/*
 * Solve P(N).  Outputs x ((N+1)*nx), w (N*nu), lam ((N+1)*nx), obj (1).
 * Optional outputs (NULL to skip), indexed like the paper:
 *   P_all   (N+1)*nx*nx   P_t,   t = 0..N
 *   Psi_all (N+1)*nx      Psi_t, t = 0..N
 *   cbar_all (N+1)        cbar_t
 *   K_all   N*nu*nx       K_{t+1} stored at block t (policy used at stage t)
 *   k_all   N*nu          k_{t+1} stored at block t
 *   G_all   N*nu*nu       G_{t+1} stored at block t
 * Returns 0, -(t+1) if G_{t+1} is not positive definite, or -1000000 if
 * memory could not be allocated.
 */
int oracle_riccati_solve(int nx, int nu, int N,
                         const double *Qx, const double *Qw, const double *Qxw,
                         const double *A, const double *B, const double *a,
                         const double *lx, const double *lw, const double *c,
                         const double *QxN, const double *lN, double cN,
                         const double *xbar0,
                         double *x, double *w, double *lam, double *obj,
                         double *P_all, double *Psi_all, double *cbar_all,
                         double *K_all, double *k_all, double *G_all)
{
    const int n = nx, m = nu;
    const size_t nn = (size_t)n * n, mm = (size_t)m * m, nm = (size_t)n * m;
    double *P = malloc(sizeof(double) * (N + 1) * nn);
    double *Psi = malloc(sizeof(double) * (N + 1) * n);
    double *cb = malloc(sizeof(double) * (N + 1));
    double *K = malloc(sizeof(double) * (N > 0 ? N : 1) * nm);
    double *kk = malloc(sizeof(double) * (N > 0 ? N : 1) * m);
    double *G = malloc(sizeof(double) * mm);
    double *Lg = malloc(sizeof(double) * mm);
    double *F = malloc(sizeof(double) * nn);
    double *H = malloc(sizeof(double) * nm);
    double *PA = malloc(sizeof(double) * nn);
    double *PB = malloc(sizeof(double) * nm);
    double *GK = malloc(sizeof(double) * nm);
    double *KGK = malloc(sizeof(double) * nn);
    double *Pa = malloc(sizeof(double) * n);
    double *tn = malloc(sizeof(double) * n);
    double *tm = malloc(sizeof(double) * m);
    double *tm2 = malloc(sizeof(double) * m);
    int status = 0;
    if (!P || !Psi || !cb || !K || !kk || !G || !Lg || !F || !H || !PA || !PB ||
        !GK || !KGK || !Pa || !tn || !tm || !tm2) {
        status = -1000000;
        goto done;
    }

    /* Alg. 1 line 1 and Alg. 2 line 1: terminal cost to go */
    memcpy(P + (size_t)N * nn, QxN, sizeof(double) * nn);
    for (int i = 0; i < n; ++i) Psi[(size_t)N * n + i] = lN ? -lN[i] : 0.0;
    cb[N] = cN;

    for (int t = N - 1; t >= 0; --t) {
        const double *At = A + (size_t)t * nn, *Bt = B + (size_t)t * nm;
        const double *Pn = P + (size_t)(t + 1) * nn, *Psin = Psi + (size_t)(t + 1) * n;
        /* Alg. 1: F = Qx + A'PA, G = Qw + B'PB, H = Qxw + A'PB */
        mat_mat(n, n, n, Pn, At, PA);
        mat_mat(n, n, m, Pn, Bt, PB);
        matT_mat(n, n, n, At, PA, F);
        matT_mat(n, m, m, Bt, PB, G);
        matT_mat(n, n, m, At, PB, H);
        for (size_t e = 0; e < nn; ++e) F[e] += Qx[(size_t)t * nn + e];
        for (size_t e = 0; e < mm; ++e) G[e] += Qw[(size_t)t * mm + e];
        if (Qxw)
            for (size_t e = 0; e < nm; ++e) H[e] += Qxw[(size_t)t * nm + e];
        if (G_all) memcpy(G_all + (size_t)t * mm, G, sizeof(double) * mm);
        /* factor G */
        if (cholesky(m, G, Lg) != 0) {
            status = -(t + 1);
            goto done;
        }
        /* G K = -H'  (K is m x n) */
        double *Kt = K + (size_t)t * nm;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) Kt[i * n + j] = -H[j * m + i];
        chol_solve(m, n, Lg, Kt);
        /* Alg. 2: G k = B'Psi - lw - B'P a */
        if (a) mat_vec(n, n, Pn, a + (size_t)t * n, Pa);
        else memset(Pa, 0, sizeof(double) * n);
        for (int i = 0; i < n; ++i) tn[i] = Psin[i] - Pa[i];
        matT_vec(n, m, Bt, tn, tm);          /* B'Psi - B'Pa */
        double *kt = kk + (size_t)t * m;
        for (int i = 0; i < m; ++i) kt[i] = tm[i] - (lw ? lw[(size_t)t * m + i] : 0.0);
        chol_solve(m, 1, Lg, kt);
        /* Psi_t = A'Psi - H k - lx - A'P a */
        double *Psit = Psi + (size_t)t * n;
        matT_vec(n, n, At, tn, Psit);        /* A'Psi - A'Pa */
        mat_vec(n, m, H, kt, Pa);            /* reuse Pa as H k */
        for (int i = 0; i < n; ++i)
            Psit[i] -= Pa[i] + (lx ? lx[(size_t)t * n + i] : 0.0);
        /* cbar_t = cbar + 1/2 a'Pa - Psi'a - 1/2 k'Gk + c */
        double cbt = cb[t + 1] + (c ? c[t] : 0.0);
        if (a) {
            const double *at = a + (size_t)t * n;
            mat_vec(n, n, Pn, at, tn);
            double aPa = 0.0, Psia = 0.0;
            for (int i = 0; i < n; ++i) {
                aPa += at[i] * tn[i];
                Psia += Psin[i] * at[i];
            }
            cbt += 0.5 * aPa - Psia;
        }
        mat_vec(m, m, G, kt, tm2);
        double kGk = 0.0;
        for (int i = 0; i < m; ++i) kGk += kt[i] * tm2[i];
        cb[t] = cbt - 0.5 * kGk;
        /* Alg. 1: P_t = F - K' G K, then symmetrise */
        mat_mat(m, m, n, G, Kt, GK);
        matT_mat(m, n, n, Kt, GK, KGK);
        double *Pt = P + (size_t)t * nn;
        for (size_t e = 0; e < nn; ++e) Pt[e] = F[e] - KGK[e];
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                double s = 0.5 * (Pt[i * n + j] + Pt[j * n + i]);
                Pt[i * n + j] = s;
                Pt[j * n + i] = s;
            }
    }

    /* Alg. 3: forward recursion */
    memcpy(x, xbar0, sizeof(double) * n);
    for (int t = 0; t < N; ++t) {
        const double *xt = x + (size_t)t * n;
        double *wt = w + (size_t)t * m;
        mat_vec(m, n, K + (size_t)t * nm, xt, wt);
        for (int i = 0; i < m; ++i) wt[i] += kk[(size_t)t * m + i];
        double *xn = x + (size_t)(t + 1) * n;
        mat_vec(n, n, A + (size_t)t * nn, xt, xn);
        mat_vec(n, m, B + (size_t)t * nm, wt, tn);
        for (int i = 0; i < n; ++i) xn[i] += tn[i] + (a ? a[(size_t)t * n + i] : 0.0);
    }
    for (int t = 0; t <= N; ++t) {
        double *lt = lam + (size_t)t * n;
        mat_vec(n, n, P + (size_t)t * nn, x + (size_t)t * n, lt);
        for (int i = 0; i < n; ++i) lt[i] -= Psi[(size_t)t * n + i];
    }
    if (obj) {
        mat_vec(n, n, P, xbar0, tn);
        double v = cb[0];
        for (int i = 0; i < n; ++i) v += 0.5 * xbar0[i] * tn[i] - Psi[i] * xbar0[i];
        *obj = v;
    }
    if (P_all) memcpy(P_all, P, sizeof(double) * (N + 1) * nn);
    if (Psi_all) memcpy(Psi_all, Psi, sizeof(double) * (N + 1) * n);
    if (cbar_all) memcpy(cbar_all, cb, sizeof(double) * (N + 1));
    if (K_all) memcpy(K_all, K, sizeof(double) * N * nm);
    if (k_all) memcpy(k_all, kk, sizeof(double) * N * m);

done:
    free(P); free(Psi); free(cb); free(K); free(kk); free(G); free(Lg); free(F);
    free(H); free(PA); free(PB); free(GK); free(KGK); free(Pa); free(tn); free(tm);
    free(tm2);
    return status;
}
