/*
 * okr_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference ("oracle") of the segment-exhaustive
 * Kron-reduction search.  Only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg may load it; the product library never does.
 * It shares no code with the HIP path.
 *
 * Every step follows the paper (Mokhtari, Chevalier, Almassalkhi,
 * "Opti-KRON for three-phase distribution feeders", arXiv 2510.19608):
 *
 *   network, I = Y V ............................ Section II.A, eq. (KCL-3phase)
 *   Kron reduction Y_K = Y_KK - Y_KR Y_RR^+ Y_RK  Section II.B, eq. (Y_kron)
 *     (pseudo-inverse on the present-phase block, node-level reduction)
 *   assignment / aggregation I_agg = (A (x) I3) I Section II.C, eq. (i_agg)
 *   candidate solve Y V^c = I^c, voltage copy ... Algorithm 1 parallel block
 *   error ||V^|-|V^c||, bound E_bar ............. eq. (v_abs), eq. (iter_obj)
 *   scenario library from AC load flow .......... Section III (library L)
 *
 * Readings of points the paper leaves open (segments, assignment direction,
 * lexicographic objective, tie rule, band margins) are stated at the
 * functions that use them.
 *
 * Parity status: every function here is pinned by CPU tests (dense pinv
 * brute force, closed forms, invariants); see tests/test_oracle.py.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cx;

#define OKRO_OK 0
#define OKRO_E_ARG (-1)
#define OKRO_E_SINGULAR (-4)
#define OKRO_E_PF_DIVERGED (-5)
#define OKRO_W_BASE_OUT_OF_BAND 1

/* ------------------------------------------------------------------ */
/* 3x3 complex blocks, row-major                                       */
/* ------------------------------------------------------------------ */

/* Moore-Penrose pseudo-inverse of a block whose support is the principal
 * submatrix on the phases in `mask` (absent-phase rows and columns are zero,
 * Section II.A).  For that structure the pseudo-inverse is the ordinary
 * inverse of the present-phase submatrix, zero-padded; computed here by
 * Gauss-Jordan elimination with partial pivoting. */
static int blk_pinv(const cx *A, unsigned mask, cx *out)
{
    int idx[3], m = 0;
    for (int p = 0; p < 3; ++p)
        if (mask >> p & 1u) idx[m++] = p;
    cx a[3][6];
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) {
            a[r][c] = A[idx[r] * 3 + idx[c]];
            a[r][m + c] = (r == c) ? 1.0 : 0.0;
        }
    for (int col = 0; col < m; ++col) {
        int piv = col;
        for (int r = col + 1; r < m; ++r)
            if (cabs(a[r][col]) > cabs(a[piv][col])) piv = r;
        if (cabs(a[piv][col]) == 0.0) return OKRO_E_SINGULAR;
        if (piv != col)
            for (int c = 0; c < 2 * m; ++c) {
                cx t = a[col][c]; a[col][c] = a[piv][c]; a[piv][c] = t;
            }
        cx d = a[col][col];
        for (int c = 0; c < 2 * m; ++c) a[col][c] /= d;
        for (int r = 0; r < m; ++r) {
            if (r == col) continue;
            cx f = a[r][col];
            for (int c = 0; c < 2 * m; ++c) a[r][c] -= f * a[col][c];
        }
    }
    for (int i = 0; i < 9; ++i) out[i] = 0.0;
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) out[idx[r] * 3 + idx[c]] = a[r][m + c];
    return OKRO_OK;
}

/* exported for the pin tests of the restricted pseudo-inverse */
int okro_pinv3(const double *A, unsigned mask, double *out)
{
    return blk_pinv((const cx *)A, mask, (cx *)out);
}

static void blk_mul(const cx *A, const cx *B, cx *C)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            cx s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[r * 3 + k] * B[k * 3 + c];
            C[r * 3 + c] = s;
        }
}

static void blk_matvec(const cx *A, const cx *x, cx *y)
{
    for (int r = 0; r < 3; ++r)
        y[r] = A[r * 3 + 0] * x[0] + A[r * 3 + 1] * x[1] + A[r * 3 + 2] * x[2];
}

/* ------------------------------------------------------------------ */
/* Network context                                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int n, S;
    const int32_t *parent;
    const uint8_t *phase;
    const int32_t *segment;
    const cx *Ydiag; /* [n][9] */
    const cx *Yoff;  /* [n][9], Y_{i,parent(i)} */
    int *child_off, *child;  /* CSR children, increasing id */
    int *bfs;                /* parents before children */
    int *pre;                /* DFS preorder, children in increasing id */
    cx *z;                   /* [n][9] branch impedance (pinv of the branch admittance) */
} okro_net;

static void net_free(okro_net *N)
{
    if (!N) return;
    free(N->child_off); free(N->child); free(N->bfs); free(N->pre); free(N->z);
    free(N);
}

static okro_net *net_new(int n, const int32_t *parent, const uint8_t *phase,
                         const int32_t *segment, const double *Ydiag,
                         const double *Yoff, int *status)
{
    okro_net *N = (okro_net *)calloc(1, sizeof(okro_net));
    N->n = n;
    N->parent = parent; N->phase = phase; N->segment = segment;
    N->Ydiag = (const cx *)Ydiag; N->Yoff = (const cx *)Yoff;
    N->child_off = (int *)calloc((size_t)n + 1, sizeof(int));
    N->child = (int *)calloc((size_t)n, sizeof(int));
    N->bfs = (int *)calloc((size_t)n, sizeof(int));
    N->pre = (int *)calloc((size_t)n, sizeof(int));
    N->z = (cx *)calloc((size_t)n * 9, sizeof(cx));
    for (int i = 1; i < n; ++i) N->child_off[parent[i] + 1]++;
    for (int i = 0; i < n; ++i) N->child_off[i + 1] += N->child_off[i];
    int *fill = (int *)calloc((size_t)n, sizeof(int));
    for (int i = 1; i < n; ++i) {
        int p = parent[i];
        N->child[N->child_off[p] + fill[p]++] = i;
    }
    free(fill);
    /* BFS order */
    int head = 0, tail = 0;
    N->bfs[tail++] = 0;
    while (head < tail) {
        int v = N->bfs[head++];
        for (int e = N->child_off[v]; e < N->child_off[v + 1]; ++e) N->bfs[tail++] = N->child[e];
    }
    /* DFS preorder with an explicit stack */
    int *stack = (int *)malloc(sizeof(int) * (size_t)n);
    int sp = 0, np = 0;
    stack[sp++] = 0;
    while (sp) {
        int v = stack[--sp];
        N->pre[np++] = v;
        for (int e = N->child_off[v + 1] - 1; e >= N->child_off[v]; --e) stack[sp++] = N->child[e];
    }
    free(stack);
    /* branch impedance z_i = (y_i)^+ with y_i = -Y_{i,parent(i)} */
    *status = OKRO_OK;
    for (int i = 1; i < n; ++i) {
        cx y[9];
        for (int q = 0; q < 9; ++q) y[q] = -N->Yoff[(size_t)i * 9 + q];
        if (blk_pinv(y, phase[i], N->z + (size_t)i * 9) != OKRO_OK) *status = OKRO_E_SINGULAR;
    }
    return N;
}

/* ------------------------------------------------------------------ */
/* AC load flow: the scenario library (V^_l, I^_l) of Section III.     */
/* Constant-PQ wye loads; backward/forward sweep on the radial tree:   */
/* load currents conj(S/V), branch currents by backward accumulation,  */
/* V_child = V_parent - z J; repeat until max|dV| <= tol.              */
/* I^ is the injection (= -load current), so that Y V^ = I^ off the    */
/* slack; the slack row holds the current the substation supplies.     */
/* ------------------------------------------------------------------ */
int okro_powerflow(int n, const int32_t *parent, const uint8_t *phase,
                   const double *Ydiag, const double *Yoff, int S,
                   const double *Sload_, const double *V0_, double tol, int maxit,
                   double *Vhat_, double *Ihat_, int *iters_out)
{
    int st;
    okro_net *N = net_new(n, parent, phase, NULL, Ydiag, Yoff, &st);
    if (st != OKRO_OK) { net_free(N); return st; }
    const cx *Sload = (const cx *)Sload_;
    const cx *V0 = (const cx *)V0_;
    cx *Vhat = (cx *)Vhat_, *Ihat = (cx *)Ihat_;
    cx *J = (cx *)malloc(sizeof(cx) * (size_t)n * 3);
    cx *Vn = (cx *)malloc(sizeof(cx) * (size_t)n * 3);
    int worst_iters = 0, status = OKRO_OK;
    for (int l = 0; l < S; ++l) {
        const cx *Sl = Sload + (size_t)l * n * 3;
        cx *V = Vhat + (size_t)l * n * 3;
        for (int i = 0; i < n; ++i)
            for (int p = 0; p < 3; ++p) V[i * 3 + p] = (phase[i] >> p & 1u) ? V0[p] : 0.0;
        int it, conv = 0;
        for (it = 1; it <= maxit; ++it) {
            for (int i = 0; i < n; ++i)
                for (int p = 0; p < 3; ++p)
                    J[i * 3 + p] = (i > 0 && (phase[i] >> p & 1u)) ? conj(Sl[i * 3 + p] / V[i * 3 + p]) : 0.0;
            for (int b = n - 1; b >= 1; --b) {
                int v = N->bfs[b], pv = parent[v];
                for (int p = 0; p < 3; ++p) J[pv * 3 + p] += J[v * 3 + p];
            }
            for (int p = 0; p < 3; ++p) Vn[p] = V[p];
            double dmax = 0.0;
            for (int b = 1; b < n; ++b) {
                int v = N->bfs[b], pv = parent[v];
                cx d[3];
                blk_matvec(N->z + (size_t)v * 9, J + v * 3, d);
                for (int p = 0; p < 3; ++p) {
                    cx nv = (phase[v] >> p & 1u) ? Vn[pv * 3 + p] - d[p] : 0.0;
                    Vn[v * 3 + p] = nv;
                    double dd = cabs(nv - V[v * 3 + p]);
                    if (!(dd <= dmax)) dmax = dd; /* NaN-propagating max */
                }
            }
            memcpy(V, Vn, sizeof(cx) * (size_t)n * 3);
            if (!isfinite(dmax) || dmax > 1e3) break;
            if (dmax <= tol) { conv = 1; break; }
        }
        if (!conv) status = OKRO_E_PF_DIVERGED;
        if (it > worst_iters) worst_iters = it;
        /* injections at the converged voltages */
        cx *Il = Ihat + (size_t)l * n * 3;
        for (int i = 0; i < n * 3; ++i) Il[i] = 0.0;
        for (int i = 1; i < n; ++i)
            for (int p = 0; p < 3; ++p)
                if (phase[i] >> p & 1u) Il[i * 3 + p] = -conj(Sl[i * 3 + p] / V[i * 3 + p]);
        for (int i = 1; i < n; ++i)
            for (int p = 0; p < 3; ++p) Il[p] -= Il[i * 3 + p];
    }
    if (iters_out) *iters_out = worst_iters;
    free(J); free(Vn); net_free(N);
    return status;
}

/* ------------------------------------------------------------------ */
/* Sparse symmetric block matrix and block Gaussian elimination.       */
/* Eliminating node r replaces, for every pair of live neighbours a,b, */
/* Y_ab by Y_ab - Y_ar Y_rr^+ Y_rb: the Schur complement of Y_rr       */
/* (eq. Y_kron).  The same step with a right-hand side is Gaussian     */
/* elimination for the linear solve.                                   */
/* ------------------------------------------------------------------ */

typedef struct { int nbr; cx b[9]; } sp_ent;

typedef struct {
    int n;
    int *deg, *cap;
    sp_ent **row;
    cx *diag;
    uint8_t *alive;
} spmat;

static void sp_free(spmat *M)
{
    if (!M) return;
    for (int i = 0; i < M->n; ++i) free(M->row[i]);
    free(M->row); free(M->deg); free(M->cap); free(M->diag); free(M->alive);
    free(M);
}

static spmat *sp_from_net(const okro_net *N)
{
    int n = N->n;
    spmat *M = (spmat *)calloc(1, sizeof(spmat));
    M->n = n;
    M->deg = (int *)calloc((size_t)n, sizeof(int));
    M->cap = (int *)calloc((size_t)n, sizeof(int));
    M->row = (sp_ent **)calloc((size_t)n, sizeof(sp_ent *));
    M->diag = (cx *)malloc(sizeof(cx) * (size_t)n * 9);
    M->alive = (uint8_t *)malloc((size_t)n);
    memset(M->alive, 1, (size_t)n);
    memcpy(M->diag, N->Ydiag, sizeof(cx) * (size_t)n * 9);
    for (int i = 0; i < n; ++i) {
        int nc = N->child_off[i + 1] - N->child_off[i];
        M->cap[i] = nc + 2;
        M->row[i] = (sp_ent *)malloc(sizeof(sp_ent) * (size_t)M->cap[i]);
    }
    for (int i = 1; i < n; ++i) {
        int p = N->parent[i];
        const cx *Yip = N->Yoff + (size_t)i * 9;
        sp_ent *e = &M->row[i][M->deg[i]++];
        e->nbr = p;
        memcpy(e->b, Yip, sizeof(cx) * 9);
        sp_ent *f = &M->row[p][M->deg[p]++];
        f->nbr = i;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) f->b[r * 3 + c] = Yip[c * 3 + r]; /* Y_pi = Y_ip^T */
    }
    return M;
}

static sp_ent *sp_find(spmat *M, int a, int b, int create)
{
    for (int e = 0; e < M->deg[a]; ++e)
        if (M->row[a][e].nbr == b) return &M->row[a][e];
    if (!create) return NULL;
    if (M->deg[a] == M->cap[a]) {
        M->cap[a] = 2 * M->cap[a] + 2;
        M->row[a] = (sp_ent *)realloc(M->row[a], sizeof(sp_ent) * (size_t)M->cap[a]);
    }
    sp_ent *e = &M->row[a][M->deg[a]++];
    e->nbr = b;
    for (int q = 0; q < 9; ++q) e->b[q] = 0.0;
    return e;
}

static void sp_drop(spmat *M, int a, int b)
{
    for (int e = 0; e < M->deg[a]; ++e)
        if (M->row[a][e].nbr == b) {
            M->row[a][e] = M->row[a][--M->deg[a]];
            return;
        }
}

/* Eliminate node r.  If rhs != NULL (nrhs columns of [n][3]), it is updated
 * as well.  If `keep_row` != NULL the pivot pseudo-inverse and r's row at
 * elimination time are copied out for back-substitution. */
typedef struct { int r; cx piv[9]; int m; int nb[64]; cx blk[64][9]; } elim_rec;

static int sp_eliminate(spmat *M, const uint8_t *phase, int r, cx *rhs, int nrhs,
                        int n, elim_rec *rec)
{
    cx piv[9];
    if (blk_pinv(M->diag + (size_t)r * 9, phase[r], piv) != OKRO_OK) return OKRO_E_SINGULAR;
    int d = M->deg[r];
    if (rec) {
        if (d > 64) return OKRO_E_ARG;
        rec->r = r;
        memcpy(rec->piv, piv, sizeof piv);
        rec->m = d;
    }
    /* W_a = Y_ar piv for each neighbour a */
    cx (*W)[9] = (cx(*)[9])malloc(sizeof(cx) * 9 * (size_t)(d ? d : 1));
    int *nb = (int *)malloc(sizeof(int) * (size_t)(d ? d : 1));
    for (int e = 0; e < d; ++e) {
        int a = M->row[r][e].nbr;
        nb[e] = a;
        sp_ent *ar = sp_find(M, a, r, 0);
        blk_mul(ar->b, piv, W[e]);
        if (rec) {
            memcpy(rec->blk[e], M->row[r][e].b, sizeof(cx) * 9);
            rec->nb[e] = a;
        }
    }
    for (int ea = 0; ea < d; ++ea) {
        int a = nb[ea];
        for (int eb = 0; eb < d; ++eb) {
            int b = nb[eb];
            cx T[9];
            blk_mul(W[ea], M->row[r][eb].b, T);
            cx *dst = (a == b) ? M->diag + (size_t)a * 9 : sp_find(M, a, b, 1)->b;
            for (int q = 0; q < 9; ++q) dst[q] -= T[q];
        }
        if (rhs)
            for (int c = 0; c < nrhs; ++c) {
                cx t[3];
                blk_matvec(W[ea], rhs + ((size_t)c * n + r) * 3, t);
                for (int p = 0; p < 3; ++p) rhs[((size_t)c * n + a) * 3 + p] -= t[p];
            }
    }
    for (int ea = 0; ea < d; ++ea) sp_drop(M, nb[ea], r);
    M->deg[r] = 0;
    M->alive[r] = 0;
    free(W); free(nb);
    return OKRO_OK;
}

/* Kron reduction (eq. Y_kron): eliminate every node with keep[i] == 0, in
 * increasing node id.  The result is the Schur complement Y_Kron over the
 * kept nodes, independent of the order up to rounding. */
static int kron_reduce(const okro_net *N, const uint8_t *keep, spmat **out)
{
    spmat *M = sp_from_net(N);
    for (int i = 0; i < N->n; ++i)
        if (!keep[i]) {
            int st = sp_eliminate(M, N->phase, i, NULL, 0, N->n, NULL);
            if (st != OKRO_OK) { sp_free(M); return st; }
        }
    *out = M;
    return OKRO_OK;
}

/* Solve Y_K V_K = I_K (eq. Ik-YkVk) on the reduced matrix with the slack
 * voltage V0 held fixed (Dirichlet): move the slack column to the right-hand
 * side, eliminate the remaining nodes leaves-first, back-substitute.
 * I is [nrhs][n][3]; V receives [nrhs][n][3] for the kept nodes. */
static int solve_reduced(const okro_net *N, spmat *M, const cx *Iinj, const cx *V0,
                         int nrhs, cx *V)
{
    int n = N->n, st = OKRO_OK;
    cx *rhs = (cx *)malloc(sizeof(cx) * (size_t)nrhs * n * 3);
    memcpy(rhs, Iinj, sizeof(cx) * (size_t)nrhs * n * 3);
    for (int e = 0; e < M->deg[0]; ++e) {
        int a = M->row[0][e].nbr;
        sp_ent *a0 = sp_find(M, a, 0, 0);
        cx t[3];
        blk_matvec(a0->b, V0, t);
        for (int c = 0; c < nrhs; ++c)
            for (int p = 0; p < 3; ++p) rhs[((size_t)c * n + a) * 3 + p] -= t[p];
        sp_drop(M, a, 0);
    }
    M->deg[0] = 0;
    M->alive[0] = 0;
    elim_rec *recs = (elim_rec *)malloc(sizeof(elim_rec) * (size_t)n);
    int nrec = 0;
    for (int b = n - 1; b >= 1; --b) {
        int v = N->bfs[b];
        if (!M->alive[v]) continue;
        st = sp_eliminate(M, N->phase, v, rhs, nrhs, n, &recs[nrec]);
        if (st != OKRO_OK) goto done;
        ++nrec;
    }
    for (int c = 0; c < nrhs; ++c) {
        cx *Vc = V + (size_t)c * n * 3;
        for (int p = 0; p < 3; ++p) Vc[p] = V0[p];
        for (int q = nrec - 1; q >= 0; --q) {
            elim_rec *R = &recs[q];
            cx acc[3];
            for (int p = 0; p < 3; ++p) acc[p] = rhs[((size_t)c * n + R->r) * 3 + p];
            for (int e = 0; e < R->m; ++e) {
                cx t[3];
                blk_matvec(R->blk[e], Vc + R->nb[e] * 3, t);
                for (int p = 0; p < 3; ++p) acc[p] -= t[p];
            }
            blk_matvec(R->piv, acc, Vc + R->r * 3);
        }
    }
done:
    free(recs); free(rhs);
    return st;
}

/* super(i): nearest kept ancestor, inclusive (connectivity and uniqueness
 * rules of Section II.C; the reading "towards the slack" makes A a function
 * of the kept set). */
static void compute_super(const okro_net *N, const uint8_t *keep, int *sup)
{
    for (int b = 0; b < N->n; ++b) {
        int v = N->bfs[b];
        sup[v] = keep[v] ? v : sup[N->parent[v]];
    }
}

/* Candidate voltages for a kept set (Algorithm 1 parallel block):
 *   I^c = (A (x) I3) I^  (eq. i_agg: each reduced node's injection moves to
 *                         its super-node)
 *   Y_Kron from eq. (Y_kron); solve Y_Kron V_K = I^c_K with the slack fixed
 *   V^c_i = V^c_super(i) for reduced nodes (voltage assignment).
 * Vc is [S][n][3]; absent phases are zero. */
int okro_candidate_voltages(int n, const int32_t *parent, const uint8_t *phase,
                            const double *Ydiag, const double *Yoff, int S,
                            const double *Ihat_, const double *V0_,
                            const uint8_t *keep, double *Vc_)
{
    int st;
    okro_net *N = net_new(n, parent, phase, NULL, Ydiag, Yoff, &st);
    if (st != OKRO_OK) { net_free(N); return st; }
    const cx *Ihat = (const cx *)Ihat_;
    cx *Vc = (cx *)Vc_;
    int *sup = (int *)malloc(sizeof(int) * (size_t)n);
    compute_super(N, keep, sup);
    cx *Iagg = (cx *)calloc((size_t)S * n * 3, sizeof(cx));
    for (int l = 0; l < S; ++l)
        for (int i = 0; i < n; ++i)
            for (int p = 0; p < 3; ++p)
                Iagg[((size_t)l * n + sup[i]) * 3 + p] += Ihat[((size_t)l * n + i) * 3 + p];
    spmat *M = NULL;
    st = kron_reduce(N, keep, &M);
    if (st == OKRO_OK) {
        cx *VK = (cx *)calloc((size_t)S * n * 3, sizeof(cx));
        st = solve_reduced(N, M, Iagg, (const cx *)V0_, S, VK);
        for (int l = 0; l < S && st == OKRO_OK; ++l)
            for (int i = 0; i < n; ++i)
                for (int p = 0; p < 3; ++p)
                    Vc[((size_t)l * n + i) * 3 + p] =
                        (phase[i] >> p & 1u) ? VK[((size_t)l * n + sup[i]) * 3 + p] : 0.0;
        free(VK);
    }
    sp_free(M);
    free(Iagg); free(sup); net_free(N);
    return st;
}

/* Kron-reduced network of a kept set as radial blocks: for every kept node
 * x, Yk_diag[x] = Y_Kron(x,x) and, for x != 0, Yk_off[x] = Y_Kron(x, kp[x])
 * where kp[x] is the nearest kept proper ancestor.  extra_blocks receives the
 * number of nonzero off-diagonal blocks of Y_Kron that are not such tree
 * edges (0 when the reduction stays radial, Section V).  Rows of removed
 * nodes are zero. */
int okro_kron_blocks(int n, const int32_t *parent, const uint8_t *phase,
                     const double *Ydiag, const double *Yoff, const uint8_t *keep,
                     int32_t *kp, double *Yk_diag_, double *Yk_off_, int *extra_blocks)
{
    int st;
    okro_net *N = net_new(n, parent, phase, NULL, Ydiag, Yoff, &st);
    if (st != OKRO_OK) { net_free(N); return st; }
    spmat *M = NULL;
    st = kron_reduce(N, keep, &M);
    if (st != OKRO_OK) { net_free(N); return st; }
    cx *Yk_diag = (cx *)Yk_diag_, *Yk_off = (cx *)Yk_off_;
    int *sup = (int *)malloc(sizeof(int) * (size_t)n);
    compute_super(N, keep, sup);
    for (int i = 0; i < n; ++i) kp[i] = (keep[i] && i > 0) ? sup[parent[i]] : -1;
    int extra = 0;
    for (int i = 0; i < n; ++i) {
        for (int q = 0; q < 9; ++q) { Yk_diag[(size_t)i * 9 + q] = 0.0; Yk_off[(size_t)i * 9 + q] = 0.0; }
        if (!keep[i]) continue;
        memcpy(Yk_diag + (size_t)i * 9, M->diag + (size_t)i * 9, sizeof(cx) * 9);
        for (int e = 0; e < M->deg[i]; ++e) {
            int b = M->row[i][e].nbr;
            if (b == kp[i]) {
                memcpy(Yk_off + (size_t)i * 9, M->row[i][e].b, sizeof(cx) * 9);
            } else if (kp[b] != i) {
                double mx = 0;
                for (int q = 0; q < 9; ++q) mx = fmax(mx, cabs(M->row[i][e].b[q]));
                if (mx > 0) ++extra;
            }
        }
    }
    *extra_blocks = extra;
    free(sup); sp_free(M); net_free(N);
    return OKRO_OK;
}

/* ------------------------------------------------------------------ */
/* The segment-exhaustive search.                                       */
/* ------------------------------------------------------------------ */

typedef struct {
    double e_bar, v_min, v_max, tie_tol, amb_tol;
} okro_margins;

typedef struct {
    double e_glob, e_loc, slack_glob, slack_loc;
    double smice; /* sum over snapshots and clusters of the cluster's largest error */
    int feasible;
} okro_score;

typedef struct {
    okro_net *N;
    int S;
    const cx *Vhat, *Ihat, *V0;
    double *absVhat; /* [S][n][3] */
    cx *Vc;          /* work [S][n][3] */
    cx *Iagg;        /* work */
    int *sup;
    uint8_t *omega;  /* work: node in Omega_g */
    double *mice;    /* work [n]: MICE of the cluster whose super-node is i */
} okro_ctx;

/* Omega_g: for every e in the segment, c(e) is the highest node on e's root
 * path such that every node from c(e) down to e is in the segment or already
 * reduced; Omega_g is the union of the subtrees of the c(e).  It holds every
 * node whose candidate voltage or super-node can depend on the mask. */
static void omega_of_segment(const okro_net *N, const uint8_t *keep, int g,
                             const int *nodes, int k, uint8_t *omega)
{
    memset(omega, 0, (size_t)N->n);
    int *stack = (int *)malloc(sizeof(int) * (size_t)N->n);
    for (int j = 0; j < k; ++j) {
        int c = nodes[j];
        while (N->parent[c] >= 0) {
            int p = N->parent[c];
            if (N->segment[p] == g || !keep[p]) c = p; else break;
        }
        int sp = 0;
        stack[sp++] = c;
        while (sp) {
            int v = stack[--sp];
            if (omega[v]) continue;
            omega[v] = 1;
            for (int e = N->child_off[v]; e < N->child_off[v + 1]; ++e) stack[sp++] = N->child[e];
        }
    }
    free(stack);
}

/* Exported for the pin tests of Omega_g: omega_out[i] = 1 for the nodes of
 * segment g's affected region against the kept flags `keep`. */
int okro_omega(int n, const int32_t *parent, const uint8_t *phase,
               const int32_t *segment, const double *Ydiag, const double *Yoff,
               const uint8_t *keep, int g, uint8_t *omega_out)
{
    int st;
    okro_net *N = net_new(n, parent, phase, segment, Ydiag, Yoff, &st);
    if (st != OKRO_OK) { net_free(N); return st; }
    int *nodes = (int *)malloc(sizeof(int) * (size_t)n);
    int k = 0;
    for (int q = 0; q < n; ++q)
        if (segment[N->pre[q]] == g) nodes[k++] = N->pre[q];
    omega_of_segment(N, keep, g, nodes, k, omega_out);
    free(nodes); net_free(N);
    return OKRO_OK;
}

/* Score one kept set: errors per eq. (iter_obj) / Algorithm 1
 * (e = ||V^|-|V^c|| per node-phase-snapshot), the E_bar bound (eq. v_abs,
 * inclusive) and the voltage band on every node-phase.  Globals run over all
 * nodes; locals over Omega_g (slack_loc over the kept nodes in Omega_g).
 * SMICE (Algorithm 1's selection key, MICE of Section II.C): per snapshot,
 * every kept node's cluster (itself and the nodes whose super-node it is)
 * contributes its largest error over members and phases; summed over the
 * clusters and the snapshots. */
static int score_keepset(okro_ctx *C, const uint8_t *keep2, const uint8_t *omega,
                         const okro_margins *mg, okro_score *out)
{
    okro_net *N = C->N;
    int n = N->n, S = C->S;
    compute_super(N, keep2, C->sup);
    memset(C->Iagg, 0, sizeof(cx) * (size_t)S * n * 3);
    for (int l = 0; l < S; ++l)
        for (int i = 0; i < n; ++i)
            for (int p = 0; p < 3; ++p)
                C->Iagg[((size_t)l * n + C->sup[i]) * 3 + p] += C->Ihat[((size_t)l * n + i) * 3 + p];
    spmat *M = NULL;
    int st = kron_reduce(N, keep2, &M);
    if (st != OKRO_OK) return st;
    st = solve_reduced(N, M, C->Iagg, C->V0, S, C->Vc);
    sp_free(M);
    if (st != OKRO_OK) return st;
    double eg = 0, el = 0, sg = INFINITY, sl = INFINITY, smice = 0;
    for (int l = 0; l < S; ++l) {
        for (int i = 0; i < n; ++i) C->mice[i] = 0.0;
        for (int i = 0; i < n; ++i) {
            int s = C->sup[i];
            for (int p = 0; p < 3; ++p) {
                if (!(N->phase[i] >> p & 1u)) continue;
                double mag = cabs(C->Vc[((size_t)l * n + s) * 3 + p]);
                double e = fabs(mag - C->absVhat[((size_t)l * n + i) * 3 + p]);
                double sk = fmin(mag - mg->v_min, mg->v_max - mag);
                if (e > eg) eg = e;
                if (sk < sg) sg = sk;
                if (e > C->mice[s]) C->mice[s] = e;
                if (omega[i]) {
                    if (e > el) el = e;
                    if (keep2[i] && sk < sl) sl = sk;
                }
            }
        }
        for (int i = 0; i < n; ++i)
            if (C->sup[i] == i) smice += C->mice[i];
    }
    out->e_glob = eg; out->e_loc = el; out->slack_glob = sg; out->slack_loc = sl;
    out->smice = smice;
    out->feasible = (eg <= mg->e_bar) && (sg >= 0.0);
    return OKRO_OK;
}

static okro_ctx *ctx_new(okro_net *N, int S, const double *Vhat, const double *Ihat,
                         const double *V0)
{
    okro_ctx *C = (okro_ctx *)calloc(1, sizeof(okro_ctx));
    int n = N->n;
    C->N = N; C->S = S;
    C->Vhat = (const cx *)Vhat; C->Ihat = (const cx *)Ihat; C->V0 = (const cx *)V0;
    C->absVhat = (double *)malloc(sizeof(double) * (size_t)S * n * 3);
    for (size_t q = 0; q < (size_t)S * n * 3; ++q) C->absVhat[q] = cabs(C->Vhat[q]);
    C->Vc = (cx *)malloc(sizeof(cx) * (size_t)S * n * 3);
    C->Iagg = (cx *)malloc(sizeof(cx) * (size_t)S * n * 3);
    C->sup = (int *)malloc(sizeof(int) * (size_t)n);
    C->omega = (uint8_t *)malloc((size_t)n);
    C->mice = (double *)malloc(sizeof(double) * (size_t)n);
    return C;
}

static void ctx_free(okro_ctx *C)
{
    if (!C) return;
    free(C->absVhat); free(C->Vc); free(C->Iagg); free(C->sup); free(C->omega); free(C->mice);
    free(C);
}

/* Segment nodes in DFS preorder: bit j of a mask is the j-th of them. */
static int segment_nodes(const okro_net *N, int g, int *nodes)
{
    int k = 0;
    for (int q = 0; q < N->n; ++q) {
        int v = N->pre[q];
        if (N->segment[v] == g) nodes[k++] = v;
    }
    return k;
}

/* Score an explicit list of masks of segment g against a given kept state
 * (the kept flags before the segment).  Outputs are [nmask] arrays. */
int okro_score_masks(int n, const int32_t *parent, const uint8_t *phase,
                     const int32_t *segment, const double *Ydiag, const double *Yoff,
                     int S, const double *Vhat, const double *Ihat, const double *V0,
                     const uint8_t *keep_before, int g, const uint32_t *masks, int nmask,
                     double e_bar, double v_min, double v_max,
                     double *e_glob, double *e_loc, double *slack_glob,
                     double *slack_loc, int32_t *feasible, double *smice)
{
    int st;
    okro_net *N = net_new(n, parent, phase, segment, Ydiag, Yoff, &st);
    if (st != OKRO_OK) { net_free(N); return st; }
    okro_ctx *C = ctx_new(N, S, Vhat, Ihat, V0);
    okro_margins mg = {e_bar, v_min, v_max, 0, 0};
    int *nodes = (int *)malloc(sizeof(int) * (size_t)n);
    int k = segment_nodes(N, g, nodes);
    omega_of_segment(N, keep_before, g, nodes, k, C->omega);
    uint8_t *keep2 = (uint8_t *)malloc((size_t)n);
    for (int q = 0; q < nmask && st == OKRO_OK; ++q) {
        memcpy(keep2, keep_before, (size_t)n);
        for (int j = 0; j < k; ++j)
            if (masks[q] >> j & 1u) keep2[nodes[j]] = 0;
        okro_score sc;
        st = score_keepset(C, keep2, C->omega, &mg, &sc);
        e_glob[q] = sc.e_glob; e_loc[q] = sc.e_loc;
        slack_glob[q] = sc.slack_glob; slack_loc[q] = sc.slack_loc;
        feasible[q] = sc.feasible;
        if (smice) smice[q] = sc.smice;
    }
    free(keep2); free(nodes); ctx_free(C); net_free(N);
    return st;
}

/* Per-segment decision record. */
typedef struct {
    int32_t segment, k;
    uint32_t mask;
    int32_t popcount;
    double e_loc, e_min;
    int32_t ambiguous, n_scored;
    double key_gap; /* margin of the decision under the selection key: the smallest key above
                       the tie window at the chosen level minus the smallest key (inf if none) */
    double smice_rise; /* SMICE of the chosen mask minus SMICE of mask 0 (nothing reduced) */
} okro_decision;

static int popc(uint32_t m) { int c = 0; while (m) { m &= m - 1; ++c; } return c; }

/* Full search (the readings taken where the paper is open):
 *  - segments in increasing id, each against the cumulative kept state left
 *    by the earlier ones (Algorithm 1's "assign previously reduced" and
 *    I <- A I^);
 *  - feasible <=> e_glob <= E_bar and v_min <= |V^c| <= v_max everywhere;
 *  - objective: most reduced nodes, then the smallest key, then lowest mask.
 *    secondary 0: the key is e_loc (eq. iter_obj over Omega_g), masks with
 *    e_loc <= e_min + tie_tol tie; secondary 1: the key is SMICE over the
 *    whole network (Algorithm 1's selection), masks within smice_tol of the
 *    smallest tie;
 *  - a segment is flagged ambiguous when a feasible mask at the chosen level
 *    has its key within the ambiguity window (amb_tol for e_loc, smice_tol /
 *    100 for SMICE) of the tie-window edge, or a mask at that level or above
 *    has e_loc or its band slack over Omega_g within amb_tol of the E_bar or
 *    band boundary.
 * mode 0 scores all 2^k masks; mode 1 scores levels from popcount k down and
 * stops after the first level holding a feasible mask (same decision).
 * Returns OKRO_W_BASE_OUT_OF_BAND (and reduces nothing) when the full
 * network itself violates the band. */
int okro_search(int n, const int32_t *parent, const uint8_t *phase,
                const int32_t *segment, const double *Ydiag, const double *Yoff,
                int S, const double *Vhat, const double *Ihat, const double *V0,
                double e_bar, double v_min, double v_max, double tie_tol,
                double amb_tol, int mode, int secondary, double smice_tol,
                uint8_t *keep_out, okro_decision *dec, int max_segments,
                int *n_segments_out)
{
    int st;
    okro_net *N = net_new(n, parent, phase, segment, Ydiag, Yoff, &st);
    if (st != OKRO_OK) { net_free(N); return st; }
    okro_ctx *C = ctx_new(N, S, Vhat, Ihat, V0);
    okro_margins mg = {e_bar, v_min, v_max, tie_tol, amb_tol};
    int nseg = 0;
    for (int i = 0; i < n; ++i)
        if (segment[i] + 1 > nseg) nseg = segment[i] + 1;
    *n_segments_out = nseg;
    if (nseg > max_segments) { ctx_free(C); net_free(N); return OKRO_E_ARG; }
    memset(keep_out, 1, (size_t)n);
    /* the full network must itself satisfy the margins */
    okro_score base;
    memset(C->omega, 0, (size_t)n);
    st = score_keepset(C, keep_out, C->omega, &mg, &base);
    int warn = (st == OKRO_OK && !base.feasible) ? 1 : 0;
    int *nodes = (int *)malloc(sizeof(int) * (size_t)n);
    uint8_t *keep2 = (uint8_t *)malloc((size_t)n);
    for (int g = 0; g < nseg && st == OKRO_OK; ++g) {
        int k = segment_nodes(N, g, nodes);
        okro_decision *D = &dec[g];
        memset(D, 0, sizeof *D);
        D->segment = g; D->k = k;
        if (warn || k == 0 || k > 24) continue;
        omega_of_segment(N, keep_out, g, nodes, k, C->omega);
        uint32_t nm = 1u << k;
        double *el = (double *)malloc(sizeof(double) * nm);
        double *sm = (double *)malloc(sizeof(double) * nm);
        int8_t *fe = (int8_t *)malloc(nm);
        int8_t *near = (int8_t *)malloc(nm);
        uint8_t *done = (uint8_t *)calloc(nm, 1);
        int best_level = -1, nscored = 0;
        for (int level = k; level >= 0 && st == OKRO_OK; --level) {
            for (uint32_t m = 0; m < nm; ++m) {
                if (popc(m) != level) continue;
                memcpy(keep2, keep_out, (size_t)n);
                for (int j = 0; j < k; ++j)
                    if (m >> j & 1u) keep2[nodes[j]] = 0;
                okro_score sc;
                st = score_keepset(C, keep2, C->omega, &mg, &sc);
                if (st != OKRO_OK) break;
                ++nscored;
                done[m] = 1;
                el[m] = sc.e_loc;
                sm[m] = sc.smice;
                fe[m] = (int8_t)sc.feasible;
                int robust_in = sc.e_loc <= e_bar - amb_tol && sc.slack_loc >= amb_tol;
                int robust_out = sc.e_loc > e_bar + amb_tol || sc.slack_loc < -amb_tol;
                near[m] = (int8_t)(!robust_in && !robust_out);
                if (sc.feasible && best_level < 0) best_level = level;
            }
            if (mode == 1 && best_level >= 0) break;
        }
        /* mask 0 (nothing of the segment reduced), for the SMICE rise */
        double smice0 = 0.0;
        if (st == OKRO_OK) {
            if (done[0]) smice0 = sm[0];
            else {
                okro_score sc;
                st = score_keepset(C, keep_out, C->omega, &mg, &sc);
                smice0 = sc.smice;
            }
        }
        if (st == OKRO_OK) {
            D->n_scored = nscored;
            if (best_level < 0) {
                D->mask = 0; D->popcount = 0; D->e_loc = el[0]; D->e_min = el[0];
                D->ambiguous = 1; D->key_gap = INFINITY; D->smice_rise = 0.0;
            } else {
                /* the selection key of every feasible mask of the chosen level */
                const double *key = secondary ? sm : el;
                const double tol = secondary ? smice_tol : tie_tol;
                const double atol = secondary ? smice_tol / 100.0 : amb_tol;
                double emin = INFINITY, kmin = INFINITY;
                for (uint32_t m = 0; m < nm; ++m)
                    if (done[m] && fe[m] && popc(m) == best_level) {
                        if (el[m] < emin) emin = el[m];
                        if (key[m] < kmin) kmin = key[m];
                    }
                uint32_t pick = 0;
                int found = 0, amb = 0;
                for (uint32_t m = 0; m < nm; ++m) {
                    if (!done[m]) continue;
                    int pc = popc(m);
                    if (pc >= best_level && near[m]) amb = 1;
                    if (pc != best_level || !fe[m]) continue;
                    if (fabs(key[m] - (kmin + tol)) <= atol) amb = 1;
                    if (!found && key[m] <= kmin + tol) { pick = m; found = 1; }
                }
                /* the margin of the decision: the best feasible mask of the
                 * chosen level outside the tie window */
                double runner = INFINITY;
                for (uint32_t m = 0; m < nm; ++m)
                    if (done[m] && fe[m] && popc(m) == best_level && key[m] > kmin + tol && key[m] < runner)
                        runner = key[m];
                D->mask = pick; D->popcount = best_level; D->e_loc = el[pick];
                D->e_min = emin; D->ambiguous = amb;
                D->key_gap = runner - kmin;
                D->smice_rise = sm[pick] - smice0;
                for (int j = 0; j < k; ++j)
                    if (pick >> j & 1u) keep_out[nodes[j]] = 0;
            }
        }
        free(el); free(sm); free(fe); free(near); free(done);
    }
    free(nodes); free(keep2); ctx_free(C); net_free(N);
    if (st != OKRO_OK) return st;
    return warn ? OKRO_W_BASE_OUT_OF_BAND : OKRO_OK;
}

/* Per-snapshot maximum error of a final kept set over all nodes. */
int okro_final_errors(int n, const int32_t *parent, const uint8_t *phase,
                      const double *Ydiag, const double *Yoff, int S,
                      const double *Vhat_, const double *Ihat, const double *V0,
                      const uint8_t *keep, double *err_per_snapshot, double *Vc_out)
{
    int st = okro_candidate_voltages(n, parent, phase, Ydiag, Yoff, S, Ihat, V0, keep, Vc_out);
    if (st != OKRO_OK) return st;
    const cx *Vhat = (const cx *)Vhat_;
    const cx *Vc = (const cx *)Vc_out;
    for (int l = 0; l < S; ++l) {
        double e = 0;
        for (int i = 0; i < n; ++i)
            for (int p = 0; p < 3; ++p) {
                if (!(phase[i] >> p & 1u)) continue;
                size_t q = ((size_t)l * n + i) * 3 + p;
                double d = fabs(cabs(Vc[q]) - cabs(Vhat[q]));
                if (d > e) e = d;
            }
        err_per_snapshot[l] = e;
    }
    return OKRO_OK;
}

/* ------------------------------------------------------------------ */
/* The whole reduction in one call, with the argument contents of the  */
/* GPU library's reduce_feeder (topology, Y blocks, loads, margins in; */
/* aggregation map, Kron-reduced radial blocks, errors and per-segment */
/* decisions out), minus its workspace and stream.  The oracle's own   */
/* structs: it includes no header of the GPU path.                     */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t n;
    const int32_t *parent;
    const uint8_t *phase;
    const uint8_t *eligible;  /* not read: segment[] >= 0 marks the eligible nodes */
    const int32_t *segment;
} okro_topology;

typedef struct {
    const double *Y_diag;  /* [n][3][3] complex128 */
    const double *Y_off;   /* [n][3][3] complex128, Y_{i,parent(i)} */
} okro_yblocks;

typedef struct {
    int32_t S;
    const double *S_load;  /* [S][n][3] complex128, consumed power */
    const double *V0;      /* [3] complex128, slack */
    const double *Vhat;    /* [S][n][3] complex128 scenario voltages, or NULL: load flow */
} okro_loads;

typedef struct {
    double e_bar, v_min, v_max, tie_tol, amb_tol, pf_tol;
    int32_t pf_maxit;
    int32_t secondary;     /* 0: largest error over Omega_g, 1: SMICE */
    double smice_tol;      /* 0 = 1e-9 */
} okro_rmargins;

typedef struct {
    int32_t *super;            /* [n] nearest kept ancestor (itself when kept) */
    int32_t *kept_parent;      /* [n] kept parent in the reduced network (-1: reduced or slack) */
    double *Yk_diag, *Yk_off;  /* [n][3][3] complex128 (zero for reduced nodes) */
    double *err_per_snapshot;  /* [S] */
    double *Vhat;              /* [S][n][3] complex128 or NULL */
    okro_decision *seg;        /* [max(segment) + 1] */
    int32_t n_segments, n_kept;
    double max_err;
} okro_rresult;

int okr_oracle_reduce_feeder(const okro_yblocks *Y, const okro_topology *T,
                             const okro_loads *L, const okro_rmargins *mg,
                             okro_rresult *out)
{
    if (!Y || !T || !L || !mg || !out || !out->super || !out->kept_parent || !out->Yk_diag ||
        !out->Yk_off || !out->err_per_snapshot || !out->seg || T->n < 1 || L->S < 1)
        return OKRO_E_ARG;
    const int n = T->n, S = L->S;
    const size_t c3 = (size_t)S * n * 3;
    double *Vh = (double *)malloc(sizeof(cx) * c3);
    double *Ih = (double *)malloc(sizeof(cx) * c3);
    int st = OKRO_OK;
    if (L->Vhat) {
        /* injections of the given scenario voltages: -conj(S/V) at every
         * load node-phase, the slack supplying the rest (Section III) */
        memcpy(Vh, L->Vhat, sizeof(cx) * c3);
        const cx *Vc = (const cx *)Vh, *Sl = (const cx *)L->S_load;
        cx *Ic = (cx *)Ih;
        for (int l = 0; l < S; ++l) {
            cx *Il = Ic + (size_t)l * n * 3;
            for (int q = 0; q < n * 3; ++q) Il[q] = 0.0;
            for (int i = 1; i < n; ++i)
                for (int p = 0; p < 3; ++p)
                    if (T->phase[i] >> p & 1u) {
                        size_t q = ((size_t)l * n + i) * 3 + p;
                        Il[i * 3 + p] = -conj(Sl[q] / Vc[q]);
                    }
            for (int i = 1; i < n; ++i)
                for (int p = 0; p < 3; ++p) Il[p] -= Il[i * 3 + p];
        }
    } else {
        int it = 0;
        st = okro_powerflow(n, T->parent, T->phase, Y->Y_diag, Y->Y_off, S, L->S_load, L->V0,
                            mg->pf_tol > 0 ? mg->pf_tol : 1e-13, mg->pf_maxit > 0 ? mg->pf_maxit : 100,
                            Vh, Ih, &it);
    }
    uint8_t *keep = (uint8_t *)malloc((size_t)n);
    int nseg = 0;
    if (st == OKRO_OK)
        st = okro_search(n, T->parent, T->phase, T->segment, Y->Y_diag, Y->Y_off, S, Vh, Ih, L->V0,
                         mg->e_bar, mg->v_min, mg->v_max, mg->tie_tol, mg->amb_tol, 1, mg->secondary,
                         mg->smice_tol > 0 ? mg->smice_tol : 1e-9, keep, out->seg, n, &nseg);
    const int warn = st == OKRO_W_BASE_OUT_OF_BAND;
    if (st >= 0) {
        double *Vc = (double *)malloc(sizeof(cx) * c3);
        st = okro_final_errors(n, T->parent, T->phase, Y->Y_diag, Y->Y_off, S, Vh, Ih, L->V0, keep,
                               out->err_per_snapshot, Vc);
        free(Vc);
    }
    int extra = 0;
    if (st >= 0) st = okro_kron_blocks(n, T->parent, T->phase, Y->Y_diag, Y->Y_off, keep, out->kept_parent,
                                       out->Yk_diag, out->Yk_off, &extra);
    if (st >= 0) {
        int nk = 0;
        for (int i = 0; i < n; ++i) {
            int v = i;
            while (!keep[v]) v = T->parent[v];
            out->super[i] = v;
            nk += keep[i] ? 1 : 0;
        }
        out->n_kept = nk;
        out->n_segments = nseg;
        out->max_err = 0.0;
        for (int l = 0; l < S; ++l) out->max_err = fmax(out->max_err, out->err_per_snapshot[l]);
        if (out->Vhat) memcpy(out->Vhat, Vh, sizeof(cx) * c3);
    }
    free(Vh); free(Ih); free(keep);
    if (st < 0) return st;
    return warn ? OKRO_W_BASE_OUT_OF_BAND : OKRO_OK;
}
