/*
 * CPU oracle for the string-based CASCI path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow and deliberately straightforward: it builds matrix elements of
 * the fermionic Hamiltonian of eq. (hamiltonian) in Sec. II of the paper,
 *
 *     H = V + sum_pq h_pq a+_p a_q + 1/4 sum_pqrs <pq||rs> a+_p a+_q a_s a_r,
 *
 * between Slater determinants with the textbook Slater-Condon rules, in the
 * spin-orbital basis. It shares no code with the HIP library.
 *
 * Determinants (Sec. II.A.1, eq. model_space_det; occupation-number
 * representation of Sec. III.C): a 64-bit mask over 2n spin orbitals. Spin
 * orbital P < n is orbital P with spin alpha, P >= n is orbital P-n with spin
 * beta. A determinant is a+_{P1} a+_{P2} ... |-> with P1 < P2 < ..., i.e. all
 * alpha creators to the left of all beta creators, each group ascending --
 * the canonical operator order the paper uses for its operator strings
 * (Sec. III.C).
 *
 * Integrals: h[p*n+q] and chemists' (pq|rs) at eri[((p*n+q)*n+r)*n+s]. The
 * physicists' integral <PQ|RS> of the paper is (pr|qs) times spin deltas, and
 * <PQ||RS> = <PQ|RS> - <PQ|SR> (Sec. III.B).
 *
 * Permutation signs are never taken from a closed-form string formula: every
 * phase is obtained by applying the creation / annihilation operators one at
 * a time to the occupation list and counting the occupied spin orbitals each
 * operator has to pass.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t det_t;

typedef struct {
    int n;              /* spatial orbitals */
    const double* h;    /* n*n */
    const double* eri;  /* n^4 chemists' (pq|rs) */
    double ecore;
} ints_t;

static int occ(det_t d, int P) { return (int)((d >> P) & 1u); }

/* a_P |d>: returns 0 when P is empty; otherwise updates d and flips *sign
   once per occupied spin orbital Q < P that the operator passes. */
static int apply_annihilate(det_t* d, int P, int* sign)
{
    if (!occ(*d, P)) return 0;
    for (int Q = 0; Q < P; ++Q)
        if (occ(*d, Q)) *sign = -*sign;
    *d &= ~((det_t)1 << P);
    return 1;
}

/* a+_P |d> */
static int apply_create(det_t* d, int P, int* sign)
{
    if (occ(*d, P)) return 0;
    for (int Q = 0; Q < P; ++Q)
        if (occ(*d, Q)) *sign = -*sign;
    *d |= ((det_t)1 << P);
    return 1;
}

static int spin_of(const ints_t* I, int P) { return P >= I->n; }
static int orb_of(const ints_t* I, int P) { return P >= I->n ? P - I->n : P; }

/* one-electron integral between spin orbitals */
static double h_so(const ints_t* I, int P, int Q)
{
    if (spin_of(I, P) != spin_of(I, Q)) return 0.0;
    return I->h[orb_of(I, P) * I->n + orb_of(I, Q)];
}

/* <PQ|RS> = (pr|qs) delta(sP,sR) delta(sQ,sS) */
static double g_so(const ints_t* I, int P, int Q, int R, int S)
{
    if (spin_of(I, P) != spin_of(I, R) || spin_of(I, Q) != spin_of(I, S)) return 0.0;
    int n = I->n;
    int p = orb_of(I, P), q = orb_of(I, Q), r = orb_of(I, R), s = orb_of(I, S);
    return I->eri[((size_t)(p * n + r) * n + q) * n + s];
}

/* <PQ||RS> */
static double ga_so(const ints_t* I, int P, int Q, int R, int S)
{
    return g_so(I, P, Q, R, S) - g_so(I, P, Q, S, R);
}

static int popcount64(det_t x)
{
    int c = 0;
    while (x) { x &= x - 1; ++c; }
    return c;
}

/* <A|H|B> by the Slater-Condon rules. nso = 2n. */
static double h_element(const ints_t* I, det_t A, det_t B)
{
    const int nso = 2 * I->n;
    det_t diff = A ^ B;
    int ndiff = popcount64(diff);
    if (ndiff == 0) {
        double e = I->ecore;
        for (int P = 0; P < nso; ++P) {
            if (!occ(A, P)) continue;
            e += h_so(I, P, P);
            for (int Q = 0; Q < nso; ++Q)
                if (occ(A, Q)) e += 0.5 * ga_so(I, P, Q, P, Q);
        }
        return e;
    }
    if (ndiff == 2) {
        int M = -1, R = -1; /* M in A only, R in B only */
        for (int P = 0; P < nso; ++P) {
            if (!occ(diff, P)) continue;
            if (occ(A, P)) M = P; else R = P;
        }
        /* Gamma = <A| a+_M a_R |B> */
        det_t d = B;
        int sign = 1;
        if (!apply_annihilate(&d, R, &sign) || !apply_create(&d, M, &sign) || d != A) return 0.0;
        double v = h_so(I, M, R);
        for (int Q = 0; Q < nso; ++Q)
            if (occ(B, Q) && Q != R) v += ga_so(I, M, Q, R, Q);
        return sign * v;
    }
    if (ndiff == 4) {
        int Ms[2], Rs[2], nm = 0, nr = 0;
        for (int P = 0; P < nso; ++P) {
            if (!occ(diff, P)) continue;
            if (occ(A, P)) Ms[nm++] = P; else Rs[nr++] = P;
        }
        if (nm != 2 || nr != 2) return 0.0;
        /* Gamma = <A| a+_M1 a+_M2 a_R2 a_R1 |B>, rightmost operator acts first */
        det_t d = B;
        int sign = 1;
        if (!apply_annihilate(&d, Rs[0], &sign) || !apply_annihilate(&d, Rs[1], &sign) ||
            !apply_create(&d, Ms[1], &sign) || !apply_create(&d, Ms[0], &sign) || d != A)
            return 0.0;
        return sign * ga_so(I, Ms[0], Ms[1], Rs[0], Rs[1]);
    }
    return 0.0;
}

/* spin-orbital determinant of (alpha string a, beta string b) */
static det_t make_det(int n, uint64_t a, uint64_t b) { return (det_t)a | ((det_t)b << n); }

/* position of key in the ascending array arr[0..N), or -1 */
static long find_string(const uint64_t* arr, long N, uint64_t key)
{
    long lo = 0, hi = N - 1;
    while (lo <= hi) {
        long mid = (lo + hi) / 2;
        if (arr[mid] == key) return mid;
        if (arr[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/*
 * Dense H over the determinant basis (Ia, Ib) -> index Ia*Nb + Ib, with the
 * string arrays given in ascending order. H is Ndet x Ndet row-major.
 */
int oracle_dense_h(int n, const double* h, const double* eri, double ecore,
                   const uint64_t* astr, long Na, const uint64_t* bstr, long Nb, double* H)
{
    if (n < 1 || 2 * n > 64) return -1;
    ints_t I = {n, h, eri, ecore};
    long Nd = Na * Nb;
    for (long x = 0; x < Nd; ++x) {
        det_t A = make_det(n, astr[x / Nb], bstr[x % Nb]);
        for (long y = 0; y < Nd; ++y) {
            det_t B = make_det(n, astr[y / Nb], bstr[y % Nb]);
            H[x * Nd + y] = (popcount64(A ^ B) <= 4) ? h_element(&I, A, B) : 0.0;
        }
    }
    return 0;
}

/*
 * sigma_I = sum_J H_IJ C_J for the determinant indices rows[0..nrows),
 * enumerating every determinant J reachable from I by at most two
 * spin-orbital substitutions that keep the numbers of alpha and beta
 * electrons. C has Na*Nb entries; out has nrows entries.
 */
int oracle_sigma_rows(int n, const double* h, const double* eri, double ecore,
                      const uint64_t* astr, long Na, const uint64_t* bstr, long Nb,
                      const double* C, const long* rows, long nrows, double* out)
{
    if (n < 1 || 2 * n > 64) return -1;
    ints_t I = {n, h, eri, ecore};
    const int nso = 2 * n;
    det_t amask = (n == 64) ? ~(det_t)0 : (((det_t)1 << n) - 1);
    int* holes = (int*)malloc(sizeof(int) * nso);
    int* parts = (int*)malloc(sizeof(int) * nso);
    if (!holes || !parts) { free(holes); free(parts); return -2; }
    for (long t = 0; t < nrows; ++t) {
        long x = rows[t];
        det_t A = make_det(n, astr[x / Nb], bstr[x % Nb]);
        int nh = 0, np = 0;
        for (int P = 0; P < nso; ++P) {
            if (occ(A, P)) holes[nh++] = P; else parts[np++] = P;
        }
        double acc = h_element(&I, A, A) * C[x];
        /* singles */
        for (int i = 0; i < nh; ++i)
            for (int a = 0; a < np; ++a) {
                if (spin_of(&I, holes[i]) != spin_of(&I, parts[a])) continue;
                det_t B = (A & ~((det_t)1 << holes[i])) | ((det_t)1 << parts[a]);
                long ia = find_string(astr, Na, B & amask);
                long ib = find_string(bstr, Nb, B >> n);
                if (ia < 0 || ib < 0) continue;
                acc += h_element(&I, A, B) * C[ia * Nb + ib];
            }
        /* doubles */
        for (int i = 0; i < nh; ++i)
            for (int j = i + 1; j < nh; ++j)
                for (int a = 0; a < np; ++a)
                    for (int b = a + 1; b < np; ++b) {
                        int sh = spin_of(&I, holes[i]) + spin_of(&I, holes[j]);
                        int sp = spin_of(&I, parts[a]) + spin_of(&I, parts[b]);
                        if (sh != sp) continue;
                        det_t B = A & ~((det_t)1 << holes[i]) & ~((det_t)1 << holes[j]);
                        B |= ((det_t)1 << parts[a]) | ((det_t)1 << parts[b]);
                        long ia = find_string(astr, Na, B & amask);
                        long ib = find_string(bstr, Nb, B >> n);
                        if (ia < 0 || ib < 0) continue;
                        acc += h_element(&I, A, B) * C[ia * Nb + ib];
                    }
        out[t] = acc;
    }
    free(holes);
    free(parts);
    return 0;
}

/*
 * Rows of H in sparse form: for each determinant index rows[t], every
 * determinant J reachable by at most two spin-orbital substitutions (same
 * enumeration as oracle_sigma_rows) and the element H_IJ. Row t writes
 * count[t] <= maxc pairs into cols[t*maxc ...] and vals[t*maxc ...].
 */
int oracle_h_rows(int n, const double* h, const double* eri, double ecore,
                  const uint64_t* astr, long Na, const uint64_t* bstr, long Nb,
                  const long* rows, long nrows, long maxc, long* cols, double* vals, long* count)
{
    if (n < 1 || 2 * n > 64) return -1;
    ints_t I = {n, h, eri, ecore};
    const int nso = 2 * n;
    det_t amask = (((det_t)1 << n) - 1);
    int* holes = (int*)malloc(sizeof(int) * nso);
    int* parts = (int*)malloc(sizeof(int) * nso);
    if (!holes || !parts) { free(holes); free(parts); return -2; }
    for (long t = 0; t < nrows; ++t) {
        long x = rows[t];
        det_t A = make_det(n, astr[x / Nb], bstr[x % Nb]);
        int nh = 0, np = 0;
        for (int P = 0; P < nso; ++P) {
            if (occ(A, P)) holes[nh++] = P; else parts[np++] = P;
        }
        long c = 0;
        long* cr = cols + t * maxc;
        double* vr = vals + t * maxc;
        cr[c] = x; vr[c] = h_element(&I, A, A); ++c;
        for (int i = 0; i < nh; ++i)
            for (int a = 0; a < np; ++a) {
                if (spin_of(&I, holes[i]) != spin_of(&I, parts[a])) continue;
                det_t B = (A & ~((det_t)1 << holes[i])) | ((det_t)1 << parts[a]);
                long ia = find_string(astr, Na, B & amask);
                long ib = find_string(bstr, Nb, B >> n);
                if (ia < 0 || ib < 0) continue;
                if (c >= maxc) { free(holes); free(parts); return -3; }
                cr[c] = ia * Nb + ib; vr[c] = h_element(&I, A, B); ++c;
            }
        for (int i = 0; i < nh; ++i)
            for (int j = i + 1; j < nh; ++j)
                for (int a = 0; a < np; ++a)
                    for (int b = a + 1; b < np; ++b) {
                        int sh = spin_of(&I, holes[i]) + spin_of(&I, holes[j]);
                        int sp = spin_of(&I, parts[a]) + spin_of(&I, parts[b]);
                        if (sh != sp) continue;
                        det_t B = A & ~((det_t)1 << holes[i]) & ~((det_t)1 << holes[j]);
                        B |= ((det_t)1 << parts[a]) | ((det_t)1 << parts[b]);
                        long ia = find_string(astr, Na, B & amask);
                        long ib = find_string(bstr, Nb, B >> n);
                        if (ia < 0 || ib < 0) continue;
                        if (c >= maxc) { free(holes); free(parts); return -3; }
                        cr[c] = ia * Nb + ib; vr[c] = h_element(&I, A, B); ++c;
                    }
        count[t] = c;
    }
    free(holes);
    free(parts);
    return 0;
}

/*
 * Dense S^2 over the same basis: S^2 = Sz^2 + Sz + S- S+, with
 * S+ = sum_p a+_{p alpha} a_{p beta} and S- = sum_p a+_{p beta} a_{p alpha},
 * each operator applied to the occupation list one at a time.
 */
int oracle_dense_s2(int n, const uint64_t* astr, long Na, const uint64_t* bstr, long Nb, double* S2)
{
    if (n < 1 || 2 * n > 64) return -1;
    long Nd = Na * Nb;
    det_t amask = (n == 64) ? ~(det_t)0 : (((det_t)1 << n) - 1);
    memset(S2, 0, sizeof(double) * (size_t)Nd * (size_t)Nd);
    for (long y = 0; y < Nd; ++y) {
        det_t B = make_det(n, astr[y / Nb], bstr[y % Nb]);
        int na = popcount64(B & amask), nb = popcount64(B >> n);
        double sz = 0.5 * (na - nb);
        S2[y * Nd + y] += sz * sz + sz;
        for (int q = 0; q < n; ++q) {       /* S+ term a+_{q a} a_{q b} */
            det_t d = B;
            int sign = 1;
            if (!apply_annihilate(&d, n + q, &sign) || !apply_create(&d, q, &sign)) continue;
            for (int p = 0; p < n; ++p) {   /* S- term a+_{p b} a_{p a} */
                det_t e = d;
                int s2 = sign;
                if (!apply_annihilate(&e, p, &s2) || !apply_create(&e, n + p, &s2)) continue;
                long ia = find_string(astr, Na, e & amask);
                long ib = find_string(bstr, Nb, e >> n);
                if (ia < 0 || ib < 0) continue;
                S2[(ia * Nb + ib) * Nd + y] += s2;
            }
        }
    }
    return 0;
}

/*
 * Single-substitution list of every string of one spin (Sec. II.A.1): for
 * string I = strs[t] and each entry, in the order p over the occupied orbitals
 * of I ascending and, for each p, q over (unoccupied orbitals of I) + {p}
 * ascending, the string J = I - p + q and sign = <I| a+_p a_q |J>, obtained by
 * applying a_q and then a+_p to J one operator at a time. Outputs are [N][s]
 * with s = ne (n - ne + 1); J is the position of the string in strs.
 */
int oracle_single_list(int n, const uint64_t* strs, long N, int s, long* J, long* sign, long* P, long* Q)
{
    if (n < 1 || n > 64) return -1;
    for (long t = 0; t < N; ++t) {
        const det_t I = strs[t];
        long e = 0;
        for (int p = 0; p < n; ++p) {
            if (!occ(I, p)) continue;
            for (int q = 0; q < n; ++q) {
                if (occ(I, q) && q != p) continue;
                det_t d = (I & ~((det_t)1 << p)) | ((det_t)1 << q);
                const long jj = find_string(strs, N, d);
                int sg = 1;
                if (jj < 0 || !apply_annihilate(&d, q, &sg) || !apply_create(&d, p, &sg) || d != I) return -2;
                if (e >= s) return -3;
                J[t * s + e] = jj;
                sign[t * s + e] = sg;
                P[t * s + e] = p;
                Q[t * s + e] = q;
                ++e;
            }
        }
        if (e != s) return -3;
    }
    return 0;
}

/*
 * Spin-resolved one- and two-particle reduced density matrices of a real CI
 * vector C over the determinants (Ia, Ib) -> Ia*Nb + Ib (Sec. II.A.1, the
 * density matrices the multireference methods consume), by applying the
 * operators to each determinant one at a time:
 *   g1[s][p][q]          = <C| a+_{p s} a_{q s} |C>,                    s = alpha, beta
 *   g2[st][((p n + q) n + r) n + u] = <C| a+_{p s} a+_{r t} a_{u t} a_{q s} |C>,
 *                                                            st = (alpha alpha), (alpha beta), (beta beta)
 * The rightmost operator acts first. Spin orbital of orbital p with spin s:
 * p + s n (alpha creators left of beta creators, as for the determinants).
 */
static long det_index(int n, const uint64_t* astr, long Na, const uint64_t* bstr, long Nb, det_t d)
{
    det_t amask = (((det_t)1 << n) - 1);
    long ia = find_string(astr, Na, d & amask);
    long ib = find_string(bstr, Nb, d >> n);
    if (ia < 0 || ib < 0) return -1;
    return ia * Nb + ib;
}

int oracle_rdm(int n, const uint64_t* astr, long Na, const uint64_t* bstr, long Nb, const double* C,
               double* g1, double* g2)
{
    if (n < 1 || 2 * n > 64) return -1;
    const long Nd = Na * Nb;
    const long n2 = (long)n * n, n4 = n2 * n2;
    memset(g1, 0, sizeof(double) * 2 * n2);
    if (g2) memset(g2, 0, sizeof(double) * 3 * n4);
    const int spins[3][2] = {{0, 0}, {0, 1}, {1, 1}};
    for (long y = 0; y < Nd; ++y) {
        const double cj = C[y];
        if (cj == 0.0) continue;
        const det_t B = make_det(n, astr[y / Nb], bstr[y % Nb]);
        for (int s = 0; s < 2; ++s)
            for (int q = 0; q < n; ++q) {
                det_t d = B;
                int sign = 1;
                if (!apply_annihilate(&d, q + s * n, &sign)) continue;
                for (int p = 0; p < n; ++p) {
                    det_t e = d;
                    int sg = sign;
                    if (!apply_create(&e, p + s * n, &sg)) continue;
                    const long x = det_index(n, astr, Na, bstr, Nb, e);
                    if (x < 0) return -2;
                    g1[(s * n + p) * n + q] += sg * C[x] * cj;
                }
            }
        if (!g2) continue;
        for (int k = 0; k < 3; ++k) {
            const int s = spins[k][0], t = spins[k][1];
            for (int q = 0; q < n; ++q) {
                det_t d1 = B;
                int s1 = 1;
                if (!apply_annihilate(&d1, q + s * n, &s1)) continue;
                for (int u = 0; u < n; ++u) {
                    det_t d2 = d1;
                    int s2 = s1;
                    if (!apply_annihilate(&d2, u + t * n, &s2)) continue;
                    for (int r = 0; r < n; ++r) {
                        det_t d3 = d2;
                        int s3 = s2;
                        if (!apply_create(&d3, r + t * n, &s3)) continue;
                        for (int p = 0; p < n; ++p) {
                            det_t d4 = d3;
                            int s4 = s3;
                            if (!apply_create(&d4, p + s * n, &s4)) continue;
                            const long x = det_index(n, astr, Na, bstr, Nb, d4);
                            if (x < 0) return -2;
                            g2[k * n4 + ((p * n + q) * n + r) * n + u] += s4 * C[x] * cj;
                        }
                    }
                }
            }
        }
    }
    return 0;
}
