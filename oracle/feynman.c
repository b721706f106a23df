/*
 * oracle/feynman.c -- CPU oracle for the reduced-history Feynman method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU library.
 *
 * What it computes (paper, Section IV):
 *   - the internal-wire formulation (Section II-A): every gate/qubit incidence
 *     that is not wire-preserving opens a new binary wire segment; wire-
 *     preserving incidences (diagonal gates, control roles) keep the segment;
 *   - gate roles (Section II-A): diagonal -> wire-preserving, exactly one
 *     nonzero per column -> deterministic, otherwise branching;
 *   - source placement by one sweep (Section IV-A; Section IV-F, Table I):
 *     backward (the paper's choice): an artificial source sits on the
 *     input-side segment of every branching gate whose input segment is not
 *     a natural input segment, numbered in the output->input sweep order;
 *     forward: on the output-side segment of every branching gate whose
 *     output segment is not a natural output segment, numbered in the
 *     input->output sweep order; source k is bit k of the history index h,
 *     and the sweep direction is the evaluation order;
 *   - the reduced sum of Eq. (7) (Algorithm 1) and its checkpointed form
 *     (Algorithm 2), both as one walk over evaluation-order regions: the
 *     boundary values and everything they imply are fixed first; then, region
 *     by region, each assignment of the region's sources is fixed, what it
 *     implies is propagated inside the region, and the region's gate factors
 *     are multiplied in, before the later regions are walked; one region is
 *     Algorithm 1, the cuts c1 <= c2 give Algorithm 2's prefix, root and
 *     suffix;
 *   - Eq. (8) gate-operation estimate and its argmin over all cut pairs
 *     (Section IV-C, "Autotuned Partitioning"), in exact 128-bit integers.
 *
 * PropagateKnownValues is a fixpoint over local gate relations (each
 * deterministic gate admits only the (in,out) pairs of its permutation),
 * swept forward and backward until nothing changes.  This is deliberately a
 * different mechanism from the GPU's straight-line backward program.
 *
 * Readings where the paper leaves the arithmetic open:
 *   - threshold pruning: a history is dropped iff M < t, where M is the
 *     product, in evaluation order, of min(1, |U_g[out,in]|)
 *     over branching gates g; M never grows, so where the test sits does not
 *     change the result; t = 0 prunes nothing;
 *   - a history is valid iff propagation never conflicts, no gate factor is an
 *     exact zero, and M >= t;
 *   - cuts c1 <= c2 index evaluation order: prefix [0,c1), root [c1,c2),
 *     suffix [c2,G); Eq. (8) ties break to the lexicographically smallest
 *     (c1,c2).
 *
 * Bitstrings: ceil(n/64) uint64 words, qubit q is bit q (little-endian).
 */
#include <ctype.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXQ 128
#define ORC_OK 0
#define ORC_EPARSE 1
#define ORC_ERANGE 2
#define ORC_EINVAL 3
#define ORC_EINTERNAL 4

typedef struct { double re, im; } cplx;

enum { ROLE_PRESERVE = 0, ROLE_DET = 1, ROLE_BRANCH = 2 };
enum { KIND_DENSE = 0, KIND_MCX = 1, KIND_MCZ = 2 };

typedef struct {
    int kind;
    int k;                  /* number of qubits touched */
    int *q;                 /* q[j] = qubit of local bit j (MCX: q[0] is target) */
    unsigned char *neg;     /* MCX/MCZ polarity per local qubit */
    cplx m[64];             /* dense: U[out*dim + in], dim = 2^k, k <= 3 */
    int role;
    unsigned char preserve[3];  /* dense: local wire j is preserved */
    int *in_seg, *out_seg;  /* segment id per local qubit */
} ogate;

typedef struct {
    int n, G, A, nseg;
    int forward;            /* 1: forward placement, evaluation order = time order */
    int global;             /* 1: placement by reachability (sources anywhere the sweep
                               reaches them): propagation always spans the whole circuit */
    ogate *g;               /* time order */
    int out_seg[ORC_MAXQ];  /* segment carrying each qubit at the output */
    int *src_seg;           /* [A] segment fixed by source k */
    int *src_gate;          /* [A] time index of the gate of source k */
    int *src_eval;          /* [A] evaluation position of that gate */
} orc_circuit;

/* ------------------------------------------------------------------ */
/* parsing and gate matrices                                           */
/* ------------------------------------------------------------------ */

static cplx C(double re, double im) { cplx z = {re, im}; return z; }

static void set_dense(ogate *g, int k) {
    g->kind = KIND_DENSE;
    g->k = k;
    memset(g->m, 0, sizeof(g->m));
}

#define M_AT(g, out, in) ((g)->m[(out) * (1 << (g)->k) + (in)])

static int build_gate(ogate *g, const char *name, int *qs, unsigned char *ng,
                      int nq, double ang, int has_ang) {
    const double h = sqrt(0.5);
    int need_ang = 0, nq_expect = -1;
    g->q = (int *)malloc(sizeof(int) * (nq > 0 ? nq : 1));
    g->neg = (unsigned char *)calloc(nq > 0 ? nq : 1, 1);
    memcpy(g->q, qs, sizeof(int) * nq);
    memcpy(g->neg, ng, nq);
    for (int j = 0; j < nq; ++j)
        if (ng[j] && strcmp(name, "MCX") && strcmp(name, "MCZ")) return ORC_EPARSE;
    if (!strcmp(name, "MCX")) {
        if (nq < 1 || ng[0]) return ORC_EPARSE;
        g->kind = KIND_MCX; g->k = nq;
        return has_ang ? ORC_EPARSE : ORC_OK;
    }
    if (!strcmp(name, "MCZ")) {
        if (nq < 1) return ORC_EPARSE;
        g->kind = KIND_MCZ; g->k = nq;
        return has_ang ? ORC_EPARSE : ORC_OK;
    }
    if (!strcmp(name, "H") || !strcmp(name, "X") || !strcmp(name, "Y") ||
        !strcmp(name, "Z") || !strcmp(name, "S") || !strcmp(name, "SDG") ||
        !strcmp(name, "T") || !strcmp(name, "TDG")) nq_expect = 1;
    else if (!strcmp(name, "P") || !strcmp(name, "RX") || !strcmp(name, "RY") ||
             !strcmp(name, "RZ")) { nq_expect = 1; need_ang = 1; }
    else if (!strcmp(name, "CX") || !strcmp(name, "CZ") || !strcmp(name, "SWAP")) nq_expect = 2;
    else if (!strcmp(name, "CP") || !strcmp(name, "RZZ")) { nq_expect = 2; need_ang = 1; }
    else if (!strcmp(name, "CCX") || !strcmp(name, "CSWAP")) nq_expect = 3;
    else return ORC_EPARSE;
    if (nq != nq_expect || need_ang != has_ang) return ORC_EPARSE;
    set_dense(g, nq);
    if (!strcmp(name, "H")) {
        M_AT(g, 0, 0) = C(h, 0); M_AT(g, 0, 1) = C(h, 0);
        M_AT(g, 1, 0) = C(h, 0); M_AT(g, 1, 1) = C(-h, 0);
    } else if (!strcmp(name, "X")) {
        M_AT(g, 1, 0) = C(1, 0); M_AT(g, 0, 1) = C(1, 0);
    } else if (!strcmp(name, "Y")) {
        M_AT(g, 1, 0) = C(0, 1); M_AT(g, 0, 1) = C(0, -1);
    } else if (!strcmp(name, "Z")) {
        M_AT(g, 0, 0) = C(1, 0); M_AT(g, 1, 1) = C(-1, 0);
    } else if (!strcmp(name, "S")) {
        M_AT(g, 0, 0) = C(1, 0); M_AT(g, 1, 1) = C(0, 1);
    } else if (!strcmp(name, "SDG")) {
        M_AT(g, 0, 0) = C(1, 0); M_AT(g, 1, 1) = C(0, -1);
    } else if (!strcmp(name, "T")) {
        M_AT(g, 0, 0) = C(1, 0); M_AT(g, 1, 1) = C(h, h);
    } else if (!strcmp(name, "TDG")) {
        M_AT(g, 0, 0) = C(1, 0); M_AT(g, 1, 1) = C(h, -h);
    } else if (!strcmp(name, "P")) {
        M_AT(g, 0, 0) = C(1, 0); M_AT(g, 1, 1) = C(cos(ang), sin(ang));
    } else if (!strcmp(name, "RX")) {
        double c = cos(0.5 * ang), s = sin(0.5 * ang);
        M_AT(g, 0, 0) = C(c, 0); M_AT(g, 1, 1) = C(c, 0);
        M_AT(g, 0, 1) = C(0, -s); M_AT(g, 1, 0) = C(0, -s);
    } else if (!strcmp(name, "RY")) {
        double c = cos(0.5 * ang), s = sin(0.5 * ang);
        M_AT(g, 0, 0) = C(c, 0); M_AT(g, 1, 1) = C(c, 0);
        M_AT(g, 0, 1) = C(-s, 0); M_AT(g, 1, 0) = C(s, 0);
    } else if (!strcmp(name, "RZ")) {
        double c = cos(0.5 * ang), s = sin(0.5 * ang);
        M_AT(g, 0, 0) = C(c, -s); M_AT(g, 1, 1) = C(c, s);
    } else if (!strcmp(name, "CX")) {          /* local bit 0 control, bit 1 target */
        for (int x = 0; x < 4; ++x) {
            int y = (x & 1) ? (x ^ 2) : x;
            M_AT(g, y, x) = C(1, 0);
        }
    } else if (!strcmp(name, "CZ")) {
        for (int x = 0; x < 4; ++x) M_AT(g, x, x) = C(x == 3 ? -1 : 1, 0);
    } else if (!strcmp(name, "SWAP")) {
        for (int x = 0; x < 4; ++x) {
            int y = ((x & 1) << 1) | ((x >> 1) & 1);
            M_AT(g, y, x) = C(1, 0);
        }
    } else if (!strcmp(name, "CP")) {
        for (int x = 0; x < 3; ++x) M_AT(g, x, x) = C(1, 0);
        M_AT(g, 3, 3) = C(cos(ang), sin(ang));
    } else if (!strcmp(name, "RZZ")) {
        double c = cos(0.5 * ang), s = sin(0.5 * ang);
        for (int x = 0; x < 4; ++x) {
            int par = (x ^ (x >> 1)) & 1;
            M_AT(g, x, x) = par ? C(c, s) : C(c, -s);
        }
    } else if (!strcmp(name, "CCX")) {         /* bits 0,1 controls, bit 2 target */
        for (int x = 0; x < 8; ++x) {
            int y = ((x & 3) == 3) ? (x ^ 4) : x;
            M_AT(g, y, x) = C(1, 0);
        }
    } else if (!strcmp(name, "CSWAP")) {       /* bit 0 control, bits 1,2 swapped */
        for (int x = 0; x < 8; ++x) {
            int y = x;
            if (x & 1) y = (x & 1) | (((x >> 2) & 1) << 1) | (((x >> 1) & 1) << 2);
            M_AT(g, y, x) = C(1, 0);
        }
    }
    return ORC_OK;
}

static int is_zero(cplx z) { return z.re == 0.0 && z.im == 0.0; }

/* Role of a gate from its matrix (Section II-A) and, per local wire, whether
 * every nonzero transition leaves that wire's value unchanged. */
static void classify(ogate *g) {
    if (g->kind == KIND_MCX) { g->role = ROLE_DET; return; }
    if (g->kind == KIND_MCZ) { g->role = ROLE_PRESERVE; return; }
    int dim = 1 << g->k, offdiag = 0, multi = 0;
    for (int x = 0; x < dim; ++x) {
        int nz = 0;
        for (int y = 0; y < dim; ++y) {
            if (is_zero(M_AT(g, y, x))) continue;
            ++nz;
            if (y != x) offdiag = 1;
        }
        if (nz > 1) multi = 1;
    }
    g->role = !offdiag ? ROLE_PRESERVE : (multi ? ROLE_BRANCH : ROLE_DET);
    for (int j = 0; j < g->k; ++j) {
        int keep = 1;
        for (int x = 0; x < dim; ++x)
            for (int y = 0; y < dim; ++y)
                if (!is_zero(M_AT(g, y, x)) && (((x ^ y) >> j) & 1)) keep = 0;
        g->preserve[j] = (unsigned char)keep;
    }
}

static int local_preserved(const ogate *g, int j) {
    if (g->kind == KIND_MCX) return j != 0;
    if (g->kind == KIND_MCZ) return 1;
    return g->preserve[j];
}

void orc_free(orc_circuit *c) {
    if (!c) return;
    for (int i = 0; i < c->G; ++i) {
        free(c->g[i].q); free(c->g[i].neg);
        free(c->g[i].in_seg); free(c->g[i].out_seg);
    }
    free(c->g); free(c->src_seg); free(c->src_gate); free(c->src_eval);
    free(c);
}

/* ------------------------------------------------------------------ */
/* source placement by reachability (Section IV-B, Fig. 3)              */
/* ------------------------------------------------------------------ */

/* Determinism-propagation relations between internal-wire segments,
 * independent of the values: a pair (one segment fixes the other: a
 * one-qubit deterministic gate, the two swapped wires of a SWAP) or a triple
 * (a CNOT's control, target input and target output: any two fix the
 * third).  Returns -1 for a circuit outside the gate set this analysis
 * covers (branching gates on one qubit; deterministic gates on one qubit,
 * CNOT and SWAP). */
typedef struct { int n; int seg[3]; } relation;

static int is_swap_matrix(const ogate *g) {
    for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) {
            int sw = ((x & 1) << 1) | ((x >> 1) & 1);
            if (is_zero(M_AT(g, y, x)) != (y != sw)) return 0;
        }
    return 1;
}

static int build_relations(const orc_circuit *c, relation *rel, int *nrel) {
    int nr = 0;
    for (int t = 0; t < c->G; ++t) {
        const ogate *g = &c->g[t];
        if (g->role == ROLE_PRESERVE) continue;
        if (g->role == ROLE_BRANCH) {
            if (g->k != 1) return -1;
            continue;
        }
        if (g->k == 1) {
            rel[nr].n = 2; rel[nr].seg[0] = g->in_seg[0]; rel[nr].seg[1] = g->out_seg[0]; ++nr;
        } else if (g->k == 2 && g->kind == KIND_MCX) {          /* MCX with one control */
            rel[nr].n = 3;
            rel[nr].seg[0] = g->in_seg[1]; rel[nr].seg[1] = g->in_seg[0]; rel[nr].seg[2] = g->out_seg[0];
            ++nr;
        } else if (g->k == 2 && g->kind == KIND_DENSE && local_preserved(g, 0) != local_preserved(g, 1)) {
            int jc = local_preserved(g, 0) ? 0 : 1, jt = 1 - jc, flips = 0;
            /* a CNOT: the target flips for exactly one value of the kept
             * wire (a flip for both would leave the kept wire unfixed by
             * the other two) */
            for (int v = 0; v < 2; ++v) {
                const int x = v << jc;
                if (!is_zero(M_AT(g, x | (1 << jt), x))) ++flips;
            }
            if (flips != 1) return -1;
            rel[nr].n = 3;
            rel[nr].seg[0] = g->in_seg[jc]; rel[nr].seg[1] = g->in_seg[jt]; rel[nr].seg[2] = g->out_seg[jt];
            ++nr;
        } else if (g->k == 2 && g->kind == KIND_DENSE && is_swap_matrix(g)) {
            rel[nr].n = 2; rel[nr].seg[0] = g->in_seg[0]; rel[nr].seg[1] = g->out_seg[1]; ++nr;
            rel[nr].n = 2; rel[nr].seg[0] = g->in_seg[1]; rel[nr].seg[1] = g->out_seg[0]; ++nr;
        } else {
            return -1;
        }
    }
    *nrel = nr;
    return 0;
}

/* Mark everything the relations reach from the segments already marked;
 * returns how many are marked. */
static int reach(const orc_circuit *c, const relation *rel, int nrel, unsigned char *known) {
    for (;;) {
        int changed = 0;
        for (int r = 0; r < nrel; ++r) {
            const relation *x = &rel[r];
            int nk = 0, miss = -1;
            for (int i = 0; i < x->n; ++i) {
                if (known[x->seg[i]]) ++nk;
                else miss = x->seg[i];
            }
            if (nk == x->n - 1 && miss >= 0) { known[miss] = 1; changed = 1; }
        }
        if (!changed) break;
    }
    int total = 0;
    for (int i = 0; i < c->nseg; ++i) total += known[i];
    return total;
}

/* The natural sources (input and output boundary segments) plus the chosen
 * candidates, closed under the relations. */
static int reach_from(const orc_circuit *c, const relation *rel, int nrel, const int *cand,
                      const int *pick, int npick, unsigned char *known) {
    memset(known, 0, (size_t)c->nseg);
    for (int q = 0; q < c->n; ++q) { known[q] = 1; known[c->out_seg[q]] = 1; }
    for (int i = 0; i < npick; ++i) known[cand[pick[i]]] = 1;
    return reach(c, rel, nrel, known);
}

/* Sources on the input segments of branching gates (the values the sweep
 * from the output needs), as few as reach every segment: `greedy` adds, one
 * at a time, the candidate that reaches the most segments (the smallest
 * evaluation position on ties); otherwise the smallest set by exhaustive
 * search in increasing size (candidates in evaluation order, the first set
 * found kept).  Sources are numbered in evaluation order of their gates. */
static int place_by_reach(orc_circuit *c, int greedy) {
    relation *rel = (relation *)malloc(sizeof(relation) * (size_t)(2 * c->G + 1));
    int nrel = 0;
    if (build_relations(c, rel, &nrel)) { free(rel); return ORC_EINVAL; }
    int *cand = (int *)malloc(sizeof(int) * (size_t)(c->G + 1));
    int *cgate = (int *)malloc(sizeof(int) * (size_t)(c->G + 1));
    int nc = 0;
    for (int e = 0; e < c->G; ++e) {                 /* evaluation order: from the output */
        int t = c->G - 1 - e;
        const ogate *g = &c->g[t];
        if (g->role != ROLE_BRANCH || g->in_seg[0] < c->n) continue;
        cand[nc] = g->in_seg[0]; cgate[nc] = t; ++nc;
    }
    unsigned char *known = (unsigned char *)malloc((size_t)c->nseg);
    int *pick = (int *)malloc(sizeof(int) * (size_t)(nc + 1));
    int npick = 0, rc = ORC_OK;
    if (greedy) {
        unsigned char *used = (unsigned char *)calloc((size_t)nc + 1, 1);
        while (reach_from(c, rel, nrel, cand, pick, npick, known) < c->nseg) {
            int best = -1, best_n = -1;
            for (int i = 0; i < nc; ++i) {
                if (used[i]) continue;
                pick[npick] = i;
                int m = reach_from(c, rel, nrel, cand, pick, npick + 1, known);
                if (m > best_n) { best_n = m; best = i; }
            }
            used[best] = 1;
            pick[npick++] = best;
        }
        free(used);
        /* evaluation order */
        for (int i = 1; i < npick; ++i)
            for (int j = i; j > 0 && pick[j - 1] > pick[j]; --j) { int tmp = pick[j]; pick[j] = pick[j - 1]; pick[j - 1] = tmp; }
    } else {
        long budget = 20000000;
        int found = 0;
        for (int k = 0; k <= nc && !found; ++k) {
            for (int i = 0; i < k; ++i) pick[i] = i;
            for (;;) {
                if (--budget < 0) { rc = ORC_ERANGE; break; }
                if (reach_from(c, rel, nrel, cand, pick, k, known) == c->nseg) { found = 1; npick = k; break; }
                int i = k - 1;                       /* next combination, lexicographic */
                while (i >= 0 && pick[i] == nc - k + i) --i;
                if (i < 0) break;
                ++pick[i];
                for (int j = i + 1; j < k; ++j) pick[j] = pick[j - 1] + 1;
            }
            if (rc) break;
        }
        if (!found && !rc) rc = ORC_EINTERNAL;
    }
    if (rc == ORC_OK) {
        c->A = npick;
        for (int i = 0; i < npick; ++i) {
            c->src_seg[i] = cand[pick[i]];
            c->src_gate[i] = cgate[pick[i]];
            c->src_eval[i] = c->G - 1 - cgate[pick[i]];
        }
    }
    free(rel); free(cand); free(cgate); free(known); free(pick);
    return rc;
}

int orc_load_ex(const char *text, int forward, orc_circuit **out) {
    *out = NULL;
    /* placement: 0 backward sweep, 1 forward sweep, 2 fewest sources by
     * reachability (exhaustive), 3 greedy by reachability */
    const int mode = forward;
    if (mode < 0 || mode > 3) return ORC_EINVAL;
    forward = mode == 1;
    orc_circuit *c = (orc_circuit *)calloc(1, sizeof(orc_circuit));
    int cap = 64, rc = ORC_OK;
    c->g = (ogate *)calloc(cap, sizeof(ogate));
    c->n = -1;
    const char *p = text;
    char line[8192];
    while (*p) {
        size_t len = strcspn(p, "\n");
        if (len >= sizeof(line)) { rc = ORC_EPARSE; break; }
        memcpy(line, p, len); line[len] = 0;
        p += len; if (*p == '\n') ++p;
        char *hash = strchr(line, '#'); if (hash) *hash = 0;
        char *tok[260]; int nt = 0;
        for (char *s = strtok(line, " \t\r"); s && nt < 260; s = strtok(NULL, " \t\r")) tok[nt++] = s;
        if (nt == 0) continue;
        if (!strcmp(tok[0], "qubits")) {
            if (nt != 2 || c->n >= 0) { rc = ORC_EPARSE; break; }
            c->n = atoi(tok[1]);
            if (c->n < 1 || c->n > ORC_MAXQ) { rc = ORC_ERANGE; break; }
            continue;
        }
        if (c->n < 0) { rc = ORC_EPARSE; break; }
        int qs[260]; unsigned char ng[260]; int nq = 0, has_ang = 0; double ang = 0;
        for (int i = 1; i < nt; ++i) {
            const char *s = tok[i];
            int neg = 0;
            if (s[0] == '~') { neg = 1; ++s; }
            if (s[0] && strspn(s, "0123456789") == strlen(s)) {
                int q = atoi(s);
                if (q < 0 || q >= c->n) { rc = ORC_ERANGE; break; }
                for (int j = 0; j < nq; ++j) if (qs[j] == q) rc = ORC_EPARSE;
                qs[nq] = q; ng[nq] = (unsigned char)neg; ++nq;
            } else {
                char *end;
                if (neg || i != nt - 1) { rc = ORC_EPARSE; break; }
                ang = strtod(s, &end);
                if (*end || !isfinite(ang)) { rc = ORC_EPARSE; break; }
                has_ang = 1;
            }
        }
        if (rc) break;
        if (c->G == cap) { cap *= 2; c->g = (ogate *)realloc(c->g, sizeof(ogate) * cap); memset(c->g + c->G, 0, sizeof(ogate) * (cap - c->G)); }
        ogate *g = &c->g[c->G++];
        memset(g, 0, sizeof(*g));
        rc = build_gate(g, tok[0], qs, ng, nq, ang, has_ang);
        if (rc) break;
        classify(g);
    }
    if (!rc && c->n < 0) rc = ORC_EPARSE;
    if (rc) { orc_free(c); return rc; }

    /* internal-wire segments (Section II-A) */
    int cur[ORC_MAXQ];
    for (int q = 0; q < c->n; ++q) cur[q] = q;   /* segment q = input segment of qubit q */
    int next = c->n;
    for (int t = 0; t < c->G; ++t) {
        ogate *g = &c->g[t];
        g->in_seg = (int *)malloc(sizeof(int) * g->k);
        g->out_seg = (int *)malloc(sizeof(int) * g->k);
        for (int j = 0; j < g->k; ++j) {
            int q = g->q[j];
            g->in_seg[j] = cur[q];
            g->out_seg[j] = local_preserved(g, j) ? cur[q] : next++;
            cur[q] = g->out_seg[j];
        }
    }
    for (int q = 0; q < c->n; ++q) c->out_seg[q] = cur[q];
    c->nseg = next;

    /* source placement: one sweep; a branching gate whose segment on the
     * side the sweep reaches last (input side for the backward sweep,
     * output side for the forward one) is not a boundary segment gets a
     * source there */
    c->forward = forward;
    c->src_seg = (int *)malloc(sizeof(int) * (c->G + 1));
    c->src_gate = (int *)malloc(sizeof(int) * (c->G + 1));
    c->src_eval = (int *)malloc(sizeof(int) * (c->G + 1));
    c->A = 0;
    for (int e = 0; e < c->G; ++e) {
        int t = forward ? e : c->G - 1 - e;
        ogate *g = &c->g[t];
        if (g->role != ROLE_BRANCH) continue;
        for (int j = 0; j < g->k; ++j) {
            if (local_preserved(g, j)) continue;
            int seg = forward ? g->out_seg[j] : g->in_seg[j];
            int natural = forward ? seg == c->out_seg[g->q[j]] : seg < c->n;
            if (natural) continue;
            if (c->A >= c->G) { orc_free(c); return ORC_EINTERNAL; }
            c->src_seg[c->A] = seg;
            c->src_gate[c->A] = t;
            c->src_eval[c->A] = e;
            c->A++;
        }
    }
    if (mode >= 2) {
        c->global = 1;
        int prc = place_by_reach(c, mode == 3);
        if (prc) { orc_free(c); return prc; }
    }
    *out = c;
    return ORC_OK;
}

int orc_load(const char *text, orc_circuit **out) { return orc_load_ex(text, 0, out); }

int orc_info(const orc_circuit *c, int *n, int *G, int *A, int *nseg) {
    *n = c->n; *G = c->G; *A = c->A; *nseg = c->nseg;
    return ORC_OK;
}

int orc_sources(const orc_circuit *c, int *eval_pos) {
    for (int k = 0; k < c->A; ++k) eval_pos[k] = c->src_eval[k];
    return ORC_OK;
}

int orc_gate_role(const orc_circuit *c, int t) { return c->g[t].role; }

/* ------------------------------------------------------------------ */
/* wire-value propagation                                              */
/* ------------------------------------------------------------------ */

static int getbit(const uint64_t *w, int q) { return (int)((w[q >> 6] >> (q & 63)) & 1u); }

/* set a segment; 0 = ok, -1 = conflict; *changed set when newly known */
static int setv(signed char *val, int seg, int v, int *changed) {
    if (val[seg] < 0) { val[seg] = (signed char)v; if (changed) *changed = 1; return 0; }
    return val[seg] == v ? 0 : -1;
}

/* Local consistency of one deterministic gate: keep the (in,out) pairs of
 * its permutation that agree with the known values, fix every wire on which
 * all surviving pairs agree.  Returns -1 if no pair survives. */
static int rule_dense(const ogate *g, signed char *val, int *changed) {
    int dim = 1 << g->k, nsurv = 0;
    int and_in = dim - 1, or_in = 0, and_out = dim - 1, or_out = 0;
    for (int x = 0; x < dim; ++x) {
        int ok = 1;
        for (int j = 0; j < g->k && ok; ++j) {
            int v = val[g->in_seg[j]];
            if (v >= 0 && v != ((x >> j) & 1)) ok = 0;
        }
        if (!ok) continue;
        int y = -1;
        for (int yy = 0; yy < dim; ++yy) if (!is_zero(M_AT(g, yy, x))) { y = yy; break; }
        for (int j = 0; j < g->k && ok; ++j) {
            int v = val[g->out_seg[j]];
            if (v >= 0 && v != ((y >> j) & 1)) ok = 0;
        }
        if (!ok) continue;
        ++nsurv;
        and_in &= x; or_in |= x; and_out &= y; or_out |= y;
    }
    if (nsurv == 0) return -1;
    for (int j = 0; j < g->k; ++j) {
        if (((and_in ^ or_in) >> j & 1) == 0 && val[g->in_seg[j]] < 0)
            if (setv(val, g->in_seg[j], (and_in >> j) & 1, changed)) return -1;
        if (((and_out ^ or_out) >> j & 1) == 0 && val[g->out_seg[j]] < 0)
            if (setv(val, g->out_seg[j], (and_out >> j) & 1, changed)) return -1;
    }
    return 0;
}

/* Multi-controlled X: target_out = target_in XOR [every control matches]. */
static int rule_mcx(const ogate *g, signed char *val, int *changed) {
    int tin = g->in_seg[0], tout = g->out_seg[0];
    int mismatch = 0, unknown = 0, last_unknown = -1;
    for (int j = 1; j < g->k; ++j) {
        int v = val[g->in_seg[j]];
        int want = g->neg[j] ? 0 : 1;
        if (v < 0) { ++unknown; last_unknown = j; }
        else if (v != want) mismatch = 1;
    }
    int vi = val[tin], vo = val[tout];
    if (mismatch || unknown == 0) {
        int flip = mismatch ? 0 : 1;
        if (vi >= 0 && setv(val, tout, vi ^ flip, changed)) return -1;
        if (vo >= 0 && setv(val, tin, vo ^ flip, changed)) return -1;
        return 0;
    }
    if (vi < 0 || vo < 0) return 0;
    if (vi != vo) {            /* every control must match */
        for (int j = 1; j < g->k; ++j)
            if (setv(val, g->in_seg[j], g->neg[j] ? 0 : 1, changed)) return -1;
    } else if (unknown == 1) { /* the one unknown control must mismatch */
        if (setv(val, g->in_seg[last_unknown], g->neg[last_unknown] ? 1 : 0, changed)) return -1;
    }
    return 0;
}

/* PropagateKnownValues over time indices [t0, t1): sweep backward then
 * forward until no value changes.  Returns -1 on a conflict. */
static int propagate(const orc_circuit *c, signed char *val, int t0, int t1) {
    for (;;) {
        int changed = 0;
        for (int pass = 0; pass < 2; ++pass) {
            for (int i = 0; i < t1 - t0; ++i) {
                int t = pass == 0 ? t1 - 1 - i : t0 + i;
                const ogate *g = &c->g[t];
                if (g->role != ROLE_DET) continue;
                int r = g->kind == KIND_MCX ? rule_mcx(g, val, &changed)
                                            : rule_dense(g, val, &changed);
                if (r) return -1;
            }
        }
        if (!changed) return 0;
    }
}

static int set_boundary(const orc_circuit *c, signed char *val,
                        const uint64_t *bin, const uint64_t *bout) {
    memset(val, -1, (size_t)c->nseg);
    for (int q = 0; q < c->n; ++q) {
        if (setv(val, q, getbit(bin, q), NULL)) return -1;
        if (setv(val, c->out_seg[q], getbit(bout, q), NULL)) return -1;
    }
    return 0;
}

/* SetArtificialSources for sources [k0, k0+na) from the bits of hbits. */
static int set_sources(const orc_circuit *c, signed char *val, int k0, int na, uint64_t hbits) {
    for (int i = 0; i < na; ++i)
        if (setv(val, c->src_seg[k0 + i], (int)((hbits >> i) & 1u), NULL)) return -1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* history evaluation                                                  */
/* ------------------------------------------------------------------ */

typedef struct { cplx amp; double M; } partial;

static cplx cmul(cplx a, cplx b) {
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

static double modulus1(cplx z) {
    double m = sqrt(z.re * z.re + z.im * z.im);
    return m > 1.0 ? 1.0 : m;
}

/* Time index of evaluation position e (backward sweep: from the output). */
static int time_of(const orc_circuit *c, int e) { return c->forward ? e : c->G - 1 - e; }

/* The time indices [t0, t1) that evaluation positions [e0, e1) cover. */
static void time_span(const orc_circuit *c, int e0, int e1, int *t0, int *t1) {
    if (c->forward) { *t0 = e0; *t1 = e1; }
    else { *t0 = c->G - e1; *t1 = c->G - e0; }
}

/* Multiply the gate factors of evaluation positions [e0, e1), in evaluation
 * order, into the partial history (Eq. (4)); every wire must be resolved.
 * Returns 0 ok, 1 zero factor, 2 pruned. */
static int evaluate(const orc_circuit *c, const signed char *val, int e0, int e1,
                    double thr, partial *pa, uint64_t *gate_evals) {
    for (int e = e0; e < e1; ++e) {
        const int t = time_of(c, e);
        const ogate *g = &c->g[t];
        cplx f;
        for (int j = 0; j < g->k; ++j) {
            if (val[g->in_seg[j]] < 0 || val[g->out_seg[j]] < 0) {
                fprintf(stderr, "oracle: unresolved wire at gate %d\n", t);
                abort();
            }
        }
        ++*gate_evals;
        if (g->kind == KIND_MCX) {
            int match = 1;
            for (int j = 1; j < g->k; ++j)
                if (val[g->in_seg[j]] != (g->neg[j] ? 0 : 1)) match = 0;
            int ti = val[g->in_seg[0]], to = val[g->out_seg[0]];
            f = (to == (ti ^ match)) ? C(1, 0) : C(0, 0);
        } else if (g->kind == KIND_MCZ) {
            int match = 1;
            for (int j = 0; j < g->k; ++j)
                if (val[g->in_seg[j]] != (g->neg[j] ? 0 : 1)) match = 0;
            f = match ? C(-1, 0) : C(1, 0);
        } else {
            int x = 0, y = 0;
            for (int j = 0; j < g->k; ++j) {
                x |= val[g->in_seg[j]] << j;
                y |= val[g->out_seg[j]] << j;
            }
            f = M_AT(g, y, x);
        }
        if (is_zero(f)) return 1;
        pa->amp = cmul(pa->amp, f);
        if (g->role == ROLE_BRANCH) {
            pa->M = pa->M * modulus1(f);
            if (pa->M < thr) return 2;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Neumaier-compensated accumulation and statistics                    */
/* ------------------------------------------------------------------ */

typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/* SplitMix64 finaliser (Steele, Lea, Flood 2014), used to hash valid sets. */
static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

typedef struct {
    nsum re, im;
    uint64_t n_valid, sum_h, xor_h, gate_evals;
} acc_t;

static void acc_history(acc_t *a, cplx amp, uint64_t h) {
    nadd(&a->re, amp.re); nadd(&a->im, amp.im);
    a->n_valid += 1; a->sum_h += h; a->xor_h ^= mix64(h);
}

/* ------------------------------------------------------------------ */
/* the reduced sum over artificial sources, region by region            */
/* ------------------------------------------------------------------ */

/* Evaluation-order regions [cut[r], cut[r+1]) and the sources whose gates
 * they contain: na[r] consecutive source numbers from k0[r] (sources are
 * numbered in evaluation order). */
typedef struct { int nr; int cut[4]; int k0[3]; int na[3]; } regions_t;

static void make_regions(const orc_circuit *c, const int *cuts, int nr, regions_t *R) {
    R->nr = nr;
    for (int r = 0; r <= nr; ++r) R->cut[r] = cuts[r];
    int k = 0;
    for (int r = 0; r < nr; ++r) {
        R->k0[r] = k;
        R->na[r] = 0;
        while (k < c->A && c->src_eval[k] < cuts[r + 1]) { ++R->na[r]; ++k; }
    }
}

/* Add to `acc` every valid history that extends a partial one: `val` holds
 * the wire values fixed by the boundary and by the sources of regions
 * before r (with everything they imply), `pa` the product of those regions'
 * factors and `h` their source bits.  Each assignment of region r's sources
 * (only those in [lo, hi) for the first region) is fixed and propagated
 * inside the region, the region's factors are multiplied in, and the later
 * regions are walked the same way; a conflict, a zero factor or a pruned
 * product drops the subtree.  bufs[r] is region r's scratch copy. */
static void walk_regions(const orc_circuit *c, const regions_t *R, int r, const signed char *val,
                         partial pa, uint64_t h, uint64_t lo, uint64_t hi, double thr, acc_t *acc,
                         signed char **bufs) {
    if (r == R->nr) {
        acc_history(acc, pa.amp, h);
        return;
    }
    const uint64_t n = 1ULL << R->na[r];
    const uint64_t x0 = r == 0 ? lo : 0, x1 = (r == 0 && hi < n) ? hi : n;
    int t0, t1;
    time_span(c, R->cut[r], R->cut[r + 1], &t0, &t1);
    if (c->global) { t0 = 0; t1 = c->G; }
    signed char *v = bufs[r];
    for (uint64_t x = x0; x < x1; ++x) {
        memcpy(v, val, (size_t)c->nseg);
        if (set_sources(c, v, R->k0[r], R->na[r], x)) continue;
        if (propagate(c, v, t0, t1)) continue;
        partial p2 = pa;
        if (evaluate(c, v, R->cut[r], R->cut[r + 1], thr, &p2, &acc->gate_evals)) continue;
        walk_regions(c, R, r + 1, v, p2, h | (x << R->k0[r]), lo, hi, thr, acc, bufs);
    }
}

/* The transition amplitude of one (b_in, b_out) pair as the reduced sum of
 * Eq. (7), walked over the given evaluation-order cuts (nr regions; first
 * region's assignments restricted to [lo, hi)).  The boundary values and
 * what they imply are fixed once; a pair they already contradict has no
 * valid history. */
static void reduced_sum(const orc_circuit *c, const uint64_t *bin, const uint64_t *bout, double thr,
                        const int *cuts, int nr, uint64_t lo, uint64_t hi, acc_t *acc) {
    regions_t R;
    make_regions(c, cuts, nr, &R);
    size_t ns = (size_t)c->nseg;
    signed char *v0 = (signed char *)malloc(ns);
    signed char *bufs[3];
    for (int r = 0; r < 3; ++r) bufs[r] = (signed char *)malloc(ns);
    if (set_boundary(c, v0, bin, bout) == 0 && propagate(c, v0, 0, c->G) == 0) {
        partial one = {{1.0, 0.0}, 1.0};
        walk_regions(c, &R, 0, v0, one, 0, lo, hi, thr, acc, bufs);
    }
    free(v0);
    for (int r = 0; r < 3; ++r) free(bufs[r]);
}

/* One transition amplitude.  c1 < 0 selects Algorithm 1.
 * stats[4] = n_valid, sum_h (mod 2^64), xor of mix64(h), gate evaluations. */
int orc_pair(const orc_circuit *c, const uint64_t *bin, const uint64_t *bout,
             double thr, int c1, int c2, double *amp, uint64_t *stats) {
    if (!(thr >= 0.0) || !isfinite(thr)) return ORC_EINVAL;
    if (c->A > 62) return ORC_ERANGE;
    if (c1 >= 0 && (c1 > c2 || c2 > c->G)) return ORC_EINVAL;
    if (c1 >= 0 && c->global) return ORC_EINVAL;     /* reachability placements: Algorithm 1 only */
    acc_t a;
    memset(&a, 0, sizeof(a));
    if (c1 < 0) {
        const int cuts[2] = {0, c->G};               /* Algorithm 1: one region */
        reduced_sum(c, bin, bout, thr, cuts, 1, 0, ~0ULL, &a);
    } else {
        const int cuts[4] = {0, c1, c2, c->G};       /* Algorithm 2: prefix, root, suffix */
        reduced_sum(c, bin, bout, thr, cuts, 3, 0, ~0ULL, &a);
    }
    amp[0] = a.re.s + a.re.c;
    amp[1] = a.im.s + a.im.c;
    stats[0] = a.n_valid; stats[1] = a.sum_h; stats[2] = a.xor_h; stats[3] = a.gate_evals;
    return ORC_OK;
}

/* Eq. (2) for a batch: amps[j] = sum_i coeff_i * alpha(in_i, out_j), inputs
 * summed in order; stats[j] = (n_valid, sum_h, xor_h, gate_evals) over the
 * pairs of output j.  OpenMP over outputs with nthreads threads. */
int orc_evaluate(const orc_circuit *c, const uint64_t *inputs, const double *coeffs, int S,
                 const uint64_t *outputs, int M, double thr, int c1, int c2,
                 double *amps, uint64_t *stats, int nthreads) {
    if (!(thr >= 0.0) || !isfinite(thr) || S < 0 || M < 0) return ORC_EINVAL;
    if (c->A > 62) return ORC_ERANGE;
    if (c1 >= 0 && (c1 > c2 || c2 > c->G)) return ORC_EINVAL;
    int W = (c->n + 63) / 64;
    int rc = ORC_OK;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int j = 0; j < M; ++j) {
        double re = 0.0, im = 0.0;
        uint64_t st[4] = {0, 0, 0, 0};
        for (int i = 0; i < S; ++i) {
            double a[2];
            uint64_t s[4];
            if (orc_pair(c, inputs + (size_t)i * W, outputs + (size_t)j * W, thr, c1, c2, a, s)) {
                rc = ORC_EINTERNAL;
                continue;
            }
            double cr = coeffs[2 * i], ci = coeffs[2 * i + 1];
            re += cr * a[0] - ci * a[1];
            im += cr * a[1] + ci * a[0];
            st[0] += s[0]; st[1] += s[1]; st[2] ^= s[2]; st[3] += s[3];
        }
        amps[2 * j] = re; amps[2 * j + 1] = im;
        for (int k = 0; k < 4; ++k) stats[4 * (size_t)j + k] = st[k];
    }
    return rc;
}

/* A bounded sample of Algorithm 2 for timing: prefix assignments
 * h_p in [hp_lo, hp_hi) only, for each of the M outputs (one input b_in),
 * OpenMP over outputs.  amps/stats as orc_evaluate (partial sums). */
int orc_sample(const orc_circuit *c, const uint64_t *bin, const uint64_t *outputs, int M,
               double thr, int c1, int c2, uint64_t hp_lo, uint64_t hp_hi,
               double *amps, uint64_t *stats, int nthreads) {
    if (!(thr >= 0.0) || !isfinite(thr) || M < 0) return ORC_EINVAL;
    if (c->A > 62) return ORC_ERANGE;
    if (c1 < 0 || c1 > c2 || c2 > c->G) return ORC_EINVAL;
    int W = (c->n + 63) / 64;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
    for (int j = 0; j < M; ++j) {
        acc_t a;
        memset(&a, 0, sizeof(a));
        const int cuts[4] = {0, c1, c2, c->G};
        reduced_sum(c, bin, outputs + (size_t)j * W, thr, cuts, 3, hp_lo, hp_hi, &a);
        amps[2 * j] = a.re.s + a.re.c;
        amps[2 * j + 1] = a.im.s + a.im.c;
        stats[4 * (size_t)j] = a.n_valid;
        stats[4 * (size_t)j + 1] = a.sum_h;
        stats[4 * (size_t)j + 2] = a.xor_h;
        stats[4 * (size_t)j + 3] = a.gate_evals;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Eq. (8) and its argmin                                              */
/* ------------------------------------------------------------------ */

typedef unsigned __int128 u128;

static void region_counts(const orc_circuit *c, int c1, int c2, int *A3) {
    A3[0] = A3[1] = A3[2] = 0;
    for (int k = 0; k < c->A; ++k) {
        int e = c->src_eval[k];
        A3[e < c1 ? 0 : (e < c2 ? 1 : 2)]++;
    }
}

static u128 eq8(int Ap, int Ar, int As, int Gp, int Gr, int Gs) {
    u128 inner = (u128)Gr + ((u128)1 << As) * (u128)Gs;
    return ((u128)1 << Ap) * ((u128)Gp + ((u128)1 << Ar) * inner);
}

int orc_eq8(const orc_circuit *c, int c1, int c2, uint64_t *cost2) {
    if (c1 < 0 || c1 > c2 || c2 > c->G) return ORC_EINVAL;
    if (c->A > 100) return ORC_ERANGE;
    int A3[3];
    region_counts(c, c1, c2, A3);
    u128 v = eq8(A3[0], A3[1], A3[2], c1, c2 - c1, c->G - c2);
    cost2[0] = (uint64_t)v; cost2[1] = (uint64_t)(v >> 64);
    return ORC_OK;
}

/* Exhaustive argmin of Eq. (8) over 0 <= c1 <= c2 <= G, smallest (c1,c2) on ties. */
int orc_eq8_argmin(const orc_circuit *c, int *c1o, int *c2o, uint64_t *cost2) {
    if (c->A > 100) return ORC_ERANGE;
    int G = c->G;
    int *before = (int *)calloc((size_t)G + 1, sizeof(int)); /* sources with eval pos < e */
    for (int k = 0; k < c->A; ++k) before[c->src_eval[k] + 1]++;
    for (int e = 1; e <= G; ++e) before[e] += before[e - 1];
    u128 best = 0; int b1 = 0, b2 = 0, have = 0;
    for (int c1 = 0; c1 <= G; ++c1)
        for (int c2 = c1; c2 <= G; ++c2) {
            int Ap = before[c1], Ar = before[c2] - before[c1], As = c->A - before[c2];
            u128 v = eq8(Ap, Ar, As, c1, c2 - c1, G - c2);
            if (!have || v < best) { best = v; b1 = c1; b2 = c2; have = 1; }
        }
    free(before);
    *c1o = b1; *c2o = b2;
    cost2[0] = (uint64_t)best; cost2[1] = (uint64_t)(best >> 64);
    return ORC_OK;
}
