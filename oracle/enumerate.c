/* Oracle diagram enumerator in plain C (test infrastructure): the brute force of
 * oracle/diagrams.py (enumerate_topologies with is_sigma_diagram and canonical), for orders up
 * to 6, where the Python loop over (2n)! = 479 001 600 permutations is too slow.
 *
 * Same definitions, written out again (a reading of Sec. II.A, eq. sigma_integration, and of
 * the q != 0 restriction of eq. ueg_action):
 *   - a labelled contraction is a permutation sigma of the 2n vertices; the propagator leaving v
 *     enters sigma[v]; interaction line i joins 2i and 2i+1; the out-vertex o has sigma[o] = 0
 *     and o -> 0 is the amputated external pair, not an internal edge;
 *   - a self-energy diagram's internal graph (the 2n - 1 propagators other than o -> 0 and the
 *     n interaction lines) is connected and has no bridge: removing any one edge keeps it
 *     connected (an interaction bridge is a q = 0 tadpole, a propagator bridge makes the
 *     diagram one-particle reducible); checked by brute force, one search per removed edge;
 *   - canonical form: breadth-first relabelling from the in-vertex (0 -> 0, its partner -> 1;
 *     labelled vertices visited in label order; the target of the visited vertex's propagator,
 *     if new, gets the next even label 2m and its partner 2m + 1).
 * Output: a header line "# order n: T topologies, L labelled permutations", then the T
 * distinct canonical permutations in lexicographic order, one per line.
 *
 * Usage: enumerate_topologies n   (n in 1..6; OpenMP threads over the value of sigma[0]). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXV 12

static int n2;

/* connectivity of the internal graph with edge `skip` removed (-1: none), bitmask search */
static int connected_without(const int* ea, const int* eb, int ne, int skip) {
    uint32_t adj[MAXV];
    for (int v = 0; v < n2; ++v) adj[v] = 0;
    for (int e = 0; e < ne; ++e) {
        if (e == skip) continue;
        adj[ea[e]] |= 1u << eb[e];
        adj[eb[e]] |= 1u << ea[e];
    }
    uint32_t seen = 1u, frontier = 1u;
    while (frontier) {
        uint32_t next = 0;
        for (int v = 0; v < n2; ++v)
            if (frontier & (1u << v)) next |= adj[v];
        frontier = next & ~seen;
        seen |= next;
    }
    return seen == (1u << n2) - 1u;
}

static int is_sigma_diagram(const int* sigma) {
    int ea[3 * MAXV], eb[3 * MAXV], ne = 0;
    for (int v = 0; v < n2; ++v) {
        if (sigma[v] == 0) continue; /* the external o -> 0 */
        ea[ne] = v;
        eb[ne] = sigma[v];
        ++ne;
    }
    for (int i = 0; i < n2 / 2; ++i) {
        ea[ne] = 2 * i;
        eb[ne] = 2 * i + 1;
        ++ne;
    }
    if (!connected_without(ea, eb, ne, -1)) return 0;
    for (int e = 0; e < ne; ++e)
        if (!connected_without(ea, eb, ne, e)) return 0;
    return 1;
}

static uint64_t canonical_key(const int* sigma) {
    int lab[MAXV], order[MAXV], no = 0, nxt = 1;
    for (int v = 0; v < n2; ++v) lab[v] = -1;
    lab[0] = 0;
    lab[1] = 1;
    order[no++] = 0;
    order[no++] = 1;
    for (int j = 0; j < no; ++j) {
        int w = sigma[order[j]];
        if (lab[w] < 0) {
            lab[w] = 2 * nxt;
            lab[w ^ 1] = 2 * nxt + 1;
            order[no++] = w;
            order[no++] = w ^ 1;
            ++nxt;
        }
    }
    int out[MAXV];
    for (int v = 0; v < n2; ++v) out[lab[v]] = lab[sigma[v]];
    uint64_t key = 0;
    for (int v = 0; v < n2; ++v) key = (key << 4) | (uint64_t)out[v];
    return key;
}

static int next_permutation(int* a, int m) {
    int i = m - 2;
    while (i >= 0 && a[i] >= a[i + 1]) --i;
    if (i < 0) return 0;
    int j = m - 1;
    while (a[j] <= a[i]) --j;
    int t = a[i];
    a[i] = a[j];
    a[j] = t;
    for (int l = i + 1, r = m - 1; l < r; ++l, --r) {
        t = a[l];
        a[l] = a[r];
        a[r] = t;
    }
    return 1;
}

static int cmp_u64(const void* x, const void* y) {
    uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
    return a < b ? -1 : a > b;
}

/* append keys to a growable array */
typedef struct {
    uint64_t* k;
    size_t n, cap;
} keys_t;

static void push(keys_t* s, uint64_t v) {
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 1024;
        s->k = (uint64_t*)realloc(s->k, s->cap * sizeof(uint64_t));
        if (!s->k) {
            fprintf(stderr, "out of memory\n");
            exit(2);
        }
    }
    s->k[s->n++] = v;
}

/* sort and drop duplicates */
static void unique(keys_t* s) {
    if (!s->n) return;
    qsort(s->k, s->n, sizeof(uint64_t), cmp_u64);
    size_t w = 1;
    for (size_t i = 1; i < s->n; ++i)
        if (s->k[i] != s->k[w - 1]) s->k[w++] = s->k[i];
    s->n = w;
}

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s n\n", argv[0]);
        return 1;
    }
    int n = atoi(argv[1]);
    if (n < 1 || n > 6) {
        fprintf(stderr, "n must be in 1..6\n");
        return 1;
    }
    n2 = 2 * n;
    keys_t all = {0, 0, 0};
    long long labelled = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : labelled)
    for (int first = 0; first < n2; ++first) {
        keys_t mine = {0, 0, 0};
        int sigma[MAXV], rest[MAXV], m = 0;
        for (int v = 0; v < n2; ++v)
            if (v != first) rest[m++] = v;
        sigma[0] = first;
        do {
            for (int i = 0; i < m; ++i) sigma[i + 1] = rest[i];
            if (is_sigma_diagram(sigma)) {
                ++labelled;
                push(&mine, canonical_key(sigma));
                if (mine.n > (1u << 20)) unique(&mine);
            }
        } while (next_permutation(rest, m));
        unique(&mine);
#pragma omp critical
        {
            for (size_t i = 0; i < mine.n; ++i) push(&all, mine.k[i]);
        }
        free(mine.k);
    }
    unique(&all);
    printf("# order %d: %zu topologies, %lld labelled permutations (oracle/enumerate.c)\n", n, all.n, labelled);
    for (size_t i = 0; i < all.n; ++i) {
        for (int v = 0; v < n2; ++v) {
            int x = (int)((all.k[i] >> (4 * (n2 - 1 - v))) & 15u);
            printf(v ? " %d" : "%d", x);
        }
        printf("\n");
    }
    free(all.k);
    return 0;
}
