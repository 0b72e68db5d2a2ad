/*
 * mphx_oracle.c -- plain, slow, single-threaded CPU reference for the MWHC build path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls this
 * file; only the test-suite, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no code, header, table or constant generator with the GPU path: every step is
 * written out here from the paper's definitions, in the paper's order.
 *
 * Paper: Belazzougui, Boldi, Ottaviano, Venturini, Vigna, "Cache-Oblivious Peeling of Random
 * Hypergraphs" (arXiv 1312.0526).  Section references below are to that paper.
 *
 *  - Section 3 (MWHC): three hash functions map key x to the edge {h0(x), h1(x), h2(x)} of a
 *    3-hypergraph on gamma*n vertices; vertex values u solve f(x) = u[h0]+u[h1]+u[h2] mod
 *    sigma by backward substitution along a peeling order; for an MPHF, f(x) is the index i
 *    of a vertex h_i(x) that had degree 1 when x's edge was peeled, and a ranking structure
 *    over the used vertices makes h_f(x)(x) minimal.
 *  - Section 4.1 (packed incidence lists, the XOR trick, labelled variant): each vertex keeps
 *    its degree d and the XOR of the labels (here: edge ids) of its incident edges; when
 *    d = 1 the XOR is the only incident edge.
 *  - Section 4.2 (layered peeling): each round removes the edges of all vertices that have
 *    degree 1 at the start of the round; an edge found from several degree-1 vertices is
 *    removed once; concatenated layers form a peeling order whatever the order inside a layer.
 *  - Section 4.3 (tripartition): h_i maps into part i = [i*P, (i+1)*P) of the vertex set, so
 *    the three vertices of an edge are distinct.  (Avoiding backward scans): assignment walks
 *    the layers in reverse round order, each layer in any order.
 *  - Section 5 (lookups): ranking counts the non-zero 2-bit pairs of 64-bit words with a
 *    broadword expression.
 *
 * Readings where the paper is silent (each one is listed with its reason in the design notes):
 *  - key hashing: SplitMix64 replaces the paper's Jenkins hash (Section 3, footnote); edge
 *    vertex k of a key is k*P + floor(z_k * P / 2^64), z_k = fin(s + (k+1)*GAMMA), where
 *    s = key XOR seed for u64 keys; byte-string keys use the 128-bit digest (a, b) defined
 *    below and z_0, z_1 come from a, z_2 from b (a = b = key XOR seed reproduces u64 keys);
 *  - P = ceil(n * gamma_num / (3 * gamma_den)), m = 3P vertices;
 *  - hinge of an edge = the lowest tuple position (= part) among its vertices with degree 1
 *    at the start of the round that removes it; rounds are numbered from 0;
 *  - canonical order: edges by round, ascending id inside a round, then the edges that were
 *    never removed (the 2-core) in ascending id;
 *  - vertex values: g = 0 for vertices that are no hinge; 2-bit code 0 = not a hinge,
 *    1 / 2 = hinge with g = 1 / 2, 3 = hinge with g = 0;
 *  - rank table: one u64 per 512 vertices holding the number of hinge vertices strictly
 *    before the block (exclusive rank), so the MPHF maps onto [0, n);
 *  - retries: seed, seed+1, ... up to max_tries; degree above 255 is an error;
 *  - HEM split (Section 3, "Practical workarounds", signatures chosen so that no two keys
 *    share one): a u64 key's signature is the 64-bit fin(s + 4*GAMMA) (s = key XOR seed, a
 *    bijection) and a byte string's the whole 128-bit digest (a, b) under the seed; the top k
 *    bits of the signature's first word pick one of 2^k buckets; inside its bucket the key is
 *    the digest pair (swap(first word), second word) -- (swap(sig), swap(sig)) for u64 keys,
 *    (swap(a), b) for strings, swap exchanging the 32-bit halves -- whose edge under seed t is
 *    the edge of the digest (x XOR t, y XOR t); each bucket gets the MWHC MPHF of its keys
 *    (hash seed = the build's seed, retries seed+1, ...); f(x) = (keys in earlier buckets) +
 *    the bucket MPHF's value; a bucket that fails (max_tries 2-cores) fails the build, which
 *    the caller redoes with another seed;
 *  - static functions (Section 3, any sigma in [1, 2^32]): values must lie in [0, sigma);
 *    u = 0 on vertices that are no hinge; each u is stored in b = (bits of sigma - 1) bits,
 *    vertex v's field at bits [v*b, v*b + b) of the little-endian bit string of the u64
 *    words (b = 0 when sigma = 1: nothing is stored and every lookup is 0).
 *
 * No floating point anywhere.  All arithmetic is on unsigned integers.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-2)
#define ORC_ENOMEM (-3)
#define ORC_ECORE 1
#define ORC_EDUP 2

#define ORC_NONE 0xFFFFFFFFu
#define ORC_MAX_DEGREE 255u

static const uint64_t ORC_GAMMA = 0x9E3779B97F4A7C15ull;

/* Progress lines on stderr from the peel and the assignment (long runs only; off by default). */
static int orc_progress = 0;
void orc_set_progress(int on) { orc_progress = on; }

/* SplitMix64 output function (Steele, Lea & Flood 2014; Stafford's "Mix13" constants). */
static uint64_t orc_fin(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Output t (1-based) of the SplitMix64 stream seeded at state s. */
uint64_t orc_splitmix(uint64_t s, uint64_t t)
{
    return orc_fin(s + t * ORC_GAMMA);
}

/* floor(z * p / 2^64): maps a uniform 64-bit value into [0, p). */
static uint64_t orc_range(uint64_t z, uint64_t p)
{
    return (uint64_t)(((unsigned __int128)z * p) >> 64);
}

/* Vertices per part: P = ceil(n * gamma / 3) with gamma = gnum / gden (Section 3: gamma*n
 * vertices in total, Section 4.3: three equal parts). */
uint64_t orc_part_size(uint64_t n, uint32_t gnum, uint32_t gden)
{
    unsigned __int128 num = (unsigned __int128)n * gnum;
    unsigned __int128 den = (unsigned __int128)3 * gden;
    return (uint64_t)((num + den - 1) / den);
}

/* Edge of a key from its 128-bit digest (a, b): vertex k lies in part k (Section 4.3). */
static void orc_edge_of_digest(uint64_t a, uint64_t b, uint64_t P, uint32_t out[3])
{
    uint64_t z0 = orc_fin(a + 1 * ORC_GAMMA);
    uint64_t z1 = orc_fin(a + 2 * ORC_GAMMA);
    uint64_t z2 = orc_fin(b + 3 * ORC_GAMMA);
    out[0] = (uint32_t)(0 * P + orc_range(z0, P));
    out[1] = (uint32_t)(1 * P + orc_range(z1, P));
    out[2] = (uint32_t)(2 * P + orc_range(z2, P));
}

void orc_hash_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t P, uint32_t* edges)
{
    for (uint64_t i = 0; i < n; i++) {
        uint64_t s = keys[i] ^ seed;
        orc_edge_of_digest(s, s, P, edges + 3 * i);
    }
}

/* 128-bit digest of a byte string.  Word j is bytes [8j, 8j+8) read little-endian, the bytes
 * past the end of the key taken as zero.  Lane A and lane B each sum fin(w_j XOR salt_j) over
 * the words, with salt_j = s + j*GAMMA and s the lane's own seed-derived start; each lane
 * then folds in the length. */
void orc_digest_str(const uint8_t* x, uint64_t len, uint64_t seed, uint64_t* a_out, uint64_t* b_out)
{
    uint64_t sa = orc_splitmix(seed, 1);
    uint64_t sb = orc_splitmix(seed, 2);
    uint64_t A = 0, B = 0;
    uint64_t nwords = (len + 7) / 8;
    for (uint64_t j = 0; j < nwords; j++) {
        uint64_t w = 0;
        for (uint64_t t = 0; t < 8; t++) {
            uint64_t p = 8 * j + t;
            if (p < len)
                w |= (uint64_t)x[p] << (8 * t);
        }
        A += orc_fin(w ^ (sa + j * ORC_GAMMA));
        B += orc_fin(w ^ (sb + j * ORC_GAMMA));
    }
    *a_out = orc_fin(A ^ sa ^ len);
    *b_out = orc_fin(B ^ sb ^ len);
}

void orc_hash_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint64_t P,
                  uint32_t* edges)
{
    for (uint64_t i = 0; i < n; i++) {
        uint64_t a, b;
        orc_digest_str(bytes + offs[i], offs[i + 1] - offs[i], seed, &a, &b);
        orc_edge_of_digest(a, b, P, edges + 3 * i);
    }
}

/* Keys given as 128-bit digests (x_i, y_i): under seed t the edge is that of the digest
 * (x_i XOR t, y_i XOR t).  A u64 key is the pair (key, key). */
void orc_hash_pairs(const uint64_t* x, const uint64_t* y, uint64_t n, uint64_t seed, uint64_t P, uint32_t* edges)
{
    for (uint64_t i = 0; i < n; i++)
        orc_edge_of_digest(x[i] ^ seed, y[i] ^ seed, P, edges + 3 * i);
}

/* ------------------------------------------------------------------------------------------
 * Layered peeling (Section 4.2) over packed incidence lists with edge-id labels (Section 4.1).
 *
 * part_size != 0 declares the edges tripartite (vertex k of every edge in part k); the
 * position of a degree-1 vertex inside its edge is then its part.  part_size == 0 means a
 * generic edge list, where the position is found by comparing with the edge's vertices.
 *
 * Outputs (all caller-owned, length n): order, round (ORC_NONE for 2-core edges),
 * core_mask (1 for 2-core edges), hinge (0..2, 0xFF for 2-core edges; may be NULL).
 * info[0] = number of peeled edges, info[1] = number of rounds (non-empty layers),
 * info[2] = maximum vertex degree.
 * ------------------------------------------------------------------------------------------ */
int orc_peel(const uint32_t* edges, uint64_t n, uint64_t m, uint64_t part_size, uint32_t* order,
             uint32_t* round, uint8_t* core_mask, uint8_t* hinge_out, uint64_t* info)
{
    if (n > 0xFFFFFFFFull || m > 0x100000000ull)
        return ORC_EINVAL;
    for (uint64_t e = 0; e < n; e++) {
        const uint32_t* t = edges + 3 * e;
        if (t[0] >= m || t[1] >= m || t[2] >= m)
            return ORC_EINVAL;
        if (t[0] == t[1] || t[0] == t[2] || t[1] == t[2])
            return ORC_EINVAL;
        if (part_size) {
            for (int k = 0; k < 3; k++)
                if (t[k] / part_size != (uint64_t)k)
                    return ORC_EINVAL;
        }
    }

    uint32_t* deg = calloc(m ? m : 1, sizeof(uint32_t)); /* Degree(L_v) */
    uint32_t* lab = calloc(m ? m : 1, sizeof(uint32_t)); /* XOR of incident edge labels */
    uint8_t* hinge = malloc(n ? n : 1);
    uint32_t* frontier = malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* next = malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* layer = malloc((n ? n : 1) * sizeof(uint32_t));
    if (!deg || !lab || !hinge || !frontier || !next || !layer) {
        free(deg); free(lab); free(hinge); free(frontier); free(next); free(layer);
        return ORC_ENOMEM;
    }

    /* AddEdge for every edge at every one of its vertices. */
    uint32_t maxdeg = 0;
    for (uint64_t e = 0; e < n; e++) {
        for (int k = 0; k < 3; k++) {
            uint32_t v = edges[3 * e + k];
            deg[v] += 1;
            lab[v] ^= (uint32_t)e;
            if (deg[v] > maxdeg)
                maxdeg = deg[v];
        }
    }
    if (maxdeg > ORC_MAX_DEGREE) {
        free(deg); free(lab); free(hinge); free(frontier); free(next); free(layer);
        if (info) { info[0] = 0; info[1] = 0; info[2] = maxdeg; }
        return ORC_ERANGE;
    }
    if (orc_progress) {
        fprintf(stderr, "[oracle] %llu incidence records built, maximum degree %u\n", (unsigned long long)(3 * n), maxdeg);
        fflush(stderr);
    }

    for (uint64_t e = 0; e < n; e++) {
        round[e] = ORC_NONE;
        hinge[e] = 0xFF;
    }

    /* Round 0 candidates: every vertex of degree 1. */
    uint64_t nf = 0;
    for (uint64_t v = 0; v < m; v++)
        if (deg[v] == 1)
            frontier[nf++] = (uint32_t)v;

    uint32_t r = 0;
    uint64_t peeled = 0;
    for (;;) {
        /* Pass A (no mutation): RetrieveEdge at every vertex that has degree 1 now, i.e. at
         * the start of round r.  Each edge enters the layer once; its hinge is the lowest
         * position among the vertices that found it. */
        uint64_t nl = 0;
        for (uint64_t i = 0; i < nf; i++) {
            uint32_t v = frontier[i];
            if (deg[v] != 1)
                continue;
            uint32_t e = lab[v];
            uint8_t k;
            if (part_size) {
                k = (uint8_t)(v / part_size);
            } else {
                k = edges[3 * (uint64_t)e] == v ? 0 : (edges[3 * (uint64_t)e + 1] == v ? 1 : 2);
            }
            if (round[e] == ORC_NONE) {
                round[e] = r;
                hinge[e] = k;
                layer[nl++] = e;
            } else if (k < hinge[e]) {
                hinge[e] = k;
            }
        }
        if (nl == 0)
            break;
        /* Pass B: DeleteEdge of every layer edge at its three vertices; a vertex whose
         * degree drops to exactly 1 becomes a candidate for the next round. */
        uint64_t nn = 0;
        for (uint64_t i = 0; i < nl; i++) {
            uint32_t e = layer[i];
            for (int k = 0; k < 3; k++) {
                uint32_t u = edges[3 * (uint64_t)e + k];
                deg[u] -= 1;
                lab[u] ^= e;
                if (deg[u] == 1)
                    next[nn++] = u;
            }
        }
        peeled += nl;
        if (orc_progress) {
            fprintf(stderr, "[oracle] round %u: %llu edges peeled (%llu in all)\n", r, (unsigned long long)nl,
                    (unsigned long long)peeled);
            fflush(stderr);
        }
        uint32_t* tmp = frontier;
        frontier = next;
        next = tmp;
        nf = nn;
        r += 1;
    }

    /* Canonical order: counting sort by round (stable, so ascending id inside a round),
     * then the 2-core edges in ascending id. */
    uint64_t* start = calloc((uint64_t)r + 2, sizeof(uint64_t));
    if (!start) {
        free(deg); free(lab); free(hinge); free(frontier); free(next); free(layer);
        return ORC_ENOMEM;
    }
    for (uint64_t e = 0; e < n; e++) {
        uint64_t slot = round[e] == ORC_NONE ? r : round[e];
        start[slot + 1] += 1;
    }
    for (uint64_t j = 0; j <= r; j++)
        start[j + 1] += start[j];
    for (uint64_t e = 0; e < n; e++) {
        uint64_t slot = round[e] == ORC_NONE ? r : round[e];
        order[start[slot]++] = (uint32_t)e;
    }
    for (uint64_t e = 0; e < n; e++) {
        core_mask[e] = round[e] == ORC_NONE ? 1 : 0;
        if (hinge_out)
            hinge_out[e] = hinge[e];
    }
    if (info) {
        info[0] = peeled;
        info[1] = r;
        info[2] = maxdeg;
    }
    free(start);
    free(deg); free(lab); free(hinge); free(frontier); free(next); free(layer);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------
 * Assignment (Section 3, solved along the layers in reverse round order as in Section 4.3)
 * and the 2-bit code vector.  order/round/hinge are orc_peel's outputs; every edge must be
 * peeled.  codes8 (length m, caller-owned) receives one 2-bit code per vertex.
 * ------------------------------------------------------------------------------------------ */
int orc_assign(const uint32_t* edges, uint64_t n, uint64_t m, const uint32_t* order,
               const uint32_t* round, const uint8_t* hinge, uint8_t* codes8)
{
    uint8_t* g = calloc(m ? m : 1, 1);
    uint8_t* used = calloc(m ? m : 1, 1);
    if (!g || !used) {
        free(g); free(used);
        return ORC_ENOMEM;
    }
    /* Walk layers from the last round to round 0; inside a layer any order is valid, here
     * the canonical ascending order. */
    uint64_t end = n;
    while (end > 0) {
        uint32_t rr = round[order[end - 1]];
        if (rr == ORC_NONE) {
            free(g); free(used);
            return ORC_ECORE;
        }
        uint64_t begin = end;
        while (begin > 0 && round[order[begin - 1]] == rr)
            begin--;
        for (uint64_t i = begin; i < end; i++) {
            uint64_t e = order[i];
            uint32_t k = hinge[e];
            uint32_t vk = edges[3 * e + k];
            uint32_t v1 = edges[3 * e + (k + 1) % 3];
            uint32_t v2 = edges[3 * e + (k + 2) % 3];
            /* f(x) = k requires g[vk] + g[v1] + g[v2] = k (mod 3). */
            g[vk] = (uint8_t)((k + 6 - g[v1] - g[v2]) % 3);
            used[vk] = 1;
        }
        if (orc_progress) {
            fprintf(stderr, "[oracle] layer of round %u assigned (%llu edges)\n", rr, (unsigned long long)(end - begin));
            fflush(stderr);
        }
        end = begin;
    }
    for (uint64_t v = 0; v < m; v++)
        codes8[v] = used[v] ? (g[v] ? g[v] : 3) : 0;
    free(g);
    free(used);
    return ORC_OK;
}

/* Pack 32 codes per u64 word (vertex v at bits 2*(v%32) of word v/32) and build the rank
 * samples: rank[b] = number of non-zero codes among vertices [0, 512*b). */
void orc_pack_rank(const uint8_t* codes8, uint64_t m, uint64_t* words, uint64_t* rank)
{
    uint64_t nwords = (m + 31) / 32;
    for (uint64_t w = 0; w < nwords; w++) {
        uint64_t x = 0;
        for (uint64_t t = 0; t < 32; t++) {
            uint64_t v = 32 * w + t;
            if (v < m)
                x |= (uint64_t)(codes8[v] & 3) << (2 * t);
        }
        words[w] = x;
    }
    uint64_t nblocks = (m + 511) / 512;
    uint64_t count = 0;
    for (uint64_t b = 0; b < nblocks; b++) {
        rank[b] = count;
        for (uint64_t v = 512 * b; v < 512 * (b + 1) && v < m; v++)
            count += codes8[v] != 0;
    }
}

/* Number of non-zero 2-bit pairs of a word (broadword, Section 5). */
static uint64_t orc_nzpairs(uint64_t w)
{
    uint64_t x = (w | (w >> 1)) & 0x5555555555555555ull;
    return (uint64_t)__builtin_popcountll(x);
}

static uint64_t orc_rank_of(const uint64_t* words, const uint64_t* rank, uint64_t h)
{
    uint64_t r = rank[h >> 9];
    for (uint64_t w = (h >> 9) * 16; w < (h >> 5); w++)
        r += orc_nzpairs(words[w]);
    uint64_t below = 2 * (h & 31);
    uint64_t mask = below ? ((1ull << below) - 1) : 0;
    return r + orc_nzpairs(words[h >> 5] & mask);
}

static uint32_t orc_code_at(const uint64_t* words, uint64_t v)
{
    return (uint32_t)((words[v >> 5] >> (2 * (v & 31))) & 3);
}

/* MPHF value of a key with edge t: i = (g0 + g1 + g2) mod 3, value = rank of vertex t[i]. */
static uint64_t orc_eval_edge(const uint64_t* words, const uint64_t* rank, const uint32_t t[3])
{
    uint32_t s = 0;
    for (int k = 0; k < 3; k++)
        s += orc_code_at(words, t[k]) % 3; /* code 3 stands for g = 0 */
    return orc_rank_of(words, rank, t[s % 3]);
}

void orc_lookup_u64(const uint64_t* words, const uint64_t* rank, uint64_t P, uint64_t seed,
                    const uint64_t* keys, uint64_t n, uint64_t* out)
{
    for (uint64_t i = 0; i < n; i++) {
        uint32_t t[3];
        orc_hash_u64(keys + i, 1, seed, P, t);
        out[i] = orc_eval_edge(words, rank, t);
    }
}

void orc_lookup_str(const uint64_t* words, const uint64_t* rank, uint64_t P, uint64_t seed,
                    const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t* out)
{
    for (uint64_t i = 0; i < n; i++) {
        uint64_t a, b;
        uint32_t t[3];
        orc_digest_str(bytes + offs[i], offs[i + 1] - offs[i], seed, &a, &b);
        orc_edge_of_digest(a, b, P, t);
        out[i] = orc_eval_edge(words, rank, t);
    }
}

/* ------------------------------------------------------------------------------------------
 * Static function (Section 3): u in [sigma]^m with f(x) = u[h0(x)] + u[h1(x)] + u[h2(x)]
 * (mod sigma) for every key, solved like the MPHF's g along the layers in reverse round order:
 * the hinge vertex of x's edge takes f(x) minus the other two vertices' values.
 * ------------------------------------------------------------------------------------------ */
uint32_t orc_sf_bits(uint64_t sigma)
{
    uint32_t b = 0;
    while (b < 64 && ((sigma - 1) >> b) != 0)
        b++;
    return b;
}

int orc_sf_assign(const uint32_t* edges, uint64_t n, uint64_t m, const uint32_t* order, const uint32_t* round,
                  const uint8_t* hinge, const uint32_t* values, uint64_t sigma, uint32_t* u)
{
    for (uint64_t v = 0; v < m; v++)
        u[v] = 0;
    uint64_t end = n;
    while (end > 0) {
        uint32_t rr = round[order[end - 1]];
        if (rr == ORC_NONE)
            return ORC_ECORE;
        uint64_t begin = end;
        while (begin > 0 && round[order[begin - 1]] == rr)
            begin--;
        for (uint64_t i = begin; i < end; i++) {
            uint64_t e = order[i];
            uint32_t k = hinge[e];
            uint32_t vh = edges[3 * e + k];
            uint32_t va = edges[3 * e + (k + 1) % 3];
            uint32_t vb = edges[3 * e + (k + 2) % 3];
            /* f(x) = u[vh] + u[va] + u[vb] (mod sigma) */
            u[vh] = (uint32_t)((values[e] + 2 * sigma - u[va] - u[vb]) % sigma);
        }
        end = begin;
    }
    return ORC_OK;
}

/* Fields of b bits, vertex v at bit v*b of the little-endian bit string of the words. */
void orc_sf_pack(const uint32_t* u, uint64_t m, uint32_t b, uint64_t* words)
{
    uint64_t nwords = (m * b + 63) / 64;
    for (uint64_t w = 0; w < nwords; w++)
        words[w] = 0;
    for (uint64_t v = 0; v < m; v++)
        for (uint32_t t = 0; t < b; t++) {
            uint64_t bit = v * b + t;
            words[bit / 64] |= (uint64_t)((u[v] >> t) & 1u) << (bit % 64);
        }
}

static uint64_t orc_sf_field(const uint64_t* words, uint32_t b, uint64_t v)
{
    uint64_t x = 0;
    for (uint32_t t = 0; t < b; t++) {
        uint64_t bit = v * b + t;
        x |= ((words[bit / 64] >> (bit % 64)) & 1u) << t;
    }
    return x;
}

static uint64_t orc_sf_eval_edge(const uint64_t* words, uint64_t sigma, const uint32_t t[3])
{
    uint32_t b = orc_sf_bits(sigma);
    return (orc_sf_field(words, b, t[0]) + orc_sf_field(words, b, t[1]) + orc_sf_field(words, b, t[2])) % sigma;
}

void orc_sf_lookup_u64(const uint64_t* words, uint64_t sigma, uint64_t P, uint64_t seed, const uint64_t* keys,
                       uint64_t n, uint64_t* out)
{
    for (uint64_t i = 0; i < n; i++) {
        uint32_t t[3];
        orc_hash_u64(keys + i, 1, seed, P, t);
        out[i] = orc_sf_eval_edge(words, sigma, t);
    }
}

void orc_sf_lookup_str(const uint64_t* words, uint64_t sigma, uint64_t P, uint64_t seed, const uint8_t* bytes,
                       const uint64_t* offs, uint64_t n, uint64_t* out)
{
    for (uint64_t i = 0; i < n; i++) {
        uint64_t a, b;
        uint32_t t[3];
        orc_digest_str(bytes + offs[i], offs[i + 1] - offs[i], seed, &a, &b);
        orc_edge_of_digest(a, b, P, t);
        out[i] = orc_sf_eval_edge(words, sigma, t);
    }
}

/* ------------------------------------------------------------------------------------------
 * Ranked static-function layout (Section 3: ceil(log sigma) n + gamma n + o(n) bits with a
 * ranking structure).  Only the vertices whose value u[v] is not zero keep a field; u is zero
 * off the hinges, so there are at most n of them.
 *   marks: m bits, bit v % 64 of word v / 64 set iff u[v] != 0;
 *   rank:  rank[j] = the number of marked vertices below vertex ORC_SFR_BLOCK * j, for
 *          j = 0 .. ceil(m / ORC_SFR_BLOCK); the last entry is the number of fields;
 *   vals:  the fields of the marked vertices in vertex order, field i at bits [i b, i b + b)
 *          of the little-endian bit string of the words.
 * A vertex without a mark has u = 0.  Built here from the packed plain layout (one field per
 * vertex, as orc_sf_pack writes it).
 * ------------------------------------------------------------------------------------------ */
#define ORC_SFR_BLOCK 1024

uint64_t orc_sfr_rank_words(uint64_t m)
{
    return (m + ORC_SFR_BLOCK - 1) / ORC_SFR_BLOCK + 1;
}

static void orc_put_field(uint64_t* words, uint32_t b, uint64_t i, uint64_t x)
{
    for (uint32_t t = 0; t < b; t++) {
        uint64_t bit = i * b + t;
        words[bit / 64] |= ((x >> t) & 1u) << (bit % 64);
    }
}

/* Returns the number of fields; vals must hold ceil(fields * b / 64) words. */
uint64_t orc_sf_rank_layout(const uint64_t* words, uint64_t m, uint32_t b, uint64_t* marks, uint64_t* rank,
                            uint64_t* vals)
{
    for (uint64_t w = 0; w < (m + 63) / 64; w++)
        marks[w] = 0;
    uint64_t count = 0;
    for (uint64_t v = 0; v < m; v++) {
        if (v % ORC_SFR_BLOCK == 0)
            rank[v / ORC_SFR_BLOCK] = count;
        if (orc_sf_field(words, b, v) != 0) {
            marks[v / 64] |= 1ull << (v % 64);
            count++;
        }
    }
    rank[(m + ORC_SFR_BLOCK - 1) / ORC_SFR_BLOCK] = count;
    for (uint64_t w = 0; w < (count * b + 63) / 64; w++)
        vals[w] = 0;
    uint64_t i = 0;
    for (uint64_t v = 0; v < m; v++)
        if ((marks[v / 64] >> (v % 64)) & 1u)
            orc_put_field(vals, b, i++, orc_sf_field(words, b, v));
    return count;
}

/* u[v] through the ranking structure: zero without a mark, else the field whose index is the
 * number of marked vertices below v (the block's sample plus the marks in the block before v,
 * counted one by one). */
static uint64_t orc_sfr_value(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint32_t b,
                              uint64_t v)
{
    if (!((marks[v / 64] >> (v % 64)) & 1u))
        return 0;
    uint64_t r = rank[v / ORC_SFR_BLOCK];
    for (uint64_t x = v - v % ORC_SFR_BLOCK; x < v; x++)
        r += (marks[x / 64] >> (x % 64)) & 1u;
    return orc_sf_field(vals, b, r);
}

static uint64_t orc_sfr_eval_edge(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint64_t sigma,
                                  const uint32_t t[3])
{
    uint32_t b = orc_sf_bits(sigma);
    return (orc_sfr_value(marks, rank, vals, b, t[0]) + orc_sfr_value(marks, rank, vals, b, t[1]) +
            orc_sfr_value(marks, rank, vals, b, t[2])) % sigma;
}

void orc_sfr_lookup_u64(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint64_t sigma, uint64_t P,
                        uint64_t seed, const uint64_t* keys, uint64_t n, uint64_t* out)
{
    for (uint64_t i = 0; i < n; i++) {
        uint32_t t[3];
        orc_hash_u64(keys + i, 1, seed, P, t);
        out[i] = orc_sfr_eval_edge(marks, rank, vals, sigma, t);
    }
}

void orc_sfr_lookup_str(const uint64_t* marks, const uint64_t* rank, const uint64_t* vals, uint64_t sigma, uint64_t P,
                        uint64_t seed, const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t* out)
{
    for (uint64_t i = 0; i < n; i++) {
        uint64_t a, b;
        uint32_t t[3];
        orc_digest_str(bytes + offs[i], offs[i + 1] - offs[i], seed, &a, &b);
        orc_edge_of_digest(a, b, P, t);
        out[i] = orc_sfr_eval_edge(marks, rank, vals, sigma, t);
    }
}

/* ------------------------------------------------------------------------------------------
 * Whole MPHF build: hash (Section 3 / 4.3), peel (Section 4.2), retry with the next seed
 * while a 2-core remains, assign (Section 3 / 4.3), pack and rank (Section 5).
 * info[0] = P, info[1] = m, info[2] = seed used, info[3] = tries, info[4] = rounds,
 * info[5] = 2-core edges on the last try.
 * ------------------------------------------------------------------------------------------ */
static int orc_keys_equal(int kind, const void* keys, const uint64_t* offs, uint64_t i, uint64_t j)
{
    if (kind == 0)
        return ((const uint64_t*)keys)[i] == ((const uint64_t*)keys)[j];
    if (kind == 2) /* digest pairs: first words in keys, second words in offs */
        return ((const uint64_t*)keys)[i] == ((const uint64_t*)keys)[j] && offs[i] == offs[j];
    uint64_t li = offs[i + 1] - offs[i], lj = offs[j + 1] - offs[j];
    if (li != lj)
        return 0;
    return memcmp((const uint8_t*)keys + offs[i], (const uint8_t*)keys + offs[j], li) == 0;
}

static const uint32_t* orc_sort_edges;
static int orc_cmp_triple(const void* pa, const void* pb)
{
    uint32_t a = *(const uint32_t*)pa, b = *(const uint32_t*)pb;
    for (int k = 0; k < 3; k++) {
        uint32_t x = orc_sort_edges[3 * (uint64_t)a + k], y = orc_sort_edges[3 * (uint64_t)b + k];
        if (x != y)
            return x < y ? -1 : 1;
    }
    return a < b ? -1 : (a > b);
}

/* kind 0: u64 keys; 1: byte strings (keys = bytes, offs = offsets); 2: digest pairs (keys =
 * first words, offs = second words).  values == NULL: the MPHF (words = 2-bit codes, rank =
 * samples); else the static function with those values in [0, sigma) (words = packed u, rank
 * unused). */
static int orc_build(int kind, const void* keys, const uint64_t* offs, uint64_t n, const uint32_t* values,
                     uint64_t sigma, uint64_t seed, uint32_t gnum, uint32_t gden, uint32_t max_tries,
                     uint64_t* words, uint64_t* rank, uint64_t* info)
{
    if (gden == 0 || gnum == 0 || max_tries == 0 || n > 0xFFFFFFFFull)
        return ORC_EINVAL;
    if (values) {
        if (sigma == 0 || sigma > 0x100000000ull)
            return ORC_EINVAL;
        for (uint64_t i = 0; i < n; i++)
            if (values[i] >= sigma)
                return ORC_EINVAL;
    }
    uint64_t P = orc_part_size(n, gnum, gden);
    uint64_t m = 3 * P;
    if (m > 0x100000000ull)
        return ORC_EINVAL;
    uint32_t* edges = malloc((n ? n : 1) * 3 * sizeof(uint32_t));
    uint32_t* order = malloc((n ? n : 1) * sizeof(uint32_t));
    uint32_t* round = malloc((n ? n : 1) * sizeof(uint32_t));
    uint8_t* core = malloc(n ? n : 1);
    uint8_t* hinge = malloc(n ? n : 1);
    uint8_t* codes8 = malloc(m ? m : 1);
    if (!edges || !order || !round || !core || !hinge || !codes8) {
        free(edges); free(order); free(round); free(core); free(hinge); free(codes8);
        return ORC_ENOMEM;
    }
    int status = ORC_ECORE;
    uint64_t pinfo[3] = {0, 0, 0};
    uint32_t t;
    for (t = 0; t < max_tries; t++) {
        uint64_t s = seed + t;
        if (kind == 0)
            orc_hash_u64((const uint64_t*)keys, n, s, P, edges);
        else if (kind == 2)
            orc_hash_pairs((const uint64_t*)keys, offs, n, s, P, edges);
        else
            orc_hash_str((const uint8_t*)keys, offs, n, s, P, edges);
        int rc = orc_peel(edges, n, m, P, order, round, core, hinge, pinfo);
        if (rc != ORC_OK) {
            status = rc;
            break;
        }
        if (pinfo[0] == n) {
            if (values) {
                uint32_t* u = malloc((m ? m : 1) * sizeof(uint32_t));
                if (!u) {
                    status = ORC_ENOMEM;
                    break;
                }
                rc = orc_sf_assign(edges, n, m, order, round, hinge, values, sigma, u);
                if (rc == ORC_OK)
                    orc_sf_pack(u, m, orc_sf_bits(sigma), words);
                free(u);
            } else {
                rc = orc_assign(edges, n, m, order, round, hinge, codes8);
                if (rc == ORC_OK)
                    orc_pack_rank(codes8, m, words, rank);
            }
            status = rc;
            break;
        }
    }
    if (status == ORC_ECORE) {
        /* Identical core edges with equal keys can never peel under any seed. */
        t = max_tries - 1;
        uint64_t nc = n - pinfo[0];
        uint32_t* ids = malloc((nc ? nc : 1) * sizeof(uint32_t));
        if (ids) {
            uint64_t c = 0;
            for (uint64_t e = 0; e < n; e++)
                if (core[e])
                    ids[c++] = (uint32_t)e;
            orc_sort_edges = edges;
            qsort(ids, c, sizeof(uint32_t), orc_cmp_triple);
            for (uint64_t i = 0; i + 1 < c && status == ORC_ECORE; i++) {
                uint64_t j = i + 1;
                int same = 1;
                for (int k = 0; k < 3; k++)
                    same &= edges[3 * (uint64_t)ids[i] + k] == edges[3 * (uint64_t)ids[j] + k];
                if (same && orc_keys_equal(kind, keys, offs, ids[i], ids[j]))
                    status = ORC_EDUP;
            }
            free(ids);
        }
    }
    if (info) {
        info[0] = P;
        info[1] = m;
        info[2] = seed + t;
        info[3] = (uint64_t)t + 1;
        info[4] = pinfo[1];
        info[5] = n - pinfo[0];
    }
    free(edges); free(order); free(round); free(core); free(hinge); free(codes8);
    return status;
}

int orc_mphf_build_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint32_t gnum, uint32_t gden,
                       uint32_t max_tries, uint64_t* words, uint64_t* rank, uint64_t* info)
{
    return orc_build(0, keys, NULL, n, NULL, 0, seed, gnum, gden, max_tries, words, rank, info);
}

int orc_mphf_build_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed,
                       uint32_t gnum, uint32_t gden, uint32_t max_tries, uint64_t* words,
                       uint64_t* rank, uint64_t* info)
{
    return orc_build(1, bytes, offs, n, NULL, 0, seed, gnum, gden, max_tries, words, rank, info);
}

int orc_sf_build_u64(const uint64_t* keys, const uint32_t* values, uint64_t n, uint64_t sigma, uint64_t seed,
                     uint32_t gnum, uint32_t gden, uint32_t max_tries, uint64_t* words, uint64_t* info)
{
    return orc_build(0, keys, NULL, n, values, sigma, seed, gnum, gden, max_tries, words, NULL, info);
}

int orc_sf_build_str(const uint8_t* bytes, const uint64_t* offs, const uint32_t* values, uint64_t n,
                     uint64_t sigma, uint64_t seed, uint32_t gnum, uint32_t gden, uint32_t max_tries,
                     uint64_t* words, uint64_t* info)
{
    return orc_build(1, bytes, offs, n, values, sigma, seed, gnum, gden, max_tries, words, NULL, info);
}

/* ------------------------------------------------------------------------------------------
 * HEM split (Section 3): signatures, buckets by their top bits, one MWHC MPHF per bucket.
 * ------------------------------------------------------------------------------------------ */
uint64_t orc_hem_signature_u64(uint64_t key, uint64_t seed) { return orc_fin((key ^ seed) + 4 * ORC_GAMMA); }

/* A byte string's signature: its whole 128-bit digest (a, b) under the seed. */
void orc_hem_signature_str(const uint8_t* x, uint64_t len, uint64_t seed, uint64_t* a, uint64_t* b)
{
    orc_digest_str(x, len, seed, a, b);
}

/* Signatures of n keys (the per-key functions above, in a loop). */
void orc_hem_signatures_u64(const uint64_t* keys, uint64_t n, uint64_t seed, uint64_t* out)
{
    for (uint64_t i = 0; i < n; i++)
        out[i] = orc_hem_signature_u64(keys[i], seed);
}

void orc_hem_signatures_str(const uint8_t* bytes, const uint64_t* offs, uint64_t n, uint64_t seed, uint64_t* a,
                            uint64_t* b)
{
    for (uint64_t i = 0; i < n; i++)
        orc_hem_signature_str(bytes + offs[i], offs[i + 1] - offs[i], seed, a + i, b + i);
}

/* The first word of the pair a signature stands for inside its bucket: the signature's first
 * word with its two 32-bit halves swapped. */
static uint64_t orc_hem_bucket_key(uint64_t sig) { return (sig << 32) | (sig >> 32); }

/* The bucket key of signature i: (swap(sigs[i]), sigs2[i]), or (swap, swap) without sigs2. */
static void orc_hem_pair(const uint64_t* sigs, const uint64_t* sigs2, uint64_t i, uint64_t* x, uint64_t* y)
{
    *x = orc_hem_bucket_key(sigs[i]);
    *y = sigs2 ? sigs2[i] : *x;
}

/* sigs: the n signatures' first words; sigs2: their second words (string keys) or NULL (u64
 * keys).  k in [0, 32].  Outputs: bucket_off (2^k + 1 key offsets), code_off
 * and rank_off (2^k + 1: where bucket b's ceil(m_b/32) codes and ceil(m_b/512) rank samples
 * start), seeds (2^k: each bucket's seed used), codes and rank (sized by code_off[2^k] and
 * rank_off[2^k]: the caller calls with codes == NULL first to learn them).  Returns ORC_OK,
 * or the first failing bucket's status (ORC_ECORE / ORC_EDUP / ORC_ERANGE). */
int orc_hem_build(const uint64_t* sigs, const uint64_t* sigs2, uint64_t n, uint32_t k, uint64_t seed, uint32_t gnum,
                  uint32_t gden, uint32_t max_tries, uint64_t* bucket_off, uint64_t* code_off, uint64_t* rank_off,
                  uint64_t* seeds, uint64_t* codes, uint64_t* rank)
{
    if (k > 32 || gnum == 0 || gden == 0 || max_tries == 0)
        return ORC_EINVAL;
    const uint64_t B = 1ull << k;
    for (uint64_t b = 0; b <= B; b++)
        bucket_off[b] = 0;
    for (uint64_t i = 0; i < n; i++)
        bucket_off[(k ? sigs[i] >> (64 - k) : 0) + 1]++;
    for (uint64_t b = 0; b < B; b++)
        bucket_off[b + 1] += bucket_off[b];
    code_off[0] = rank_off[0] = 0;
    for (uint64_t b = 0; b < B; b++) {
        uint64_t m = 3 * orc_part_size(bucket_off[b + 1] - bucket_off[b], gnum, gden);
        code_off[b + 1] = code_off[b] + (m + 31) / 32;
        rank_off[b + 1] = rank_off[b] + (m + 511) / 512;
    }
    if (!codes)
        return ORC_OK;
    /* counting sort of the bucket keys (digest pairs) by bucket, stable in key order */
    uint64_t* kx = malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t* ky = malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t* fill = malloc(B * sizeof(uint64_t));
    if (!kx || !ky || !fill) {
        free(kx); free(ky); free(fill);
        return ORC_ENOMEM;
    }
    for (uint64_t b = 0; b < B; b++)
        fill[b] = bucket_off[b];
    for (uint64_t i = 0; i < n; i++) {
        uint64_t at = fill[k ? sigs[i] >> (64 - k) : 0]++;
        orc_hem_pair(sigs, sigs2, i, &kx[at], &ky[at]);
    }
    int status = ORC_OK;
    for (uint64_t b = 0; b < B && status == ORC_OK; b++) {
        uint64_t info[6];
        uint64_t lo = bucket_off[b];
        status = orc_build(2, kx + lo, ky + lo, bucket_off[b + 1] - lo, NULL, 0, seed, gnum, gden, max_tries,
                           codes + code_off[b], rank + rank_off[b], info);
        seeds[b] = info[2];
    }
    free(kx);
    free(ky);
    free(fill);
    return status;
}

/* f(x) for the key of signature i. */
static uint64_t orc_hem_eval(const uint64_t* sigs, const uint64_t* sigs2, uint64_t i, uint32_t k,
                             const uint64_t* bucket_off, const uint64_t* code_off, const uint64_t* rank_off,
                             const uint64_t* seeds, const uint64_t* codes, const uint64_t* rank, uint32_t gnum,
                             uint32_t gden)
{
    uint64_t sig = sigs[i];
    uint64_t b = k ? sig >> (64 - k) : 0;
    uint64_t nb = bucket_off[b + 1] - bucket_off[b];
    uint64_t x, y;
    uint32_t t[3];
    orc_hem_pair(sigs, sigs2, i, &x, &y);
    orc_hash_pairs(&x, &y, 1, seeds[b], orc_part_size(nb, gnum, gden), t);
    return bucket_off[b] + orc_eval_edge(codes + code_off[b], rank + rank_off[b], t);
}

void orc_hem_lookup(const uint64_t* sigs, const uint64_t* sigs2, uint64_t n, uint32_t k, const uint64_t* bucket_off,
                    const uint64_t* code_off, const uint64_t* rank_off, const uint64_t* seeds,
                    const uint64_t* codes, const uint64_t* rank, uint32_t gnum, uint32_t gden, uint64_t* out)
{
    for (uint64_t i = 0; i < n; i++)
        out[i] = orc_hem_eval(sigs, sigs2, i, k, bucket_off, code_off, rank_off, seeds, codes, rank, gnum, gden);
}

/* ------------------------------------------------------------------------------------------
 * Peeling of an r-hypergraph, 2 <= r <= 8 (Section 2 defines r-hypergraphs; the paper works
 * with r = 3 and notes the generalization is direct).  The same definitions as orc_peel on a
 * generic edge list: edge e is edges[r*e .. r*e + r), a labelled incidence record per vertex
 * (degree and XOR of incident edge ids, Section 4.1), synchronous rounds (Section 4.2) whose
 * layer is every edge holding a vertex of degree 1 at the round's start, the hinge the lowest
 * tuple position among those vertices, and the canonical order (by round, ascending id inside
 * a round, the 2-core edges last in ascending id).  Statuses as orc_peel.
 * ------------------------------------------------------------------------------------------ */
int orc_peel_r(const uint32_t* edges, uint64_t n, uint64_t m, uint32_t r, uint32_t* order, uint32_t* round,
               uint8_t* core_mask, uint8_t* hinge_out, uint64_t* info)
{
    if (r < 2 || r > 8 || n > 0xFFFFFFFFull || m > 0x100000000ull)
        return ORC_EINVAL;
    for (uint64_t e = 0; e < n; e++) {
        const uint32_t* t = edges + (uint64_t)r * e;
        for (uint32_t a = 0; a < r; a++) {
            if (t[a] >= m)
                return ORC_EINVAL;
            for (uint32_t b = a + 1; b < r; b++)
                if (t[a] == t[b])
                    return ORC_EINVAL;
        }
    }
    uint32_t* deg = calloc(m ? m : 1, sizeof(uint32_t));
    uint32_t* lab = calloc(m ? m : 1, sizeof(uint32_t));
    uint8_t* hinge = malloc(n ? n : 1);
    uint32_t* frontier = malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* next = malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t* layer = malloc((n ? n : 1) * sizeof(uint32_t));
    if (!deg || !lab || !hinge || !frontier || !next || !layer) {
        free(deg); free(lab); free(hinge); free(frontier); free(next); free(layer);
        return ORC_ENOMEM;
    }
    uint32_t maxdeg = 0;
    for (uint64_t e = 0; e < n; e++)
        for (uint32_t k = 0; k < r; k++) {
            uint32_t v = edges[(uint64_t)r * e + k];
            deg[v] += 1;
            lab[v] = lab[v] ^ (uint32_t)e;
            if (deg[v] > maxdeg)
                maxdeg = deg[v];
        }
    if (ORC_MAX_DEGREE < maxdeg) {  /* some degree above the limit */
        free(deg); free(lab); free(hinge); free(frontier); free(next); free(layer);
        if (info) { info[0] = 0; info[1] = 0; info[2] = maxdeg; }
        return ORC_ERANGE;
    }
    for (uint64_t e = 0; e < n; e++) {
        round[e] = ORC_NONE;
        hinge[e] = 0xFF;
    }
    uint64_t nf = 0;
    for (uint64_t v = 0; v < m; v++)
        if (deg[v] == 1)
            frontier[nf++] = (uint32_t)v;
    uint32_t rd = 0;
    uint64_t peeled = 0;
    for (;;) {
        /* retrieve at every vertex of degree 1 at the round's start (no mutation) */
        uint64_t nl = 0;
        for (uint64_t i = 0; i < nf; i++) {
            uint32_t v = frontier[i];
            if (deg[v] != 1)  /* no longer of degree 1 */
                continue;
            uint32_t e = lab[v];
            uint8_t k = 0;
            while (edges[(uint64_t)r * e + k] != v)
                k++;
            if (round[e] == ORC_NONE) {
                round[e] = rd;
                hinge[e] = k;
                layer[nl++] = e;
            } else if (hinge[e] > k) {  /* a lower position also found it */
                hinge[e] = k;
            }
        }
        if (nl == 0)
            break;
        /* delete every layer edge at all of its r vertices */
        uint64_t nn = 0;
        for (uint64_t i = 0; i < nl; i++) {
            uint32_t e = layer[i];
            for (uint32_t k = 0; k < r; k++) {
                uint32_t u = edges[(uint64_t)r * e + k];
                deg[u] -= 1;
                lab[u] ^= e;
                if (deg[u] == 1)  /* a candidate of the next round */
                    next[nn++] = u;
            }
        }
        peeled += nl;
        if (orc_progress) {
            fprintf(stderr, "[oracle] round %u: %llu edges peeled (%llu in all)\n", r, (unsigned long long)nl,
                    (unsigned long long)peeled);
            fflush(stderr);
        }
        uint32_t* tmp = frontier;
        frontier = next;
        next = tmp;
        nf = nn;
        rd += 1;
    }
    uint64_t* start = calloc((uint64_t)rd + 2, sizeof(uint64_t));
    if (!start) {
        free(deg); free(lab); free(hinge); free(frontier); free(next); free(layer);
        return ORC_ENOMEM;
    }
    for (uint64_t e = 0; e < n; e++)
        start[(round[e] == ORC_NONE ? rd : round[e]) + 1] += 1;
    for (uint64_t j = 0; j <= rd; j++)
        start[j + 1] += start[j];
    for (uint64_t e = 0; e < n; e++)
        order[start[round[e] == ORC_NONE ? rd : round[e]]++] = (uint32_t)e;
    for (uint64_t e = 0; e < n; e++) {
        core_mask[e] = round[e] == ORC_NONE ? 1 : 0;
        if (hinge_out)
            hinge_out[e] = hinge[e];
    }
    if (info) {
        info[0] = peeled;
        info[1] = rd;
        info[2] = maxdeg;
    }
    free(start);
    free(deg); free(lab); free(hinge); free(frontier); free(next); free(layer);
    return ORC_OK;
}
