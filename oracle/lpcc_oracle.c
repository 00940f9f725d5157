/*
 * CPU oracle for the integer-only octree context model and its range coder.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reading of the
 * paper ("Towards Practical Lossless Neural Compression for LiDAR Point
 * Clouds", arXiv 2603.25260) that the GPU library is checked against.  Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the GPU library shares no code, header or table with it.
 *
 * Everything is integer arithmetic except the construction of the softmax
 * exponent table, which follows its plain definition round(2^15 e^{-i/16})
 * in double precision (checked against 60-digit decimals by the tests).
 *
 * Readings of the paper that fix what it leaves open (layer internals,
 * rounding, CDF rule, coder, stream layout) are listed in the design notes;
 * each function below cites the passage it follows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVAL -1
#define ORC_E_CAPACITY -2
#define ORC_E_CORRUPT -3
#define ORC_E_MODEL -4
#define ORC_E_NOMEM -6

#define MAXD 21
#define NSYM 255

enum { K_EMB = 1, K_DOWN, K_CONV1, K_CONV2, K_SKIP, K_UP, K_FC1, K_FC2 };

/* ------------------------------------------------------------------------ */
/* Morton keys (Sec. S3.2 "Coordinate Sampling"): bit 3b+2 of the key is    */
/* bit b of x, bit 3b+1 is y, bit 3b is z, so the three low bits of a key   */
/* are the child slot o = 4(x&1) + 2(y&1) + (z&1) within its parent.        */
/* ------------------------------------------------------------------------ */
static uint64_t morton_encode(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint64_t k = 0;
    for (int b = 0; b < bits; b++) {
        k |= (uint64_t)((x >> b) & 1u) << (3 * b + 2);
        k |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
        k |= (uint64_t)((z >> b) & 1u) << (3 * b);
    }
    return k;
}

static void morton_decode(uint64_t k, int bits, int64_t *x, int64_t *y, int64_t *z)
{
    int64_t X = 0, Y = 0, Z = 0;
    for (int b = 0; b < bits; b++) {
        X |= (int64_t)((k >> (3 * b + 2)) & 1u) << b;
        Y |= (int64_t)((k >> (3 * b + 1)) & 1u) << b;
        Z |= (int64_t)((k >> (3 * b)) & 1u) << b;
    }
    *x = X; *y = Y; *z = Z;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* Octree (Sec. S3.2): sort in Morton order, then repeatedly halve the      */
/* coordinates (key >> 3) and drop consecutive duplicates.  The occupancy   */
/* code of a node sets bit o for every occupied child slot o (the fixed     */
/* 2x2x2 stride-2 convolution over an all-ones input).                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int D;
    int64_t N[MAXD + 1];
    uint64_t *key[MAXD + 1];  /* V_d, ascending */
    uint8_t *code[MAXD];      /* X_d in [1,255] */
} octree_t;

static void octree_free(octree_t *T)
{
    for (int d = 0; d <= MAXD; d++) { free(T->key[d]); T->key[d] = NULL; }
    for (int d = 0; d < MAXD; d++) { free(T->code[d]); T->code[d] = NULL; }
}

static int octree_build(const int32_t *xyz, int64_t n, int D, octree_t *T)
{
    memset(T, 0, sizeof(*T));
    T->D = D;
    int64_t side = (int64_t)1 << D;
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++)
            if (xyz[3 * i + a] < 0 || xyz[3 * i + a] >= side) return ORC_E_INVAL;
    uint64_t *k = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    if (!k) return ORC_E_NOMEM;
    for (int64_t i = 0; i < n; i++)
        k[i] = morton_encode((uint32_t)xyz[3 * i], (uint32_t)xyz[3 * i + 1], (uint32_t)xyz[3 * i + 2], D);
    qsort(k, (size_t)n, sizeof(uint64_t), cmp_u64);
    int64_t u = 0;
    for (int64_t i = 0; i < n; i++)
        if (u == 0 || k[i] != k[u - 1]) k[u++] = k[i];
    T->key[D] = k;
    T->N[D] = u;
    for (int d = D - 1; d >= 0; d--) {
        int64_t Nc = T->N[d + 1];
        uint64_t *pk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(Nc > 0 ? Nc : 1));
        uint8_t *pc = (uint8_t *)calloc((size_t)(Nc > 0 ? Nc : 1), 1);
        if (!pk || !pc) { free(pk); free(pc); return ORC_E_NOMEM; }
        int64_t m = 0;
        for (int64_t i = 0; i < Nc; i++) {
            uint64_t parent = T->key[d + 1][i] >> 3;
            if (m == 0 || pk[m - 1] != parent) pk[m++] = parent;
            pc[m - 1] |= (uint8_t)(1u << (T->key[d + 1][i] & 7u));
        }
        T->key[d] = pk;
        T->code[d] = pc;
        T->N[d] = m;
    }
    return ORC_OK;
}

/* first child row in V_{d+1} of every node of V_d, plus a sentinel */
static int64_t *child_starts(const octree_t *T, int d)
{
    int64_t N = T->N[d];
    int64_t *cs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    if (!cs) return NULL;
    int64_t r = 0;
    for (int64_t p = 0; p < N; p++) {
        cs[p] = r;
        for (int o = 0; o < 8; o++)
            if (T->code[d][p] & (1u << o)) r++;
    }
    cs[N] = r;
    return cs;
}

/* ------------------------------------------------------------------------ */
/* 3x3x3 neighbourhood of every node of V_j (the occupied-neighbour         */
/* statistic of Sec. 1 and the sparse convolutions of Sec. 3.3): row of the */
/* neighbour at offset (dx,dy,dz), tap index 9(dx+1)+3(dy+1)+(dz+1), or -1  */
/* when that voxel is empty or outside [0, 2^j)^3.  Plain binary search.    */
/* ------------------------------------------------------------------------ */
static int64_t find_key(const uint64_t *keys, int64_t N, uint64_t k)
{
    int64_t lo = 0, hi = N - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] == k) return mid;
        if (keys[mid] < k) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static void kernel_map(const uint64_t *keys, int64_t N, int j, int32_t *nbr)
{
    int64_t side = (int64_t)1 << j;
    for (int64_t i = 0; i < N; i++) {
        int64_t x, y, z;
        morton_decode(keys[i], j, &x, &y, &z);
        for (int dx = -1; dx <= 1; dx++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dz = -1; dz <= 1; dz++) {
                    int t = 9 * (dx + 1) + 3 * (dy + 1) + (dz + 1);
                    int64_t X = x + dx, Y = y + dy, Z = z + dz;
                    int64_t r = -1;
                    if (X >= 0 && X < side && Y >= 0 && Y < side && Z >= 0 && Z < side)
                        r = find_key(keys, N, morton_encode((uint32_t)X, (uint32_t)Y, (uint32_t)Z, j));
                    nbr[27 * i + t] = (int32_t)r;
                }
    }
}

/* ------------------------------------------------------------------------ */
/* Weight blob                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind, depth, j, taps, cin, cout;
    int64_t m_pos, m_neg;
    int r, z_in, z_out;
    const int32_t *bias;
    const int8_t *W;  /* [taps][cin][cout] */
    int own;          /* the weights are stored in this layer's record */
} layer_t;

typedef struct {
    int C, D, n_deep, k0;
    int xfp;  /* 1: cross-scale feature propagation (blob version 1); 0: the ablation without it (version 2) */
    uint32_t blob_id;
    int n_layers;
    layer_t *L;
    int first[MAXD + 1];
} model_t;

static uint32_t fnv1a32(const uint8_t *p, size_t n)
{
    uint32_t h = 2166136261u;
    for (size_t i = 0; i < n; i++) { h ^= p[i]; h *= 16777619u; }
    return h;
}

static uint32_t rd32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

/* expected (kind, j, taps, cin, cout) sequence of one coded depth; without */
/* cross-scale propagation (xfp = 0) a shallow depth first embeds X_{d-1}   */
/* and the deep ResBlock reads G alone (C -> C, identity skip)              */
static int expected_layers(int C, int D, int n_deep, int xfp, int d, int out[][5])
{
    int k0 = D - n_deep - 1, n = 0;
    if (d >= 1 && d <= k0) {
        if (!xfp) { int e[5] = {K_EMB, d - 1, 1, 8, C}; memcpy(out[n++], e, sizeof(e)); }
        int a[3][5] = {{K_CONV1, 0, 27, C, C}, {K_CONV2, 0, 27, C, C}, {K_UP, d - 1, 1, C + 8, 8 * C}};
        for (int i = 0; i < 3; i++) memcpy(out[n++], a[i], sizeof(a[i]));
    } else if (d > k0) {
        int e[5] = {K_EMB, d - 1, 1, 8, C};
        memcpy(out[n++], e, sizeof(e));
        for (int j = d - 1; j > k0; j--) { int t[5] = {K_DOWN, j, 8, C, C}; memcpy(out[n++], t, sizeof(t)); }
        int cin = xfp ? 2 * C : C;
        int r1[5] = {K_CONV1, k0, 27, cin, C}, r2[5] = {K_CONV2, k0, 27, C, C}, sk[5] = {K_SKIP, k0, 1, 2 * C, C};
        memcpy(out[n++], r1, sizeof(r1)); memcpy(out[n++], r2, sizeof(r2));
        if (xfp) memcpy(out[n++], sk, sizeof(sk));
        for (int j = k0; j < d; j++) { int t[5] = {K_UP, j, 1, C + 8, 8 * C}; memcpy(out[n++], t, sizeof(t)); }
    }
    int f1[5] = {K_FC1, d, 1, C, C}, f2[5] = {K_FC2, d, 1, C, NSYM};
    memcpy(out[n++], f1, sizeof(f1)); memcpy(out[n++], f2, sizeof(f2));
    return n;
}

static void model_free(model_t *M) { free(M->L); M->L = NULL; }

static int model_parse(const uint8_t *b, size_t len, model_t *M)
{
    memset(M, 0, sizeof(*M));
    if (!b || len < 32 || rd32(b) != 0x5743504Cu) return ORC_E_MODEL;
    uint32_t ver = rd32(b + 4);
    if (((ver & 0xFFu) != 1 && (ver & 0xFFu) != 2) || (ver & ~0x1FFu)) return ORC_E_MODEL;
    /* version flag 0x100: level-aware parameter sharing (the future work of  */
    /* Sec. S2, last paragraph; reading in the design notes): each record     */
    /* names the layer whose weights it uses, and only that layer stores them */
    int shared = (ver & 0x100u) != 0;
    M->xfp = (ver & 0xFFu) == 1;
    M->C = (int)rd32(b + 8); M->D = (int)rd32(b + 12); M->n_deep = (int)rd32(b + 16);
    M->n_layers = (int)rd32(b + 20);
    if (M->C < 1 || M->C > 256 || M->D < 1 || M->D > MAXD || M->n_deep < 0 || M->n_deep > M->D - 1)
        return ORC_E_MODEL;
    M->k0 = M->D - M->n_deep - 1;
    M->blob_id = fnv1a32(b, len);
    M->L = (layer_t *)calloc((size_t)(M->n_layers > 0 ? M->n_layers : 1), sizeof(layer_t));
    if (!M->L) return ORC_E_NOMEM;
    size_t off = 32;
    int li = 0;
    int exp[64][5];
    for (int d = 0; d < M->D; d++) {
        M->first[d] = li;
        int ne = expected_layers(M->C, M->D, M->n_deep, M->xfp, d, exp);
        for (int e = 0; e < ne; e++, li++) {
            if (li >= M->n_layers || off + 44 > len) goto bad;
            layer_t *L = &M->L[li];
            L->kind = (int)rd32(b + off); L->depth = (int)rd32(b + off + 4); L->j = (int)rd32(b + off + 8);
            L->taps = (int)rd32(b + off + 12); L->cin = (int)rd32(b + off + 16); L->cout = (int)rd32(b + off + 20);
            L->m_pos = (int32_t)rd32(b + off + 24); L->m_neg = (int32_t)rd32(b + off + 28);
            L->r = (int)rd32(b + off + 32); L->z_in = (int32_t)rd32(b + off + 36); L->z_out = (int32_t)rd32(b + off + 40);
            if (L->kind != exp[e][0] || L->depth != d || L->j != exp[e][1] || L->taps != exp[e][2] ||
                L->cin != exp[e][3] || L->cout != exp[e][4]) goto bad;
            if (L->m_pos < 0 || L->m_neg < 0 || L->r < 0 || L->r > 62 || L->z_in < -128 || L->z_in > 127 ||
                L->z_out < -128 || L->z_out > 127) goto bad;
            off += 44;
            int owner = li;
            if (shared) {
                if (off + 4 > len) goto bad;
                owner = (int)rd32(b + off);
                off += 4;
                if (owner < 0 || owner > li) goto bad;
            }
            size_t nb = (size_t)L->cout * 4, nw = owner == li ? (size_t)L->taps * L->cin * L->cout : 0;
            if (off + nb + nw > len) goto bad;
            L->bias = (const int32_t *)(b + off);
            for (int o = 0; o < L->cout; o++) {
                int32_t v = (int32_t)rd32(b + off + 4 * (size_t)o);
                if (v <= -(1 << 24) || v >= (1 << 24)) goto bad;
            }
            off += nb;
            if (owner == li) {
                L->W = (const int8_t *)(b + off);
                L->own = 1;
            } else {
                /* the weights of an earlier layer of the same shape that owns them */
                const layer_t *O = &M->L[owner];
                if (!O->own || O->taps != L->taps || O->cin != L->cin || O->cout != L->cout) goto bad;
                L->W = O->W;
            }
            off += nw;
            off = (off + 3) & ~(size_t)3;
        }
    }
    M->first[M->D] = li;
    if (li != M->n_layers || off != len) goto bad;
    return ORC_OK;
bad:
    model_free(M);
    return ORC_E_MODEL;
}

/* ------------------------------------------------------------------------ */
/* Requantisation, Eq. 14: clip(round(acc * m / 2^r) + z_y, -128, 127).     */
/* Rounding is half up (add 2^(r-1), then floor).  The activation is folded */
/* into the multiplier: m = m_pos for acc >= 0 and m_neg otherwise (ReLU:   */
/* m_neg = 0, identity: m_neg = m_pos, PReLU: the slope times m_pos).       */
/* ------------------------------------------------------------------------ */
static int64_t floor_div_pow2(int64_t v, int r)
{
    int64_t q = v / ((int64_t)1 << r);            /* truncates toward zero */
    if (v < 0 && q * ((int64_t)1 << r) != v) q -= 1;
    return q;
}

static int8_t requant(int64_t acc, const layer_t *L)
{
    int64_t m = acc >= 0 ? L->m_pos : L->m_neg;
    int64_t p = acc * m;
    int64_t q = L->r > 0 ? floor_div_pow2(p + ((int64_t)1 << (L->r - 1)), L->r) : p;
    q += L->z_out;
    if (q < -128) q = -128;
    if (q > 127) q = 127;
    return (int8_t)q;
}

static int8_t clamp8(int64_t v) { return (int8_t)(v < -128 ? -128 : (v > 127 ? 127 : v)); }

/* accumulator of Eq. 13 must fit int32 (32-bit accumulation) */
static int acc_ok(int64_t a) { return a >= INT32_MIN && a <= INT32_MAX; }

/* Dense integer linear layer, Eq. 13 (weights symmetric, z_w = 0). */
static int linear(const layer_t *L, const int8_t *x, int64_t rows, int8_t *y)
{
    for (int64_t i = 0; i < rows; i++)
        for (int o = 0; o < L->cout; o++) {
            int64_t acc = L->bias[o];
            for (int c = 0; c < L->cin; c++)
                acc += (int64_t)(x[i * L->cin + c] - L->z_in) * L->W[(size_t)c * L->cout + o];
            if (!acc_ok(acc)) return ORC_E_MODEL;
            y[i * L->cout + o] = requant(acc, L);
        }
    return ORC_OK;
}

/* Submanifold 3x3x3 sparse convolution as indexed linear transforms        */
/* (Sec. 3.3): outputs only at occupied sites; an empty neighbour adds      */
/* nothing (the zero padding of the re-densified map, Sec. 3.1).            */
static int conv3(const layer_t *L, const int8_t *x, const int32_t *nbr, int64_t rows, int8_t *y)
{
    for (int64_t i = 0; i < rows; i++)
        for (int o = 0; o < L->cout; o++) {
            int64_t acc = L->bias[o];
            for (int t = 0; t < 27; t++) {
                int32_t r = nbr[27 * i + t];
                if (r < 0) continue;
                for (int c = 0; c < L->cin; c++)
                    acc += (int64_t)(x[(int64_t)r * L->cin + c] - L->z_in) *
                           L->W[((size_t)t * L->cin + c) * L->cout + o];
            }
            if (!acc_ok(acc)) return ORC_E_MODEL;
            y[i * L->cout + o] = requant(acc, L);
        }
    return ORC_OK;
}

/* Kernel-2 stride-2 sparse convolution from depth j to depth j-1 (the      */
/* Downsampling of Eq. 4): a parent sums its occupied children, each child  */
/* with the weight slice of its slot o.                                     */
static int down_k2s2(const layer_t *L, const int8_t *x, const uint64_t *ckeys, const int64_t *cs,
                     int64_t parents, int8_t *y)
{
    for (int64_t q = 0; q < parents; q++)
        for (int o = 0; o < L->cout; o++) {
            int64_t acc = L->bias[o];
            for (int64_t c = cs[q]; c < cs[q + 1]; c++) {
                int slot = (int)(ckeys[c] & 7u);
                for (int ch = 0; ch < L->cin; ch++)
                    acc += (int64_t)(x[c * L->cin + ch] - L->z_in) * L->W[((size_t)slot * L->cin + ch) * L->cout + o];
            }
            if (!acc_ok(acc)) return ORC_E_MODEL;
            y[q * L->cout + o] = requant(acc, L);
        }
    return ORC_OK;
}

/* bits(X): the 8 occupancy bits as int8 channels, 127 where set (the       */
/* occupancy channels of Concat(., X), Eq. 9 and 11).                       */
static void code_bits(uint8_t code, int8_t *out)
{
    for (int o = 0; o < 8; o++) out[o] = (code >> o) & 1u ? 127 : 0;
}

/* Upsampling + Pruning (Eq. 6/9/11): Linear(C+8 -> 8C) + PReLU over        */
/* [Z | bits(X)], output block o belongs to child slot o; only occupied     */
/* children are kept, parents in order and slots ascending, which is the    */
/* Morton order of the next depth (Sec. S3.2).                              */
static int up_prune(const layer_t *L, int C, const int8_t *Z, const uint8_t *code, int64_t parents,
                    int8_t *y, int64_t *rows_out)
{
    int8_t in[512 + 8];
    int64_t r = 0;
    for (int64_t p = 0; p < parents; p++) {
        memcpy(in, Z + p * C, (size_t)C);
        code_bits(code[p], in + C);
        for (int o = 0; o < 8; o++) {
            if (!(code[p] & (1u << o))) continue;
            for (int oc = 0; oc < C; oc++) {
                int col = o * C + oc;
                int64_t acc = L->bias[col];
                for (int c = 0; c < C + 8; c++)
                    acc += (int64_t)(in[c] - L->z_in) * L->W[(size_t)c * L->cout + col];
                if (!acc_ok(acc)) return ORC_E_MODEL;
                y[r * C + oc] = requant(acc, L);
            }
            r++;
        }
    }
    *rows_out = r;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Integer softmax (Eq. 15) and the coder's frequency table.                */
/* The exponent table covers only the non-positive domain max - l_i >= 0;  */
/* one logit unit is 1/16 nat, so E[i] = round(2^15 e^{-i/16}).             */
/* ------------------------------------------------------------------------ */
static int32_t LUT[256];
static int lut_ready = 0;

static void lut_init(void)
{
    if (lut_ready) return;
    for (int i = 0; i < 256; i++) LUT[i] = (int32_t)floor(32768.0 * exp(-(double)i / 16.0) + 0.5);
    lut_ready = 1;
}

/* Frequencies f_s >= 1 summing to exactly 2^16:                            */
/*   E_i = LUT[M - l_i],  S = sum E_i,  f_i = 1 + floor(E_i * 65281 / S),    */
/*   the remainder 65536 - sum f goes to the lowest index holding max l.    */
/* CDF: cdf[0] = 0, cdf[s+1] = cdf[s] + f_s, cdf[255] = 65536.              */
static void logits_to_cdf(const int8_t *l, int32_t *cdf)
{
    lut_init();
    int M = -128, arg = 0;
    for (int i = 0; i < NSYM; i++)
        if (l[i] > M) { M = l[i]; arg = i; }
    int64_t S = 0, E[NSYM];
    for (int i = 0; i < NSYM; i++) { E[i] = LUT[M - l[i]]; S += E[i]; }
    int64_t f[NSYM], tot = 0;
    for (int i = 0; i < NSYM; i++) { f[i] = 1 + (E[i] * 65281) / S; tot += f[i]; }
    f[arg] += 65536 - tot;
    cdf[0] = 0;
    for (int i = 0; i < NSYM; i++) cdf[i + 1] = cdf[i] + (int32_t)f[i];
}

/* Base geometry (Sec. S2, "Detailed Model Structure", last paragraph: the  */
/* levels that are not modelled are coded directly from the frequencies of  */
/* their symbols).  For a depth d < B the counts n_s of its occupancy codes */
/* give the frequencies by the same rule as the softmax above, with the     */
/* counts in place of the exponentials:                                     */
/*   N = sum n_s, f_s = 1 + floor(n_s * 65281 / N), the remainder goes to   */
/*   the lowest index holding max n.  Every f_s >= 1, total exactly 2^16.   */
static void counts_to_cdf(const uint32_t *n, int32_t *cdf)
{
    int64_t N = 0;
    int arg = 0;
    for (int i = 0; i < NSYM; i++) {
        N += n[i];
        if (n[i] > n[arg]) arg = i;
    }
    int64_t f[NSYM], tot = 0;
    for (int i = 0; i < NSYM; i++) { f[i] = 1 + ((int64_t)n[i] * 65281) / (N > 0 ? N : 1); tot += f[i]; }
    f[arg] += 65536 - tot;
    cdf[0] = 0;
    for (int i = 0; i < NSYM; i++) cdf[i + 1] = cdf[i] + (int32_t)f[i];
}

/* ------------------------------------------------------------------------ */
/* Model: features F_d for coded depth d (Sec. 3.1-3.2, Eq. 4-11).          */
/*   d = B        : F_B = 0 (the first modelled depth has no coarser        */
/*                  context; B = 0 models every depth from the root)        */
/*   B < d <= k0  : S = ResBlock(F_{d-1}) on V_{d-1};                       */
/*                  F_d = Prune(Up([S | bits(X_{d-1})]), X_{d-1})           */
/*   d > k0       : G = Down(X_{d-1}) at depth k0;                          */
/*                  H = ResBlock([F_k0 | G]) on V_k0;                       */
/*                  Z_k0 = H, Z_{j+1} = Prune(Up([Z_j | bits(X_j)]), X_j)   */
/*                  for j = k0 .. d-1; F_d = Z_d.                           */
/* ResBlock(x) = clamp(rq(conv2(relu-rq(conv1(x)))) + skip(x)), skip = x    */
/* when the widths agree, else a requantised 2C -> C linear layer.          */
/* Without cross-scale propagation (the ablation of Sec. 4.4, Table 4;     */
/* blob version 2) nothing is carried from F_{d-1} or F_k0:                 */
/*   B < d <= k0  : E = Emb(bits(X_{d-1})) on V_{d-1}, S = ResBlock(E);     */
/*                  F_d = Prune(Up([S | bits(X_{d-1})]), X_{d-1})           */
/*   d > k0       : H = ResBlock(G) on V_k0 (identity skip), then as above. */
/* With n_deep = 0 (no re-densified depth) this is the ablation baseline.   */
/* ------------------------------------------------------------------------ */
static int resblock(const model_t *M, const layer_t *c1, const layer_t *c2, const layer_t *sk,
                    const octree_t *T, int j, const int8_t *x, int8_t *out)
{
    int C = M->C;
    int64_t N = T->N[j];
    int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * 27 * (size_t)(N > 0 ? N : 1));
    int8_t *h = (int8_t *)malloc((size_t)(N > 0 ? N : 1) * C);
    int8_t *y = (int8_t *)malloc((size_t)(N > 0 ? N : 1) * C);
    int8_t *s = (int8_t *)malloc((size_t)(N > 0 ? N : 1) * C);
    int st = ORC_E_NOMEM;
    if (!nbr || !h || !y || !s) goto done;
    kernel_map(T->key[j], N, j, nbr);
    if ((st = conv3(c1, x, nbr, N, h)) != ORC_OK) goto done;
    if ((st = conv3(c2, h, nbr, N, y)) != ORC_OK) goto done;
    if (sk) {
        if ((st = linear(sk, x, N, s)) != ORC_OK) goto done;
    } else {
        memcpy(s, x, (size_t)N * C);
    }
    for (int64_t i = 0; i < N * C; i++) out[i] = clamp8((int64_t)y[i] + s[i]);
    st = ORC_OK;
done:
    free(nbr); free(h); free(y); free(s);
    return st;
}

/* F_d into *F (malloc'ed N_d x C).  Needs V_0..V_d, X_0..X_{d-1},          */
/* F_{d-1} (shallow) and F_k0 (deep): only already-coded data (Sec. 3.1).   */
static int features(const model_t *M, const octree_t *T, int d, int B, const int8_t *F_prev,
                    const int8_t *F_k0, int8_t **F)
{
    int C = M->C, k0 = M->k0;
    int64_t Nd = T->N[d];
    *F = NULL;
    int8_t *out = (int8_t *)calloc((size_t)(Nd > 0 ? Nd : 1) * C, 1);
    if (!out) return ORC_E_NOMEM;
    if (d == B) { *F = out; return ORC_OK; }
    const layer_t *L = &M->L[M->first[d]];
    int st = ORC_OK;
    if (d <= k0) {
        int64_t Np = T->N[d - 1], rows;
        int8_t *S = (int8_t *)malloc((size_t)(Np > 0 ? Np : 1) * C);
        if (!S) { free(out); return ORC_E_NOMEM; }
        int li = 0;
        const int8_t *x = F_prev;
        int8_t *E = NULL;
        if (!M->xfp) {
            /* the ResBlock input is the embedding of the parent codes */
            int8_t *bits = (int8_t *)malloc((size_t)(Np > 0 ? Np : 1) * 8);
            E = (int8_t *)malloc((size_t)(Np > 0 ? Np : 1) * C);
            if (!bits || !E) { free(bits); free(E); free(S); free(out); return ORC_E_NOMEM; }
            for (int64_t i = 0; i < Np; i++) code_bits(T->code[d - 1][i], bits + 8 * i);
            st = linear(&L[li++], bits, Np, E);
            free(bits);
            x = E;
        }
        if (st == ORC_OK) st = resblock(M, &L[li], &L[li + 1], NULL, T, d - 1, x, S);
        if (st == ORC_OK) st = up_prune(&L[li + 2], C, S, T->code[d - 1], Np, out, &rows);
        if (st == ORC_OK && rows != Nd) st = ORC_E_CORRUPT;
        free(S);
        free(E);
    } else {
        /* Down: embed bits(X_{d-1}) at depth d-1, then k2s2 steps to k0 */
        int li = 0;
        const layer_t *emb = &L[li++];
        int64_t Ne = T->N[d - 1];
        int8_t *bits = (int8_t *)malloc((size_t)(Ne > 0 ? Ne : 1) * 8);
        int8_t *G = (int8_t *)malloc((size_t)(Ne > 0 ? Ne : 1) * C);
        if (!bits || !G) { free(bits); free(G); free(out); return ORC_E_NOMEM; }
        for (int64_t i = 0; i < Ne; i++) code_bits(T->code[d - 1][i], bits + 8 * i);
        st = linear(emb, bits, Ne, G);
        free(bits);
        for (int j = d - 1; j > k0 && st == ORC_OK; j--) {
            const layer_t *dn = &L[li++];
            int64_t *cs = child_starts(T, j - 1);
            int8_t *G2 = (int8_t *)malloc((size_t)(T->N[j - 1] > 0 ? T->N[j - 1] : 1) * C);
            if (!cs || !G2) { free(cs); free(G2); st = ORC_E_NOMEM; break; }
            st = down_k2s2(dn, G, T->key[j], cs, T->N[j - 1], G2);
            free(cs); free(G); G = G2;
        }
        /* ResBlock on [F_k0 | G] at depth k0 (on G alone without propagation) */
        int64_t Nk = T->N[k0];
        int8_t *cat = (int8_t *)malloc((size_t)(Nk > 0 ? Nk : 1) * 2 * C);
        int8_t *Z = (int8_t *)malloc((size_t)(Nk > 0 ? Nk : 1) * C);
        if (st == ORC_OK && (!cat || !Z)) st = ORC_E_NOMEM;
        if (st == ORC_OK && M->xfp) {
            for (int64_t i = 0; i < Nk; i++) {
                memcpy(cat + i * 2 * C, F_k0 + i * C, (size_t)C);
                memcpy(cat + i * 2 * C + C, G + i * C, (size_t)C);
            }
            st = resblock(M, &L[li], &L[li + 1], &L[li + 2], T, k0, cat, Z);
            li += 3;
        } else if (st == ORC_OK) {
            st = resblock(M, &L[li], &L[li + 1], NULL, T, k0, G, Z);
            li += 2;
        }
        free(G); free(cat);
        /* Re-sparsification: upsample and prune from k0 to d */
        for (int j = k0; j < d && st == ORC_OK; j++) {
            int64_t rows;
            int8_t *Z2 = (int8_t *)malloc((size_t)(T->N[j + 1] > 0 ? T->N[j + 1] : 1) * C);
            if (!Z2) { st = ORC_E_NOMEM; break; }
            st = up_prune(&L[li++], C, Z, T->code[j], T->N[j], Z2, &rows);
            if (st == ORC_OK && rows != T->N[j + 1]) st = ORC_E_CORRUPT;
            free(Z); Z = Z2;
        }
        if (st == ORC_OK) memcpy(out, Z, (size_t)Nd * C);
        free(Z);
    }
    if (st != ORC_OK) { free(out); return st; }
    *F = out;
    return ORC_OK;
}

/* Predictor (Eq. 7): two-layer MLP, C -> C (ReLU) -> 255 int8 logits. */
static int predict_logits(const model_t *M, int d, const int8_t *F, int64_t N, int8_t *logits)
{
    const layer_t *L = &M->L[M->first[d + 1] - 2];
    int8_t *h = (int8_t *)malloc((size_t)(N > 0 ? N : 1) * M->C);
    if (!h) return ORC_E_NOMEM;
    int st = linear(&L[0], F, N, h);
    if (st == ORC_OK) st = linear(&L[1], h, N, logits);
    free(h);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Range coder: G. N. N. Martin (1979), byte-oriented with a cache byte and */
/* carry propagation; 32-bit range, 16-bit totals.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t low;
    uint32_t range;
    uint8_t cache;
    uint64_t pending;
    uint8_t *out;
    size_t cap, len;
} rc_enc_t;

static void rc_put(rc_enc_t *e, uint8_t b)
{
    if (e->len < e->cap) e->out[e->len] = b;
    e->len++;
}

static void rc_shift_low(rc_enc_t *e)
{
    if (e->low < 0xFF000000ull || e->low >= 0x100000000ull) {
        uint8_t carry = (uint8_t)(e->low >> 32);
        rc_put(e, (uint8_t)(e->cache + carry));
        for (; e->pending > 1; e->pending--) rc_put(e, (uint8_t)(0xFF + carry));
        e->pending = 0;
        e->cache = (uint8_t)((e->low >> 24) & 0xFF);
    }
    e->pending++;
    e->low = (e->low & 0x00FFFFFFull) << 8;
}

static void rc_enc_init(rc_enc_t *e, uint8_t *out, size_t cap)
{
    e->low = 0; e->range = 0xFFFFFFFFu; e->cache = 0; e->pending = 1;
    e->out = out; e->cap = cap; e->len = 0;
}

static void rc_encode(rc_enc_t *e, uint32_t start, uint32_t freq)
{
    uint32_t r = e->range >> 16;
    e->low += (uint64_t)r * start;
    e->range = r * freq;
    while (e->range < (1u << 24)) { e->range <<= 8; rc_shift_low(e); }
}

static void rc_flush(rc_enc_t *e)
{
    for (int i = 0; i < 5; i++) rc_shift_low(e);
}

typedef struct {
    uint32_t range, code;
    const uint8_t *in;
    size_t len, pos;
} rc_dec_t;

static uint8_t rc_byte(rc_dec_t *dd) { return dd->pos < dd->len ? dd->in[dd->pos++] : (dd->pos++, 0); }

static void rc_dec_init(rc_dec_t *dd, const uint8_t *in, size_t len)
{
    dd->in = in; dd->len = len; dd->pos = 0; dd->range = 0xFFFFFFFFu; dd->code = 0;
    for (int i = 0; i < 5; i++) dd->code = (dd->code << 8) | rc_byte(dd);
}

/* symbol s with r*cdf[s] <= code < r*cdf[s+1]; -1 if the stream is corrupt */
static int rc_decode(rc_dec_t *dd, const int32_t *cdf)
{
    uint32_t r = dd->range >> 16;
    if ((uint64_t)dd->code >= (uint64_t)r * 65536u) return -1;
    int s = 0;
    for (int t = 0; t < NSYM; t++)
        if ((uint64_t)r * (uint32_t)cdf[t] <= dd->code) s = t;
    dd->code -= r * (uint32_t)cdf[s];
    dd->range = r * (uint32_t)(cdf[s + 1] - cdf[s]);
    while (dd->range < (1u << 24)) { dd->code = (dd->code << 8) | rc_byte(dd); dd->range <<= 8; }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Bitstream (little-endian):                                               */
/*   u32 'LPC1', u8 version (1, or 2 with base geometry), u8 D, u8 n_deep,  */
/*   u8 c, u32 blob_id, u32 N_D, u32 N_d (d = 0..D-1);                      */
/*   version 2 only: u8 B, then for d = 0..B-1 u8 m and m pairs             */
/*   (u8 code, u32 count), codes ascending, counts >= 1 summing to N_d;     */
/*   u16 chunk length for each chunk (depth ascending, chunk ascending),    */
/*   then the chunk payloads.                                               */
/* Chunk k of depth d codes nodes [k 2^c, min((k+1) 2^c, N_d)).             */
/* ------------------------------------------------------------------------ */
static void wr32(uint8_t *p, uint32_t v) { p[0] = v & 0xFF; p[1] = (v >> 8) & 0xFF; p[2] = (v >> 16) & 0xFF; p[3] = v >> 24; }
static int64_t nchunks(int64_t N, int c) { return (N + ((int64_t)1 << c) - 1) >> c; }

/* ======================================================================== */
/* Exported entry points                                                    */
/* ======================================================================== */

int orc_lut(int32_t *out)
{
    lut_init();
    memcpy(out, LUT, sizeof(LUT));
    return ORC_OK;
}

int orc_morton(const int32_t *xyz, int64_t n, int bits, uint64_t *keys)
{
    for (int64_t i = 0; i < n; i++)
        keys[i] = morton_encode((uint32_t)xyz[3 * i], (uint32_t)xyz[3 * i + 1], (uint32_t)xyz[3 * i + 2], bits);
    return ORC_OK;
}

/* counts[D+1]; keys (concatenated V_0..V_D) and codes (X_0..X_{D-1}) may be NULL to query sizes */
int orc_octree(const int32_t *xyz, int64_t n, int D, int64_t *counts, uint64_t *keys, uint8_t *codes)
{
    if (D < 1 || D > MAXD || n < 0) return ORC_E_INVAL;
    octree_t T;
    int st = octree_build(xyz, n, D, &T);
    if (st != ORC_OK) { octree_free(&T); return st; }
    int64_t ko = 0, co = 0;
    for (int d = 0; d <= D; d++) {
        counts[d] = T.N[d];
        if (keys) memcpy(keys + ko, T.key[d], sizeof(uint64_t) * (size_t)T.N[d]);
        if (codes && d < D) memcpy(codes + co, T.code[d], (size_t)T.N[d]);
        ko += T.N[d];
        if (d < D) co += T.N[d];
    }
    octree_free(&T);
    return ORC_OK;
}

int orc_kernel_map(const uint64_t *keys, int64_t N, int j, int32_t *nbr)
{
    kernel_map(keys, N, j, nbr);
    return ORC_OK;
}

/* one requantisation (Eq. 14) with explicit parameters */
int orc_requant(const int64_t *acc, int64_t n, int32_t m_pos, int32_t m_neg, int r, int z_out, int8_t *out)
{
    layer_t L;
    memset(&L, 0, sizeof(L));
    L.m_pos = m_pos; L.m_neg = m_neg; L.r = r; L.z_out = z_out;
    for (int64_t i = 0; i < n; i++) out[i] = requant(acc[i], &L);
    return ORC_OK;
}

/* submanifold conv of one layer given as raw arrays (W: [27][cin][cout]) */
int orc_conv3(const int8_t *x, const int32_t *nbr, int64_t rows, int cin, int cout, const int8_t *W,
              const int32_t *bias, int32_t m_pos, int32_t m_neg, int r, int z_in, int z_out, int8_t *y)
{
    layer_t L;
    memset(&L, 0, sizeof(L));
    L.taps = 27; L.cin = cin; L.cout = cout; L.W = W; L.bias = bias;
    L.m_pos = m_pos; L.m_neg = m_neg; L.r = r; L.z_in = z_in; L.z_out = z_out;
    return conv3(&L, x, nbr, rows, y);
}

int orc_counts_to_cdf(const uint32_t *counts, int32_t *cdf)
{
    counts_to_cdf(counts, cdf);
    return ORC_OK;
}

int orc_logits_to_cdf(const int8_t *logits, int64_t n, int32_t *cdf)
{
    for (int64_t i = 0; i < n; i++) logits_to_cdf(logits + i * NSYM, cdf + i * 256);
    return ORC_OK;
}

/* one range-coded chunk of symbols with the given CDF rows (n x 256) */
int orc_rc_encode(const int32_t *sym, const int32_t *cdf, int64_t n, uint8_t *out, size_t cap, size_t *len)
{
    rc_enc_t e;
    rc_enc_init(&e, out, cap);
    for (int64_t i = 0; i < n; i++) {
        const int32_t *c = cdf + i * 256;
        if (sym[i] < 0 || sym[i] >= NSYM) return ORC_E_INVAL;
        rc_encode(&e, (uint32_t)c[sym[i]], (uint32_t)(c[sym[i] + 1] - c[sym[i]]));
    }
    rc_flush(&e);
    *len = e.len;
    return e.len > cap ? ORC_E_CAPACITY : ORC_OK;
}

int orc_rc_decode(const uint8_t *in, size_t len, const int32_t *cdf, int64_t n, int32_t *sym)
{
    rc_dec_t dd;
    rc_dec_init(&dd, in, len);
    for (int64_t i = 0; i < n; i++) {
        int s = rc_decode(&dd, cdf + i * 256);
        if (s < 0) return ORC_E_CORRUPT;
        sym[i] = s;
    }
    return ORC_OK;
}

int orc_model_info(const void *blob, size_t len, int *C, int *D, int *n_deep, uint32_t *blob_id)
{
    model_t M;
    int st = model_parse((const uint8_t *)blob, len, &M);
    if (st != ORC_OK) return st;
    *C = M.C; *D = M.D; *n_deep = M.n_deep; *blob_id = M.blob_id;
    model_free(&M);
    return ORC_OK;
}

/* Run the model over a fully known octree and hand each depth's CDF rows  */
/* (or logits/features) to a callback-free sink selected by `what`.         */
/* what: 0 = CDF int32 [N_d][256], 1 = logits int8 [N_d][255],              */
/*       2 = features int8 [N_d][C]                                         */
static int run_depth(const model_t *M, const octree_t *T, int level, int what, void *dst)
{
    int8_t *Fprev = NULL, *Fk0 = NULL, *F = NULL;
    int st = ORC_OK;
    for (int d = 0; d <= level && st == ORC_OK; d++) {
        /* deep depths read only F_k0; shallow ones need the chain */
        if (d > M->k0 && d < level) continue;
        st = features(M, T, d, 0, Fprev, Fk0, &F);
        if (st != ORC_OK) break;
        if (d == M->k0) {
            free(Fk0);
            Fk0 = (int8_t *)malloc((size_t)(T->N[d] > 0 ? T->N[d] : 1) * M->C);
            if (!Fk0) { st = ORC_E_NOMEM; break; }
            memcpy(Fk0, F, (size_t)T->N[d] * M->C);
        }
        if (d == level) break;
        free(Fprev);
        Fprev = F;
        F = NULL;
    }
    if (st == ORC_OK) {
        int64_t N = T->N[level];
        if (what == 2) {
            memcpy(dst, F, (size_t)N * M->C);
        } else {
            int8_t *lg = (int8_t *)malloc((size_t)(N > 0 ? N : 1) * NSYM);
            if (!lg) st = ORC_E_NOMEM;
            if (st == ORC_OK) st = predict_logits(M, level, F, N, lg);
            if (st == ORC_OK) {
                if (what == 1) memcpy(dst, lg, (size_t)N * NSYM);
                else for (int64_t i = 0; i < N; i++) logits_to_cdf(lg + i * NSYM, (int32_t *)dst + i * 256);
            }
            free(lg);
        }
    }
    free(Fprev); free(Fk0); free(F);
    return st;
}

/* what = 0 CDF, 1 logits, 2 features of depth `level` */
int orc_level_output(const void *blob, size_t blob_len, const int32_t *xyz, int64_t n, int level, int what,
                     void *out, int64_t cap, int64_t *n_nodes)
{
    model_t M;
    int st = model_parse((const uint8_t *)blob, blob_len, &M);
    if (st != ORC_OK) return st;
    if (level < 0 || level >= M.D || n < 0 || what < 0 || what > 2) { model_free(&M); return ORC_E_INVAL; }
    octree_t T;
    st = octree_build(xyz, n, M.D, &T);
    if (st == ORC_OK) {
        *n_nodes = T.N[level];
        if (T.N[level] > cap) st = ORC_E_CAPACITY;
        else if (T.N[level] > 0) st = run_depth(&M, &T, level, what, out);
    }
    octree_free(&T);
    model_free(&M);
    return st;
}

int orc_level_probs(const void *blob, size_t blob_len, const int32_t *xyz, int64_t n, int level,
                    int32_t *cdf_out, int64_t cap, int64_t *n_nodes)
{
    return orc_level_output(blob, blob_len, xyz, n, level, 0, cdf_out, cap, n_nodes);
}

/* Encode with the depths d < B coded from their own symbol counts and the  */
/* model applied from depth B on (B = 0: every depth modelled, version 1).  */
int orc_encode_base(const void *blob, size_t blob_len, const int32_t *xyz, int64_t n, int c, int B,
                    uint8_t *out, size_t cap, size_t *out_len)
{
    model_t M;
    int st = model_parse((const uint8_t *)blob, blob_len, &M);
    if (st != ORC_OK) return st;
    if (n < 0 || c < 4 || c > 14 || B < 0 || B > M.k0) { model_free(&M); return ORC_E_INVAL; }
    int D = M.D;
    octree_t T;
    st = octree_build(xyz, n, D, &T);
    if (st != ORC_OK) { octree_free(&T); model_free(&M); return st; }
    int64_t nch = 0;
    for (int d = 0; d < D; d++) nch += nchunks(T.N[d], c);
    /* symbol counts of the base depths */
    uint32_t (*cnt)[NSYM] = (uint32_t (*)[NSYM])calloc((size_t)(B > 0 ? B : 1), sizeof(uint32_t[NSYM]));
    size_t tables = 0;
    if (!cnt) st = ORC_E_NOMEM;
    for (int d = 0; d < B && st == ORC_OK; d++) {
        for (int64_t i = 0; i < T.N[d]; i++) cnt[d][T.code[d][i] - 1]++;
        tables += 1;
        for (int s2 = 0; s2 < NSYM; s2++) tables += cnt[d][s2] ? 5 : 0;
    }
    size_t pre = 16 + 4 * (size_t)D + (B > 0 ? 1 + tables : 0);
    size_t hdr = pre + 2 * (size_t)nch;
    /* the payload is built in a scratch buffer; worst case 2 bytes/symbol + 5/chunk */
    size_t worst = 0;
    for (int d = 0; d < D; d++) worst += 2 * (size_t)T.N[d];
    worst += 5 * (size_t)nch + 16;
    uint8_t *pay = (uint8_t *)malloc(worst);
    uint16_t *lens = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(nch > 0 ? nch : 1));
    int32_t *cdf = (int32_t *)malloc(sizeof(int32_t) * 256);
    if (!pay || !lens || !cdf) st = ORC_E_NOMEM;
    size_t plen = 0;
    int64_t ci = 0;
    int8_t *Fprev = NULL, *Fk0 = NULL;
    for (int d = 0; d < D && st == ORC_OK; d++) {
        int64_t N = T.N[d];
        int8_t *F = NULL, *lg = NULL;
        if (d < B) {
            counts_to_cdf(cnt[d], cdf);
        } else {
            st = features(&M, &T, d, B, Fprev, Fk0, &F);
            if (st != ORC_OK) break;
            lg = (int8_t *)malloc((size_t)(N > 0 ? N : 1) * NSYM);
            if (!lg) { free(F); st = ORC_E_NOMEM; break; }
            st = predict_logits(&M, d, F, N, lg);
        }
        for (int64_t k = 0; k < nchunks(N, c) && st == ORC_OK; k++) {
            int64_t a = k << c, b = a + ((int64_t)1 << c) < N ? a + ((int64_t)1 << c) : N;
            rc_enc_t e;
            rc_enc_init(&e, pay + plen, worst - plen);
            for (int64_t i = a; i < b; i++) {
                if (d >= B) logits_to_cdf(lg + i * NSYM, cdf);
                int s = T.code[d][i] - 1;
                rc_encode(&e, (uint32_t)cdf[s], (uint32_t)(cdf[s + 1] - cdf[s]));
            }
            rc_flush(&e);
            if (e.len > 65535) { st = ORC_E_INVAL; break; }
            lens[ci++] = (uint16_t)e.len;
            plen += e.len;
        }
        free(lg);
        if (d >= B && d <= M.k0) { free(Fprev); Fprev = F; if (d == M.k0) { free(Fk0); Fk0 = (int8_t *)malloc((size_t)(N > 0 ? N : 1) * M.C); if (Fk0) memcpy(Fk0, F, (size_t)N * M.C); else st = ORC_E_NOMEM; } }
        else free(F);
    }
    if (st == ORC_OK) {
        *out_len = hdr + plen;
        if (hdr + plen > cap) st = ORC_E_CAPACITY;
    }
    if (st == ORC_OK) {
        out[0] = 'L'; out[1] = 'P'; out[2] = 'C'; out[3] = '1';
        out[4] = B > 0 ? 2 : 1; out[5] = (uint8_t)D; out[6] = (uint8_t)M.n_deep; out[7] = (uint8_t)c;
        wr32(out + 8, M.blob_id);
        wr32(out + 12, (uint32_t)T.N[D]);
        for (int d = 0; d < D; d++) wr32(out + 16 + 4 * d, (uint32_t)T.N[d]);
        if (B > 0) {
            size_t o = 16 + 4 * (size_t)D;
            out[o++] = (uint8_t)B;
            for (int d = 0; d < B; d++) {
                int m = 0;
                for (int s2 = 0; s2 < NSYM; s2++) m += cnt[d][s2] ? 1 : 0;
                out[o++] = (uint8_t)m;
                for (int s2 = 0; s2 < NSYM; s2++)
                    if (cnt[d][s2]) { out[o] = (uint8_t)(s2 + 1); wr32(out + o + 1, cnt[d][s2]); o += 5; }
            }
        }
        for (int64_t k = 0; k < nch; k++) {
            out[pre + 2 * k] = lens[k] & 0xFF;
            out[pre + 2 * k + 1] = lens[k] >> 8;
        }
        memcpy(out + hdr, pay, plen);
    }
    free(Fprev); free(Fk0); free(pay); free(lens); free(cdf); free(cnt);
    octree_free(&T);
    model_free(&M);
    return st;
}

int orc_encode(const void *blob, size_t blob_len, const int32_t *xyz, int64_t n, int c, uint8_t *out,
               size_t cap, size_t *out_len)
{
    return orc_encode_base(blob, blob_len, xyz, n, c, 0, out, cap, out_len);
}

int orc_peek_header(const uint8_t *bs, size_t len, int *D, int64_t *n_points)
{
    if (!bs || len < 16) return ORC_E_CORRUPT;
    if (bs[0] != 'L' || bs[1] != 'P' || bs[2] != 'C' || bs[3] != '1' || (bs[4] != 1 && bs[4] != 2))
        return ORC_E_CORRUPT;
    *D = bs[5];
    *n_points = rd32(bs + 12);
    return ORC_OK;
}

/* Decode level by level (Sec. 3.1: the decoder only sees coded levels):    */
/* model -> CDFs of depth d -> symbols -> X_d -> children V_{d+1}.          */
int orc_decode(const void *blob, size_t blob_len, const uint8_t *bs, size_t len, int32_t *xyz_out, int64_t cap,
               int64_t *n_out)
{
    model_t M;
    int st = model_parse((const uint8_t *)blob, blob_len, &M);
    if (st != ORC_OK) return st;
    int D = M.D;
    if (!bs || len < 16 || bs[0] != 'L' || bs[1] != 'P' || bs[2] != 'C' || bs[3] != '1' ||
        (bs[4] != 1 && bs[4] != 2)) {
        model_free(&M); return ORC_E_CORRUPT;
    }
    if (bs[5] != D || bs[6] != M.n_deep || rd32(bs + 8) != M.blob_id) { model_free(&M); return ORC_E_MODEL; }
    int c = bs[7];
    if (c < 4 || c > 14 || len < 16 + 4 * (size_t)D) { model_free(&M); return ORC_E_CORRUPT; }
    octree_t T;
    memset(&T, 0, sizeof(T));
    T.D = D;
    int64_t NDh = rd32(bs + 12);
    int64_t Nh[MAXD + 1];
    for (int d = 0; d < D; d++) Nh[d] = rd32(bs + 16 + 4 * d);
    Nh[D] = NDh;
    /* counts must describe an octree: N_0 in {0,1}, N_d <= N_{d+1} <= 8 N_d */
    if (Nh[0] > 1 || (Nh[0] == 0) != (NDh == 0)) { model_free(&M); return ORC_E_CORRUPT; }
    for (int d = 0; d < D; d++)
        if (Nh[d + 1] < Nh[d] || Nh[d + 1] > 8 * Nh[d]) { model_free(&M); return ORC_E_CORRUPT; }
    int64_t nch = 0;
    for (int d = 0; d < D; d++) nch += nchunks(Nh[d], c);
    /* version 2: base depth and the symbol counts of every base depth */
    int B = 0;
    size_t pre = 16 + 4 * (size_t)D;
    uint32_t (*cnt)[NSYM] = NULL;
    if (bs[4] == 2) {
        if (len < pre + 1) { model_free(&M); return ORC_E_CORRUPT; }
        B = bs[pre++];
        if (B < 1 || B > M.k0) { model_free(&M); return ORC_E_CORRUPT; }
        cnt = (uint32_t (*)[NSYM])calloc((size_t)B, sizeof(uint32_t[NSYM]));
        if (!cnt) { model_free(&M); return ORC_E_NOMEM; }
        for (int d = 0; d < B && st == ORC_OK; d++) {
            if (len < pre + 1) { st = ORC_E_CORRUPT; break; }
            int m = bs[pre++], last = 0;
            int64_t sum = 0;
            if (len < pre + 5 * (size_t)m) { st = ORC_E_CORRUPT; break; }
            for (int k = 0; k < m; k++, pre += 5) {
                int code = bs[pre];
                uint32_t v = rd32(bs + pre + 1);
                if (code <= last || v == 0) { st = ORC_E_CORRUPT; break; }
                cnt[d][code - 1] = v;
                sum += v;
                last = code;
            }
            if (st == ORC_OK && sum != Nh[d]) st = ORC_E_CORRUPT;
        }
        if (st != ORC_OK) { free(cnt); model_free(&M); return st; }
    }
    size_t hdr = pre + 2 * (size_t)nch;
    if (len < hdr) { free(cnt); model_free(&M); return ORC_E_CORRUPT; }
    size_t total = 0;
    for (int64_t k = 0; k < nch; k++) total += (size_t)bs[pre + 2 * k] | ((size_t)bs[pre + 2 * k + 1] << 8);
    if (hdr + total != len) { free(cnt); model_free(&M); return ORC_E_CORRUPT; }
    *n_out = NDh;
    if (NDh > cap) { free(cnt); model_free(&M); return ORC_E_CAPACITY; }
    if (NDh == 0) { free(cnt); model_free(&M); return ORC_OK; }

    T.N[0] = 1;
    T.key[0] = (uint64_t *)calloc(1, sizeof(uint64_t));
    int8_t *Fprev = NULL, *Fk0 = NULL;
    int32_t *cdf = (int32_t *)malloc(sizeof(int32_t) * 256);
    size_t pos = hdr;
    int64_t ci = 0;
    if (!T.key[0] || !cdf) st = ORC_E_NOMEM;
    for (int d = 0; d < D && st == ORC_OK; d++) {
        int64_t N = T.N[d];
        int8_t *F = NULL, *lg = NULL;
        T.code[d] = (uint8_t *)malloc((size_t)(N > 0 ? N : 1));
        if (!T.code[d]) { st = ORC_E_NOMEM; break; }
        if (d < B) {
            counts_to_cdf(cnt[d], cdf);
        } else {
            st = features(&M, &T, d, B, Fprev, Fk0, &F);
            if (st != ORC_OK) break;
            lg = (int8_t *)malloc((size_t)(N > 0 ? N : 1) * NSYM);
            if (!lg) { free(F); st = ORC_E_NOMEM; break; }
            st = predict_logits(&M, d, F, N, lg);
        }
        for (int64_t k = 0; k < nchunks(N, c) && st == ORC_OK; k++, ci++) {
            size_t cl = (size_t)bs[pre + 2 * ci] | ((size_t)bs[pre + 2 * ci + 1] << 8);
            rc_dec_t dd;
            rc_dec_init(&dd, bs + pos, cl);
            int64_t a = k << c, b = a + ((int64_t)1 << c) < N ? a + ((int64_t)1 << c) : N;
            for (int64_t i = a; i < b; i++) {
                if (d >= B) logits_to_cdf(lg + i * NSYM, cdf);
                int s = rc_decode(&dd, cdf);
                if (s < 0) { st = ORC_E_CORRUPT; break; }
                T.code[d][i] = (uint8_t)(s + 1);
            }
            pos += cl;
        }
        free(lg);
        if (st != ORC_OK) { free(F); break; }
        /* children: parent order, slots ascending (Sec. S3.2) */
        int64_t Nc = 0;
        for (int64_t p = 0; p < N; p++)
            for (int o = 0; o < 8; o++) Nc += (T.code[d][p] >> o) & 1u;
        if (Nc != Nh[d + 1]) { free(F); st = ORC_E_CORRUPT; break; }
        T.key[d + 1] = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(Nc > 0 ? Nc : 1));
        if (!T.key[d + 1]) { free(F); st = ORC_E_NOMEM; break; }
        int64_t r = 0;
        for (int64_t p = 0; p < N; p++)
            for (int o = 0; o < 8; o++)
                if ((T.code[d][p] >> o) & 1u) T.key[d + 1][r++] = (T.key[d][p] << 3) | (uint64_t)o;
        T.N[d + 1] = Nc;
        if (d < B) {
            /* base depth: no features */
        } else if (d <= M.k0) {
            free(Fprev); Fprev = F;
            if (d == M.k0) {
                free(Fk0);
                Fk0 = (int8_t *)malloc((size_t)(N > 0 ? N : 1) * M.C);
                if (Fk0) memcpy(Fk0, F, (size_t)N * M.C); else st = ORC_E_NOMEM;
            }
        } else {
            free(F);
        }
    }
    if (st == ORC_OK) {
        for (int64_t i = 0; i < T.N[D]; i++) {
            int64_t x, y, z;
            morton_decode(T.key[D][i], D, &x, &y, &z);
            xyz_out[3 * i] = (int32_t)x; xyz_out[3 * i + 1] = (int32_t)y; xyz_out[3 * i + 2] = (int32_t)z;
        }
    }
    free(Fprev); free(Fk0); free(cdf); free(cnt);
    octree_free(&T);
    model_free(&M);
    return st;
}
