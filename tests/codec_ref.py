"""A second, independent numpy transcription of the per-depth integer model.

Test-only.  It is not a pin of the method (it encodes the same readings as the
C oracle); it guards against transcription slips in either implementation
(weight layouts, zero points, concat order, child order).  Tiny inputs only.
"""
import struct

import numpy as np

from paper_2603_25260_amd import synth


def parse_blob(blob):
    version = struct.unpack_from("<I", blob, 4)[0]
    shared = bool(version & 0x100)  # records name the layer whose weights they use
    C, D, n_deep, n_layers = struct.unpack_from("<4I", blob, 8)
    off = 32
    layers, order = {}, []
    for li in range(n_layers):
        kind, depth, j, taps, cin, cout, m_pos, m_neg, r, z_in, z_out = struct.unpack_from("<6I2iI2i", blob, off)
        off += 44
        owner = li
        if shared:
            owner = struct.unpack_from("<I", blob, off)[0]
            off += 4
        b = np.frombuffer(blob, np.int32, cout, off).astype(np.int64)
        off += 4 * cout
        if owner == li:
            W = np.frombuffer(blob, np.int8, taps * cin * cout, off).reshape(taps, cin, cout).astype(np.int64)
            off += taps * cin * cout
        else:
            W = layers[order[owner]]["W"]
        off = (off + 3) & ~3
        layers[(kind, depth, j)] = dict(W=W, b=b, m_pos=m_pos, m_neg=m_neg, r=r, z_in=z_in, z_out=z_out)
        order.append((kind, depth, j))
    return C, D, n_deep, layers


def rq(acc, L):
    acc = np.asarray(acc, np.int64)
    m = np.where(acc >= 0, L["m_pos"], L["m_neg"]).astype(np.int64)
    p = acc * m
    if L["r"] > 0:
        p = (p + (1 << (L["r"] - 1))) >> L["r"]   # numpy >> on int64 is a floor shift
    return np.clip(p + L["z_out"], -128, 127).astype(np.int64)


def bits(codes):
    return np.array([[127 if (c >> o) & 1 else 0 for o in range(8)] for c in codes], np.int64).reshape(-1, 8)


def level_logits_all(blob, xyz):
    C, D, n_deep, Ls = parse_blob(blob)
    k0 = D - n_deep - 1
    u = np.unique(np.asarray(xyz).reshape(-1, 3), axis=0).astype(np.int64)
    # per depth: coordinates in Morton order (sort by key via lexsort of interleaved bits)
    def key(c, d):
        k = np.zeros(len(c), np.int64)
        for b in range(d):
            k |= ((c[:, 0] >> b) & 1) << (3 * b + 2)
            k |= ((c[:, 1] >> b) & 1) << (3 * b + 1)
            k |= ((c[:, 2] >> b) & 1) << (3 * b)
        return k
    V = []
    for d in range(D + 1):
        cells = np.unique(u >> (D - d), axis=0)
        V.append(cells[np.argsort(key(cells, d))])
    index = [{tuple(c): i for i, c in enumerate(V[d])} for d in range(D + 1)]
    X = []
    for d in range(D):
        codes = np.zeros(len(V[d]), np.int64)
        for c in V[d + 1]:
            o = 4 * (c[0] & 1) + 2 * (c[1] & 1) + (c[2] & 1)
            codes[index[d][tuple(c >> 1)]] |= 1 << o
        X.append(codes)

    def conv(L, x, d):
        out = np.tile(L["b"], (len(V[d]), 1))
        for i, c in enumerate(V[d]):
            for t in range(27):
                dd = np.array([t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1])
                r = index[d].get(tuple(c + dd))
                if r is not None:
                    out[i] += (x[r] - L["z_in"]) @ L["W"][t]
        return rq(out, L)

    def lin(L, x):
        return rq((x - L["z_in"]) @ L["W"][0] + L["b"], L)

    def up(L, Z, d):
        inp = np.concatenate([Z, bits(X[d])], 1)
        full = (inp - L["z_in"]) @ L["W"][0] + L["b"]
        rows = []
        for p in range(len(V[d])):
            for o in range(8):
                if (X[d][p] >> o) & 1:
                    rows.append(full[p, o * C:(o + 1) * C])
        return rq(np.array(rows).reshape(-1, C), L)

    def down(L, G, j):  # depth j -> j-1
        out = np.tile(L["b"], (len(V[j - 1]), 1))
        for i, c in enumerate(V[j]):
            o = 4 * (c[0] & 1) + 2 * (c[1] & 1) + (c[2] & 1)
            out[index[j - 1][tuple(c >> 1)]] += (G[i] - L["z_in"]) @ L["W"][o]
        return rq(out, L)

    F = {0: np.zeros((len(V[0]), C), np.int64)}
    logits = []
    for d in range(D):
        if 1 <= d <= k0:
            x = F[d - 1]
            h = conv(Ls[(3, d, 0)], x, d - 1)
            y = conv(Ls[(4, d, 0)], h, d - 1)
            S = np.clip(y + x, -128, 127)
            F[d] = up(Ls[(6, d, d - 1)], S, d - 1)
        elif d > k0:
            G = lin(Ls[(1, d, d - 1)], bits(X[d - 1]))
            for j in range(d - 1, k0, -1):
                G = down(Ls[(2, d, j)], G, j)
            cat = np.concatenate([F[k0], G], 1)
            h = conv(Ls[(3, d, k0)], cat, k0)
            y = conv(Ls[(4, d, k0)], h, k0)
            s = lin(Ls[(5, d, k0)], cat)
            Z = np.clip(y + s, -128, 127)
            for j in range(k0, d):
                Z = up(Ls[(6, d, j)], Z, j)
            F[d] = Z
        h = lin(Ls[(7, d, d)], F[d])
        logits.append(lin(Ls[(8, d, d)], h).astype(np.int8))
    return logits
