"""CPU emulation of the split DSS index scheme (NUMA_STAGE_SPLIT: the element
kernel's tail and the face kernel k_fin_split), N = 1..8.

The DSS (the sum over elements in Eq. (discstrongform), Code example 1) is
split between the element kernel, which adds the x-face pairs inside its run
of EB consecutive elements and finishes the nodes whose copies it then holds,
and the face kernel, which gathers the rest from the row-ordered face
contributions (Fa) and the run-boundary copies (Fb).  This test replays the
index arithmetic of both kernels on the host for small meshes (runs inside a
row, runs wrapping onto the next row or layer, nx smaller than a run, walls
and periodic z) and checks:

* every Fa / Fb / state index is in bounds, and Fa and Fb fit the
  contribution scratch of (N+1)^3 values per element;
* no Fa or Fb entry is written twice, every entry the face kernel reads was
  written;
* every unique node is finished exactly once, by one of the two kernels;
* the copies summed for a node are exactly that node's element-local copies
  (the gather map computed here from the lattice).

The run length and workgroup width follow the element kernel: 256 lanes of
(N+1)^2 columns, at N >= 5 also at most an 80 KB FP64 five-field tile.
"""
from collections import defaultdict

import pytest


def split_eb(N):
    PP = (N + 1) ** 2
    lanes = 256 // PP
    return lanes if N <= 4 else min(lanes, 2048 // (PP * (N + 1)))


def split_threads(N):
    return ((split_eb(N) * (N + 1) ** 2 + 63) // 64) * 64


def split_fp(N, j, k):
    """face pair index of local (j, k) on an element face in y or z"""
    if k == 0:
        return j
    if k == N:
        return N + 1 + j
    return 2 * (N + 1) + 2 * (k - 1) + (1 if j == N else 0)


def split_fp_jk(N, fp):
    if fp <= N:
        return fp, 0
    if fp < 2 * (N + 1):
        return fp - (N + 1), N
    r = fp - 2 * (N + 1)
    return (N if r & 1 else 0), 1 + (r >> 1)


def emulate(N, nx, ny, nz, walls):
    P = N + 1
    PP = P * P
    NP = PP * P
    EB, BT = split_eb(N), split_threads(N)
    NFP, NIP = 4 * N, (N - 1) ** 2
    NB = NFP + NIP * (N + 1)
    ni, nj = nx * N, ny * N
    nk = nz * N + 1 if walls else nz * N
    nu, ne = ni * nj * nk, nx * ny * nz
    vs = nz * ny * NFP * ni
    assert 5 * vs + ne * NB * 5 == 5 * ne * NP  # Fa and Fb fill the contribution scratch

    def elem(e):
        return e % nx, (e // nx) % ny, e // (nx * ny)

    def uid(e, i, j, k):
        ex, ey, ez = elem(e)
        gi, gj, gk = (ex * N + i) % ni, (ey * N + j) % nj, ez * N + k
        if not walls:
            gk %= nk
        return gi + ni * (gj + nj * gk)

    truth = defaultdict(set)  # unique node -> its (element, local node) copies
    for e in range(ne):
        for k in range(P):
            for j in range(P):
                for i in range(P):
                    truth[uid(e, i, j, k)].add((e, i + P * j + PP * k))
    assert len(truth) == nu

    Fa, Fb = {}, {}
    finished, got = defaultdict(int), {}
    nwg = (ne + EB - 1) // EB
    for wg in range(nwg):
        e0 = wg * EB
        new = min(EB, ne - e0)
        # Fb: the east face of a run's last element (face pairs, then interior
        # pairs at i = N), the interior rows of a run's first element
        ex = elem(e0)[0]
        for qq in range(new):
            exq = (ex + qq) % nx
            base = (e0 + qq) * NB
            if qq == EB - 1 or exq == nx - 1:
                for slot in range(NFP + NIP):
                    if slot < NFP:
                        jj, kk = split_fp_jk(N, slot)
                    else:
                        jj, kk = 1 + (slot - NFP) % (N - 1), 1 + (slot - NFP) // (N - 1)
                    o = (base + slot) * 5
                    assert 0 <= o and o + 4 < ne * NB * 5 and o not in Fb
                    Fb[o] = {(e0 + qq, N + P * (jj + P * kk))}
            if NIP > 0 and (qq == 0 or exq == 0):
                for nd in range(NIP * N):
                    ip, ii = divmod(nd, N)
                    jj, kk = 1 + ip % (N - 1), 1 + ip // (N - 1)
                    o = (base + NFP + NIP + nd) * 5
                    assert o + 4 < ne * NB * 5 and o not in Fb
                    Fb[o] = {(e0 + qq, ii + P * (jj + P * kk))}
        # Fa: every face pair's row, the run's x pairs added
        for nd in range(EB * N):
            qq, ii = divmod(nd, N)
            if qq >= new:
                continue
            exq, ey, ez = elem(e0 + qq)
            pair = ii == 0 and qq > 0 and exq != 0
            for fp in range(NFP):
                jj, kk = split_fp_jk(N, fp)
                assert split_fp(N, jj, kk) == fp
                o = ((ez * ny + ey) * NFP + fp) * ni + exq * N + ii
                assert 0 <= o < vs and o not in Fa
                cs = {(e0 + qq, ii + P * (jj + P * kk))}
                if pair:
                    cs.add((e0 + qq - 1, N + P * (jj + P * kk)))
                Fa[o] = cs
        # run-interior nodes finished by the element kernel
        NIN = NIP * EB * N
        SPL = (NIN + BT - 1) // BT if NIN > 0 else 1
        for t in range(BT):
            for p in range(SPL):
                n = t + p * BT
                if n >= NIN:
                    continue
                ip, m = divmod(n, EB * N)
                qq, ii = divmod(m, N)
                if qq >= new:
                    continue
                exq, ey, ez = elem(e0 + qq)
                if qq == 0 or exq == 0:
                    continue
                jj, kk = 1 + ip % (N - 1), 1 + ip // (N - 1)
                I = exq * N + ii + ni * (ey * N + jj + nj * (ez * N + kk))
                assert 0 <= I < nu
                cs = {(e0 + qq, ii + P * (jj + P * kk))}
                if ii == 0:
                    cs.add((e0 + qq - 1, N + P * (jj + P * kk)))
                finished[I] += 1
                got[I] = cs

    # the face kernel: face-row blocks, run-start blocks interleaved
    rl = nj + (N - 1) * ny
    rows = nz * rl + (nj if walls else 0)
    mblk = (rows * ni + 255) // 256
    nbb = ((nwg + ny * nz) * NIP * N + 255) // 256
    seen_a, seen_b = set(), set()
    for g in range(mblk + nbb):
        lb, runstart = g, False
        if nbb > 0:
            S = (mblk + nbb) // nbb
            if lb < nbb * S:
                k = lb // S
                runstart = lb - k * S == S - 1
                lb = k if runstart else lb - k
            else:
                lb -= nbb
        (seen_b if runstart else seen_a).add(lb)
        for th in range(256):
            idv = lb * 256 + th
            if not runstart:
                if idv >= rows * ni:
                    continue
                R, gi = divmod(idv, ni)
                ezr, rr = divmod(R, rl)
                if ezr == nz:
                    gk, gj = nz * N, rr
                elif rr < nj:
                    gk, gj = ezr * N, rr
                else:
                    kk, r2 = divmod(rr - nj, ny)
                    gj, gk = r2 * N, ezr * N + 1 + kk
                zc, kc, nzc = [gk // N] * 2, [gk % N] * 2, 1
                if kc[0] == 0:
                    if walls and gk == nz * N:
                        zc[0], kc[0] = nz - 1, N
                    elif not (walls and gk == 0):
                        zc[1], kc[1], nzc = (nz - 1 if zc[0] == 0 else zc[0] - 1), N, 2
                yc, jc, nyc = [gj // N] * 2, [gj % N] * 2, 1
                if jc[0] == 0:
                    yc[1], jc[1], nyc = (ny - 1 if yc[0] == 0 else yc[0] - 1), N, 2
                ex, xface = gi // N, gi % N == 0
                cs = set()
                for z in range(nzc):
                    for y in range(nyc):
                        fp = split_fp(N, jc[y], kc[z])
                        o = ((zc[z] * ny + yc[y]) * NFP + fp) * ni + gi
                        assert o in Fa
                        assert not (Fa[o] & cs)
                        cs |= Fa[o]
                        ec = ex + nx * (yc[y] + ny * zc[z])
                        if xface and (ex == 0 or ec % EB == 0):
                            ob = ((ec + nx - 1 if ex == 0 else ec - 1) * NB + fp) * 5
                            assert ob in Fb and not (Fb[ob] & cs)
                            cs |= Fb[ob]
            else:
                if NIP == 0:
                    continue
                cand, rr = divmod(idv, NIP * N)
                ip, i = divmod(rr, N)
                if cand >= nwg + ny * nz:
                    continue
                if cand < nwg:
                    e = cand * EB
                else:
                    e = (cand - nwg) * nx
                    if e % EB == 0:  # a workgroup start: taken above
                        continue
                ex, ey, ez = elem(e)
                jj, kk = 1 + ip % (N - 1), 1 + ip // (N - 1)
                gi, gj, gk = ex * N + i, ey * N + jj, ez * N + kk
                ew = e + nx - 1 if ex == 0 else e - 1
                o0 = (e * NB + NFP + NIP + ip * N + i) * 5
                assert o0 in Fb
                cs = set(Fb[o0])
                if i == 0:
                    o1 = (ew * NB + NFP + ip) * 5
                    assert o1 in Fb
                    cs |= Fb[o1]
            I = gi + ni * (gj + nj * gk)
            assert 0 <= I < nu
            finished[I] += 1
            got[I] = cs
    assert seen_a == set(range(mblk)) and seen_b == set(range(nbb))
    twice = [I for I in range(nu) if finished[I] != 1]
    assert not twice, (twice[:5], [finished[I] for I in twice[:5]])
    for I in range(nu):
        assert got[I] == truth[I], (I, got[I], truth[I])


# (N, nx, ny, nz, walls): runs inside a row, wrapping onto the next row or
# layer, nx smaller than a run, periodic z
CASES = [
    (1, 4, 4, 2, True), (1, 3, 2, 2, False), (1, 70, 1, 2, True),
    (2, 30, 2, 2, True), (2, 3, 5, 2, False),
    (3, 16, 4, 3, True), (3, 17, 2, 2, True), (3, 6, 3, 3, False),
    (4, 20, 2, 3, False), (4, 12, 3, 2, True), (4, 5, 3, 2, True), (4, 2, 2, 2, False),
    (5, 7, 3, 2, True), (5, 3, 2, 3, False), (5, 10, 2, 2, True),
    (6, 5, 3, 2, True), (6, 4, 2, 2, False),
    (7, 5, 2, 2, True), (7, 3, 2, 2, False),
    (8, 4, 2, 2, True), (8, 3, 2, 2, False),
]


@pytest.mark.parametrize("N,nx,ny,nz,walls", CASES)
def test_split_layout(N, nx, ny, nz, walls):
    emulate(N, nx, ny, nz, walls)


def test_split_run_lengths():
    """The runs the element kernel takes: 64, 28, 16, 10, 7, 5, 4, 2 elements
    at N = 1..8, at most 256 lanes and (N >= 5) 80 KB of five FP64 fields."""
    assert [split_eb(N) for N in range(1, 9)] == [64, 28, 16, 10, 7, 5, 4, 2]
    for N in range(5, 9):
        assert split_eb(N) * 5 * (N + 1) ** 3 * 8 <= 81920
