"""Host replay of the single-launch factorisation's schedule (the state
machine of Resident::run in csrc/resident_kernels.hpp), without arithmetic.

Every workgroup runs its loop with the kernel's waits: a bulk or deferred
projection by q_k waits until column k has been normalised and stored to Q
(its owner's own_norm), a critical-path step by column k waits until k has
been copied to U (its owner's store_u).  The replay checks, for every shape:

* termination: all workgroups finish, none waits forever (no deadlock for
  any interleaving the replay produces: workgroups run until they block,
  in round-robin order);
* Figure 1's order: column j (b included) receives the projections
  k = 0, 1, ..., min(j, n) - 1, each once, in ascending order, and every
  column j < n is normalised once, after its last projection.

The placement helpers (res_trade, res_position) and the loop are restated
from the kernel; a change there without the same change here fails these
tests.
"""
import pytest

RES_SEP = 25
NONE = 1 << 30


def res_trade(g, odd, G):
    if G < 6 * RES_SEP:
        return g
    if odd:
        if g < RES_SEP:
            return g + 2 * RES_SEP
        if 2 * RES_SEP <= g < 3 * RES_SEP:
            return g - 2 * RES_SEP
    else:
        if g >= G - RES_SEP:
            return g - 2 * RES_SEP
        if G - 3 * RES_SEP <= g < G - 2 * RES_SEP:
            return g + 2 * RES_SEP
    return g


def res_position(i, g, G):
    odd = (i & 1) == 1
    gg = res_trade(g, odd, G)
    return 2 * G * (i // 2) + ((2 * G - 1 - gg) if odd else gg)


class Machine:
    """Shared state: which columns are in Q (normalised) and in U (handed
    on), and the projections each column has received."""

    def __init__(self, n, ncols):
        self.n, self.ncols = n, ncols
        self.in_q = [False] * ncols
        self.in_u = [False] * ncols
        self.normalised = [0] * ncols
        self.received = [[] for _ in range(ncols)]


class Workgroup:
    def __init__(self, g, G, n, ncols, defer, mach):
        self.g, self.G, self.n, self.ncols, self.defer, self.m = g, G, n, ncols, defer, mach
        self.np = ncols  # panels of one column
        nq = 0
        while res_position(nq, g, G) < self.np:
            nq += 1
        self.nq = nq
        self.owned = [self.panel(i)[0] for i in range(nq)]  # ascending columns
        self.last = max(self.owned) if self.owned else -1
        self.kend = (self.last + 1) if self.last < n else n
        self.st, self.nxt, self.k = 0, 0, 0
        self.ps, self.pe, self.kd, self.dc = 0, 0, -1, 0
        self.handed = -1
        self.done = self.last < 0

    def panel(self, i):
        if i >= self.nq:
            return NONE, NONE
        qi = res_position(self.nq - 1 - i, self.g, self.G)
        ps = self.np - 1 - qi
        return ps, min(ps + 1, self.ncols)

    def apply(self, k, lo):
        for j in self.owned:
            if j > k and j >= lo:
                self.m.received[j].append(k)

    def store_u(self, x):
        assert not self.m.in_u[x], "column %d handed on twice" % x
        self.m.in_u[x] = True

    def own_norm(self, x):
        assert self.m.received[x] == list(range(x)), "column %d normalised before its projections" % x
        self.m.normalised[x] += 1
        self.m.in_q[x] = True

    def run(self):
        """Passes until the loop ends or a wait cannot be satisfied yet;
        returns the number of passes made."""
        passes = 0
        n = self.n
        while not self.done:
            mode, opk, lo, qsrc = 0, -1, 0, 3
            if self.st == 0:
                if self.k >= self.kend:
                    self.done = True
                    break
                self.ps, self.pe = self.panel(self.nxt)
                if self.k == self.ps:
                    self.st = 1
                    passes += 1
                    continue
                opk = self.k
                if self.ps < n and self.k + self.defer >= self.ps:
                    if self.kd < 0:
                        self.kd = self.k
                    mode, qsrc = 2, 4
                else:
                    mode, qsrc, lo = 1, 0, self.k + 1
            elif self.st == 1:
                mode, opk = 3, self.ps
            else:
                mode, opk = 1, self.dc
                qsrc = 2 if self.dc < self.ps else 1
                lo = self.pe
            # the waits: Q column published, or U column handed on
            if qsrc in (0, 2) and not self.m.in_q[opk]:
                break
            if qsrc == 4 and not self.m.in_u[opk]:
                break
            if mode == 1:
                self.apply(opk, lo)
            elif mode == 2:
                self.m.received[self.ps].append(opk)
                if opk + 1 == self.ps:
                    self.store_u(self.ps)
                    self.handed = self.ps
            else:
                if self.handed != self.ps:
                    self.store_u(self.ps)
                self.own_norm(self.ps)
            passes += 1
            if self.st == 0:
                self.k += 1
                if self.k == self.ps and self.ps < n:
                    self.st = 1
            elif self.st == 1:
                if self.last >= self.pe:
                    self.st, self.dc = 2, (self.kd if self.kd >= 0 else self.ps)
                else:
                    self.st, self.k, self.nxt, self.kd = 0, self.pe, self.nxt + 1, -1
            else:
                self.dc += 1
                if self.dc >= self.pe:
                    self.st, self.k, self.nxt, self.kd = 0, self.pe, self.nxt + 1, -1
        return passes


def replay(n, augmented, G, defer=12):
    ncols = n + 1 if augmented else n
    mach = Machine(n, ncols)
    wgs = [Workgroup(g, G, n, ncols, defer, mach) for g in range(G)]
    owners = sorted(c for w in wgs for c in w.owned)
    assert owners == list(range(ncols)), "every column owned exactly once"
    while True:
        progress = sum(w.run() for w in wgs)
        if all(w.done for w in wgs):
            break
        assert progress > 0, "deadlock: n=%d G=%d, stuck workgroups %s" % (
            n, G, [(w.g, w.st, w.k, w.ps) for w in wgs if not w.done][:5])
    for j in range(ncols):
        assert mach.received[j] == list(range(min(j, n))), j
        if j < n:
            assert mach.normalised[j] == 1 and mach.in_u[j], j
    return mach


@pytest.mark.parametrize("n,augmented,G", [
    (1024, True, 256),   # the 1024 x 1024 dd system with b on 256 compute units
    (1023, False, 256),
    (500, True, 256),    # 1 x 700 x 500 FP64 shape
    (255, True, 256),    # fewer columns than workgroups: one column each
    (299, True, 150),    # the trades near the reflection points start at G = 150
    (700, True, 151),
    (2047, False, 240),
    (64, False, 64),     # a 64-column precision-form panel
    (33, True, 34),      # Newton-sized
    (1, True, 2),
    (2, False, 2),
])
def test_schedule_terminates_in_figure_1_order(n, augmented, G):
    replay(n, augmented, G)


@pytest.mark.parametrize("defer", [1, 2, 5, 25])
def test_schedule_with_other_lookahead_windows(defer):
    replay(400, True, 200, defer=defer)
