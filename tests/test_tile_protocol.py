"""The tile kernel's LDS labeling protocol under arbitrary interleavings (CPU).

The bond kernel labels a tile with its waves working on one LDS forest P at
once: each wave runs a Hoshen-Kopelman pass over its strip of rows (every run
entry written first, then one row at a time: the run's label lowered to the
labels above it, each other touched label lowered to the run's, and a lowered
label's old parent joined one row later), then the strips are joined at their
boundaries with lock-free unions (atomic minimum, path halving), and after a
workgroup barrier every site walks read-only to its root.  This file models
those steps as they are written in the kernel, with every LDS access an atomic
step and a random scheduler interleaving the accesses of all lanes of all
waves (a stronger adversary than the hardware, where a wave's lanes move
together).  Each site's root must be the smallest site index of its
component in the tile's bond graph (Sec. 2: the smallest label), for every
schedule.

The strip joins' finds halve paths while other waves' unions run, so the
positive cases also cover path halving concurrent with unions.  Two mutants
check that the test can fail: dropping the join of a lowered label's old
parent, and root walks (with path halving, as the kernel's first version had
them) started without the barrier after the strip joins, which then read a
forest that other waves are still joining.
"""
import numpy as np
import pytest

W = 16          # lanes (columns) of the model tile
WAVES = 4
RPW = 4         # rows per wave
H = WAVES * RPW


def components_min(br, bd):
    """Smallest site index of each site's component; br[y, x]: bond to the
    right inside the tile, bd[y, x]: bond down inside the tile."""
    par = list(range(H * W))

    def find(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    for y in range(H):
        for x in range(W):
            i = y * W + x
            if x + 1 < W and br[y, x]:
                a, b = find(i), find(i + 1)
                par[max(a, b)] = min(a, b)
            if y + 1 < H and bd[y, x]:
                a, b = find(i), find(i + W)
                par[max(a, b)] = min(a, b)
    return np.array([find(i) for i in range(H * W)])


# LDS primitives: every access is one atomic step (a yield follows it).
def find(P, x):
    p = P[x]
    yield
    while p != x:
        gp = P[p]
        yield
        if gp == p:
            return p
        P[x] = gp  # path halving
        yield
        x = gp
        p = P[x]
        yield
    return x


def union(P, a, b):
    while True:
        a = yield from find(P, a)
        b = yield from find(P, b)
        if a == b:
            return
        if a < b:
            a, b = b, a
        old = P[a]
        P[a] = min(old, b)  # atomic minimum, returns the old word
        yield
        if old == a:
            return
        a = old


def run_starts(rmask_row):
    """First site (column) of each lane's run: the right bonds of the row
    inside the tile join a lane to the next one."""
    out, start = [], 0
    for x in range(W):
        if x == 0 or not rmask_row[x - 1]:
            start = x
        out.append(start)
    return out


def instruction(lanes, body):
    """One wave instruction: its lanes' accesses, in any order."""
    return [body(ln) for ln in lanes]


def wave_program(w, P, br, bd, mutant):
    """The steps of wave w: each step is a list of lane threads (generators)
    that run concurrently; a step ends when all of them have; 'barrier' waits
    for every wave."""
    ly0 = w * RPW
    node = [[ly0 * W + r * W + s for s in run_starts(br[ly0 + r])] for r in range(RPW)]
    lanes = range(W)

    def store(i, v):
        def g():
            P[i] = v
            yield
        return g()

    # pre-pass: every site points at its run's first site
    for r in range(RPW):
        yield instruction(lanes, lambda ln, r=r: store((ly0 + r) * W + ln, node[r][ln]))
    lab_prev = list(node[0])
    pend = None  # (need, old, target, lab) of the previous row
    for r in range(1, RPW):
        up = [bool(bd[ly0 + r - 1, ln]) for ln in lanes]

        def amin(ln, r=r):
            def g():
                P[node[r][ln]] = min(P[node[r][ln]], lab_prev[ln])
                yield
            return g()

        yield instruction([ln for ln in lanes if up[ln]], amin)
        lab = [0] * W

        def load(ln, r=r):
            def g():
                lab[ln] = P[node[r][ln]]
                yield
            return g()

        yield instruction(lanes, load)
        if pend is not None and mutant != "no_parent_join":
            need, old, tgt, lp = pend
            yield [union(P, old[ln], lp[ln]) for ln in lanes if need[ln] and old[ln] != tgt[ln] and old[ln] != lp[ln]]
        need = [up[ln] and lab_prev[ln] != lab[ln] for ln in lanes]
        old = list(lab_prev)

        def fmin(ln):
            def g():
                old[ln] = P[lab_prev[ln]]
                P[lab_prev[ln]] = min(old[ln], lab[ln])
                yield
            return g()

        yield instruction([ln for ln in lanes if need[ln]], fmin)
        pend = (need, old, list(lab_prev), list(lab))
        lab_prev = lab
    if mutant != "no_parent_join":
        need, old, tgt, lp = pend
        yield [union(P, old[ln], lp[ln]) for ln in lanes if need[ln] and old[ln] != tgt[ln] and old[ln] != lp[ln]]
    yield "barrier"
    # strip boundaries: the last row of this strip with the first of the next
    if w + 1 < WAVES:
        ly = ly0 + RPW - 1
        ends = {}

        def load2(ln):
            def g():
                ends[ln] = [P[ly * W + ln]]
                yield
                ends[ln].append(P[(ly + 1) * W + ln])
                yield
            return g()

        act = [ln for ln in lanes if bd[ly, ln] and not (ln > 0 and bd[ly, ln - 1] and br[ly, ln - 1] and br[ly + 1, ln - 1])]
        yield instruction(act, load2)
        yield [union(P, ends[ln][0], ends[ln][1]) for ln in act]
    if mutant != "halving_roots_no_barrier":
        yield "barrier"


def roots_read_only(P):
    out = []
    for i in range(H * W):
        x = P[i]
        for _ in range(H * W):
            if P[x] == x:
                break
            x = P[x]
        out.append(x)
    return np.array(out)


def roots_halving(P):
    """Root walks with path halving stores (the mutant's phase 3)."""
    def walk(i, res):
        x = yield from find(P, i)
        res[i] = x
    return walk


def simulate(br, bd, rng, mutant=None):
    P = [0] * (H * W)
    progs = [wave_program(w, P, br, bd, mutant) for w in range(WAVES)]
    cur = [[] for _ in range(WAVES)]
    state = ["run"] * WAVES  # run, barrier, done, roots
    roots = [None] * (H * W)
    walk = roots_halving(P)

    def next_step(w):
        try:
            s = next(progs[w])
        except StopIteration:
            if mutant == "halving_roots_no_barrier":
                # this wave's sites walk to their roots at once, while other
                # waves may still be joining their strips
                cur[w] = [walk(i, roots) for i in range(w * RPW * W, (w + 1) * RPW * W)]
                state[w] = "roots"
            else:
                state[w] = "done"
            return
        if s == "barrier":
            state[w] = "barrier"
        else:
            cur[w] = list(s)

    for w in range(WAVES):
        next_step(w)
    while True:
        # waves whose step is over take their next one
        for w in range(WAVES):
            while state[w] == "run" and not cur[w]:
                next_step(w)
            if state[w] == "roots" and not cur[w]:
                state[w] = "done"
        if all(s == "barrier" for s in state):
            for w in range(WAVES):
                state[w] = "run"
                next_step(w)
            continue
        live = [w for w in range(WAVES) if state[w] in ("run", "roots") and cur[w]]
        if not live:
            assert all(s in ("done", "barrier") for s in state)
            if all(s == "done" for s in state):
                break
            raise AssertionError("a wave waits at a barrier the others never reach")
        w = live[rng.integers(len(live))]
        k = rng.integers(len(cur[w]))
        try:
            next(cur[w][k])
        except StopIteration:
            cur[w].pop(k)
    if mutant == "halving_roots_no_barrier":
        return np.array(roots)
    return roots_read_only(P)


def random_bonds(rng, p):
    br = rng.random((H, W)) < p
    bd = rng.random((H, W)) < p
    br[:, W - 1] = False  # bonds that leave the tile are not part of the tile forest
    bd[H - 1, :] = False
    return br, bd


@pytest.mark.parametrize("p", [0.3, 0.5, 0.6, 0.75, 0.95])
def test_protocol_gives_smallest_index_under_any_interleaving(p):
    rng = np.random.default_rng(int(p * 1000) + 11)
    for trial in range(40):
        br, bd = random_bonds(rng, p)
        want = components_min(br, bd)
        for sched in range(3):
            got = simulate(br, bd, np.random.default_rng(1000 * trial + sched))
            assert np.array_equal(got, want), (p, trial, sched)


def test_protocol_special_shapes():
    # a comb whose teeth join only through the bottom row (many lowered
    # labels), a spiral, and a tile with every bond active
    rng = np.random.default_rng(5)
    shapes = []
    br = np.zeros((H, W), bool)
    bd = np.zeros((H, W), bool)
    bd[: H - 1, ::2] = True
    br[H - 1, : W - 1] = True
    shapes.append((br, bd))
    br = np.zeros((H, W), bool)
    bd = np.zeros((H, W), bool)
    y0, x0, y1, x1 = 0, 0, H - 1, W - 1
    while y0 <= y1 and x0 <= x1:
        br[y0, x0:x1] = True
        bd[y0:y1, x1] = True
        br[y1, x0:x1] = True
        bd[y0 + 2:y1, x0] = True
        y0, x0, y1, x1 = y0 + 2, x0 + 2, y1 - 2, x1 - 2
    br[:, W - 1] = False
    bd[H - 1, :] = False
    shapes.append((br, bd))
    br = np.ones((H, W), bool)
    bd = np.ones((H, W), bool)
    br[:, W - 1] = False
    bd[H - 1, :] = False
    shapes.append((br, bd))
    for br, bd in shapes:
        want = components_min(br, bd)
        for sched in range(20):
            assert np.array_equal(simulate(br, bd, np.random.default_rng(rng.integers(1 << 30))), want)


@pytest.mark.parametrize("mutant", ["no_parent_join", "halving_roots_no_barrier"])
def test_mutants_are_caught(mutant):
    rng = np.random.default_rng(17)
    caught = False
    for trial in range(300):
        br, bd = random_bonds(rng, 0.6)
        want = components_min(br, bd)
        for sched in range(4):
            if not np.array_equal(simulate(br, bd, np.random.default_rng(77 * trial + sched), mutant), want):
                caught = True
                break
        if caught:
            break
    assert caught, f"the {mutant} mutant was never caught"
