"""The H-ring protocols of the fused step, checked on the CPU.

TWO form (BF16/FP16, and FP32 with 12 waves):

The kernel's step loop (one workgroup of NW waves, R = (m - 1) / 2, a ring of
NW + 2R H slots, nq = ty + 2R q-rows) is modelled action by action: in step st
wave w computes q-row st NW + w and writes it into slot (st NW + w) mod
(NW + 2R) after waiting until waves w - 2R .. w have finished the output rows
of step st - 1; then all waves meet at a barrier; then wave w finishes output
row st NW - 2R + w, which reads the q-rows orow .. orow + 2R, and publishes
its count of finished output-row phases.  Random schedules of the waves (any
interleaving the barrier and the waits allow) must never let an output row
read a slot that does not hold the q-row it needs, from the start to the end
of its reads, and every schedule must finish (no wave waits forever).  A
window one wave too narrow must be caught.

One-barrier form (FP32 with 8 waves): a ring of 2 NW + 2R slots; step st
finishes the output rows of step st - 1 and then writes q-row st NW + w, with
one barrier at the end of each step and no other wait.
"""
import random

import pytest


def _run(nw, r, ty, rng, window):
    hr = nw + 2 * r
    nq = ty + 2 * r
    nsteps = (nq + nw - 1) // nw
    slot = [None] * hr
    fdone = [0] * nw
    arrived = [0] * nsteps            # waves at the barrier of each step
    # per wave: (step, phase); phases: 0 write, 1 barrier, 2 read start,
    # 3 read end + release
    state = [(0, 0) for _ in range(nw)]
    held = {}                         # wave -> q-rows its output row reads

    def runnable(w):
        st, ph = state[w]
        if st >= nsteps:
            return False
        if ph == 0:
            qr = st * nw + w
            if st == 0 or qr >= nq:
                return True
            return all(fdone[v] >= st for v in range(max(0, w - window), w + 1))
        if ph == 1:
            return True               # arriving at the barrier
        if ph == 2:
            return arrived[st] == nw  # past the barrier once all arrived
        return True

    def step(w):
        st, ph = state[w]
        if ph == 0:
            qr = st * nw + w
            if qr < nq:
                slot[qr % hr] = qr
            state[w] = (st, 1)
        elif ph == 1:
            arrived[st] += 1
            state[w] = (st, 2)
        elif ph == 2:
            orow = st * nw - 2 * r + w
            need = [q for q in range(orow, orow + 2 * r + 1) if 0 <= orow < ty]
            for q in need:
                if slot[q % hr] != q:
                    return "read of q-row %d found %r" % (q, slot[q % hr])
            held[w] = need
            state[w] = (st, 3)
        else:
            for q in held.pop(w, []):
                if slot[q % hr] != q:
                    return "q-row %d overwritten during its reads" % q
            fdone[w] = st + 1
            state[w] = (st + 1, 0)
        return None

    while True:
        ready = [w for w in range(nw) if runnable(w)]
        if not ready:
            done = all(state[w][0] >= nsteps for w in range(nw))
            return None if done else "deadlock"
        err = step(rng.choice(ready))
        if err:
            return err


@pytest.mark.parametrize("nw", [8, 12])
@pytest.mark.parametrize("r", [1, 2, 3])
def test_ring_wait_protocol(nw, r):
    rng = random.Random(nw * 10 + r)
    for trial in range(150):
        ty = rng.randint(1, 100)
        err = _run(nw, r, ty, rng, 2 * r)
        assert err is None, (nw, r, ty, trial, err)


def test_narrow_window_is_caught():
    """Waiting on one neighbour fewer lets a q-row overwrite a slot that an
    output row of the previous step still reads."""
    rng = random.Random(7)
    found = False
    for trial in range(300):
        if _run(12, 3, rng.randint(20, 100), rng, 2 * 3 - 1):
            found = True
            break
    assert found


def _run_one_barrier(nw, r, ty, rng, hr):
    nq = ty + 2 * r
    nsteps = (nq + nw - 1) // nw
    slot = [None] * hr
    arrived = [0] * (nsteps + 1)
    # phases per step st = 0 .. nsteps: 0 read start (output rows of st - 1),
    # 1 read end, 2 write q-row st, 3 barrier arrival, 4 past the barrier
    state = [(0, 0) for _ in range(nw)]
    held = {}

    def runnable(w):
        st, ph = state[w]
        if st > nsteps:
            return False
        if ph == 4:
            return arrived[st] == nw
        return True

    def step(w):
        st, ph = state[w]
        if ph == 0:
            orow = (st - 1) * nw - 2 * r + w
            need = [q for q in range(orow, orow + 2 * r + 1) if st > 0 and 0 <= orow < ty]
            for q in need:
                if slot[q % hr] != q:
                    return "read of q-row %d found %r" % (q, slot[q % hr])
            held[w] = need
            state[w] = (st, 1)
        elif ph == 1:
            for q in held.pop(w, []):
                if slot[q % hr] != q:
                    return "q-row %d overwritten during its reads" % q
            state[w] = (st, 2)
        elif ph == 2:
            qr = st * nw + w
            if st < nsteps and qr < nq:
                slot[qr % hr] = qr
            state[w] = (st, 3)
        elif ph == 3:
            arrived[st] += 1
            state[w] = (st, 4)
        else:
            state[w] = (st + 1, 0)
        return None

    while True:
        ready = [w for w in range(nw) if runnable(w)]
        if not ready:
            return None if all(state[w][0] > nsteps for w in range(nw)) else "deadlock"
        err = step(rng.choice(ready))
        if err:
            return err


@pytest.mark.parametrize("r", [1, 2, 3])
def test_one_barrier_ring(r):
    nw = 8
    rng = random.Random(100 + r)
    for trial in range(150):
        ty = rng.randint(1, 120)
        err = _run_one_barrier(nw, r, ty, rng, 2 * nw + 2 * r)
        assert err is None, (r, ty, trial, err)


def test_one_barrier_ring_too_small_is_caught():
    """With NW + 2R slots and one barrier per step, a q-row of step st
    overwrites a slot that an output row of step st - 1 still reads."""
    rng = random.Random(11)
    assert any(_run_one_barrier(8, 3, rng.randint(20, 120), rng, 8 + 2 * 3)
               for _ in range(300))
