"""Pipelining order for CPU->GPU transfer and on-GPU decode (Sec. 3.3).

Test infrastructure only (see ``oracle/__init__.py``).

Each data block i is a two-stage job: transfer a[i] (PCIe copy), then decode
b[i] (GPU kernel); the copy engine and the GPU each run one job at a time, in
the same order.  The paper orders the blocks with Johnson's rule for the
two-machine flow shop; Johnson (1954) proved that rule gives the smallest
makespan when the buffer between the stages is unlimited.
"""
import itertools


def johnson_order(a, b):
    """Johnson's rule: jobs whose transfer is shorter than their decode go
    first, by increasing transfer time; the others follow, by decreasing
    decode time.  Ties keep the lower job index first."""
    n = len(a)
    first = sorted((i for i in range(n) if a[i] < b[i]), key=lambda i: (a[i], i))
    rest = sorted((i for i in range(n) if a[i] >= b[i]), key=lambda i: (-b[i], i))
    return first + rest


def makespan(order, a, b, slots=None):
    """Completion time of the last decode when the jobs run in `order`.

    Stage 1 (copy) of job k starts when the previous copy is done and, with a
    bounded number of staging slots, when the decode that last used the same
    slot (job k - slots) has finished.  Stage 2 (decode) starts when its own
    copy and the previous decode are done."""
    c1 = 0.0
    done2 = []
    for k, i in enumerate(order):
        start1 = c1
        if slots is not None and k >= slots:
            start1 = max(start1, done2[k - slots])
        c1 = start1 + a[i]
        prev2 = done2[-1] if done2 else 0.0
        done2.append(max(prev2, c1) + b[i])
    return done2[-1] if done2 else 0.0


def brute_force_best(a, b, slots=None):
    """Smallest makespan over all orders (small n only)."""
    best = None
    for perm in itertools.permutations(range(len(a))):
        m = makespan(perm, a, b, slots)
        if best is None or m < best[0]:
            best = (m, perm)
    return best
