"""Host-side model of the balanced drain schedule of the symmetric P2P kernel
(`k_p2p_sym`, Stokeslet-only form): per batch of 32 ring entries a lane keeps up to
R = ceil(Q / 64) pairs of its own target, taken in cyclic order starting at its
(lane mod c)-th accepted entry (c its pair count; lowest rotated bit first), and queues the
rest (highest rotated bits first); lanes with fewer
than R pairs take queue entries in order in their spare rounds.  The first min over lanes
of the own-pair counts are rounds in which every lane takes its own pair; the kernel runs
them as a separate loop (no ballot, no queue) and starts the general rounds after them.
The model checks that every accepted (target, entry) pair is evaluated exactly once within
R rounds, that every lane has a pair of its own in each of the separate loop's rounds, and
that the queue never exceeds its 512 entries, on random, sparse and adversarial masks."""
import numpy as np
import pytest

K, LANES, QUEUE = 32, 64, 512


def schedule(acc):
    """Pairs (lane, entry) in the order the kernel's rounds evaluate them; queue length."""
    cnt = acc.shape[1]
    m = [sum(int(acc[l, j]) << j for j in range(cnt)) for l in range(LANES)]
    qn = int(acc.sum())
    rounds = (qn + LANES - 1) // LANES
    # start of each lane's cyclic order: its (lane mod c)-th set bit (0 for an empty mask)
    rot = []
    for l in range(LANES):
        bits = [j for j in range(K) if m[l] >> j & 1]
        rot.append(bits[l % len(bits)] if bits else 0)
    rm = [((m[l] >> rot[l]) | (m[l] << (K - rot[l]))) & 0xFFFFFFFF for l in range(LANES)]
    c = [bin(x).count("1") for x in m]
    own_n = [min(x, rounds) for x in c]
    ex = [c[l] - own_n[l] for l in range(LANES)]
    queue = []
    while any(e > 0 for e in ex):           # one pass per iteration of the kernel's excess loop
        for l in range(LANES):
            if ex[l] > 0:
                pb = rm[l].bit_length() - 1  # highest set bit
                rm[l] ^= 1 << pb
                queue.append((l, (pb + rot[l]) & (K - 1)))
                ex[l] -= 1
    done, qb = [], 0
    own_all = min(own_n)
    for r in range(own_all):                # every lane pops its own lowest rotated bit
        for l in range(LANES):
            assert rm[l] != 0
            pb = (rm[l] & -rm[l]).bit_length() - 1
            rm[l] &= rm[l] - 1
            done.append((l, (pb + rot[l]) & (K - 1)))
    for r in range(own_all, rounds):
        rank = 0
        for l in range(LANES):
            if r < own_n[l]:
                pb = (rm[l] & -rm[l]).bit_length() - 1  # lowest set bit
                rm[l] &= rm[l] - 1
                done.append((l, (pb + rot[l]) & (K - 1)))
            else:
                q = qb + rank
                rank += 1
                if q < len(queue):
                    done.append(queue[q])
        qb += rank
    return done, len(queue), rounds, own_all


def masks(seed):
    rng = np.random.default_rng(seed)
    for trial in range(300):
        cnt = K if trial % 3 else int(rng.integers(1, K + 1))
        kind = trial % 4
        if kind == 0:
            acc = rng.random((LANES, cnt)) < rng.random() ** 2
        elif kind == 1:  # half the lanes inactive (a partial chunk)
            acc = rng.random((LANES, cnt)) < 0.6
            acc[LANES // 2:] = False
        elif kind == 2:  # k full lanes, the rest empty: the queue's worst case at k = 32
            acc = np.zeros((LANES, cnt), bool)
            acc[: int(rng.integers(0, LANES + 1))] = True
        else:  # geometric: acceptance falling with a lane coordinate
            acc = rng.random((LANES, cnt)) < np.linspace(1.0, 0.0, LANES)[:, None]
        yield acc


@pytest.mark.parametrize("seed", [0, 1])
def test_every_pair_once_and_queue_bound(seed):
    for acc in masks(seed):
        done, qlen, rounds, _ = schedule(acc)
        want = sorted((l, j) for l in range(LANES) for j in range(acc.shape[1]) if acc[l, j])
        assert sorted(done) == want
        assert len(done) <= rounds * LANES
        assert qlen <= QUEUE


def test_queue_worst_case_is_reached():
    acc = np.zeros((LANES, K), bool)
    acc[:32] = True
    _, qlen, rounds, own_all = schedule(acc)
    assert (qlen, rounds, own_all) == (512, 16, 0)


def test_dense_batches_run_mostly_in_the_all_own_loop():
    # every lane accepts 24..32 of the 32 entries (a target deep inside the cutoff sphere of
    # the batch): R <= 32 and every lane holds at least 24 pairs, so the separate loop takes
    # min(R, 24) rounds and the general rounds only balance the remainder
    rng = np.random.default_rng(5)
    for _ in range(20):
        k = rng.integers(24, K + 1, LANES)
        acc = np.zeros((LANES, K), bool)
        for l in range(LANES):
            acc[l, rng.choice(K, k[l], replace=False)] = True
        done, qlen, rounds, own_all = schedule(acc)
        assert own_all == min(rounds, int(k.min()))
        assert sorted(done) == sorted((l, j) for l in range(LANES) for j in range(K) if acc[l, j])
        assert qlen <= QUEUE
