"""The sieve's wave-cooperative walk, modelled on the CPU.

A wave takes the multiples o = f + p (lane + 64 i) < 2^17 of one prime (or
square) p with f < p: the word address of o in the permuted byte layout
(32-y group g, word t mod 8, byte t div 8 for o = 32 g + t) advances by 64p
per step, the wave repeats while lane 63's multiple is below 2^17, and each
lane then takes at most one more.  The model checks that this visits every
multiple of the segment exactly once, at its own word and byte, and never an
address outside the segment.  The device sums are checked against the
oracle by the GPU parity tests; this pins the walk's bounds by themselves.
"""
import numpy as np

SEG = 1 << 17


def _addr(o):
    return (o & ~31) | ((o & 7) << 2)


def _walk(f, p):
    step = 64 * p
    out = []
    for lane in range(64):
        o = f + lane * p
        a = _addr(o)
        o63 = f + 63 * p
        while o63 < SEG:
            assert a < SEG
            out.append((a, o & 24))
            a += step
            o63 += step
        if a < SEG:
            out.append((a, o & 24))
    return out


def _reference(f, p):
    return [(_addr(o), o & 24) for o in range(f, SEG, p)]


def test_step_keeps_word_and_byte():
    rng = np.random.default_rng(21)
    for _ in range(20000):
        p = int(rng.integers(5, 2**15))
        o = int(rng.integers(0, SEG))
        assert _addr(o + 64 * p) == _addr(o) + 64 * p
        assert (o + 64 * p) & 24 == o & 24


def test_walk_visits_each_multiple_once():
    rng = np.random.default_rng(22)
    primes = [17, 19, 23, 29, 101, 1009, 1021, 2003, 2039]
    primes += [int(v) for v in rng.integers(17, 2048, 60)]
    squares = [25, 49, 121, 169, 97 * 97, 359 * 359]
    for p in primes + squares:
        for f in {0, 1, p // 2, p - 1, int(rng.integers(0, p))}:
            got = _walk(f, p)
            assert len(got) == len(set(got))
            assert sorted(got) == sorted(_reference(f, p))
