"""Reference genetic cut search (Algorithm 1 of Sec. III B), test infrastructure.

Follows the algorithm's steps in the paper's order with these readings (the
paper leaves them open or garbled):
  * an individual is an ordered list of M distinct cut variables; the fitness
    of a cut set C is the exact cost of eliminating G - C with the min-fill
    order: (width, work), lower is better, ties broken by the sorted id list;
  * crossover pairs the sorted population as (1,2), (3,4), ... leaving the best
    (index 0) alone, and swaps the last floor(M/2) positions of the pair; a
    value repeated inside one individual is replaced, scanning positions in
    order, by a random variable not in the individual;
  * mutation picks one individual other than the best, one position, and puts
    a random non-member there;
  * "repeat ... until t > T" runs T+1 generations; Step 5 evaluates and returns
    the best.
Random draws come from one counter-based generator, SplitMix64 (Steele, Lea
and Flood, OOPSLA 2014), written here from its published definition; the
planner implements the same generator independently, so both searches make
the same draws.  A uniform draw in [0, m) is the 64-bit output modulo m.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

from .qaoa import min_fill_order, elimination_cost

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, counter: int) -> int:
    """Output number `counter` (0-based) of the SplitMix64 stream seeded by `seed`."""
    z = (seed + (counter + 1) * GOLDEN_GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    def __init__(self, seed: int):
        self.seed = seed & MASK64
        self.counter = 0

    def next(self) -> int:
        r = splitmix64(self.seed, self.counter)
        self.counter += 1
        return r

    def below(self, m: int) -> int:
        return self.next() % m


def cut_fitness(adj, cut: Sequence[int]) -> Tuple[int, int, Tuple[int, ...]]:
    """Exact cost of the sliced network G - C under its min-fill order."""
    order, _ = min_fill_order(adj, removed=cut)
    width, work = elimination_cost(adj, order, removed=cut)
    return width, work, tuple(sorted(cut))


def ga_cut_search(adj, M: int, N: int = 11, T: int = 4, seed: int = 0,
                  candidates: Optional[Sequence[int]] = None):
    """Algorithm 1 (Sec. III B).  Returns (sorted best cut, (width, work))."""
    cand = list(range(len(adj))) if candidates is None else list(candidates)
    if M <= 0:
        w, work, _ = cut_fitness(adj, [])
        return [], (w, work)
    if M >= len(cand):
        w, work, _ = cut_fitness(adj, cand)
        return sorted(cand), (w, work)
    rng = SplitMix64(seed)

    def nonmember(ind: List[int]) -> int:
        while True:
            u = cand[rng.below(len(cand))]
            if u not in ind:
                return u

    # initial population: N uniformly drawn M-subsets
    pop: List[List[int]] = []
    for _ in range(N):
        ind: List[int] = []
        while len(ind) < M:
            u = cand[rng.below(len(cand))]
            if u not in ind:
                ind.append(u)
        pop.append(ind)

    cache = {}

    def key(ind):
        s = tuple(sorted(ind))
        if s not in cache:
            cache[s] = cut_fitness(adj, s)
        return cache[s]

    h = M // 2
    t = 0
    while True:
        pop.sort(key=key)                                  # Step 1
        for i in range(1, N - 1, 2):                       # Step 2
            a, b = pop[i], pop[i + 1]
            ta, tb = a[M - h:], b[M - h:]
            a[M - h:], b[M - h:] = tb, ta
            for ind in (a, b):
                for pos in range(M):
                    if ind[pos] in ind[:pos]:
                        ind[pos] = nonmember(ind)
        if N > 1:                                          # Step 3
            j = 1 + rng.below(N - 1)
            pos = rng.below(M)
            pop[j][pos] = nonmember(pop[j])
        t += 1                                             # Step 4
        if t > T:
            break
    pop.sort(key=key)                                      # Step 5
    best = pop[0]
    w, work, _ = key(best)
    return sorted(best), (w, work)


def ga_min_k(adj, max_rank: int, k_max: int, N: int = 11, T: int = 4, seed: int = 0):
    """Smallest cut size k whose searched cut set meets the rank cap."""
    for k in range(0, k_max + 1):
        cut, (w, work) = ga_cut_search(adj, k, N=N, T=T, seed=seed)
        if w <= max_rank:
            return cut, (w, work)
    return None
