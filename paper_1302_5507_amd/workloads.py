"""Seeded synthetic workloads for batched read-vs-window alignment.

This module only draws inputs.  It holds none of the alignment arithmetic:
no scoring, no recurrence, no packing into the device format.  Both the GPU
path and the CPU oracle consume what it returns, so it is the single point
the two sides share.

The shapes follow the Illumina-style workloads the paper evaluates on
(Results: 100/150 bp paired-end reads, lengths 50-250 bp, insert size about
500 bp; Methods, "Simulation of single-end and paired-end reads").  The real
and Mason-simulated datasets are not available, so uniform i.i.d. ACGT
genomes stand in for GRCh37 and a simple copy-and-edit walk stands in for the
read simulator.  Bases are coded A=0, C=1, G=2, T=3 (no N).

Read model (all configs): a read is produced by walking its window from a
start offset.  At each source base an indel event starts with probability
``p_ind`` (insertion or deletion with equal odds, length from the config's
length law); an insertion emits that many uniform random bases, a deletion
skips that many source bases; otherwise the source base is copied, replaced
by one of the three other bases with probability ``p_sub``.  The walk stops
once exactly ``n`` read bases exist.  A walk that runs off the end of its
window is redrawn with a new start offset.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ALPHABET = "ACGT"


@dataclasses.dataclass
class Workload:
    """A batch of alignment tasks.  Task t aligns read t against window t.

    genome     uint8[G]   base codes of the sequence windows are cut from
    read_codes uint8[*]   all reads' base codes, concatenated
    read_off   int64[T]   start of read t in ``read_codes``
    read_len   int32[T]   n_t
    ref_off    int64[T]   start of window t in ``genome`` (a base offset)
    ref_len    int32[T]   m_t
    true_off   int32[T]   simulated start of read t in its window, -1 for a
                          random (unalignable) read
    """

    name: str
    genome: np.ndarray
    read_codes: np.ndarray
    read_off: np.ndarray
    read_len: np.ndarray
    ref_off: np.ndarray
    ref_len: np.ndarray
    true_off: np.ndarray
    seed: int = 0
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def n_tasks(self) -> int:
        return int(self.read_len.shape[0])

    @property
    def cells(self) -> int:
        return int(np.dot(self.read_len.astype(np.int64), self.ref_len.astype(np.int64)))

    def read(self, t: int) -> np.ndarray:
        o = int(self.read_off[t])
        return self.read_codes[o:o + int(self.read_len[t])]

    def window(self, t: int) -> np.ndarray:
        o = int(self.ref_off[t])
        return self.genome[o:o + int(self.ref_len[t])]

    def subset(self, idx) -> "Workload":
        """Tasks ``idx`` (in that order) as a new workload sharing the genome."""
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.read_len[idx].astype(np.int64)
        offs = np.zeros(len(idx), dtype=np.int64)
        if len(idx):
            offs[1:] = np.cumsum(lens)[:-1]
        codes = np.empty(int(lens.sum()), dtype=np.uint8)
        for k, t in enumerate(idx):
            codes[offs[k]:offs[k] + lens[k]] = self.read(int(t))
        return Workload(self.name + "[subset]", self.genome, codes, offs,
                        self.read_len[idx].copy(), self.ref_off[idx].copy(),
                        self.ref_len[idx].copy(), self.true_off[idx].copy(),
                        self.seed, dict(self.params))


def random_genome(length: int, seed: int) -> np.ndarray:
    return np.random.Generator(np.random.PCG64(seed)).integers(0, 4, size=length, dtype=np.uint8)


def _geometric_trunc(rng, p, size, cap):
    x = rng.geometric(p, size=size)
    return np.minimum(x, cap) if cap else x


def _walk(rng, genome, win_off, win_len, n, start, p_sub, p_ind, indel_len):
    """Vectorised copy-and-edit walk for a set of reads.

    All arrays have one entry per read.  ``n`` may vary per read.  Returns
    (codes[R, max_n] uint8, ok[R] bool); ``ok`` is False where the walk ran
    off the window, and such rows must be redrawn by the caller.
    """
    R = len(n)
    nmax = int(n.max()) if R else 0
    out = np.zeros((R, max(nmax, 1)), dtype=np.uint8)
    length = np.zeros(R, dtype=np.int64)
    src = start.astype(np.int64).copy()
    ins_left = np.zeros(R, dtype=np.int64)
    ok = np.ones(R, dtype=bool)
    active = length < n
    rows = np.arange(R)
    while active.any():
        a = rows[active]
        # pending inserted bases first
        ins = ins_left[a] > 0
        ai = a[ins]
        if ai.size:
            out[ai, length[ai]] = rng.integers(0, 4, size=ai.size, dtype=np.uint8)
            length[ai] += 1
            ins_left[ai] -= 1
        an = a[~ins]
        if an.size:
            u = rng.random(an.size)
            ev = u < p_ind[an] if np.ndim(p_ind) else u < p_ind
            ae = an[ev]
            if ae.size:
                lens = indel_len(rng, ae.size)
                is_ins = rng.random(ae.size) < 0.5
                ins_left[ae[is_ins]] = lens[is_ins]
                src[ae[~is_ins]] += lens[~is_ins]
            ac = an[~ev]
            if ac.size:
                off_ok = src[ac] < win_len[ac]
                bad = ac[~off_ok]
                ok[bad] = False
                length[bad] = n[bad]            # stop the walk; redrawn by caller
                ac = ac[off_ok]
                base = genome[win_off[ac] + src[ac]]
                ps = p_sub[ac] if np.ndim(p_sub) else p_sub
                sub = rng.random(ac.size) < ps
                shift = rng.integers(1, 4, size=ac.size, dtype=np.uint8)
                base = np.where(sub, (base + shift) & 3, base).astype(np.uint8)
                out[ac, length[ac]] = base
                length[ac] += 1
                src[ac] += 1
        active = length < n
    return out, ok


def _assemble(name, genome, reads2d, n, win_off, win_len, true_off, seed, params):
    T = len(n)
    offs = np.zeros(T, dtype=np.int64)
    if T:
        offs[1:] = np.cumsum(n.astype(np.int64))[:-1]
    mask = np.arange(reads2d.shape[1])[None, :] < n[:, None]
    codes = reads2d[mask]
    return Workload(name, genome, codes.astype(np.uint8), offs, n.astype(np.int32),
                    win_off.astype(np.int64), win_len.astype(np.int32),
                    true_off.astype(np.int32), seed, params)


def simulate(name, genome, n, win_len, start_law, p_sub, p_ind, indel_len, rng,
             win_off=None, random_frac=0.0, max_redraw=50, params=None):
    """Generic generator: windows at uniform genome positions (unless given),
    reads walked from ``start_law(rng, idx)`` offsets with the read model."""
    n = np.asarray(n, dtype=np.int64)
    win_len = np.asarray(win_len, dtype=np.int64)
    T = len(n)
    G = len(genome)
    if win_off is None:
        win_off = rng.integers(0, G - win_len + 1, size=T)
    win_off = np.asarray(win_off, dtype=np.int64)
    p_sub = np.broadcast_to(np.asarray(p_sub, dtype=np.float64), (T,)).copy()
    p_ind = np.broadcast_to(np.asarray(p_ind, dtype=np.float64), (T,)).copy()
    reads = np.zeros((T, max(int(n.max()) if T else 1, 1)), dtype=np.uint8)
    true_off = np.full(T, -1, dtype=np.int64)
    todo = np.arange(T)
    for _ in range(max_redraw):
        if todo.size == 0:
            break
        start = start_law(rng, todo)
        out, ok = _walk(rng, genome, win_off[todo], win_len[todo], n[todo], start,
                        p_sub[todo], p_ind[todo], indel_len)
        good = todo[ok]
        reads[good, :out.shape[1]] = out[ok]
        true_off[good] = start[ok]
        todo = todo[~ok]
    if todo.size:
        raise RuntimeError(f"{todo.size} reads could not be placed inside their windows")
    if random_frac > 0:
        rnd = rng.random(T) < random_frac
        k = int(rnd.sum())
        reads[rnd] = rng.integers(0, 4, size=(k, reads.shape[1]), dtype=np.uint8)
        true_off[rnd] = -1
    return _assemble(name, genome, reads, n, win_off, win_len, true_off, 0, params or {})


# --------------------------------------------------------------------------
# The five benchmark workloads.

def config1(seed: int = 101, genome_seed: int = 1) -> Workload:
    """1,000 reads x 100 bp vs 1,000 windows x 300 bp cut from a 1 Mbp genome;
    2% substitutions, 0.5% indel events of length uniform {1,2,3}."""
    g = random_genome(1_000_000, genome_seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    T = 1000
    n = np.full(T, 100)
    m = np.full(T, 300)
    law = lambda r, idx: r.integers(0, 300 - 100 + 1, size=idx.size)
    w = simulate("config1", g, n, m, law, 0.02, 0.005,
                 lambda r, k: r.integers(1, 4, size=k), rng,
                 params=dict(p_sub=0.02, p_ind=0.005, indel="uniform{1,2,3}"))
    w.seed = seed
    return w


def config2(seed: int = 102, genome_seed: int = 1, n_reads: int = 1_000_000) -> Workload:
    """Mate-rescue windows: reads x 100 bp vs 250 bp windows from a 1 Mbp
    genome.  Fragment F ~ N(500, 50^2) places the read at clamp(75 + F - 500,
    0, 150) in its window.  2% substitutions, 0.5% indel events with
    Geometric(1/2) length (mean 2); 10% of reads are uniform random."""
    g = random_genome(1_000_000, genome_seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.full(n_reads, 100)
    m = np.full(n_reads, 250)

    def law(r, idx):
        f = np.rint(r.normal(500.0, 50.0, size=idx.size)).astype(np.int64)
        return np.clip(75 + f - 500, 0, 150)

    w = simulate("config2", g, n, m, law, 0.02, 0.005,
                 lambda r, k: _geometric_trunc(r, 0.5, k, 0), rng, random_frac=0.10,
                 params=dict(p_sub=0.02, p_ind=0.005, indel="geometric(1/2)", random_frac=0.1))
    w.seed = seed
    return w


CONFIG3_LENGTHS = (36, 50, 75, 100, 150, 250)


def config3(seed: int = 103, genome_seed: int = 1, n_reads: int = 2_000_000,
            lengths=CONFIG3_LENGTHS) -> Workload:
    """Uneven batch: read length uniform over {36,50,75,100,150,250}, window
    m = n + 2*30 + 100; 4% substitutions, 0.5% indel events with
    Geometric(1/4) length truncated at 30."""
    g = random_genome(1_000_000, genome_seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = rng.choice(np.asarray(lengths), size=n_reads)
    m = n + 160
    law = lambda r, idx: r.integers(0, 161, size=idx.size)
    w = simulate("config3", g, n, m, law, 0.04, 0.005,
                 lambda r, k: _geometric_trunc(r, 0.25, k, 30), rng,
                 params=dict(p_sub=0.04, p_ind=0.005, indel="geometric(1/4)<=30"))
    w.seed = seed
    return w


def short_reads(n: int, n_reads: int = 2_000_000, seed: int = 108, genome_seed: int = 1) -> Workload:
    """Short reads of n bases against windows of n + 160 (the uneven batch's
    window rule and error model): the shapes with 32-64 tasks per wavefront,
    where the paper's word-interleaved read layout could matter."""
    g = random_genome(1_000_000, genome_seed)
    rng = np.random.Generator(np.random.PCG64(seed + n))
    nn = np.full(n_reads, n)
    m = nn + 160
    law = lambda r, idx: r.integers(0, 161, size=idx.size)
    w = simulate(f"short{n}", g, nn, m, law, 0.04, 0.005,
                 lambda r, k: _geometric_trunc(r, 0.25, k, 30), rng,
                 params=dict(p_sub=0.04, p_ind=0.005, indel="geometric(1/4)<=30"))
    w.seed = seed + n
    return w


def config5(seed: int = 105, genome_seed: int = 1, n_reads: int = 500_000) -> Workload:
    """Low-similarity tail: reads x 150 bp vs 1,000 bp windows; per-read
    identity p ~ U[0.60, 0.75], divergence d = 1 - p split as p_sub = 0.75 d
    and indel events p_ind = 0.05 d of Geometric(0.2) length (mean 5)
    truncated at 50."""
    g = random_genome(1_000_000, genome_seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.full(n_reads, 150)
    m = np.full(n_reads, 1000)
    ident = rng.uniform(0.60, 0.75, size=n_reads)
    d = 1.0 - ident
    law = lambda r, idx: r.integers(0, 1000 - 150 + 1, size=idx.size)
    w = simulate("config5", g, n, m, law, 0.75 * d, 0.05 * d,
                 lambda r, k: _geometric_trunc(r, 0.2, k, 50), rng,
                 params=dict(identity="U[0.60,0.75]", p_sub="0.75d", p_ind="0.05d",
                             indel="geometric(0.2)<=50"))
    w.seed = seed
    return w


@dataclasses.dataclass
class MultiWorkload:
    """Reads with lists of candidate regions (the multi-candidate call).

    read_codes, read_off, read_len   the reads (base codes, one per byte)
    cand_start int64[R+1]  read r owns candidates [cand_start[r], cand_start[r+1])
    cand_off   int64[C]    window start in ``genome`` (bases)
    cand_len   int32[C]    window length
    cand_support int32[C]  ranking key (supporting seeds)
    cand_strand uint8[C]   1: the read's reverse complement aligns to the window
    true_cand  int64[R]    the candidate the read was simulated from
    """

    name: str
    genome: np.ndarray
    read_codes: np.ndarray
    read_off: np.ndarray
    read_len: np.ndarray
    cand_start: np.ndarray
    cand_off: np.ndarray
    cand_len: np.ndarray
    cand_support: np.ndarray
    cand_strand: np.ndarray
    true_cand: np.ndarray
    seed: int = 0
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def n_reads(self) -> int:
        return int(self.read_len.size)

    @property
    def n_cands(self) -> int:
        return int(self.cand_len.size)


def multi_candidate(n_reads: int = 200_000, seed: int = 106, genome_seed: int = 1,
                    lengths=(100, 150), flank: int = 30, mean_cands: float = 12.0,
                    max_cands: int = 40, max_support: int = 20) -> MultiWorkload:
    """Candidate lists per read (stand-in for step 3's seed hits): each read
    is simulated from a window of n + 2*flank bases with config3's error
    model and is reverse-complemented with probability 1/2 (its candidate
    then has strand 1).  A read has 1 + Poisson(mean_cands - 1) candidates
    (at most max_cands): the true window and random decoy windows of the
    same length and random strand, in random order; supports are uniform
    over 1..max_support for all of them, so with a ceiling below the count
    the true window is sometimes not aligned."""
    g = random_genome(1_000_000, genome_seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = rng.choice(np.asarray(lengths), size=n_reads).astype(np.int64)
    m = n + 2 * flank
    law = lambda r, idx: r.integers(0, 2 * flank + 1, size=idx.size)
    w = simulate("multi-true", g, n, m, law, 0.03, 0.005,
                 lambda r, k: _geometric_trunc(r, 0.25, k, 30), rng)
    rc = rng.random(n_reads) < 0.5
    codes = w.read_codes.copy()
    for r in np.nonzero(rc)[0]:
        a, b = int(w.read_off[r]), int(w.read_off[r] + w.read_len[r])
        codes[a:b] = 3 - codes[a:b][::-1]
    k = np.minimum(1 + rng.poisson(mean_cands - 1.0, size=n_reads), max_cands).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(k)]).astype(np.int64)
    C = int(start[-1])
    owner = np.repeat(np.arange(n_reads), k)
    cm = m[owner].astype(np.int32)
    coff = rng.integers(0, len(g) - cm + 1).astype(np.int64)
    strand = (rng.random(C) < 0.5).astype(np.uint8)
    support = rng.integers(1, max_support + 1, size=C).astype(np.int32)
    true_pos = start[:-1] + rng.integers(0, k)          # a random slot of each read's list
    coff[true_pos] = w.ref_off
    strand[true_pos] = rc.astype(np.uint8)
    return MultiWorkload("multi", g, codes, w.read_off.copy(), w.read_len.copy(), start, coff, cm,
                         support, strand, true_pos.astype(np.int64), seed,
                         dict(lengths=list(lengths), flank=flank, mean_cands=mean_cands,
                              max_cands=max_cands, max_support=max_support, p_sub=0.03,
                              p_ind=0.005, rc_frac=0.5))


SERVE_LENGTHS = (50, 75, 100, 150, 250)


def serving_genome(seed: int = 4, length: int = 100_000_000) -> np.ndarray:
    return random_genome(length, seed)


def serving_request(genome: np.ndarray, rng, lengths=SERVE_LENGTHS, max_batch: int = 4096) -> Workload:
    """One request of the served workload: batch size floor(exp(U(0, ln 4097)))
    in [1, 4096], read lengths uniform over {50,75,100,150,250}, windows
    m = n + 160 as (offset, length) into the resident genome, error model as
    the uneven batch."""
    b = int(math.floor(math.exp(rng.uniform(0.0, math.log(max_batch + 1)))))
    b = max(1, min(max_batch, b))
    n = rng.choice(np.asarray(lengths), size=b)
    m = n + 160
    law = lambda r, idx: r.integers(0, 161, size=idx.size)
    return simulate("serve", genome, n, m, law, 0.04, 0.005,
                    lambda r, k: _geometric_trunc(r, 0.25, k, 30), rng)


def serving_pool(genome: np.ndarray, n_reads: int, seed: int = 104,
                 lengths=SERVE_LENGTHS) -> Workload:
    """A pool of served reads over the resident genome: lengths uniform over
    {50,75,100,150,250}, windows m = n + 160 at uniform genome positions, the
    uneven batch's error model.  Requests are consecutive slices of it."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = rng.choice(np.asarray(lengths), size=n_reads)
    m = n + 160
    law = lambda r, idx: r.integers(0, 161, size=idx.size)
    w = simulate("serve-pool", genome, n, m, law, 0.04, 0.005,
                 lambda r, k: _geometric_trunc(r, 0.25, k, 30), rng,
                 params=dict(p_sub=0.04, p_ind=0.005, indel="geometric(1/4)<=30"))
    w.seed = seed
    return w


def request_sizes(count: int, seed: int, max_batch: int = 4096) -> np.ndarray:
    """Batch sizes floor(exp(U(0, ln(max_batch + 1)))) in [1, max_batch]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    b = np.floor(np.exp(rng.uniform(0.0, math.log(max_batch + 1), size=count))).astype(np.int64)
    return np.clip(b, 1, max_batch)


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Open-loop arrival times (seconds from start) of a Poisson process."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def random_tasks(rng, n_tasks: int, n_range=(1, 40), m_range=(1, 60), genome_len: int = 5000,
                 related: float = 0.7) -> Workload:
    """Small mixed tasks for parity and edge-case tests: lengths uniform in the
    given ranges; a fraction of reads are edited copies of their window, the
    rest uniform random."""
    g = rng.integers(0, 4, size=genome_len, dtype=np.uint8)
    n = rng.integers(n_range[0], n_range[1] + 1, size=n_tasks)
    m = rng.integers(m_range[0], m_range[1] + 1, size=n_tasks)
    off = rng.integers(0, genome_len - m + 1)
    reads = np.zeros((n_tasks, max(int(n.max()), 1)), dtype=np.uint8)
    for t in range(n_tasks):
        win = g[off[t]:off[t] + m[t]]
        if rng.random() < related and m[t] > 0:
            s = int(rng.integers(0, m[t]))
            src = np.resize(win[s:], n[t]) if m[t] - s > 0 else rng.integers(0, 4, size=n[t])
            src = src.astype(np.uint8)
            flip = rng.random(n[t]) < 0.1
            src[flip] = rng.integers(0, 4, size=int(flip.sum()), dtype=np.uint8)
            # a few random indels
            if n[t] > 4 and rng.random() < 0.5:
                p = int(rng.integers(1, n[t] - 1))
                k = int(rng.integers(1, 4))
                if rng.random() < 0.5:
                    src = np.concatenate([src[:p], rng.integers(0, 4, size=k, dtype=np.uint8), src[p:]])[:n[t]]
                else:
                    src = np.concatenate([src[:p], src[p + k:], rng.integers(0, 4, size=k, dtype=np.uint8)])[:n[t]]
            reads[t, :n[t]] = src
        else:
            reads[t, :n[t]] = rng.integers(0, 4, size=n[t], dtype=np.uint8)
    return _assemble("random", g, reads, n, off, m, np.full(n_tasks, -1), 0, {})


def from_strings(pairs, pad: int = 0) -> Workload:
    """Tasks from (read, window) string pairs over ACGT (tests)."""
    lut = {c: i for i, c in enumerate(ALPHABET)}
    reads = [np.array([lut[c] for c in r], dtype=np.uint8) for r, _ in pairs]
    wins = [np.array([lut[c] for c in w], dtype=np.uint8) for _, w in pairs]
    g = np.concatenate(wins + [np.zeros(pad, dtype=np.uint8)]) if wins else np.zeros(max(pad, 1), np.uint8)
    n = np.array([len(r) for r in reads], dtype=np.int64)
    m = np.array([len(w) for w in wins], dtype=np.int64)
    woff = np.zeros(len(pairs), dtype=np.int64)
    if len(pairs):
        woff[1:] = np.cumsum(m)[:-1]
    roff = np.zeros(len(pairs), dtype=np.int64)
    if len(pairs):
        roff[1:] = np.cumsum(n)[:-1]
    codes = np.concatenate(reads) if reads and n.sum() else np.zeros(0, dtype=np.uint8)
    return Workload("strings", g, codes, roff, n.astype(np.int32), woff, m.astype(np.int32),
                    np.full(len(pairs), -1, dtype=np.int32))


# --------------------------------------------------------------------------
# Read pairs for mate rescue.

ORIENT_SAME = {0: False, 1: True, 2: False, 3: True}   # FR, FF, RF, FF with the mate upstream
ORIENT_UP = {0: False, 1: False, 2: True, 3: True}


@dataclasses.dataclass
class MateWorkload:
    """Pairs with one end aligned, for the mate-rescue call.

    read_codes, read_off, read_len   the unaligned ends (as sequenced)
    mate_pos   int64[R]  leftmost forward-strand base of the aligned end
    mate_len   int32[R]  its length
    mate_strand uint8[R] its strand (0 forward, 1 reverse)
    v, u, orientation    fragment length range and orientation code
    true_pos   int64[R]  leftmost forward-strand base of the unaligned end
                         before sequencing errors (-1 for random reads)
    true_strand uint8[R] its strand
    frag       int64[R]  simulated fragment length
    """

    name: str
    genome: np.ndarray
    read_codes: np.ndarray
    read_off: np.ndarray
    read_len: np.ndarray
    mate_pos: np.ndarray
    mate_len: np.ndarray
    mate_strand: np.ndarray
    v: int
    u: int
    orientation: int
    true_pos: np.ndarray
    true_strand: np.ndarray
    frag: np.ndarray
    seed: int = 0
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def n_reads(self) -> int:
        return int(self.read_len.size)


def mate_pairs(n_pairs: int = 1_000_000, seed: int = 107, genome_seed: int = 1, n: int = 100,
               n_mapped: int = 100, frag_mean: float = 500.0, frag_sd: float = 50.0,
               v: int = 425, u: int = 575, orientation: int = 0, p_sub: float = 0.02,
               p_ind: float = 0.005, random_frac: float = 0.10, genome=None) -> MateWorkload:
    """Simulated pairs: fragments of length rint(N(frag_mean, frag_sd^2))
    (at least max(n, n_mapped)) at uniform genome positions.  The aligned
    end has a random strand and sits at one outer end of its fragment, the
    unaligned end at the other, as the orientation code says (0 FR: opposite
    strand, downstream; 1 FF: same strand, downstream; 2 RF: opposite,
    upstream; 3: same strand, upstream).  The unaligned end is walked from
    the genome with config2's error model and reverse-complemented when it
    lies on the reverse strand; random_frac of them are uniform random.
    The default (1,000,000 pairs of 100 bp, v = 425, u = 575) gives
    250 bp regions, the mate-rescue batch's shape."""
    g = random_genome(1_000_000, genome_seed) if genome is None else genome
    G = len(g)
    rng = np.random.Generator(np.random.PCG64(seed))
    R = n_pairs
    frag = np.rint(rng.normal(frag_mean, frag_sd, size=R)).astype(np.int64)
    frag = np.maximum(frag, max(n, n_mapped))
    a = rng.integers(0, G - frag + 1)
    s = (rng.random(R) < 0.5).astype(np.int64)
    up = ORIENT_UP[orientation]
    higher = (s == 0) != up                  # the unaligned end lies toward higher coordinates
    mate_pos = np.where(higher, a, a + frag - n_mapped)
    true_pos = np.where(higher, a + frag - n, a)
    true_strand = s if ORIENT_SAME[orientation] else 1 - s
    nn = np.full(R, n, dtype=np.int64)
    # walk each unaligned end forward from its true start (slack for deletions)
    slack = np.minimum(G - true_pos, n + 64)
    reads, ok = _walk(rng, g, true_pos, slack, nn, np.zeros(R, np.int64), np.full(R, p_sub),
                      np.full(R, p_ind), lambda r, k: _geometric_trunc(r, 0.5, k, 0))
    bad = ~ok
    if bad.any():   # ran past the slack: redraw those without indels
        idx = np.nonzero(bad)[0]
        r2, _ = _walk(rng, g, true_pos[idx], np.full(idx.size, n), nn[idx],
                      np.zeros(idx.size, np.int64), np.full(idx.size, p_sub),
                      np.zeros(idx.size), lambda r, k: _geometric_trunc(r, 0.5, k, 0))
        reads[idx] = r2
    rev = true_strand == 1
    reads[rev] = 3 - reads[rev][:, ::-1]
    rnd = rng.random(R) < random_frac
    reads[rnd] = rng.integers(0, 4, size=(int(rnd.sum()), n), dtype=np.uint8)
    tp = np.where(rnd, -1, true_pos)
    return MateWorkload("mate", g, reads.reshape(-1).astype(np.uint8),
                        np.arange(R, dtype=np.int64) * n, nn.astype(np.int32),
                        mate_pos.astype(np.int64), np.full(R, n_mapped, np.int32),
                        s.astype(np.uint8), v, u, orientation, tp.astype(np.int64),
                        true_strand.astype(np.uint8), frag, seed,
                        dict(frag_mean=frag_mean, frag_sd=frag_sd, p_sub=p_sub, p_ind=p_ind,
                             random_frac=random_frac))
