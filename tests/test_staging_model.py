"""CPU model of the LDS staging of the main sweep kernel (staging.hpp: stage_window /
stage_pairs / read_window): the index maps that decide which lane loads which stream
position into which window slot, checked on random chunk layouts.  The invariants
are what make the shipped kernel's ordering safe:
  1. within a window every slot (segment src, position t) is written by exactly one
     lane, in one round, and read back by exactly one lane, src itself;
  2. the slot read by lane src at position t holds stream position s0 + t of src's
     own segment (or the padding (EMPTY, 0) past its end);
  3. the key-stream entry of position e is written in pass 1 and read in pass 2 by the
     same lane (the two passes stage with the same map), so pass 2 needs no fence:
     one thread's store and later load of one address stay in program order;
  4. consecutive windows reuse the same slots, so a write of window s0 + WIN must not
     move above a read of window s0 -- the wave_sync after read_window orders them."""
import numpy as np
import pytest

WAVE, WIN = 64, 16
SPR = WAVE // WIN


def stage_map(lo, hi, s0):
    """(lane, round) -> (segment src, position t, stream index e or None)."""
    out = {}
    for lane in range(WAVE):
        for r in range(WIN):
            src = r * SPR + lane // WIN
            t = lane % WIN
            e = lo[src] + s0 + t
            out[(lane, r)] = (src, t, e if e < hi[src] else None)
    return out


@pytest.mark.parametrize("seed", range(5))
def test_staging_maps(seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 130, size=WAVE)
    lo = np.concatenate([[0], np.cumsum(lens)[:-1]])
    hi = lo + lens
    maxlen = int(lens.max())
    writer = {}  # stream index -> lane that staged it (pass 1)
    for s0 in range(0, maxlen, WIN):
        m = stage_map(lo, hi, s0)
        slots = {}
        for (lane, r), (src, t, e) in m.items():
            assert (src, t) not in slots          # 1: one writer per slot
            slots[(src, t)] = (lane, e)
            if e is not None:
                assert e not in writer
                writer[e] = lane
        assert len(slots) == WAVE * WIN
        for src in range(WAVE):                   # 2: lane src reads its own positions
            for t in range(WIN):
                _, e = slots[(src, t)]
                want = lo[src] + s0 + t
                assert e == (want if want < hi[src] else None)
        m2 = stage_map(lo, hi, s0)                # 3: pass 2 uses the same map
        for (lane, r), (_, _, e) in m2.items():
            if e is not None:
                assert writer[e] == lane
    assert sorted(writer) == [e for s in range(WAVE) for e in range(lo[s], hi[s])]
