"""Batch preparation of large unsorted batches: the MSD split into buckets
followed by a sort of every bucket in LDS, and its hand-off to the LSD radix
passes (batches below the split's size, low parts wider than 32 bits, buckets
larger than one block's LDS, batches above the split's size).  Every case
inserts an unsorted batch (with repeats) into a CPMA and checks the whole
exported image against the oracle's set through the structure checker; the
path taken is read from the sort phase's algorithmic bytes per key: 48 for
the split (count 8, split 12 as it writes 32-bit low parts, bucket sort with
repeat removal 12, packing 16), 40 when the validation counted the buckets
with the bit length of the previous large batch, 24 per LSD pass plus 24 for the repeat removal after
them, 24 for a sorted batch (repeat removal only)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

MSD = "msd"


def lsd(passes):
    return 24 * passes + 24


@pytest.fixture(scope="module")
def cp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_05055_amd as p
    p.lib()
    return p


def shuffled(a, seed):
    return a[np.random.default_rng(seed).permutation(len(a))]


def clustered(n, seed):
    """Two thirds uniform 40-bit keys, one third inside one 2^20-wide window:
    that window's bucket outgrows a block's LDS."""
    u = synth.uniform_keys(n - n // 3, seed, bits=40)
    c = np.uint64(0x5A5A500000) + synth.uniform_keys(n // 3, seed + 1, bits=20)
    return shuffled(np.concatenate([u, c]), seed + 2)


CASES = [
    # (name, batch generator, expected path)
    ("threshold_40bit", lambda s: synth.uniform_keys(1 << 19, s, bits=40), MSD),
    ("below_threshold", lambda s: synth.uniform_keys((1 << 19) - 1, s, bits=40), lsd(5)),
    ("narrow_20bit_repeats", lambda s: synth.uniform_keys(1_000_000, s, bits=20), MSD),
    ("low_part_33_bits", lambda s: synth.uniform_keys(1_000_000, s, bits=41), lsd(6)),
    # (one LSD pass would also count 48 bytes per key; the sequence test below
    # tells the two apart)
    ("byte_keys_no_low_part", lambda s: synth.uniform_keys(600_000, s, bits=8), MSD),
    ("zipf_overflowing_bucket", lambda s: shuffled(synth.zipf_keys(1_000_000, s, bits=34), s + 9), lsd(5)),
    ("clustered_overflowing_bucket", lambda s: clustered(3_000_000, s), lsd(5)),
    ("top_bucket_count_40bit", lambda s: synth.uniform_keys(20_000_000, s, bits=40), MSD),
]


def sort_bytes_per_key(c, k):
    return c.stats()["sort"][2] / k


def check_image(c, expect, orc):
    b, u, h = c.export()
    code, msg = orc.check_image(b, u, h, c.geometry()[1], expect)
    assert code == 0, msg
    assert c.size() == len(expect)


@pytest.mark.parametrize("name,gen,path", CASES, ids=[c[0] for c in CASES])
def test_large_unsorted_insert(cp, orc, name, gen, path):
    seed = synth.SEED_BASE + 1200 + 10 * CASES.index((name, gen, path))
    base = synth.uniform_keys(100_000, seed, bits=40)
    batch = gen(seed + 3)
    print(f"[batch sort] {name}: k={len(batch)}", flush=True)
    assert np.any(batch[1:] < batch[:-1]), "the batch must be unsorted"
    c = cp.CPMA(base)
    S = orc.build_set(base)
    S, added = orc.insert(S, batch)
    c.stats_select(["sort"])
    assert c.insert_batch(batch) == added
    per_key = sort_bytes_per_key(c, len(batch))
    assert per_key == (48 if path == MSD else path), per_key
    c.stats_select([])
    check_image(c, S, orc)


def test_large_unsorted_delete(cp, orc):
    """A delete batch takes the same preparation: half its keys present, half
    absent, with repeats, in random order.  Building from 2e6 unsorted keys
    prepared them the same way, so the delete's validation already counts the
    buckets with their bit length (40 bytes per key)."""
    seed = synth.SEED_BASE + 1300
    base = synth.unique_uniform_keys(2_000_000, seed, bits=40)
    c = cp.CPMA(base)
    S = orc.build_set(base)
    present = base[synth.sample_indices(len(base), 400_000, seed + 1)]
    absent = synth.uniform_keys(400_000, seed + 2, bits=40)
    batch = shuffled(np.concatenate([present, present[:100_000], absent]), seed + 3)
    S, removed = orc.delete(S, batch)
    c.stats_select(["sort"])
    assert c.delete_batch(batch) == removed
    assert sort_bytes_per_key(c, len(batch)) == 40
    c.stats_select([])
    check_image(c, S, orc)


def test_counts_with_the_previous_bit_length(cp, orc):
    """From the second large batch on, validation counts the buckets with the
    previous batch's bit length: the counts are used when the batch has no
    more bits than that and its buckets still fit (40 bytes per key), and the
    batch is recounted otherwise (48); a skewed batch still falls back to the
    LSD passes.  Every batch is checked
    against the oracle."""
    seed = synth.SEED_BASE + 1400
    base = synth.uniform_keys(100_000, seed, bits=40)
    c = cp.CPMA(base)
    S = orc.build_set(base)
    steps = [
        (synth.uniform_keys(1_000_000, seed + 1, bits=40), 48),   # no earlier bit length
        (synth.uniform_keys(1_000_000, seed + 2, bits=40), 40),   # same bits
        (synth.uniform_keys(1_000_000, seed + 3, bits=39), 40),   # fewer bits: counts hold
        # three bits fewer: the old split leaves 32 buckets of ~25000 keys,
        # more than a block's LDS holds, so the batch is recounted
        (synth.uniform_keys(800_000, seed + 4, bits=36), 48),
        (synth.uniform_keys(1_000_000, seed + 5, bits=38), 48),   # more bits: recounted
        (shuffled(synth.zipf_keys(1_000_000, seed + 6, bits=34), seed + 7), lsd(5)),
        (synth.uniform_keys(1_000_000, seed + 8, bits=40), 48),   # more bits than the skewed batch
        (np.sort(synth.unique_uniform_keys(1_000_000, seed + 9, bits=40)), 24),  # sorted: no sort
        # byte keys: the 40-bit split puts them all in one bucket, so they are
        # recounted with no low part; the next byte batch uses its counts
        (synth.uniform_keys(600_000, seed + 10, bits=8), 48),
        (synth.uniform_keys(600_000, seed + 11, bits=8), 40),
        # 44-bit keys leave a 36-bit low part: LSD passes, first after counts
        # for the byte keys' bit length, then with the validation counting
        # the first digit
        (synth.uniform_keys(1_000_000, seed + 12, bits=44), lsd(6)),
        (synth.uniform_keys(1_000_000, seed + 13, bits=44), lsd(6)),
        (synth.uniform_keys(1_000_000, seed + 14, bits=40), 48),  # the split again
    ]
    for step, (batch, per_key) in enumerate(steps):
        print(f"[batch sort] sequence step {step}: k={len(batch)}", flush=True)
        S, added = orc.insert(S, batch)
        c.stats_select(["sort"])
        assert c.insert_batch(batch) == added, step
        assert sort_bytes_per_key(c, len(batch)) == per_key, step
        c.stats_select([])
        check_image(c, S, orc)
