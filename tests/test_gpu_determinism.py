"""Determinism: the same inputs give the same leaf image, bit for bit.  Two
sets built from the same keys take the same sequence of batches (large and
small, inserts and deletes, one that grows the set, one that redistributes
windows); after every batch their exported images (bytes, used counts, heads)
are identical.  The same holds for the uncompressed and key-value variants."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_05055_amd as p
    p.lib()
    return p


def same_image(a, b):
    ea, eb = a.export(), b.export()
    assert a.geometry() == b.geometry()
    for x, y in zip(ea, eb):
        assert np.array_equal(x, y)


def batches(seed):
    x0 = np.uint64(int(synth.uniform_keys(1, seed, bits=39)[0]))
    return [("i", synth.uniform_keys(200000, seed + 1, bits=40)),
            ("d", None),
            ("i", synth.uniform_keys(300, seed + 2, bits=40)),
            ("i", x0 + synth.uniform_keys(20000, seed + 3, bits=22)),
            ("i", synth.uniform_keys(600000, seed + 4, bits=40)),
            ("d", None)]


@pytest.mark.parametrize("variant", ["cpma", "pma", "kv"])
def test_same_inputs_same_images(cp, orc, variant):
    seed = synth.SEED_BASE + 5000
    base = synth.uniform_keys(300000, seed, bits=40)
    kw = {"uncompressed": variant == "pma"}
    if variant == "kv":
        kw["values"] = synth.uniform_keys(len(base), seed + 9, bits=64)
    a = cp.CPMA(base, leaf_bytes=512, **kw)
    b = cp.CPMA(base, leaf_bytes=512, **kw)
    same_image(a, b)
    present = orc.build_set(base)
    for i, (kind, keys) in enumerate(batches(seed + 10)):
        if kind == "d":
            keys = present[synth.sample_indices(len(present), len(present) // 5, seed + 20 + i)]
            assert a.delete_batch(keys) == b.delete_batch(keys)
            present = orc.delete(present, keys)[0]
        elif variant == "kv":
            vals = synth.uniform_keys(len(keys), seed + 30 + i, bits=64)
            assert a.insert_kv(keys, vals) == b.insert_kv(keys, vals)
            present = orc.insert(present, keys)[0]
        else:
            assert a.insert_batch(keys) == b.insert_batch(keys)
            present = orc.insert(present, keys)[0]
        same_image(a, b)
        if variant == "kv":
            assert np.array_equal(a.code_bytes(), b.code_bytes())
    a.close()
    b.close()
