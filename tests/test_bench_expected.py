"""The benchmark's stored oracle values (tests/golden/bench_expected.json) are
the oracle's: their offsets address the entries they claim in the block
storage of Section 2.1, and the smallest workload's values recompute bit for
bit from the oracle."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "golden", "bench_expected.json")


@pytest.fixture(scope="module")
def expected():
    with open(PATH) as f:
        return json.load(f)["cases"]


def test_cases_cover_the_benchmark(expected):
    for name in ["t-wishart-n16-t5000", "t-gamma-mix-n48-t100000", "laplace-mix-n24-t200000",
                 "ar1-garch-n64-t50000"]:
        w = workloads.WORKLOADS[name]
        rec = expected[name]
        assert (rec["n"], rec["b"], rec["t"]) == (w["n"], w["b"], w["t"])
        assert sorted(int(d) for d in rec["orders"]) == list(range(2, w["d_max"] + 1))
    assert sorted(expected["laplace-mix-n8-t20000-d10"]["orders"]) == ["10", "9"]
    assert sorted(expected["laplace-mix-n16-t20000-d8"]["orders"]) == ["7", "8"]


def test_offsets_address_every_diagonal_and_agree_with_the_library(expected):
    import paper_1701_05420_amd as pc

    for name, rec in expected.items():
        n, b = rec["n"], rec["b"]
        for ds, o in rec["orders"].items():
            d = int(ds)
            offs = np.array(o["offsets"], dtype=np.int64)
            assert len(offs) == len(o["kappa"]) == len(o["moment"]) and len(np.unique(offs)) == len(offs)
            idx = oracle.block_indices(n, d, b, offs)
            assert (idx >= 0).all()
            be = b ** d
            for off, ix in zip(offs, idx):
                # the library's canonical copy of this entry lies in the same block
                assert pc.stored_offset(n, d, b, sorted(ix.tolist())) // be == off // be
            diag = {pc.stored_offset(n, d, b, [i] * d) for i in range(n)}
            assert diag <= set(offs.tolist())


def test_values_recompute_from_the_oracle(expected):
    oracle.build()
    rec = expected["t-wishart-n16-t5000"]
    _, Xc = oracle.center(workloads.generate("t-wishart-n16-t5000"))
    for ds, o in rec["orders"].items():
        d = int(ds)
        idx = oracle.block_indices(rec["n"], d, rec["b"], np.array(o["offsets"], dtype=np.int64))
        got = oracle.cumulant_at(Xc, idx.astype(np.int32))
        assert np.array_equal(got, np.array(o["kappa"]))
        mom = np.prod(np.stack([Xc[:, idx[:, k]] for k in range(d)]), axis=0).mean(axis=0)
        assert np.allclose(mom, np.array(o["moment"]), rtol=1e-12, atol=0)
