"""The C-ABI library loads and exports every symbol include/lwe.h declares, and its
parameter registry (sizes, CDF tables) agrees with the oracle.  No device work here."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lwe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lwe_[A-Za-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    from paper_2606_01211_amd import lwe

    L = lwe.lib()
    decl = _declared()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(lwe.EXPORTS) == decl
    # argument checks that touch no device
    assert L.lwe_ctx_set_side_stream(None, 1) == lwe.LWE_EINVAL
    assert L.lwe_ctx_set_hash_lanes(None, 1) == lwe.LWE_EINVAL
    assert L.lwe_ctx_stream(None) is None


@pytest.mark.parametrize("n", [640, 976, 1344, 4096, 8192, 16384, 32768])
def test_registry_matches_oracle(orc, n):
    import paper_2606_01211_amd as L

    p = L.params(L.param_id(n))
    o = orc.params_for(n)
    assert (p.n, p.logq, p.B, p.K) == (o.n, o.logq, o.B, o.K)
    assert p.sigma == o.sigma
    assert (p.pk_bytes, p.sk_bytes, p.ct_bytes, p.mu_bytes) == (o.pk_bytes, o.sk_bytes, o.ct_bytes, o.mu_bytes)
    assert np.array_equal(L.cdf_table(p.pid), orc.cdf_table(o.K, o.sigma))


def test_register_custom_and_reject_bad():
    import paper_2606_01211_amd as L
    from paper_2606_01211_amd.lwe import LweError

    pid = L.register_params(200, 16, 2, 6, 1.4)
    assert L.register_params(200, 16, 2, 6, 1.4) == pid
    assert L.params(pid).n == 200
    for bad in [(201, 16, 2, 6, 1.4), (200, 17, 2, 6, 1.4), (200, 16, 16, 6, 1.4), (200, 16, 2, 0, 1.4),
                (200, 16, 2, 6, -1.0), (65536, 16, 2, 6, 1.4)]:
        with pytest.raises(LweError):
            L.register_params(*bad)
    with pytest.raises(KeyError):
        L.param_id(1000)


def test_sizes():
    import paper_2606_01211_amd as L

    p = L.params(L.param_id(1344))
    assert (p.pk_bytes, p.sk_bytes, p.ct_bytes, p.mu_bytes) == (21520, 43088, 21632, 32)
    p = L.params(L.param_id(32768))
    assert (p.pk_bytes, p.ct_bytes) == (524304, 524416)
