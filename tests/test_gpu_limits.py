"""Device workspace bound from the environment (NCF_WORKSPACE_LIMIT_MB).

The library reads the variable once per process, so each case runs in a
subprocess of its own. A call whose arenas would exceed the bound returns
NCF_E_NOMEM with a message naming the variable, allocates nothing, and
leaves the library usable: a smaller call in the same process still
succeeds and matches the oracle.
"""
from __future__ import annotations

import os
import subprocess
import sys
import textwrap

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASE = textwrap.dedent("""
    import sys
    sys.path.insert(0, ".")
    import numpy as np
    from oracle import oracle as O
    from paper_2609_03866_amd import ncf, synth

    def tiny():
        rng = np.random.default_rng(3)
        t = np.sort(rng.uniform(0.0, 50.0, 60))
        x = rng.normal(size=60)
        lags = np.arange(0.0, 6.0)
        c, b, n, rc = ncf.acf(t, x, lags, "rectangle", 0.5, raise_on_error=False)
        assert rc == 0, (rc, ncf.lib().ncf_last_error())
        st, oc, ob, on = O.acf(t, x, lags, "rectangle", 0.5)
        assert st == 0 and np.array_equal(n, on) and np.max(np.abs(c - oc)) <= 1e-12

    tiny()
    d = synth.c2(seed=7, n=20_000)
    c, b, n, rc = ncf.ccf(d["t"], d["x"], d["s"], d["y"], d["lags"], "gaussian", d["h"],
                          raise_on_error=False)
    msg = ncf.lib().ncf_last_error()
    assert rc == ncf.E_NOMEM, (rc, msg)
    assert b"NCF_WORKSPACE_LIMIT_MB" in msg, msg
    tiny()
    print("limit ok")
""")


def test_workspace_limit_returns_nomem_and_leaves_the_library_usable():
    env = dict(os.environ, NCF_WORKSPACE_LIMIT_MB="2")
    print("case: NCF_WORKSPACE_LIMIT_MB=2, c2-shaped CCF n=2e4 must fail, tiny ACF must pass",
          flush=True)
    r = subprocess.run([sys.executable, "-c", CASE], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "limit ok" in r.stdout
