"""Property test of the C ABI's parameter checks (no GPU needed): random
kzk_params, valid and invalid in every field, are classified the way the
header states (grid sizes first: KZK_ERR_SIZE; then KZK_ERR_ARG for the other
fields), and no rejected call leaves a plan behind.  Valid parameters go on
to device work, which needs a GPU: without one the call fails there, with one
it succeeds (and the plan is destroyed)."""
import ctypes
import math

from hypothesis import given, settings, strategies as st

from test_abi import _params

SIZE, ARG = 2, 1
POW2_TAU = [32, 64, 512, 8192]
GEN_TAU = [224, 448, 3584, 7168]
BAD_TAU = [0, 16, 48, 96, 112, 480, 14336, 16384, -64]
POW2_Y = [16, 256, 4096, 8192]
BAD_Y = [0, 8, 12, 448, 16384]
REAL = st.sampled_from([1e-3, 0.5, 0.0, -1.0, math.inf, math.nan])


def expected(k):
    size_ok = (k["n_tau"] in POW2_TAU + GEN_TAU) and (k["n_y"] in POW2_Y)
    if not size_ok:
        return SIZE
    fin = math.isfinite
    arg_ok = (k["L_tau"] > 0 and k["h"] > 0 and fin(k["h"]) and k["dtype"] in (0, 1) and k["A"] >= 0 and fin(k["A"])
              and fin(k["D"]) and fin(k["nl"]) and k["weno_eps"] > 0 and k["lf_scope"] == 0
              and not (k["cfl_max"] < 0) and k["scheme"] in (0, 1) and k["reg_eps"] >= 0 and fin(k["reg_eps"])
              and k["vel"] == 0 and k["state_fp64"] in (0, 1)
              and not (k["state_fp64"] == 1 and k["dtype"] == 0 and k["reg_eps"] > 0))
    return None if arg_ok else ARG


@settings(max_examples=400, deadline=None)
@given(n_tau=st.sampled_from(POW2_TAU + GEN_TAU + BAD_TAU), n_y=st.sampled_from(POW2_Y + BAD_Y),
       L_tau=st.sampled_from([8.0, 0.0, -8.0, math.nan]), h=REAL, dtype=st.sampled_from([0, 1, 2, -1]),
       A=st.sampled_from([0.0, 1e-4, -1e-4, math.inf, math.nan]), D=REAL, nl=REAL,
       weno_eps=st.sampled_from([1e-6, 0.0, -1e-6, math.nan]), lf_scope=st.sampled_from([0, 1]),
       cfl_max=st.sampled_from([0.0, 1.0, -1.0]), scheme=st.sampled_from([0, 1, 2]),
       reg_eps=st.sampled_from([0.0, 2.0 ** -24, -1e-9, math.inf, math.nan]), vel=st.sampled_from([0, 0, 0, 1, 2]),
       state_fp64=st.sampled_from([0, 1, 3]))
def test_create_classifies_parameters_as_documented(**k):
    from paper_2103_06080_amd import kzk
    L = kzk.lib()
    p = _params(**k)
    h = ctypes.c_void_p()
    code = L.kzk_create(ctypes.byref(p), 1, None, ctypes.byref(h))
    want = expected(k)
    if want is not None:
        assert code == want, (k, code)
        assert not h.value
    else:
        assert code not in (SIZE, ARG), (k, code)
        if code == 0:
            L.kzk_destroy(h)
        else:
            assert not h.value
