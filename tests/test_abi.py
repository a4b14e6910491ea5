"""The C ABI without a GPU: the library loads, exports what the header
declares, and its pure host functions and argument checks behave."""
import ctypes as C
import os

import pytest

from paper_2109_07527_amd import crmc

pytestmark = pytest.mark.skipif(not os.path.exists(crmc.LIB_PATH), reason="libcrmc.so not built")


def test_every_declared_symbol_is_exported():
    L = crmc.load()
    names = crmc.header_symbols()
    assert "crmc_create" in names and "crmc_sweep" in names and "crmc_observe" in names
    assert "crmc_build_cells" in names
    for n in names:
        assert hasattr(L, n), n


def test_pIX_from_salt_matches_closed_form():
    from oracle import closed_forms as cf
    for pIS, pH in [(1.0, 7.0), (2.0, 4.5), (6.0, 7.5), (3.0, 11.0), (-1.0, 2.0)]:
        assert crmc.crmc_pIX_from_salt(pIS, pH) == pytest.approx(cf.pIX_from_salt(pIS, pH), abs=1e-13)


def test_ungrouping_shares_complete_the_combined_ions():
    """With pI_X from eq. pIXgen, the salt ion and H+ make up the whole X+ at
    pH <= 7 and the salt ion and OH- the whole X- at pH >= 7; the salt share
    is 10^(pI_X - pI_S) whatever the pH, and a NULL output is an error."""
    from oracle import closed_forms as cf
    for pIS, pH in [(2.0, 4.5), (1.0, 6.9), (3.0, 2.0), (2.0, 7.0), (2.5, 9.5), (0.5, 12.0)]:
        pIX = cf.pIX_from_salt(pIS, pH)
        f = crmc.crmc_ungroup_fractions(pH, pIS, pIS, pIX, pIX)
        if pH <= 7.0:
            assert f["S_pos"] + f["H"] == pytest.approx(1.0, abs=1e-12)
            assert f["S_neg"] + f["OH"] < 1.0 or pH == 7.0
        if pH >= 7.0:
            assert f["S_neg"] + f["OH"] == pytest.approx(1.0, abs=1e-12)
        assert f["S_pos"] == pytest.approx(10.0 ** (pIX - pIS), rel=1e-12)
        assert f["S_pos"] == pytest.approx(f["S_neg"], rel=1e-12)
    L = crmc.load()
    assert L.crmc_ungroup_fractions(7.0, 14.0, 2.0, 2.0, 1.9, 1.9, None) == crmc.CRMC_E_ARG


def _params(**kw):
    p = crmc.crmc_params()
    p.n_replicas, p.precision, p.trials_per_cell, p.pairing, p.ion_coupling = 1, 32, 1, 1, 1
    p.lB, p.rc, p.eps_wca, p.rho0NA, p.pKw, p.kappa, p.pKb = 2.0, 6.0, 1.0, 0.0269424, 14.0, 0.5, 5.0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("bad", [dict(precision=16), dict(trials_per_cell=0), dict(rc=0.0),
                                 dict(n_replicas=0), dict(rho0NA=-1.0), dict(lds_records=-5),
                                 dict(lB=-1.0), dict(ion_trials=-1), dict(ion_trials=5000)])
def test_create_rejects_invalid_parameters(bad):
    L = crmc.load()
    h = C.c_void_p()
    rc = L.crmc_create(C.byref(_params(**bad)), C.byref(h))
    assert rc == crmc.CRMC_E_ARG
    assert not h.value


def test_null_arguments():
    L = crmc.load()
    assert L.crmc_create(None, None) == crmc.CRMC_E_ARG
    assert L.crmc_sweep(None, 7.0, 4.5, 1.0, 1) == crmc.CRMC_E_ARG
    n = C.c_int64(0)
    assert L.crmc_export_state(None, None, C.byref(n)) == crmc.CRMC_E_ARG
    assert L.crmc_import_state(None, None, 0) == crmc.CRMC_E_ARG
    L.crmc_destroy(None)


def test_workspace_size_and_attach_on_the_host():
    """Creating and building touch no device: the workspace size of built
    replicas is known on the host (it grows with the replicas), and the
    attach call checks its arguments and refuses a second workspace."""
    from workloads import nanoparticle_pair
    s = nanoparticle_pair(seed=4, L=40.0, R=4.0, sites=120, separation=11.0)
    S = crmc.System(n_replicas=2, lB=2.0, rc=6.0, stream=None)
    with pytest.raises(crmc.CrmcError) as ei:
        S.workspace_size()
    assert ei.value.code == crmc.CRMC_E_STATE
    S.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    S.build_cells(1, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    n2 = S.workspace_size()
    one = crmc.System(n_replicas=1, lB=2.0, rc=6.0, stream=None)
    one.build_cells(0, L=s["L"], xyz=s["xyz"], kind=s["kind"], core_xyz=s["core_xyz"], core_R=s["core_R"])
    n1 = one.workspace_size()
    # two replicas hold two sets of records (2 buffers x cells x capacity x 16 bytes)
    obs_cells = 6 ** 3
    assert n2 - n1 >= 2 * obs_cells * 16 * 64
    assert S.memory() == dict(own=0, workspace_used=0, workspace_largest_free=0)
    with pytest.raises(crmc.CrmcError):
        crmc.crmc_set_workspace(S.h, 0, n2)
    crmc.crmc_set_workspace(S.h, 1 << 40, n2)  # never dereferenced: no call here needs the device
    assert S.memory()["workspace_largest_free"] >= n2 - 256
    with pytest.raises(crmc.CrmcError) as ei:
        crmc.crmc_set_workspace(S.h, 1 << 40, n2)
    assert ei.value.code == crmc.CRMC_E_STATE
    S.close()
    one.close()
