"""The diagnostic record against the oracle's, record by record, on the
same seeded inputs (through the C ABI): per-component field energies,
per-species kinetic energy and momentum, total particle momentum, field
momentum E x B, collision and particle counts."""
import numpy as np
import pytest

import synth
from pic_cases import gpu_run, log, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-9), ("mixed", 1e-4)])
def test_diagnostic_records_match_the_oracle(pic, prec, bar):
    log(f"case diagnostics {prec}")
    wl = synth.beam_plasma((64, 64), ppc=8, u_th_beam=0.2, nu=0.05, steps=40)
    parts = synth.load(wl)
    orc = oracle_run(wl, parts)
    g = gpu_run(wl, parts, pic.PIC_PREC_FP64 if prec == "fp64" else pic.PIC_PREC_MIXED, diag_every=1)
    orecs = orc.step(wl.steps, diag=True)
    g.step(wl.steps)
    grecs = g.history()
    g.close()
    assert [r["step"] for r in grecs] == [r["step"] for r in orecs]

    def close(a, b, scale):
        return np.max(np.abs(np.asarray(a) - np.asarray(b))) <= bar * scale

    Wmax = max(float(np.max(r["W"])) for r in orecs)
    Kmax = max(float(np.max(np.abs(r["kinetic"]))) for r in orecs)
    Pmax = max(float(np.max(np.abs(r["p_species"]))) for r in orecs)
    Fmax = max(float(np.max(np.abs(r["p_field"]))) for r in orecs)
    assert Wmax > 0 and Fmax > 0
    for gr, orr in zip(grecs, orecs):
        assert close(gr["W"], orr["W"], Wmax), gr["step"]
        assert close(gr["kinetic"], orr["kinetic"], Kmax), gr["step"]
        assert close(gr["p_species"], orr["p_species"], Pmax), gr["step"]
        assert close(gr["p_particles"], orr["p_particles"], Pmax), gr["step"]
        assert close(gr["p_field"], orr["p_field"], Fmax), gr["step"]
        assert gr["collisions"] == orr["collisions"]
        assert list(gr["n_particles"]) == [p.id.size for p in parts]
