"""Comparisons shared by the GPU parity tests (no GPU code here)."""
import numpy as np


def compare_state(net, gs, os_, t):
    """Relative error 1e-5 of V against max(|V|, V_th - E) (the threshold
    distance is the voltage scale near 0 mV), of w against max(|w|, alpha);
    refractory counters exact."""
    Vg, Wg, Rg = gs
    Vo, Wo, Ro = os_
    tolV = 1e-5 * np.maximum(np.abs(Vo), net["v_th"] - net["e_rest"])
    dv = np.abs(Vg.astype(np.float64) - Vo)
    assert np.all(dv <= tolV), f"step {t}: V error {dv.max()} at {dv.argmax()} (V={Vo[dv.argmax()]})"
    tolw = 1e-5 * np.maximum(np.abs(Wo), net["alpha_w"])
    dw = np.abs(Wg.astype(np.float64) - Wo)
    assert np.all(dw <= tolw), f"step {t}: w error {dw.max()}"
    np.testing.assert_array_equal(Rg.astype(np.int32), Ro)


def pending_charge(oracle_mod, net, raster, T, j):
    """Charge queued for target j after steps 0..T-1, by arrival time T ..
    T - 1 + d_max: the oracle's synapses from the raster's recent spikers to
    j, each spike's charge placed at its step + the synapse's delay."""
    return oracle_mod.col_pending(net, int(j), raster, T)


def ring_pending(ring, net, T, j):
    """The ring's charge for target j arriving at T .. T - 1 + d_max."""
    return np.array([ring[(T + a) % ring.shape[0], j] for a in range(net["d_max"])], dtype=np.int64)
