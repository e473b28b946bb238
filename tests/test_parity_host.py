"""Host-side helpers of the parity tests (no GPU)."""
import pytest

from parity import rounding_envelope


def test_rounding_envelope_by_hand():
    rows = lambda es: [{"t": 0.1 * k, "e_kin": e, "e_pot": 0.0, "e_int": 0.0} for k, e in enumerate(es)]
    gold = rows([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    p1 = rows([1.0, 1.0, 1.02, 1.0, 1.0, 1.0, 1.0, 1.0])
    p2 = rows([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.97])
    env = rounding_envelope(gold, [p1, p2], 1.0, half_window=0.2)
    assert env == pytest.approx([0.02, 0.02, 0.02, 0.02, 0.02, 0.03, 0.03, 0.03])
    env = rounding_envelope(gold, [p1, p2], 1.0, half_window=0.0)
    assert env == pytest.approx([0.0, 0.0, 0.02, 0.0, 0.0, 0.0, 0.0, 0.03])
