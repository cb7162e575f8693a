"""Pin for the oracle's vertex move (CPU only): one step worked by hand."""
import numpy as np

from oracle import step


def test_one_step_by_hand():
    X = np.array([[1.0, -2.0], [0.5, 0.25]])
    upd = np.array([[0.1, 0.0], [-0.2, 0.3]])
    gains = np.array([[1.0, 0.5], [0.02, 2.0]])
    G = np.array([[0.01, -0.03], [-0.5, 0.0]])
    sp = step.StepParams(eta=10.0)
    Xn, un, gn = step.step(X, upd, gains, G, it=3, sp=sp)
    # (g>0, upd>0): (T,T) (F,F) / (F,F) (F,T)  ->  shrink shrink / shrink grow
    want_g = np.array([[0.8, 0.4], [0.016, 2.2]])
    want_g = np.maximum(want_g, 0.01)
    assert np.allclose(gn, want_g, rtol=1e-15)
    want_u = 0.5 * upd - 10.0 * want_g * G
    assert np.allclose(un, want_u, rtol=1e-15)
    assert np.allclose(Xn, X + want_u, rtol=1e-15)
    # late momentum and the n/12 learning rate rule
    Xn, un, gn = step.step(X, upd, gains, G, it=300, sp=step.StepParams())
    assert np.allclose(un, 0.8 * upd - 200.0 * gn * G)
    assert step.learning_rate(24000, step.StepParams()) == 2000.0


def test_gain_floor():
    X = np.zeros((1, 2))
    Xn, un, gn = step.step(X, np.array([[1.0, 1.0]]), np.array([[0.011, 0.5]]),
                           np.array([[1.0, 1.0]]), it=0, sp=step.StepParams(eta=1.0))
    assert np.allclose(gn, [[0.01, 0.4]])
