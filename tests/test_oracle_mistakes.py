"""Planted mistakes: each entry edits a copy of the oracle's C source the way
a plausible slip would (a dropped term, a wrong sign, a swapped operand) and
checks that at least one of the listed pins, which never reuse the oracle's
own formulas, now fails.  A mistake no pin catches would be a gap in the
pins.  The Python oracles get theirs by replacing a module attribute.  CPU
only: the C copies are built with gcc into a temporary directory."""

import tempfile

import numpy as np
import pytest

from tests import test_oracle_backward as B
from tests import test_oracle_pins as T

MEANS = [(0.0, 0.0, 10.0), (1.3, -0.7, 9.0), (-2.0, 1.5, 14.0)]


def _single(orc):
    for m in MEANS:
        T.test_single_gaussian_closed_form(orc, m)


PINS = {
    "decode biases": T.test_decode_biases_only,
    "decode inputs": T.test_decode_input_distance_and_direction,
    "decode relu path": T.test_decode_relu_and_feature_path,
    "single Gaussian": _single,
    "two Gaussians": T.test_two_gaussians_front_to_back,
    "partition of unity": T.test_partition_of_unity_and_weights,
    "thr2 closed form": T.test_thr2_closed_form,
    "Eq. 7 literal": T.test_threshold_form_matches_literal_eq7,
    "skip certificate": T._check_skip_certificate,
    "backward FD": B.test_full_chain_gradcheck_fd,
}

# name: ([(exact source text, replacement)], pins expected to catch it)
MISTAKES = {
    "viewing direction reversed": (
        [("for (int a = 0; a < 3; ++a) x[F + 1 + a] = d[a] / dist;",
          "for (int a = 0; a < 3; ++a) x[F + 1 + a] = -d[a] / dist;")], ["decode inputs"]),
    "distance not relative to d_max": (
        [("x[F] = dist / d_max;", "x[F] = dist;")], ["decode inputs"]),
    "offset scaled by the base scale": (
        [("out[a * G + g] = (double)pos[3 * j + a] + (double)o[a] * (double)offset_scale[3 * j + a];",
          "out[a * G + g] = (double)pos[3 * j + a] + (double)o[a] * (double)base_scale[3 * j + a];")],
        ["decode biases"]),
    "opacity through a sigmoid": (
        [("      double op = tanh(ya[i]);", "      double op = sigm(ya[i]);")], ["decode biases"]),
    "quaternion left unnormalised": (
        [("out[(6 + a) * G + g] = qn > 0 ? q[a] / qn : (a == 0 ? 1.0 : 0.0);",
          "out[(6 + a) * G + g] = qn > 0 ? q[a] : (a == 0 ? 1.0 : 0.0);")], ["decode biases"]),
    "hidden layer without ReLU": (
        [("for (int h = 0; h < Wd; ++h) s += (hpre[h] > 0 ? hpre[h] : 0.0) * (double)w2[h * out + o];",
          "for (int h = 0; h < Wd; ++h) s += hpre[h] * (double)w2[h * out + o];")],
        ["decode inputs", "decode relu path"]),
    "dilation on one axis only": (
        [("a += pp->dilation; c += pp->dilation;", "a += pp->dilation;")], ["single Gaussian"]),
    "Jacobian depth term with the wrong sign": (
        [("double J00 = k->fx / zc, J02 = -k->fx * tx / (zc * zc);",
          "double J00 = k->fx / zc, J02 = k->fx * tx / (zc * zc);")], ["single Gaussian"]),
    "transmittance multiplied by alpha": (
        [("    T *= (1.0 - a);\n    if (T < pp->t_min) break;", "    T *= a;\n    if (T < pp->t_min) break;")],
        ["two Gaussians", "partition of unity"]),
    "background not attenuated": (
        [("for (int c = 0; c < 3; ++c) out[c] = C[c] + T * pp->bg[c];",
          "for (int c = 0; c < 3; ++c) out[c] = C[c] + pp->bg[c];")], ["two Gaussians"]),
    "level bias with the wrong sign": (
        [("double t = (double)d_max * exp2((double)lod_bias[j] - (double)level[j]);",
          "double t = (double)d_max * exp2(-(double)lod_bias[j] - (double)level[j]);")],
        ["thr2 closed form", "Eq. 7 literal"]),
    "colour behind an entry not divided by (1 - a)": (
        [("double dLda = Ti * cdot - bdot / (1.0 - a);", "double dLda = Ti * cdot - bdot;")],
        ["backward FD"]),
    "mean gradient with the cross term dropped": (
        [("d[0] = dpw * (p[2] * dx + p[3] * dy);", "d[0] = dpw * (p[2] * dx);")], ["backward FD"]),
    "blend weight after the transmittance update": (
        [("      w[list[i]] += wt;", "      w[list[i]] += wt * (1.0 - a);")], ["skip certificate"]),
}


def _plant(src, edits):
    for old, new in edits:
        assert src.count(old) >= 1, old
        src = src.replace(old, new)
    return src


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_a_pin_catches_the_mistake(orc, name):
    edits, pins = MISTAKES[name]
    src = _plant(orc.source(), edits)
    caught = []
    with tempfile.TemporaryDirectory() as d:
        with orc.variant(src, d, tag="m" + str(abs(hash(name)) % 10 ** 8)):
            for p in pins:
                try:
                    PINS[p](orc)
                except AssertionError:
                    caught.append(p)
    assert caught, f"no pin catches: {name}"


def test_the_unplanted_oracle_passes_every_pin(orc):
    for p in PINS.values():
        p(orc)


# ---- the Python oracles: a mistake is planted by replacing a module
# attribute (a constant or a function) for the duration of the check ----

def _explicit_pins(orc):
    import tests.test_oracle_explicit as TE
    from oracle import explicit as EX
    TE.test_sh_basis_matches_scipy(EX)
    TE.test_sh_low_order_closed_forms(EX)
    TE.test_decode_explicit_closed_forms(EX)


def _loss_pins(orc):
    import tests.test_oracle_losses as TL
    from oracle import losses as LO
    TL.test_ssim_matches_brute_force(LO)
    TL.test_ssim_constant_images_closed_form(LO)
    TL.test_photometric_gradient_fd(LO)


def _densify_pins(orc):
    import tests.test_oracle_densify as TD
    from oracle import densify as DO
    TD.test_level_thresholds(DO)


def _sh_norm_swapped(l, m):
    import math
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l + m) / math.factorial(l - m))


PY_MISTAKES = {
    "SH normalisation with (l - m)! and (l + m)! swapped": ("oracle.explicit", "_norm",
                                                           _sh_norm_swapped, _explicit_pins),
    "SSIM window of sigma 1.0": ("oracle.losses", "SSIM_SIGMA", 1.0, _loss_pins),
    "SSIM constants swapped": ("oracle.losses", "SSIM_C1", 0.03 ** 2, _loss_pins),
    "densification thresholds from 2^(-beta L)": (
        "oracle.densify", "level_thresholds",
        lambda tau_g, beta, n_levels: np.array(
            [float(np.float32(tau_g)) * np.exp2(-float(np.float32(beta)) * L)
             for L in range(n_levels + 1)]).astype(np.float32),
        _densify_pins),
}


@pytest.mark.parametrize("name", sorted(PY_MISTAKES))
def test_a_pin_catches_the_python_mistake(orc, monkeypatch, name):
    import importlib
    mod, attr, bad, pins = PY_MISTAKES[name]
    m = importlib.import_module(mod)
    pins(orc)  # the unmodified module passes
    monkeypatch.setattr(m, attr, bad)
    with pytest.raises(AssertionError):
        pins(orc)
