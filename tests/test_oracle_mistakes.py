"""Planted mistakes: each entry edits a copy of the oracle's C source the way
a plausible slip would (a dropped term, a wrong sign, a swapped operand) and
checks that at least one of the listed pins, which never reuse the oracle's
own formulas, now fails.  A mistake no pin catches would be a gap in the
pins.  CPU only: the copies are built with gcc into a temporary directory."""

import tempfile

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
