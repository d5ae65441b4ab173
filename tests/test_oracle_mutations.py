"""The oracle's pins catch plausible mistakes (CPU only).

Each case copies the oracle's C source, plants one mistake by a textual
substitution, compiles the copy into a temporary directory and checks that
at least one pin fails against it (and that the same pins pass against the
unmodified oracle, which the pin tests themselves establish). Nothing here
touches the GPU library.
"""
import pytest

import oracle
from tests import test_oracle_pins as P

# (name, text in cloak_oracle.c, replacement, pins that must catch it)
MUTATIONS = [
    ("bottom cap normal points into the cloak",
     "if (surf == SURF_BOTTOM || surf == EV_BOTTOM) { n[0] = 0; n[1] = 0; n[2] = -1; return; }",
     "if (surf == SURF_BOTTOM || surf == EV_BOTTOM) { n[0] = 0; n[1] = 0; n[2] = 1; return; }",
     (P.test_finite_radial_ordinary_caps_closed_form, P.test_finite_azimuthal_extraordinary_caps_closed_form)),
    ("total internal reflection about the radial normal on every surface",
     "        if (w) *w *= Rref[branch];\n        reflect(y + 3, nn);",
     "        if (w) *w *= Rref[branch];\n        outward_normal(SURF_SIDE, y, nn);\n        reflect(y + 3, nn);",
     (P.test_finite_radial_ordinary_caps_closed_form, P.test_finite_azimuthal_extraordinary_caps_closed_form)),
    ("entry through the top cap accepted only over the metal disk's radius",
     "        if (s > 0.0 && x * x + y * y <= c->b * c->b && s < best) {\n            best = s; *surf = SURF_TOP;",
     "        if (s > 0.0 && x * x + y * y <= c->a * c->a && s < best) {\n            best = s; *surf = SURF_TOP;",
     (P.test_finite_radial_ordinary_caps_closed_form, P.test_finite_azimuthal_extraordinary_caps_closed_form)),
    ("Hamiltonian drift not checked at outer interfaces",
     "if (!(fabs(hamiltonian(c, branch, y) - 1.0) <= 1e-3)) { status = ORC_DIVERGED; break; }",
     "",
     (P.test_diverged_rule_at_outer_interfaces,)),
    ("goggle axes swapped",
     "    if (goggle == 0) {\n        memcpy(e, a, sizeof(a));",
     "    if (goggle != 0) {\n        memcpy(e, a, sizeof(a));",
     (P.test_goggle_axes_are_an_orthonormal_pair_along_the_camera_frame,
      P.test_inplane_goggle_passes_the_design_polarization_on_the_centre_row)),
    ("polarized entry always takes the s wave",
     "    zc Ei[3] = { e[0] / l, e[1] / l, e[2] / l };",
     "    zc Ei[3] = { w.s[0], w.s[1], w.s[2] };",
     (P.test_polarized_entry_is_textbook_fresnel_with_the_mixing_angle,
      P.test_polarized_entry_conserves_energy_and_averages_to_unpolarized)),
    ("goggle weight of a crystal path without the polarizer's half",
     "            else if (st == ORC_EXITED) wi = 0.5 * w;",
     "            else if (st == ORC_EXITED) wi = w;",
     (P.test_goggle_images_split_the_unpolarized_image,
      P.test_inplane_goggle_passes_the_design_polarization_on_the_centre_row)),
    ("reflected child followed in the other mode's medium",
     "            int sc = crystal_walk(c, bp, o, yc, &tc, &nc, &wc, NULL, rf->p_child[bp], rf->d_child[bp], &hc);",
     "            int sc = crystal_walk(c, 1 - bp, o, yc, &tc, &nc, &wc, NULL, rf->p_child[bp], rf->d_child[bp], &hc);",
     (P.test_first_order_reflection_of_the_radial_ordinary_ray_closed_form,)),
    ("reflected child without its exit transmission",
     "            int sc = crystal_walk(c, bp, o, yc, &tc, &nc, &wc, NULL, rf->p_child[bp], rf->d_child[bp], &hc);",
     "            int sc = crystal_walk(c, bp, o, yc, &tc, &nc, NULL, NULL, rf->p_child[bp], rf->d_child[bp], &hc);",
     (P.test_first_order_reflection_of_the_radial_ordinary_ray_closed_form,)),
    ("canonical Hamiltonian keeps the polynomial form's f",
     "        *f = dk(1.0);\n",
     "",
     (lambda: P.test_canonical_hamiltonian_cloaks_inplane_rays_and_is_singular_at_the_axis(0),)),
    ("step growth capped at 4 instead of 5",
     "    else fac = fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));",
     "    else fac = fmin(4.0, fmax(0.2, 0.9 * pow(err, -0.2)));",
     (P.test_dp45_controller_on_straight_chords,)),
    ("hmax ignored by the step controller",
     "            h_next = fmin(h * dp45_factor(err, after_reject), o->hmax);",
     "            h_next = h * dp45_factor(err, after_reject);",
     (P.test_dp45_controller_on_straight_chords,)),
    ("entry reflection weighted by the transmitted fraction",
     "            rf->w_ext = Rin;",
     "            rf->w_ext = Tin[branch];",
     (P.test_entry_reflection_is_the_fresnel_remainder,)),
]


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(name, old, new, pins, tmp_path):
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation site not unique: {name}"
    path = oracle.build_variant(src.replace(old, new), str(tmp_path))
    caught = []
    with oracle.use_library(path):
        for pin in pins:
            try:
                pin()
            except AssertionError:
                caught.append(pin.__name__)
    assert caught, f"no pin caught: {name}"
