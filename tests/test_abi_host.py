"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/pic.h declares, the binding names the same set, and
pic_create rejects invalid arguments before touching the device."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("pic_create", "pic_load_particles", "pic_step", "pic_get_fields",
                     "pic_get_particles"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1608_01009_amd import pic
    L = pic.library()
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(pic.ABI_SYMBOLS) == _declared()


def _create(**kw):
    from paper_1608_01009_amd import pic
    args = dict(n=(8, 8, 8), dx=(1.0, 1.0, 1.0), dt=0.25, species=[(-1.0, 1.0, 0.1, 100)],
                supercell=4, rebin_every=20)
    args.update(kw)
    n, dx, dt, sp = args.pop("n"), args.pop("dx"), args.pop("dt"), args.pop("species")
    return pic.pic_create(n, dx, dt, sp, **args)


@pytest.mark.parametrize("kw,needle", [
    (dict(dt=0.6), "Courant"),
    (dict(dt=-1.0), "dt"),
    (dict(dt=float("nan")), "dt"),
    (dict(n=(8, 8, 6)), "multiple of supercell"),
    (dict(n=(0, 8, 8)), ">= 1"),
    (dict(supercell=0), "supercell"),
    (dict(supercell=7, n=(7, 7, 7)), "LDS"),
    (dict(rebin_every=0), "rebin_every"),
    (dict(dx=(1.0, 0.0, 1.0)), "dx"),
    (dict(species=[(-1.0, 0.0, 0.1, 10)]), "mass"),
    (dict(species=[(-1.0, 1.0, -0.1, 10)]), "weight"),
    (dict(species=[(-1.0, 1.0, 0.1, -1)]), "capacity"),
    (dict(species=[(-1.0, 1.0, 0.1, 1 << 29)]), "capacity"),     # 32-bit byte offsets
    (dict(n=(2048, 1024, 1024), dt=0.25), "grid too large"),
    (dict(species=[(1e-280, 1.0, 0.1, 10)]), "charge dt"),
    (dict(precision=2), "precision"),
    (dict(precision="mixed", n=(2048, 8, 8)), "1024 cells"),
    (dict(species=[(-1.0, 1e-280, 0.1, 10)]), "charge dt"),
    (dict(species=[]), "n_species"),
    (dict(bc_x=2), "bc_x"),
    (dict(bc_x="absorbing", precision="mixed"), "PIC_BC_ABSORBING"),
    (dict(bc_x="absorbing", deterministic_j=True), "PIC_BC_ABSORBING"),
    (dict(bc_x="absorbing", supercell=1), "supercell 2 or 4"),
])
def test_create_rejects_invalid_arguments(kw, needle):
    from paper_1608_01009_amd import pic
    with pytest.raises(pic.PicError) as ei:
        _create(**kw)
    assert ei.value.code == pic.PIC_EINVAL
    assert needle in ei.value.message
    assert needle in pic.pic_last_error(None)


def test_courant_limit_is_inclusive_of_rounding():
    # dt exactly at the limit passes validation (it then needs a device, so
    # only the validation outcome is checked: any error must not be EINVAL)
    from paper_1608_01009_amd import pic
    lim = 1.0 / math.sqrt(3.0)
    try:
        ctx = _create(dt=lim)
    except pic.PicError as e:
        assert e.code != pic.PIC_EINVAL, e
    else:
        pic.pic_destroy(ctx)


def test_null_context_calls_are_rejected():
    from paper_1608_01009_amd import pic
    L = pic.library()
    assert L.pic_step(None, 1) == pic.PIC_EINVAL
    assert L.pic_set_fields(None, None) == pic.PIC_EINVAL
    L.pic_destroy(None)   # ignored
