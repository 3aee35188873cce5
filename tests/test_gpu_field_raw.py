"""GPU field arithmetic on its internal representation (nine 29-bit limbs,
Montgomery R = 2^261), checked against exact integer arithmetic through the
library's raw-limb diagnostic kernel (cases in field_cases.py)."""
import pytest

import field_cases as FC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_14497_amd import pcmm
    pcmm.lib()
    return pcmm


def test_raw_field_ops_vs_integers(dev):
    FC.check_raw_field_ops(dev.diag_field_raw)


def test_raw_products_of_extreme_carry_only_operands(dev):
    """The products that take a doubled operand (limbs < 2^30) and a
    subtracted product: operands carry-only below 4p with limbs 0..7 at or
    near 2^29 - 1, the largest column sums their bounds allow."""
    FC.check_extreme_carry_only_products(dev.diag_field_raw)


def test_loose_quotient_products(dev):
    """Products with loose quotient digits (the accumulation's mixed
    addition): random normal operands and carry-only operands at the largest
    limbs their bounds allow; exact value and normal form."""
    FC.check_loose_quotient_products(dev.diag_field_raw)


def test_raw_normalisation_of_signed_limbs(dev):
    FC.check_signed_limb_normalisation(dev.diag_field_raw)


def test_inversion_by_divsteps(dev):
    """fe_inv (divsteps) on the GPU: the modular inverse in Montgomery form on
    edge values, carry-only extremes and random operands below 4p, equal to
    the Fermat chain's result."""
    FC.check_inversion(dev.diag_field_raw)
