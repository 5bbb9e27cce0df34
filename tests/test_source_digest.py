"""The digest that ties measured figures (profiles/) to the kernels: comments
and layout do not change it, code does."""
from paper_2001_01570_amd import build as B


def test_comments_and_layout_do_not_change_the_code_tokens():
    a = 'int f(int x) {  // the "y" isn\'t used\n  return x * 2; /* twice */ }\n'
    b = 'int f(int x)\n{\n  return x * 2;\n}  // reformatted\n'
    assert B.code_tokens(a) == B.code_tokens(b)


def test_code_and_literals_change_the_code_tokens():
    assert B.code_tokens('x = 2;') != B.code_tokens('x = 3;')
    assert B.code_tokens('s = "a // b";') != B.code_tokens('s = "a";')
    assert B.code_tokens("c = '/';") == "c = '/';"


def test_digest_is_stable():
    assert B.source_digest() == B.source_digest()
    assert len(B.source_digest()) == 16
