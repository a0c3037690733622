import pytest


def pytest_collection_modifyitems(config, items):
    for it in items:
        if "/gpu/" in str(it.fspath):
            it.add_marker(pytest.mark.gpu)
